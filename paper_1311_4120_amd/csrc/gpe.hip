// Time-splitting driver for the Gross-Pitaevskii / Schroedinger-Poisson
// equation, the application that evaluates the potential of eq. gpe many times
// for a changing rho = |psi|^2 (Section 1):
//
//   i psi_t = [-1/2 Lap + V + beta |psi|^2 + lambda Phi] psi,   Phi = U * |psi|^2.
//
// One step is Strang splitting: N(dt/2), K(dt), N(dt/2), with
//   N(h): psi <- exp(-i h (V + beta |psi|^2 + lambda Phi)) psi   (|psi| unchanged)
//   K(h): psi <- IDFT(exp(-i h |k|^2 / 2) DFT(psi)),  k_j = 2 pi q_j / R_j,
// the Laplacian periodic on the box.  Phi comes from the plan's potential
// pipeline; since N keeps |psi|, the Phi of a step's second half-step serves
// the next step's first, one evaluation per step.  In imaginary time the
// factors lose their i, Phi is evaluated before each half-step and psi is
// renormalised to H sum |psi|^2 = 1 after every step.  One step is captured in
// a HIP graph and replayed, so a call of many steps costs one launch per step.
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "common.h"

namespace jgb {

Status validate(const jgb_params* p);

namespace {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {
  T x, y;
};

constexpr int kSumBlocks = 1024;  // blocks of the reduction kernels (fixed, so sums are deterministic)
constexpr int kSums = 4;          // sum |psi|^2, sum V |psi|^2, sum |psi|^4, sum Phi |psi|^2

struct Grid {
  int n0, n1, n2;
  FastDiv d12, d2;
  uint32_t npts;
  double x0[3], h[3];   // first coordinate and spacing per internal axis (unit axis: 0, 0)
  double g2[3];         // trap: gamma_a^2 per internal axis (V = sum g2 x^2 / 2)
};

__device__ inline void coords(const Grid& g, uint32_t i, int& i0, int& i1, int& i2) {
  i0 = (int)g.d12.div(i);
  const uint32_t r = i - (uint32_t)i0 * (uint32_t)(g.n1 * g.n2);
  i1 = (int)g.d2.div(r);
  i2 = (int)(r - (uint32_t)i1 * g.n2);
}

template <typename T>
__device__ inline double trap_at(const Grid& g, const T* V, uint32_t i) {
  if (V) return (double)V[i];
  int i0, i1, i2;
  coords(g, i, i0, i1, i2);
  const double x = g.x0[0] + i0 * g.h[0], y = g.x0[1] + i1 * g.h[1], z = g.x0[2] + i2 * g.h[2];
  return 0.5 * (g.g2[0] * x * x + g.g2[1] * y * y + g.g2[2] * z * z);
}

// N(h): psi <- exp(-i h theta) psi (real time) or exp(-h theta) psi (imaginary
// time), theta = V + beta |psi|^2 + lambda Phi; writes rho = |psi|^2 of the
// result when rho != nullptr.
template <typename T>
__global__ void __launch_bounds__(256) k_gpe_local(Grid g, C2<T>* psi, const T* phi, const T* V, double beta,
                                                   double lam, double h, int imaginary, T* rho) {
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < g.npts; i += gridDim.x * 256u) {
    C2<T> p = psi[i];
    const double a2 = (double)p.x * p.x + (double)p.y * p.y;
    const double theta = trap_at(g, V, i) + beta * a2 + lam * (double)phi[i];
    double fr, fi;
    if (imaginary) {
      fr = exp(-h * theta);
      fi = 0.0;
    } else {
      sincos(-h * theta, &fi, &fr);
    }
    const double re = fr * p.x - fi * p.y, im = fr * p.y + fi * p.x;
    p.x = (T)re;
    p.y = (T)im;
    psi[i] = p;
    if (rho) rho[i] = (T)(re * re + im * im);
  }
}

// Per-block partial sums of |psi|^2, V |psi|^2, |psi|^4 and Phi |psi|^2
// (phi may be null: that sum is 0), in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256) k_gpe_sums(Grid g, const C2<T>* psi, const T* phi, const T* V,
                                                  double* parts) {
  double s[kSums] = {0.0, 0.0, 0.0, 0.0};
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < g.npts; i += gridDim.x * 256u) {
    const C2<T> p = psi[i];
    const double a2 = (double)p.x * p.x + (double)p.y * p.y;
    s[0] += a2;
    s[1] += trap_at(g, V, i) * a2;
    s[2] += a2 * a2;
    if (phi) s[3] += (double)phi[i] * a2;
  }
  __shared__ double ws[kSums][4];
  for (int q = 0; q < kSums; ++q) {
    double v = s[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) ws[q][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < kSums)
    parts[threadIdx.x * kSumBlocks + blockIdx.x] =
        ((ws[threadIdx.x][0] + ws[threadIdx.x][1]) + ws[threadIdx.x][2]) + ws[threadIdx.x][3];
}

// Per-block partial sums of |k|^2 |DFT(psi)|^2.
template <typename T>
__global__ void __launch_bounds__(256) k_gpe_kin_sums(Grid g, const C2<T>* ph, const double* kt, int off1,
                                                      int off2, double* parts) {
  double s = 0.0;
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < g.npts; i += gridDim.x * 256u) {
    int i0, i1, i2;
    coords(g, i, i0, i1, i2);
    const double k0 = kt[i0], k1 = kt[off1 + i1], k2 = kt[off2 + i2];
    const C2<T> p = ph[i];
    s += (k0 * k0 + k1 * k1 + k2 * k2) * ((double)p.x * p.x + (double)p.y * p.y);
  }
  __shared__ double ws[4];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) parts[kSums * kSumBlocks + blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

// Sums of the partials (one block, fixed order) into
// out = {norm, kinetic, trap, local, nonlocal, total, mu} (mode 1) or out[0] =
// norm (mode 0).
__global__ void __launch_bounds__(256) k_gpe_finalize(const double* parts, int nsums, double H, double beta,
                                                      double lam, double inv_n, int mode, double* out) {
  __shared__ double red[256];
  __shared__ double tot[kSums + 1];
  for (int q = 0; q < nsums; ++q) {
    double v = 0.0;
    for (int b = threadIdx.x; b < kSumBlocks; b += 256) v += parts[q * kSumBlocks + b];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) tot[q] = red[0];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double nrm = H * tot[0];
  if (mode == 0) {
    out[0] = nrm;
    return;
  }
  const double etrap = H * tot[1], eloc = 0.5 * beta * H * tot[2], enl = 0.5 * lam * H * tot[3];
  const double ekin = 0.5 * H * inv_n * tot[4];
  out[0] = nrm;
  out[1] = ekin;
  out[2] = etrap;
  out[3] = eloc;
  out[4] = enl;
  out[5] = ekin + etrap + eloc + enl;
  out[6] = (ekin + etrap + 2.0 * eloc + 2.0 * enl) / nrm;
}

// psi <- psi / sqrt(norm), norm = *nrm (imaginary-time renormalisation).
template <typename T>
__global__ void __launch_bounds__(256) k_gpe_scale(Grid g, C2<T>* psi, const double* nrm) {
  const T f = (T)(1.0 / sqrt(*nrm));
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < g.npts; i += gridDim.x * 256u) {
    C2<T> p = psi[i];
    psi[i] = C2<T>{p.x * f, p.y * f};
  }
}

}  // namespace
}  // namespace jgb

using jgb::Plan;

struct jgb_gpe_s {
  jgb_plan_s* plan = nullptr;      // the potential's plan, on the driver's own stream
  hipStream_t caller = nullptr;    // params.potential.stream
  hipStream_t st = nullptr;        // the driver's stream (graphs are captured on it)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int device = 0;
  double beta = 0, lam = 0, dt = 0;
  int imaginary = 0;
  const void* V = nullptr;
  jgb::Grid g{};
  void* rho = nullptr;             // |psi|^2, real
  void* phi = nullptr;             // U * |psi|^2, real
  void* work = nullptr;            // complex copy of psi for the kinetic energy
  void* tw[3] = {nullptr, nullptr, nullptr};  // exp(-2 pi i t / n_a)
  double* kt = nullptr;            // k_a(q) per axis, concatenated
  int koff[3] = {0, 0, 0};
  double* parts = nullptr;         // (kSums + 1) x kSumBlocks partial sums
  double* nrm = nullptr;           // renormalisation: H sum |psi|^2
  std::vector<void*> allocations;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* graph_psi = nullptr;       // the psi the graph was captured for
};

namespace {

jgb_status gpe_report(jgb_status code, const std::string& msg) {
  if (code != JGB_OK) jgb::set_error(msg);
  return code;
}

jgb_status gpe_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return JGB_OK;
  (void)hipGetLastError();
  return gpe_report(JGB_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

unsigned blocks_for(uint32_t n) {
  unsigned b = (n + 255u) / 256u;
  return b < (unsigned)jgb::kSumBlocks ? (b ? b : 1u) : (unsigned)jgb::kSumBlocks;
}

void release_gpe(jgb_gpe_s* q) {
  (void)hipSetDevice(q->device);
  if (q->st) (void)hipStreamSynchronize(q->st);
  if (q->exec) (void)hipGraphExecDestroy(q->exec);
  if (q->graph) (void)hipGraphDestroy(q->graph);
  for (void* p : q->allocations) (void)hipFree(p);
  if (q->plan) (void)jgb_destroy(q->plan);
  if (q->ev_in) (void)hipEventDestroy(q->ev_in);
  if (q->ev_out) (void)hipEventDestroy(q->ev_out);
  if (q->st) (void)hipStreamDestroy(q->st);
  delete q;
}

template <typename P>
hipError_t gpe_alloc(jgb_gpe_s* q, P** ptr, size_t bytes) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes ? bytes : 16);
  if (e != hipSuccess) return e;
  q->allocations.push_back(p);
  *ptr = (P*)p;
  return hipSuccess;
}

template <typename T>
jgb_status enqueue_potential(jgb_gpe_s* q, const void* psi) {
  Plan& pl = q->plan->pl;
  hipError_t e = jgb::launch_density<T>(pl, psi, q->rho, q->st);
  if (e != hipSuccess) return gpe_hip(e, "density");
  return jgb::potential_pipeline(pl, q->rho, q->phi, nullptr, q->st);
}

template <typename T>
jgb_status enqueue_local(jgb_gpe_s* q, void* psi, double h, bool write_rho) {
  const unsigned nb = blocks_for(q->g.npts);
  hipLaunchKernelGGL(jgb::k_gpe_local<T>, dim3(nb), dim3(256), 0, q->st, q->g, (jgb::C2<T>*)psi,
                     (const T*)q->phi, (const T*)q->V, q->beta, q->lam, h, q->imaginary,
                     write_rho ? (T*)q->rho : (T*)nullptr);
  return gpe_hip(hipGetLastError(), "local step");
}

template <typename T>
jgb_status enqueue_kinetic(jgb_gpe_s* q, void* psi, double h) {
  Plan& pl = q->plan->pl;
  hipError_t e = jgb::launch_fft_periodic_kinetic<T>(pl, q->tw, psi, q->kt, q->koff, h, q->imaginary,
                                                     1.0 / (double)q->g.npts, q->st);
  return gpe_hip(e, "kinetic step");
}

// One Strang step, enqueued on q->st (the captured body of the graph).  Real
// time expects Phi of the current |psi|^2 in q->phi and leaves it so.
template <typename T>
jgb_status enqueue_step(jgb_gpe_s* q, void* psi) {
  const double h = 0.5 * q->dt;
  jgb_status c;
  if (!q->imaginary) {
    if ((c = enqueue_local<T>(q, psi, h, false)) != JGB_OK) return c;
    if ((c = enqueue_kinetic<T>(q, psi, q->dt)) != JGB_OK) return c;
    if ((c = enqueue_potential<T>(q, psi)) != JGB_OK) return c;
    return enqueue_local<T>(q, psi, h, false);
  }
  if ((c = enqueue_potential<T>(q, psi)) != JGB_OK) return c;
  if ((c = enqueue_local<T>(q, psi, h, false)) != JGB_OK) return c;
  if ((c = enqueue_kinetic<T>(q, psi, q->dt)) != JGB_OK) return c;
  if ((c = enqueue_potential<T>(q, psi)) != JGB_OK) return c;
  if ((c = enqueue_local<T>(q, psi, h, false)) != JGB_OK) return c;
  const unsigned nb = blocks_for(q->g.npts);
  const Plan& pl = q->plan->pl;
  // the sums always run kSumBlocks blocks: the finalize reads every partial
  hipLaunchKernelGGL(jgb::k_gpe_sums<T>, dim3(jgb::kSumBlocks), dim3(256), 0, q->st, q->g, (const jgb::C2<T>*)psi,
                     (const T*)nullptr, (const T*)q->V, q->parts);
  hipLaunchKernelGGL(jgb::k_gpe_finalize, dim3(1), dim3(256), 0, q->st, q->parts, 1, pl.H, q->beta, q->lam, 0.0,
                     0, q->nrm);
  hipLaunchKernelGGL(jgb::k_gpe_scale<T>, dim3(nb), dim3(256), 0, q->st, q->g, (jgb::C2<T>*)psi,
                     (const double*)q->nrm);
  return gpe_hip(hipGetLastError(), "renormalisation");
}

template <typename T>
jgb_status capture_step(jgb_gpe_s* q, void* psi) {
  if (q->exec) (void)hipGraphExecDestroy(q->exec);
  if (q->graph) (void)hipGraphDestroy(q->graph);
  q->exec = nullptr;
  q->graph = nullptr;
  q->graph_psi = nullptr;
  hipError_t e = hipStreamBeginCapture(q->st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return gpe_hip(e, "begin capture");
  jgb_status c = enqueue_step<T>(q, psi);
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(q->st, &g);
  if (c != JGB_OK || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return c != JGB_OK ? c : gpe_hip(ee, "end capture");
  }
  q->graph = g;
  e = hipGraphInstantiate(&q->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    q->graph = nullptr;
    return gpe_hip(e, "graph instantiate");
  }
  q->graph_psi = psi;
  return JGB_OK;
}

template <typename T>
jgb_status run_steps(jgb_gpe_s* q, void* psi, int nsteps, int use_graph) {
  jgb_status c;
  if (!q->imaginary && (c = enqueue_potential<T>(q, psi)) != JGB_OK) return c;
  if (use_graph && (q->graph_psi != psi || !q->exec) && (c = capture_step<T>(q, psi)) != JGB_OK) return c;
  for (int s = 0; s < nsteps; ++s) {
    if (use_graph) {
      hipError_t e = hipGraphLaunch(q->exec, q->st);
      if (e != hipSuccess) return gpe_hip(e, "graph launch");
    } else if ((c = enqueue_step<T>(q, psi)) != JGB_OK) {
      return c;
    }
  }
  return JGB_OK;
}

template <typename T>
jgb_status run_energy(jgb_gpe_s* q, const void* psi, double* out) {
  jgb_status c = enqueue_potential<T>(q, psi);
  if (c != JGB_OK) return c;
  hipLaunchKernelGGL(jgb::k_gpe_sums<T>, dim3(jgb::kSumBlocks), dim3(256), 0, q->st, q->g, (const jgb::C2<T>*)psi,
                     (const T*)q->phi, (const T*)q->V, q->parts);
  hipError_t e = hipMemcpyAsync(q->work, psi, (size_t)q->g.npts * 2 * sizeof(T), hipMemcpyDeviceToDevice, q->st);
  if (e != hipSuccess) return gpe_hip(e, "copy");
  const Plan& pl = q->plan->pl;
  if ((e = jgb::launch_fft_periodic<T>(pl, q->tw, q->work, -1, q->st)) != hipSuccess) return gpe_hip(e, "FFT");
  hipLaunchKernelGGL(jgb::k_gpe_kin_sums<T>, dim3(jgb::kSumBlocks), dim3(256), 0, q->st, q->g, (const jgb::C2<T>*)q->work,
                     q->kt, q->koff[1], q->koff[2], q->parts);
  hipLaunchKernelGGL(jgb::k_gpe_finalize, dim3(1), dim3(256), 0, q->st, q->parts, jgb::kSums + 1, pl.H, q->beta,
                     q->lam, 1.0 / (double)q->g.npts, 1, out);
  return gpe_hip(hipGetLastError(), "energy sums");
}

// order q->st after the caller's stream, and the caller after q->st
jgb_status enter(jgb_gpe_s* q) {
  hipError_t e = hipSetDevice(q->device);
  if (e == hipSuccess) e = hipEventRecord(q->ev_in, q->caller);
  if (e == hipSuccess) e = hipStreamWaitEvent(q->st, q->ev_in, 0);
  return gpe_hip(e, "stream ordering");
}

jgb_status leave(jgb_gpe_s* q) {
  hipError_t e = hipEventRecord(q->ev_out, q->st);
  if (e == hipSuccess) e = hipStreamWaitEvent(q->caller, q->ev_out, 0);
  return gpe_hip(e, "stream ordering");
}

}  // namespace

extern "C" {

jgb_status jgb_gpe_create(const jgb_gpe_params* params, jgb_gpe_t* out) {
  jgb::set_error("");
  if (!out) return gpe_report(JGB_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!params) return gpe_report(JGB_ERR_INVALID_ARG, "params is NULL");
  if (params->struct_size != sizeof(jgb_gpe_params))
    return gpe_report(JGB_ERR_INVALID_ARG, "params.struct_size != sizeof(jgb_gpe_params)");
  if (!std::isfinite(params->dt) || params->dt == 0.0) return gpe_report(JGB_ERR_INVALID_ARG, "dt must be finite and nonzero");
  if (!std::isfinite(params->beta)) return gpe_report(JGB_ERR_INVALID_ARG, "beta must be finite");
  if (params->imaginary != 0 && params->imaginary != 1) return gpe_report(JGB_ERR_INVALID_ARG, "imaginary must be 0 or 1");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(params->trap[i])) return gpe_report(JGB_ERR_INVALID_ARG, "trap must be finite");
  {
    // the potential's parameters are checked before any device work
    jgb::Status v = jgb::validate(&params->potential);
    if (v.code != JGB_OK) return gpe_report(v.code, "potential plan: " + v.msg);
  }
  jgb_gpe_s* q = new (std::nothrow) jgb_gpe_s();
  if (!q) return gpe_report(JGB_ERR_OUT_OF_MEMORY, "host allocation failed");
  q->device = params->potential.device;
  q->caller = (hipStream_t)params->potential.stream;
  q->beta = params->beta;
  q->lam = params->potential.lambda;
  q->dt = params->dt;
  q->imaginary = params->imaginary;
  q->V = params->V;
  hipError_t e = hipSetDevice(q->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&q->st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&q->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&q->ev_out, hipEventDisableTiming);
  if (e != hipSuccess) {
    jgb_status s = gpe_hip(e, "stream and events");
    release_gpe(q);
    return s;
  }
  jgb_params pp = params->potential;
  pp.stream = q->st;
  jgb_status s = jgb_plan(&pp, &q->plan);
  if (s != JGB_OK) {
    std::string msg = std::string("potential plan: ") + jgb_last_error();
    release_gpe(q);
    return gpe_report(s, msg);
  }
  const Plan& pl = q->plan->pl;
  jgb::Grid& g = q->g;
  g.n0 = pl.n[0];
  g.n1 = pl.n[1];
  g.n2 = pl.n[2];
  g.d12 = jgb::FastDiv((uint32_t)(g.n1 * g.n2));
  g.d2 = jgb::FastDiv((uint32_t)g.n2);
  g.npts = (uint32_t)((int64_t)g.n0 * g.n1 * g.n2);
  // internal axes: 3D (x1, x2, x3) -> (a0, a1, a2); 2D (x1, x2) -> (a1, a2)
  const int first = (pl.dim == 3) ? 0 : 1;
  for (int a = 0; a < 3; ++a) {
    const bool phys = a >= first;
    g.h[a] = phys ? pl.h[a] : 0.0;
    g.x0[a] = phys ? -0.5 * pl.box[a] : 0.0;
    const double gam = phys ? params->trap[a - first] : 0.0;
    g.g2[a] = gam * gam;
  }
  const size_t rb = pl.real_bytes;
  e = gpe_alloc(q, &q->rho, g.npts * rb);
  if (e == hipSuccess) e = gpe_alloc(q, &q->phi, g.npts * rb);
  if (e == hipSuccess) e = gpe_alloc(q, &q->work, g.npts * 2 * rb);
  if (e == hipSuccess) e = gpe_alloc(q, &q->parts, sizeof(double) * (jgb::kSums + 1) * jgb::kSumBlocks);
  if (e == hipSuccess) e = gpe_alloc(q, &q->nrm, sizeof(double));
  // per-axis tables: twiddles for the periodic FFT and the wavenumbers
  std::vector<double> kt;
  for (int a = 0; a < 3 && e == hipSuccess; ++a) {
    const int L = pl.n[a];
    q->koff[a] = (int)kt.size();
    for (int t = 0; t < L; ++t) {
      const int sq = (t < (L + 1) / 2) ? t : t - L;
      kt.push_back(L > 1 ? 2.0 * M_PI * sq / pl.box[a] : 0.0);
    }
    std::vector<double> twd(2 * L);
    for (int t = 0; t < L; ++t) {
      twd[2 * t] = std::cos(2.0 * M_PI * t / L);
      twd[2 * t + 1] = -std::sin(2.0 * M_PI * t / L);
    }
    if (pl.fp64) {
      e = gpe_alloc(q, &q->tw[a], sizeof(double) * 2 * L);
      if (e == hipSuccess) e = hipMemcpy(q->tw[a], twd.data(), sizeof(double) * 2 * L, hipMemcpyHostToDevice);
    } else {
      std::vector<float> twf(twd.begin(), twd.end());
      e = gpe_alloc(q, &q->tw[a], sizeof(float) * 2 * L);
      if (e == hipSuccess) e = hipMemcpy(q->tw[a], twf.data(), sizeof(float) * 2 * L, hipMemcpyHostToDevice);
    }
  }
  if (e == hipSuccess) e = gpe_alloc(q, &q->kt, sizeof(double) * kt.size());
  if (e == hipSuccess) e = hipMemcpy(q->kt, kt.data(), sizeof(double) * kt.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    jgb_status st = (e == hipErrorOutOfMemory) ? gpe_report(JGB_ERR_OUT_OF_MEMORY, "device allocation failed")
                                               : gpe_hip(e, "driver tables");
    release_gpe(q);
    return st;
  }
  *out = q;
  return JGB_OK;
}

jgb_status jgb_gpe_step(jgb_gpe_t q, void* psi, int nsteps, int use_graph) {
  if (!q) return gpe_report(JGB_ERR_INVALID_ARG, "driver is NULL");
  if (!psi) return gpe_report(JGB_ERR_INVALID_ARG, "psi is NULL");
  if (nsteps < 0) return gpe_report(JGB_ERR_INVALID_ARG, "nsteps must be >= 0");
  if (use_graph != 0 && use_graph != 1) return gpe_report(JGB_ERR_INVALID_ARG, "use_graph must be 0 or 1");
  if (nsteps == 0) return JGB_OK;
  jgb_status c = enter(q);
  if (c != JGB_OK) return c;
  c = q->plan->pl.fp64 ? run_steps<double>(q, psi, nsteps, use_graph) : run_steps<float>(q, psi, nsteps, use_graph);
  jgb_status l = leave(q);
  return c != JGB_OK ? c : l;
}

jgb_status jgb_gpe_energy(jgb_gpe_t q, const void* psi, double* out) {
  if (!q) return gpe_report(JGB_ERR_INVALID_ARG, "driver is NULL");
  if (!psi || !out) return gpe_report(JGB_ERR_INVALID_ARG, "psi and out must not be NULL");
  jgb_status c = enter(q);
  if (c != JGB_OK) return c;
  c = q->plan->pl.fp64 ? run_energy<double>(q, psi, out) : run_energy<float>(q, psi, out);
  jgb_status l = leave(q);
  return c != JGB_OK ? c : l;
}

jgb_status jgb_gpe_destroy(jgb_gpe_t q) {
  if (!q) return JGB_OK;
  release_gpe(q);
  return JGB_OK;
}

}  // extern "C"
