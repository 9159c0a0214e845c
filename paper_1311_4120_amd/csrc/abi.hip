// extern "C" entry points declared in include/jgb.h.  Each call checks its
// arguments, makes the plan's device current, enqueues kernels on the plan's
// stream and converts every failure into a status code and a thread-local
// message.  Nothing is thrown across the ABI.
#include <cmath>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>
#include <string>

#include "common.h"

namespace jgb {

Status validate(const jgb_params* p);
Status build_plan(Plan& pl, const jgb_params* p);
void free_plan(Plan& pl);

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

std::vector<LaunchRecord>*& launch_record() {
  thread_local std::vector<LaunchRecord>* rec = nullptr;
  return rec;
}
const char* get_error() { return g_last_error.c_str(); }

}  // namespace jgb

using jgb::Plan;


struct jgb_batch_s {
  std::vector<jgb_plan_s*> plans;
  hipStream_t stream = nullptr;           // the caller's stream (params[0].stream), may be the NULL stream
  std::vector<hipStream_t> branches;      // streams owned by the batch; the graph is captured on branch 0
  std::vector<hipEvent_t> events;         // fork + one join event per extra branch
  hipEvent_t ev_in = nullptr;             // caller stream -> batch, batch -> caller ordering
  hipEvent_t ev_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
  void* d_tables = nullptr;               // argument tables of the batched launches
  int nlaunch = 0;                        // launches in the graph (0: per-member branches)
};

namespace {

jgb_status report(jgb_status code, const std::string& msg) {
  if (code != JGB_OK) jgb::set_error(msg);
  return code;
}

jgb_status from_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return JGB_OK;
  return report(JGB_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + nb && y < x + na;
}

size_t grid_bytes(const Plan& pl) {
  return (size_t)pl.n[0] * pl.n[1] * pl.n[2] * pl.real_bytes;
}

// Forward FFT and, for Algorithm 2, the separation of the type-2 spectrum
// into the tiles the interpolation reads.
template <typename T>
jgb_status run_forward(Plan& pl, const void* rho, hipStream_t st) {
  hipError_t e;
  if ((e = jgb::launch_fft_forward<T>(pl, (const T*)rho, st)) != hipSuccess) return from_hip(e, "forward FFT");
  if (pl.c0 != 0.0 && (e = jgb::launch_origin(pl, st)) != hipSuccess) return from_hip(e, "origin node");
  if (pl.split && (e = jgb::launch_split_unmix<T>(pl, st)) != hipSuccess) return from_hip(e, "split separation");
  return JGB_OK;
}

template <typename T>
jgb_status run_potential(Plan& pl, const void* rho, void* u, double* energy, hipStream_t st) {
  hipError_t e;
  if (pl.split) {
    // Algorithm 2: the forward spectrum is never stored whole (the paired
    // passes along the last axis recompute it)
    if ((e = jgb::launch_split_forward<T>(pl, (const T*)rho, st)) != hipSuccess) return from_hip(e, "forward FFT");
    if (pl.c0 != 0.0 && (e = jgb::launch_origin(pl, st)) != hipSuccess) return from_hip(e, "origin node");
  } else {
    jgb_status c = run_forward<T>(pl, rho, st);
    if (c != JGB_OK) return c;
  }
  if ((e = jgb::launch_interp<T>(pl, jgb::INTERP_POTENTIAL, nullptr, st)) != hipSuccess)
    return from_hip(e, "interpolation");
  if ((e = jgb::launch_spread<T>(pl, st)) != hipSuccess) return from_hip(e, "spreading");
  if ((e = jgb::launch_fft_inverse<T>(pl, (T*)u, energy ? (const T*)rho : nullptr, st)) != hipSuccess)
    return from_hip(e, "inverse FFT");
  if (energy) {
    double scale = 0.5 * pl.p.lambda * pl.H;
    jgb::stage_mark(pl, jgb::ST_ENERGY, 0, st);
    e = jgb::launch_energy_finalize(pl.d_eparts, jgb::fft_inverse_z_blocks(pl), scale, nullptr, energy, st);
    jgb::stage_mark(pl, jgb::ST_ENERGY, 1, st);
    if (e != hipSuccess) return from_hip(e, "energy");
  }
  jgb::call_done(pl);
  return JGB_OK;
}

template <typename T>
jgb_status run_energy(Plan& pl, const void* rho, double* energy) {
  hipError_t e;
  jgb_status c = run_forward<T>(pl, rho, pl.stream);
  if (c != JGB_OK) return c;
  if ((e = jgb::launch_interp<T>(pl, jgb::INTERP_ENERGY, nullptr, pl.stream)) != hipSuccess)
    return from_hip(e, "interpolation");
  int nb = jgb::interp_blocks(pl);
  if (pl.split) {
    // I1's share, sum_q M'(q) |rho^(k_q)|^2, as partials after the interpolation's
    if ((e = jgb::launch_split_energy<T>(pl, nb, pl.stream)) != hipSuccess) return from_hip(e, "split energy");
    nb += pl.nsym_blocks;
  }
  jgb::stage_mark(pl, jgb::ST_ENERGY, 0, pl.stream);
  // the node at k = 0 adds c0 rho^(0)^2
  e = jgb::launch_energy_finalize(pl.d_eparts, nb, 0.5 * pl.p.lambda, pl.c0 != 0.0 ? pl.d_origin + 1 : nullptr,
                                  energy, pl.stream);
  jgb::stage_mark(pl, jgb::ST_ENERGY, 1, pl.stream);
  if (e != hipSuccess) return from_hip(e, "energy");
  jgb::call_done(pl);
  return JGB_OK;
}

template <typename T>
jgb_status run_transform(Plan& pl, const void* rho, void* out) {
  hipError_t e;
  jgb_status c = run_forward<T>(pl, rho, pl.stream);
  if (c != JGB_OK) return c;
  if ((e = jgb::launch_interp<T>(pl, jgb::INTERP_TRANSFORM, out, pl.stream)) != hipSuccess)
    return from_hip(e, "interpolation");
  jgb::call_done(pl);
  return JGB_OK;
}

}  // namespace

// ------------------------------------------------ the allocation-free variant
//
// jgb_potential_noalloc runs jgb_potential's pipeline with its per-call
// buffers (grids, pass intermediate, partial tiles, node values, partial
// sums) carved from one file-scope device array instead of the plan's own.
// Each device holds its own copy of the array; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.

namespace {

constexpr size_t kScratchBytes = (size_t)JGB_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// The device address of this device's scratch array, looked up once per
// device with that device current (the caller has made it current).
hipError_t scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = (unsigned char*)g_scratch_ptr[dev];
  return hipSuccess;
}

// zero n16 16-byte words (a fill kernel rather than a memset node, so that the
// call stays safe to capture in a graph)
__global__ void k_zero16(uint4* p, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// the plan's per-call buffers, swapped for views into the scratch array for
// the duration of one call and restored afterwards
struct ScratchSwap {
  Plan& pl;
  void *F, *G, *W, *partials, *uhat, *ipart;
  double *eparts, *mparts, *origin;
  explicit ScratchSwap(Plan& p)
      : pl(p), F(p.d_F), G(p.d_G), W(p.d_W), partials(p.d_partials), uhat(p.nodes.uhat), ipart(p.d_ipart),
        eparts(p.d_eparts), mparts(p.d_mparts), origin(p.d_origin) {}
  ~ScratchSwap() {
    pl.d_ipart = ipart;
    pl.d_F = F;
    pl.d_G = G;
    pl.d_W = W;
    pl.d_partials = partials;
    pl.nodes.uhat = uhat;
    pl.d_eparts = eparts;
    pl.d_mparts = mparts;
    pl.d_origin = origin;
  }
};

}  // namespace

jgb_status jgb::potential_pipeline(Plan& pl, const void* rho, void* u, double* energy, hipStream_t st) {
  return pl.fp64 ? run_potential<double>(pl, rho, u, energy, st) : run_potential<float>(pl, rho, u, energy, st);
}

namespace {

jgb_status check_plan(jgb_plan_t plan) {
  if (!plan) return report(JGB_ERR_INVALID_ARG, "plan is NULL");
  hipError_t e = hipSetDevice(plan->pl.device);
  if (e != hipSuccess) return from_hip(e, "hipSetDevice");
  return JGB_OK;
}

}  // namespace

extern "C" {

jgb_status jgb_plan(const jgb_params* params, jgb_plan_t* out) {
  jgb::set_error("");
  if (!out) return report(JGB_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  jgb::Status v = jgb::validate(params);
  if (v.code != JGB_OK) return report(v.code, v.msg);
  jgb_plan_s* h = new (std::nothrow) jgb_plan_s();
  if (!h) return report(JGB_ERR_OUT_OF_MEMORY, "host allocation failed");
  jgb::Status s;
  try {
    s = jgb::build_plan(h->pl, params);
  } catch (const std::bad_alloc&) {
    s = jgb::Status{JGB_ERR_OUT_OF_MEMORY, "host allocation failed"};
  } catch (...) {
    s = jgb::Status{JGB_ERR_DEVICE, "unexpected failure while planning"};
  }
  if (s.code != JGB_OK) {
    (void)hipStreamSynchronize(h->pl.stream);
    jgb::free_plan(h->pl);
    delete h;
    return report(s.code, s.msg);
  }
  *out = h;
  return JGB_OK;
}

jgb_status jgb_potential(jgb_plan_t plan, const void* rho, void* u, double* energy) {
  jgb_status c = check_plan(plan);
  if (c != JGB_OK) return c;
  Plan& pl = plan->pl;
  if (!rho || !u) return report(JGB_ERR_INVALID_ARG, "rho and u must not be NULL");
  size_t nb = grid_bytes(pl);
  if (overlap(rho, nb, u, nb)) return report(JGB_ERR_INVALID_ARG, "rho and u overlap");
  return pl.fp64 ? run_potential<double>(pl, rho, u, energy, pl.stream)
                 : run_potential<float>(pl, rho, u, energy, pl.stream);
}

jgb_status jgb_potential_noalloc(jgb_plan_t plan, const void* rho, void* u, double* energy) {
  jgb_status c = check_plan(plan);
  if (c != JGB_OK) return c;
  Plan& pl = plan->pl;
  if (!rho || !u) return report(JGB_ERR_INVALID_ARG, "rho and u must not be NULL");
  size_t nb = grid_bytes(pl);
  if (overlap(rho, nb, u, nb)) return report(JGB_ERR_INVALID_ARG, "rho and u overlap");
  size_t off[Plan::WS_COUNT + 1];
  off[0] = 0;
  for (int i = 0; i < Plan::WS_COUNT; ++i) off[i + 1] = off[i] + align256(pl.ws_bytes[i]);
  if (off[Plan::WS_COUNT] > kScratchBytes)
    return report(JGB_ERR_UNSUPPORTED, "the plan's per-call workspace (" + std::to_string(off[Plan::WS_COUNT]) +
                                           " bytes) exceeds the allocation-free scratch (" +
                                           std::to_string(kScratchBytes) + " bytes)");
  unsigned char* base = nullptr;
  hipError_t e = scratch_address(pl.device, &base);
  if (e != hipSuccess) return from_hip(e, "hipGetSymbolAddress(scratch)");
  // only the spreading writes G, and only the tiles some node touches: the
  // others must read zero, whatever an earlier call left in the array
  const size_t n16 = off[Plan::WS_G + 1] / 16 - off[Plan::WS_G] / 16;
  hipLaunchKernelGGL(k_zero16, dim3((unsigned)std::min<size_t>((n16 + 255) / 256, 8192)), dim3(256), 0, pl.stream,
                     (uint4*)(base + off[Plan::WS_G]), n16);
  if ((e = hipGetLastError()) != hipSuccess) return from_hip(e, "scratch clear");
  ScratchSwap keep(pl);
  pl.d_F = base + off[Plan::WS_F];
  pl.d_G = base + off[Plan::WS_G];
  pl.d_W = base + off[Plan::WS_W];
  pl.d_partials = base + off[Plan::WS_PARTIALS];
  pl.nodes.uhat = base + off[Plan::WS_UHAT];
  pl.d_eparts = (double*)(base + off[Plan::WS_EPARTS]);
  pl.d_mparts = pl.ws_bytes[Plan::WS_MPARTS] ? (double*)(base + off[Plan::WS_MPARTS]) : nullptr;
  pl.d_origin = pl.ws_bytes[Plan::WS_ORIGIN] ? (double*)(base + off[Plan::WS_ORIGIN]) : nullptr;
  pl.d_ipart = pl.ws_bytes[Plan::WS_IPART] ? base + off[Plan::WS_IPART] : nullptr;
  return pl.fp64 ? run_potential<double>(pl, rho, u, energy, pl.stream)
                 : run_potential<float>(pl, rho, u, energy, pl.stream);
}

jgb_status jgb_energy(jgb_plan_t plan, const void* rho, double* energy) {
  jgb_status c = check_plan(plan);
  if (c != JGB_OK) return c;
  Plan& pl = plan->pl;
  if (!rho || !energy) return report(JGB_ERR_INVALID_ARG, "rho and energy must not be NULL");
  return pl.fp64 ? run_energy<double>(pl, rho, energy) : run_energy<float>(pl, rho, energy);
}

jgb_status jgb_potential_backward(jgb_plan_t plan, const void* grad_u, void* grad_rho) {
  jgb_status c = check_plan(plan);
  if (c != JGB_OK) return c;
  Plan& pl = plan->pl;
  if (!grad_u || !grad_rho) return report(JGB_ERR_INVALID_ARG, "grad_u and grad_rho must not be NULL");
  size_t nb = grid_bytes(pl);
  if (overlap(grad_u, nb, grad_rho, nb)) return report(JGB_ERR_INVALID_ARG, "grad_u and grad_rho overlap");
  // A is symmetric: the vector-Jacobian product is the same operator applied to grad_u
  return pl.fp64 ? run_potential<double>(pl, grad_u, grad_rho, nullptr, pl.stream)
                 : run_potential<float>(pl, grad_u, grad_rho, nullptr, pl.stream);
}

jgb_status jgb_transform(jgb_plan_t plan, const void* rho, void* rhohat) {
  jgb_status c = check_plan(plan);
  if (c != JGB_OK) return c;
  Plan& pl = plan->pl;
  if (!rho || !rhohat) return report(JGB_ERR_INVALID_ARG, "rho and rhohat must not be NULL");
  return pl.fp64 ? run_transform<double>(pl, rho, rhohat) : run_transform<float>(pl, rho, rhohat);
}

jgb_status jgb_density(jgb_plan_t plan, const void* psi, void* rho) {
  jgb_status c = check_plan(plan);
  if (c != JGB_OK) return c;
  Plan& pl = plan->pl;
  if (!psi || !rho) return report(JGB_ERR_INVALID_ARG, "psi and rho must not be NULL");
  size_t nb = grid_bytes(pl);
  if (overlap(psi, 2 * nb, rho, nb)) return report(JGB_ERR_INVALID_ARG, "psi and rho overlap");
  hipError_t e = pl.fp64 ? jgb::launch_density<double>(pl, psi, rho, pl.stream)
                         : jgb::launch_density<float>(pl, psi, rho, pl.stream);
  return from_hip(e, "density");
}

jgb_status jgb_psi_gradient(jgb_plan_t plan, const void* psi, const void* u, const double* gscale, double factor,
                            void* grad) {
  jgb_status c = check_plan(plan);
  if (c != JGB_OK) return c;
  Plan& pl = plan->pl;
  if (!psi || !u || !grad) return report(JGB_ERR_INVALID_ARG, "psi, u and grad must not be NULL");
  if (!std::isfinite(factor)) return report(JGB_ERR_INVALID_ARG, "factor must be finite");
  size_t nb = grid_bytes(pl);
  if (overlap(grad, 2 * nb, u, nb)) return report(JGB_ERR_INVALID_ARG, "grad and u overlap");
  hipError_t e = pl.fp64 ? jgb::launch_psi_gradient<double>(pl, psi, u, gscale, factor, grad, pl.stream)
                         : jgb::launch_psi_gradient<float>(pl, psi, u, gscale, factor, grad, pl.stream);
  return from_hip(e, "psi gradient");
}

jgb_status jgb_nodes(jgb_plan_t plan, double* k, double* w, double* cc) {
  jgb_status c = check_plan(plan);
  if (c != JGB_OK) return c;
  Plan& pl = plan->pl;
  if (!k && !w && !cc) return JGB_OK;
  return from_hip(jgb::launch_node_export(pl, k, w, cc, pl.stream), "node export");
}

static void release_graph(jgb_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_tables) (void)hipFree(b->d_tables);
  b->exec = nullptr;
  b->graph = nullptr;
  b->d_tables = nullptr;
  b->nlaunch = 0;
}

// Member work for balancing batch branches: grid volume and tap work.
static double member_work(const Plan& pl) {
  return (double)pl.nf[0] * pl.nf[1] * pl.nf[2] + 8.0 * (double)pl.Mh * pl.width;
}

// One launch per pipeline site over all members of a group: every member's
// pipeline is recorded (nothing is issued), the records are merged site by
// site -- a site being a kernel and its occurrence in the member's pipeline,
// in pipeline order -- and each site becomes one launch over the group's
// members that have it, its blocks the members' blocks in turn.  With several
// branches the members are dealt to them (longest work first onto the least
// loaded branch), one chain of merged launches per branch.  Returns
// JGB_ERR_UNSUPPORTED (and captures nothing) when the members' pipelines do
// not merge.
static jgb_status bind_batched(jgb_batch_s* b, const void* const* rho, void* const* u, double* energies) {
  const int nm = (int)b->plans.size();
  std::vector<std::vector<jgb::LaunchRecord>> recs(nm);
  for (int i = 0; i < nm; ++i) {
    Plan& pl = b->plans[i]->pl;
    jgb::launch_record() = &recs[i];
    double* E = energies ? energies + i : nullptr;
    jgb_status st = pl.fp64 ? run_potential<double>(pl, rho[i], u[i], E, b->stream)
                            : run_potential<float>(pl, rho[i], u[i], E, b->stream);
    jgb::launch_record() = nullptr;
    if (st != JGB_OK) return st;
  }
  // groups, one per branch
  const int nbr = std::min((int)b->branches.size(), nm);
  std::vector<std::vector<int>> groups(nbr);
  {
    std::vector<int> order(nm);
    for (int i = 0; i < nm; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return member_work(b->plans[x]->pl) > member_work(b->plans[y]->pl);
    });
    std::vector<double> load(nbr, 0.0);
    for (int i : order) {
      const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[k] += member_work(b->plans[i]->pl);
      groups[k].push_back(i);
    }
    for (auto& g : groups) std::sort(g.begin(), g.end());
  }
  struct Site {
    jgb::BatchLaunch f;
    int occ;
    std::vector<std::pair<int, int>> members;  // (member, record)
    size_t toff = 0, boff = 0;
    unsigned blocks = 0, threads = 0;
    size_t smem = 0;
  };
  std::vector<std::vector<Site>> chains(nbr);
  std::vector<unsigned char> host;
  auto align = [&]() { host.resize((host.size() + 255) / 256 * 256, 0); };
  for (int g = 0; g < nbr; ++g) {
    std::vector<Site>& sites = chains[g];
    for (int i : groups[g]) {
      std::vector<std::pair<jgb::BatchLaunch, int>> seen;
      int prev = -1;
      for (int r = 0; r < (int)recs[i].size(); ++r) {
        const jgb::BatchLaunch f = recs[i][r].launch;
        int occ = 0;
        for (auto& q : seen)
          if (q.first == f) occ = ++q.second;
        if (occ == 0) seen.push_back({f, 0});
        int pos = -1;
        for (int k = 0; k < (int)sites.size(); ++k)
          if (sites[k].f == f && sites[k].occ == occ) pos = k;
        if (pos < 0) {
          pos = prev + 1;
          sites.insert(sites.begin() + pos, Site{f, occ, {}});
        } else if (pos <= prev) {
          return report(JGB_ERR_UNSUPPORTED, "batch members' pipelines do not merge");
        }
        sites[pos].members.push_back({i, r});
        prev = pos;
      }
    }
    // argument tables and block offsets, 256-byte aligned, in one allocation:
    // the members' first blocks (multiples of eight: each member keeps its
    // blocks' places on the eight XCDs), then their block counts
    for (Site& st : sites) {
      align();
      st.toff = host.size();
      std::vector<int> bs, cnt;
      unsigned nb = 0;
      for (auto& mr : st.members) {
        const jgb::LaunchRecord& r = recs[mr.first][mr.second];
        host.insert(host.end(), r.args.begin(), r.args.end());
        if (st.threads && st.threads != r.threads)
          return report(JGB_ERR_UNSUPPORTED, "batched launch block sizes differ");
        st.threads = r.threads;
        st.smem = std::max(st.smem, r.smem);
        bs.push_back((int)nb);
        cnt.push_back((int)r.blocks);
        nb += (r.blocks + 7) / 8 * 8;
      }
      bs.push_back((int)nb);
      bs.insert(bs.end(), cnt.begin(), cnt.end());
      st.blocks = nb;
      align();
      st.boff = host.size();
      const unsigned char* p = reinterpret_cast<const unsigned char*>(bs.data());
      host.insert(host.end(), p, p + bs.size() * sizeof(int));
    }
  }
  hipError_t e = hipMalloc(&b->d_tables, std::max<size_t>(host.size(), 16));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b->d_tables = nullptr;
    return report(JGB_ERR_OUT_OF_MEMORY, "batch tables: hipMalloc failed");
  }
  e = hipMemcpy(b->d_tables, host.data(), host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return from_hip(e, "batch tables upload");
  hipStream_t origin = b->branches[0];
  e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return from_hip(e, "begin capture");
  hipError_t ce = hipEventRecord(b->events[0], origin);
  for (int k = 1; k < nbr && ce == hipSuccess; ++k) ce = hipStreamWaitEvent(b->branches[k], b->events[0], 0);
  const unsigned char* base = static_cast<const unsigned char*>(b->d_tables);
  int nlaunch = 0;
  for (int g = 0; g < nbr && ce == hipSuccess; ++g)
    for (const Site& st : chains[g]) {
      if (ce != hipSuccess) break;
      ce = st.f(base + st.toff, reinterpret_cast<const int*>(base + st.boff), (int)st.members.size(), st.blocks,
                st.threads, st.smem, b->branches[g]);
      ++nlaunch;
    }
  for (int k = 1; k < nbr && ce == hipSuccess; ++k) {
    ce = hipEventRecord(b->events[k], b->branches[k]);
    if (ce == hipSuccess) ce = hipStreamWaitEvent(origin, b->events[k], 0);
  }
  hipGraph_t gr = nullptr;
  hipError_t ee = hipStreamEndCapture(origin, &gr);
  if (ce != hipSuccess || ee != hipSuccess) {
    if (gr) (void)hipGraphDestroy(gr);
    (void)hipGetLastError();
    return from_hip(ce != hipSuccess ? ce : ee, "capture");
  }
  b->graph = gr;
  e = hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0);
  if (e != hipSuccess) return from_hip(e, "graph instantiate");
  b->nlaunch = nlaunch;
  return JGB_OK;
}

static void release_batch(jgb_batch_s* b) {
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  for (hipStream_t s : b->branches) (void)hipStreamSynchronize(s);
  release_graph(b);
  for (hipStream_t s : b->branches) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  for (jgb_plan_s* p : b->plans) (void)jgb_destroy(p);
  delete b;
}

jgb_status jgb_batch_create(const jgb_params* params, int count, int nstreams, jgb_batch_t* out) {
  jgb::set_error("");
  if (!out) return report(JGB_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!params) return report(JGB_ERR_INVALID_ARG, "params is NULL");
  if (count < 1 || count > 65536) return report(JGB_ERR_INVALID_ARG, "count must be in [1, 65536]");
  if (nstreams < 1 || nstreams > 8) return report(JGB_ERR_INVALID_ARG, "nstreams must be in [1, 8]");
  for (int i = 1; i < count; ++i)
    if (params[i].device != params[0].device || params[i].stream != params[0].stream)
      return report(JGB_ERR_INVALID_ARG, "all members of a batch share params[0]'s device and stream");
  jgb_batch_s* b = new (std::nothrow) jgb_batch_s();
  if (!b) return report(JGB_ERR_OUT_OF_MEMORY, "host allocation failed");
  b->device = params[0].device;
  b->stream = (hipStream_t)params[0].stream;
  for (int i = 0; i < count; ++i) {
    jgb_plan_t p = nullptr;
    jgb_status st = jgb_plan(&params[i], &p);
    if (st != JGB_OK) {
      std::string msg = "member " + std::to_string(i) + ": " + jgb::get_error();
      release_batch(b);
      return report(st, msg);
    }
    b->plans.push_back(p);
  }
  (void)hipSetDevice(b->device);
  for (int k = 0; k < nstreams; ++k) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      release_batch(b);
      return report(JGB_ERR_DEVICE, "stream creation failed");
    }
    b->branches.push_back(s);
  }
  for (int k = 0; k < nstreams + 2; ++k) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      release_batch(b);
      return report(JGB_ERR_DEVICE, "event creation failed");
    }
    b->events.push_back(e);
  }
  b->ev_in = b->events.back();
  b->events.pop_back();
  b->ev_out = b->events.back();
  b->events.pop_back();

  *out = b;
  return JGB_OK;
}

jgb_status jgb_batch_bind(jgb_batch_t b, const void* const* rho, void* const* u, double* energies) {
  if (!b) return report(JGB_ERR_INVALID_ARG, "batch is NULL");
  if (!rho || !u) return report(JGB_ERR_INVALID_ARG, "rho and u must not be NULL");
  const int count = (int)b->plans.size();
  for (int i = 0; i < count; ++i) {
    if (!rho[i] || !u[i]) return report(JGB_ERR_INVALID_ARG, "rho[i] and u[i] must not be NULL");
    size_t nb = grid_bytes(b->plans[i]->pl);
    if (overlap(rho[i], nb, u[i], nb)) return report(JGB_ERR_INVALID_ARG, "rho[i] and u[i] overlap");
    if (b->plans[i]->pl.timing.on) return report(JGB_ERR_INVALID_ARG, "a member plan has timing enabled");
  }
  hipError_t e = hipSetDevice(b->device);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  for (size_t k = 0; k < b->branches.size() && e == hipSuccess; ++k) e = hipStreamSynchronize(b->branches[k]);
  if (e != hipSuccess) return from_hip(e, "batch bind");
  release_graph(b);
  // With one stream: one launch per pipeline site over all members, unless a
  // member runs Algorithm 2 (its paired passes index blocks by the whole
  // grid).  With more: the members' own pipelines, spread over the streams.
  bool merged = b->branches.size() == 1;
  for (int i = 0; i < count; ++i) merged &= !b->plans[i]->pl.split;
  if (merged) {
    jgb_status st = bind_batched(b, rho, u, energies);
    if (st != JGB_ERR_UNSUPPORTED) {
      if (st != JGB_OK) release_graph(b);
      return st;
    }
    release_graph(b);
    jgb::set_error("");
  }
  // longest-processing-time assignment of members to branches by grid volume
  const int nbr = (int)b->branches.size();
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  auto work = [&](int i) { return member_work(b->plans[i]->pl); };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
  std::vector<double> load(nbr, 0.0);
  std::vector<std::vector<int>> members(nbr);
  for (int i : order) {
    int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[k] += work(i);
    members[k].push_back(i);
  }
  hipStream_t origin = b->branches[0];
  e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return from_hip(e, "begin capture");
  jgb_status st = JGB_OK;
  hipError_t ce = hipEventRecord(b->events[0], origin);
  for (int k = 1; k < nbr && ce == hipSuccess; ++k) ce = hipStreamWaitEvent(b->branches[k], b->events[0], 0);
  for (int k = 0; k < nbr && ce == hipSuccess && st == JGB_OK; ++k) {
    for (int i : members[k]) {
      Plan& pl = b->plans[i]->pl;
      double* E = energies ? energies + i : nullptr;
      st = pl.fp64 ? run_potential<double>(pl, rho[i], u[i], E, b->branches[k])
                   : run_potential<float>(pl, rho[i], u[i], E, b->branches[k]);
      if (st != JGB_OK) break;
    }
  }
  for (int k = 1; k < nbr && ce == hipSuccess && st == JGB_OK; ++k) {
    ce = hipEventRecord(b->events[k], b->branches[k]);
    if (ce == hipSuccess) ce = hipStreamWaitEvent(origin, b->events[k], 0);
  }
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(origin, &g);
  if (st != JGB_OK || ce != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (st != JGB_OK) return st;
    return from_hip(ce != hipSuccess ? ce : ee, "capture");
  }
  b->graph = g;
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    release_graph(b);
    return from_hip(e, "graph instantiate");
  }
  return JGB_OK;
}

jgb_status jgb_batch_run(jgb_batch_t b) {
  if (!b) return report(JGB_ERR_INVALID_ARG, "batch is NULL");
  if (!b->exec) return report(JGB_ERR_INVALID_ARG, "batch has no bound buffers (call jgb_batch_bind)");
  // order after the caller's earlier work, launch on the batch's own stream,
  // and order the caller's later work after the graph
  hipStream_t origin = b->branches[0];
  hipError_t e = hipSetDevice(b->device);
  if (e == hipSuccess) e = hipEventRecord(b->ev_in, b->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(origin, b->ev_in, 0);
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, origin);
  if (e == hipSuccess) e = hipEventRecord(b->ev_out, origin);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_out, 0);
  return from_hip(e, "graph launch");
}

jgb_status jgb_batch_launches(jgb_batch_t b, int* launches) {
  if (!b || !launches) return report(JGB_ERR_INVALID_ARG, "batch and launches must not be NULL");
  if (!b->exec) return report(JGB_ERR_INVALID_ARG, "batch has no bound buffers (call jgb_batch_bind)");
  size_t n = 0;
  hipError_t e = hipGraphGetNodes(b->graph, nullptr, &n);
  if (e != hipSuccess) return from_hip(e, "graph nodes");
  *launches = b->nlaunch > 0 ? b->nlaunch : (int)n;
  return JGB_OK;
}

jgb_status jgb_batch_plan(jgb_batch_t b, int i, jgb_plan_t* plan) {
  if (!b || !plan) return report(JGB_ERR_INVALID_ARG, "batch and plan must not be NULL");
  if (i < 0 || i >= (int)b->plans.size()) return report(JGB_ERR_INVALID_ARG, "member index out of range");
  *plan = b->plans[i];
  return JGB_OK;
}

jgb_status jgb_batch_destroy(jgb_batch_t b) {
  if (!b) return JGB_OK;
  release_batch(b);
  return JGB_OK;
}

static void release_timing(Plan& pl) {
  for (hipEvent_t e : pl.timing.ev) (void)hipEventDestroy(e);
  pl.timing = jgb::Timing{};
}

jgb_status jgb_timing_begin(jgb_plan_t plan, int max_calls) {
  jgb_status c = check_plan(plan);
  if (c != JGB_OK) return c;
  if (max_calls < 1 || max_calls > 100000) return report(JGB_ERR_INVALID_ARG, "max_calls must be in [1, 100000]");
  Plan& pl = plan->pl;
  hipError_t e = hipStreamSynchronize(pl.stream);
  if (e != hipSuccess) return from_hip(e, "stream synchronize");
  release_timing(pl);
  size_t n = (size_t)max_calls * jgb::ST_COUNT * 2;
  pl.timing.ev.resize(n, nullptr);
  for (size_t i = 0; i < n; ++i) {
    if (hipEventCreate(&pl.timing.ev[i]) != hipSuccess) {
      (void)hipGetLastError();
      pl.timing.ev.resize(i);
      release_timing(pl);
      return report(JGB_ERR_OUT_OF_MEMORY, "hipEventCreate failed");
    }
  }
  pl.timing.used.assign((size_t)max_calls * jgb::ST_COUNT, 0);
  pl.timing.max_calls = max_calls;
  pl.timing.calls = 0;
  pl.timing.on = true;
  return JGB_OK;
}

jgb_status jgb_timing_end(jgb_plan_t plan, double* stage_ms, int* calls) {
  jgb_status c = check_plan(plan);
  if (c != JGB_OK) return c;
  if (!stage_ms || !calls) return report(JGB_ERR_INVALID_ARG, "stage_ms and calls must not be NULL");
  Plan& pl = plan->pl;
  jgb::Timing& t = pl.timing;
  if (!t.on) return report(JGB_ERR_INVALID_ARG, "timing was not started");
  hipError_t e = hipStreamSynchronize(pl.stream);
  if (e != hipSuccess) {
    release_timing(pl);
    return from_hip(e, "stream synchronize");
  }
  for (int s = 0; s < jgb::ST_COUNT; ++s) {
    double acc = 0.0;
    int cnt = 0;
    for (int k = 0; k < t.calls; ++k) {
      size_t i = (size_t)k * jgb::ST_COUNT + s;
      if (!t.used[i]) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]) == hipSuccess) {
        acc += ms;
        cnt++;
      } else {
        (void)hipGetLastError();
      }
    }
    stage_ms[s] = cnt ? acc / cnt : 0.0;
  }
  *calls = t.calls;
  release_timing(pl);
  return JGB_OK;
}

jgb_status jgb_plan_info(jgb_plan_t plan, jgb_info* info) {
  if (!plan) return report(JGB_ERR_INVALID_ARG, "plan is NULL");
  if (!info) return report(JGB_ERR_INVALID_ARG, "info is NULL");
  if (info->struct_size != sizeof(jgb_info)) return report(JGB_ERR_INVALID_ARG, "info.struct_size != sizeof(jgb_info)");
  const Plan& pl = plan->pl;
  info->dim = pl.dim;
  if (pl.dim == 3) {
    for (int i = 0; i < 3; ++i) {
      info->n[i] = pl.n[i];
      info->nf[i] = pl.nf[i];
    }
  } else {
    info->n[0] = pl.n[1];
    info->n[1] = pl.n[2];
    info->n[2] = 1;
    info->nf[0] = pl.nf[1];
    info->nf[1] = pl.nf[2];
    info->nf[2] = 1;
  }
  info->n_nodes = pl.M;
  info->n_half = pl.Mh;
  info->width = pl.width;
  info->beta = pl.beta;
  info->kmax = pl.K;
  info->flags = pl.p.flags;
  info->window[0] = pl.split ? pl.win[0] : 0.0;
  info->window[1] = pl.split ? pl.win[1] : 0.0;
  info->origin_coef = pl.c0;
  info->radial_c = pl.radial_c;
  info->workspace_bytes = (int64_t)pl.workspace_bytes;
  info->interp_chunk = pl.tile_interp ? 0 : pl.interp_chunk;
  info->spread_chunk = pl.ring_spread ? -pl.ring_chunk : pl.spread_chunk;
  return JGB_OK;
}

jgb_status jgb_destroy(jgb_plan_t plan) {
  if (!plan) return JGB_OK;
  (void)hipSetDevice(plan->pl.device);
  hipError_t e = hipStreamSynchronize(plan->pl.stream);
  release_timing(plan->pl);
  jgb::free_plan(plan->pl);
  delete plan;
  if (e != hipSuccess) return from_hip(e, "stream synchronize");
  return JGB_OK;
}

const char* jgb_last_error(void) { return jgb::get_error(); }

}  // extern "C"
