// Type-2 back end: interpolation from the oversampled grid to the Fourier
// nodes (Section 2, the type-2 NUFFT run as the type-1 steps in reverse),
// fused with the quadrature weight x symbol multiply of eq. 3.7 and the
// Fourier-side energy sum (lambda/2) sum_j c_j |rho^_j|^2.
//
//   rho^_j = sum_{a,b,c} phi(a - f0) phi(b - f1) phi(c - f2) F[x0+a, y0+b, z0+c]
//
// (indices periodic on the fine grid; F already carries H and the
// deconvolution, so this is the trapezoid transform of eq. 3.2 at k_j).
//
// One wavefront per node.  Lanes 0..47 first evaluate the 3 x w kernel values
// (lane 16a + i holds phi for axis a, tap i).  Lanes then own (b, c) tap pairs
// of the two inner axes and loop over the outer axis, so a wavefront reads
// w contiguous runs of w complex values per row; the per-lane partial sums
// are reduced across the wavefront.  Nodes are bin-sorted, so consecutive
// nodes of a block touch overlapping footprints in cache.
#include "common.h"

namespace jgb {

namespace {

template <typename T>
struct C2 {
  T x, y;
};

template <typename T>
struct InterpArgs {
  int64_t Mh;
  int nf0, nf1, nf2;
  int w0, w1, w2;
  T beta0, beta1, beta2;
  T tw0, tw1, tw2;  // 2 / w per axis
  const int4* hdr;
  const T* f0;
  const T* f1;
  const T* f2;
  const double* coef;
  const int* perm;
  const C2<T>* F;
  int mode;
  C2<T>* uhat;
  T* wts;
  C2<T>* out;
  double* eparts;
  int nodes_per_wave;
};

constexpr int kWavesPerBlock = 4;

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T>
__global__ void __launch_bounds__(256) k_interp(InterpArgs<T> a) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t first = ((int64_t)blockIdx.x * kWavesPerBlock + wave) * a.nodes_per_wave;
  const int npairs = a.w1 * a.w2;
  double eacc = 0.0;

  for (int nn = 0; nn < a.nodes_per_wave; ++nn) {
    const int64_t j = first + nn;
    if (j >= a.Mh) break;
    const int4 h = a.hdr[j];
    const int x0 = h.x, y0 = h.y, z0 = h.z;

    // kernel values: lane 16*axis + tap
    T wv = T(0);
    {
      int ax = lane >> 4, t = lane & 15;
      if (ax == 0 && t < a.w0) wv = (a.w0 == 1) ? T(1) : es_kernel<T>(T(t) - a.f0[j], a.tw0, a.beta0);
      if (ax == 1 && t < a.w1) wv = (a.w1 == 1) ? T(1) : es_kernel<T>(T(t) - a.f1[j], a.tw1, a.beta1);
      if (ax == 2 && t < a.w2) wv = (a.w2 == 1) ? T(1) : es_kernel<T>(T(t) - a.f2[j], a.tw2, a.beta2);
    }
    if (a.mode == INTERP_POTENTIAL && lane < 48) a.wts[j * 48 + lane] = wv;

    // this lane's (b, c) pairs
    C2<T> acc[4];
    int off[4];
    T wyz[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int p = lane + 64 * q;
      acc[q] = C2<T>{T(0), T(0)};
      int b = p / a.w2, c = p % a.w2;
      bool ok = p < npairs;
      int bb = ok ? b : 0, cc = ok ? c : 0;
      T wy = __shfl(wv, 16 + bb, 64);
      T wz = __shfl(wv, 32 + cc, 64);
      wyz[q] = ok ? wy * wz : T(0);
      int gy = y0 + bb;
      if (gy >= a.nf1) gy -= a.nf1;
      int gz = z0 + cc;
      if (gz >= a.nf2) gz -= a.nf2;
      off[q] = gy * a.nf2 + gz;
    }
    const int nq = (npairs + 63) >> 6;
    for (int ia = 0; ia < a.w0; ++ia) {
      T wa = __shfl(wv, ia, 64);
      int gx = x0 + ia;
      if (gx >= a.nf0) gx -= a.nf0;
      const C2<T>* row = a.F + (int64_t)gx * a.nf1 * a.nf2;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q < nq) {
          C2<T> v = row[off[q]];
          acc[q].x += wa * v.x;
          acc[q].y += wa * v.y;
        }
      }
    }
    T sr = T(0), si = T(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sr += wyz[q] * acc[q].x;
      si += wyz[q] * acc[q].y;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) {
      if (a.mode == INTERP_TRANSFORM) {
        a.out[a.perm[j]] = C2<T>{sr, si};
      } else {
        double c = a.coef[j];
        double re = (double)sr, im = (double)si;
        eacc += c * (re * re + im * im);
        if (a.mode == INTERP_POTENTIAL) a.uhat[j] = C2<T>{(T)(c * re), (T)(c * im)};
      }
    }
  }

  if (a.mode != INTERP_TRANSFORM && a.eparts) {
    __shared__ double ws[kWavesPerBlock];
    if (lane == 0) ws[wave] = eacc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int i = 0; i < kWavesPerBlock; ++i) s += ws[i];
      a.eparts[blockIdx.x] = s;
    }
  }
}

}  // namespace

int interp_blocks(const Plan& pl, int nodes_per_wave) {
  int64_t per_block = (int64_t)kWavesPerBlock * nodes_per_wave;
  return (int)((pl.Mh + per_block - 1) / per_block);
}

template <typename T>
hipError_t launch_interp(const Plan& pl, InterpMode mode, void* out, hipStream_t s) {
  InterpArgs<T> a{};
  a.Mh = pl.Mh;
  a.nf0 = pl.nf[0];
  a.nf1 = pl.nf[1];
  a.nf2 = pl.nf[2];
  a.w0 = pl.w[0];
  a.w1 = pl.w[1];
  a.w2 = pl.w[2];
  a.beta0 = a.beta1 = a.beta2 = (T)pl.beta;
  a.tw0 = (T)(2.0 / pl.w[0]);
  a.tw1 = (T)(2.0 / pl.w[1]);
  a.tw2 = (T)(2.0 / pl.w[2]);
  a.hdr = pl.nodes.hdr;
  a.f0 = (const T*)pl.nodes.frac[0];
  a.f1 = (const T*)pl.nodes.frac[1];
  a.f2 = (const T*)pl.nodes.frac[2];
  a.coef = pl.nodes.coef;
  a.perm = pl.nodes.perm;
  a.F = (const C2<T>*)pl.d_F;
  a.mode = mode;
  a.uhat = (C2<T>*)pl.nodes.uhat;
  a.wts = (T*)pl.nodes.wts;
  a.out = (C2<T>*)out;
  a.eparts = pl.d_eparts;
  a.nodes_per_wave = kInterpNodesPerWave;
  unsigned blocks = (unsigned)interp_blocks(pl, a.nodes_per_wave);
  if (blocks == 0) return hipSuccess;
  stage_mark(pl, ST_INTERP, 0, s);
  hipLaunchKernelGGL(k_interp<T>, dim3(blocks), dim3(256), 0, s, a);
  stage_mark(pl, ST_INTERP, 1, s);
  return hipGetLastError();
}

template hipError_t launch_interp<double>(const Plan&, InterpMode, void*, hipStream_t);
template hipError_t launch_interp<float>(const Plan&, InterpMode, void*, hipStream_t);

}  // namespace jgb
