// Type-1 front end: spreading of the weighted node values onto the
// oversampled grid (Section 2, eq. 2.6 with the exponential-of-semicircle
// kernel in place of the Gaussian), done as an owner-computes gather:
//
//   G[g] = sum_j uhat_j phi(g0 - s0_j) phi(g1 - s1_j) phi(g2 - s2_j)   (periodic)
//
// Each wavefront owns one output tile of T0 x T1 lanes by kTileZ points along
// the contiguous axis, holds the tile's accumulators in registers and walks
// the nodes of the bins that can reach the tile (nodes are bin-sorted by the
// first tap of their footprint, bins coincide with tiles).  Every test on a
// node is uniform across the wavefront, so nodes that miss the tile, and
// z-taps outside the footprint, cost scalar work only.  No atomics: every
// grid point is written once, which makes the result deterministic.
//
// Tiles whose candidate list is longer than the chunk cap (the bins near
// k = 0, where every radial shell crowds into a few cells) are split into
// work items that write partial tiles; a second kernel sums them in order.
#include "common.h"

namespace jgb {

namespace {

template <typename T>
struct C2 {
  T x, y;
};

template <typename T>
struct SpreadArgs {
  int nf0, nf1, nf2;
  int w0, w1, w2;
  int T0, T1;
  int nt1, nt2;
  const int* bin_start;
  const int* cand0;
  const int* cand1;
  const int* cand2;
  const int* coff0;
  const int* coff1;
  const int* coff2;
  const WorkItem* items;
  int nitems;
  const int4* hdr;
  const C2<T>* uhat;
  const T* wts;
  C2<T>* G;
  C2<T>* partials;
};

constexpr int kWaves = 4;

// Add the node's z taps to the tile column.  Tap t lands on tile z index O + t;
// O is the node's first tap relative to the tile, a compile-time constant per
// instantiation, so accumulators and weights are addressed statically.
// Weights past the kernel width are stored as zeros.
template <typename T, int O>
__device__ __forceinline__ void add_column(T (&ar)[kTileZ], T (&ai)[kTileZ], const T (&wz)[kMaxWidth], T pr, T pi) {
#pragma unroll
  for (int t = 0; t < kMaxWidth; ++t) {
    const int z = O + t;
    if (z >= 0 && z < kTileZ) {
      ar[z] += wz[t] * pr;
      ai[z] += wz[t] * pi;
    }
  }
}

template <typename T>
__device__ __forceinline__ void add_column_dispatch(int o, T (&ar)[kTileZ], T (&ai)[kTileZ], const T (&wz)[kMaxWidth],
                                                    T pr, T pi) {
  switch (o) {
#define JGB_CASE(O) \
  case O:           \
    add_column<T, O>(ar, ai, wz, pr, pi); \
    break;
    JGB_CASE(-15) JGB_CASE(-14) JGB_CASE(-13) JGB_CASE(-12) JGB_CASE(-11) JGB_CASE(-10) JGB_CASE(-9)
    JGB_CASE(-8) JGB_CASE(-7) JGB_CASE(-6) JGB_CASE(-5) JGB_CASE(-4) JGB_CASE(-3) JGB_CASE(-2) JGB_CASE(-1)
    JGB_CASE(0) JGB_CASE(1) JGB_CASE(2) JGB_CASE(3) JGB_CASE(4) JGB_CASE(5) JGB_CASE(6) JGB_CASE(7)
    JGB_CASE(8) JGB_CASE(9) JGB_CASE(10) JGB_CASE(11) JGB_CASE(12) JGB_CASE(13) JGB_CASE(14) JGB_CASE(15)
#undef JGB_CASE
    default:
      break;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_spread_gather(SpreadArgs<T> a) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int it = blockIdx.x * kWaves + wave;
  if (it >= a.nitems) return;
  const WorkItem item = a.items[it];
  const int tile = item.tile;
  const int t2 = tile % a.nt2;
  const int t1 = (tile / a.nt2) % a.nt1;
  const int t0 = tile / (a.nt2 * a.nt1);
  const int o0 = t0 * a.T0, o1 = t1 * a.T1, o2 = t2 * kTileZ;
  const int lx = lane / a.T1, ly = lane % a.T1;
  const bool lane_ok = (o0 + lx < a.nf0) && (o1 + ly < a.nf1);

  T ar[kTileZ], ai[kTileZ];
#pragma unroll
  for (int z = 0; z < kTileZ; ++z) {
    ar[z] = T(0);
    ai[z] = T(0);
  }

  int v = 0;
  const int vbegin = item.vbegin, vend = item.vend;
  for (int c0 = a.coff0[t0]; c0 < a.coff0[t0 + 1] && v < vend; ++c0) {
    const int b0 = a.cand0[c0];
    for (int c1 = a.coff1[t1]; c1 < a.coff1[t1 + 1] && v < vend; ++c1) {
      const int b1 = a.cand1[c1];
      for (int c2 = a.coff2[t2]; c2 < a.coff2[t2 + 1] && v < vend; ++c2) {
        const int b2 = a.cand2[c2];
        const int bin = (b0 * a.nt1 + b1) * a.nt2 + b2;
        const int s = a.bin_start[bin], e = a.bin_start[bin + 1];
        const int cnt = e - s;
        const int lo = v > vbegin ? v : vbegin;
        const int hi = (v + cnt) < vend ? (v + cnt) : vend;
        for (int vv = lo; vv < hi; ++vv) {
          const int j = s + (vv - v);
          const int4 h = a.hdr[j];
          // first tap of the footprint relative to the tile origin, modulo the grid
          int ex = h.x - o0;
          if (ex < 0) ex += a.nf0;
          int ey = h.y - o1;
          if (ey < 0) ey += a.nf1;
          int ez = h.z - o2;
          if (ez < 0) ez += a.nf2;
          const bool zin = ez < kTileZ;               // footprint starts inside the tile
          const bool zwrap = a.nf2 - ez < a.w2;       // footprint starts before it and reaches in
          if (!((ex < a.T0 || a.nf0 - ex < a.w0) && (ey < a.T1 || a.nf1 - ey < a.w1) && (zin || zwrap))) continue;
          const T* wj = a.wts + (int64_t)j * 48;
          int dx = lx - ex;
          if (dx < 0) dx += a.nf0;
          int dy = ly - ey;
          if (dy < 0) dy += a.nf1;
          const bool in = lane_ok && dx < a.w0 && dy < a.w1;
          const T wx = wj[in ? dx : 0];
          const T wy = wj[16 + (in ? dy : 0)];
          const T p = in ? wx * wy : T(0);
          const C2<T> u = a.uhat[j];
          const T pr = p * u.x, pi = p * u.y;
          T wz[kMaxWidth];
#pragma unroll
          for (int t = 0; t < kMaxWidth; ++t) wz[t] = wj[32 + t];
          if (zin) add_column_dispatch<T>(ez, ar, ai, wz, pr, pi);
          if (zwrap) add_column_dispatch<T>(ez - a.nf2, ar, ai, wz, pr, pi);
        }
        v += cnt;
      }
    }
  }

  if (!lane_ok) return;
  const int g0 = o0 + lx, g1 = o1 + ly;
  if (item.slot < 0) {
    C2<T>* dst = a.G + ((int64_t)g0 * a.nf1 + g1) * a.nf2 + o2;
#pragma unroll
    for (int z = 0; z < kTileZ; ++z)
      if (o2 + z < a.nf2) dst[z] = C2<T>{ar[z], ai[z]};
  } else {
    C2<T>* dst = a.partials + ((int64_t)item.slot * 64 + lane) * kTileZ;
#pragma unroll
    for (int z = 0; z < kTileZ; ++z) dst[z] = C2<T>{ar[z], ai[z]};
  }
}

// Sum the partial tiles of each split tile in slot order and store the tile.
template <typename T>
__global__ void __launch_bounds__(256) k_spread_reduce(const int* multi, int nmulti, int nf0, int nf1, int nf2,
                                                       int T0, int T1, int nt1, int nt2, const C2<T>* partials,
                                                       C2<T>* G) {
  const int m = blockIdx.x;
  if (m >= nmulti) return;
  const int tile = multi[3 * m], first = multi[3 * m + 1], count = multi[3 * m + 2];
  const int t2 = tile % nt2;
  const int t1 = (tile / nt2) % nt1;
  const int t0 = tile / (nt2 * nt1);
  for (int idx = threadIdx.x; idx < 64 * kTileZ; idx += blockDim.x) {
    const int lane = idx / kTileZ, z = idx % kTileZ;
    const int g0 = t0 * T0 + lane / T1, g1 = t1 * T1 + lane % T1, g2 = t2 * kTileZ + z;
    if (g0 >= nf0 || g1 >= nf1 || g2 >= nf2) continue;
    T sr = T(0), si = T(0);
    for (int c = 0; c < count; ++c) {
      C2<T> p = partials[((int64_t)(first + c) * 64 + lane) * kTileZ + z];
      sr += p.x;
      si += p.y;
    }
    G[((int64_t)g0 * nf1 + g1) * nf2 + g2] = C2<T>{sr, si};
  }
}

__global__ void k_energy_finalize(const double* parts, int n, double scale, double* out) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += parts[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = scale * s[0];
}

}  // namespace

template <typename T>
hipError_t launch_spread(const Plan& pl, hipStream_t s) {
  SpreadArgs<T> a{};
  a.nf0 = pl.nf[0];
  a.nf1 = pl.nf[1];
  a.nf2 = pl.nf[2];
  a.w0 = pl.w[0];
  a.w1 = pl.w[1];
  a.w2 = pl.w[2];
  a.T0 = pl.T[0];
  a.T1 = pl.T[1];
  a.nt1 = pl.nt[1];
  a.nt2 = pl.nt[2];
  a.bin_start = pl.d_bin_start;
  a.cand0 = pl.d_cand[0];
  a.cand1 = pl.d_cand[1];
  a.cand2 = pl.d_cand[2];
  a.coff0 = pl.d_cand_off[0];
  a.coff1 = pl.d_cand_off[1];
  a.coff2 = pl.d_cand_off[2];
  a.items = pl.d_items;
  a.nitems = pl.nitems;
  a.hdr = pl.nodes.hdr;
  a.uhat = (const C2<T>*)pl.nodes.uhat;
  a.wts = (const T*)pl.nodes.wts;
  a.G = (C2<T>*)pl.d_G;
  a.partials = (C2<T>*)pl.d_partials;
  unsigned blocks = (unsigned)((pl.nitems + kWaves - 1) / kWaves);
  stage_mark(pl, ST_SPREAD, 0, s);
  hipLaunchKernelGGL(k_spread_gather<T>, dim3(blocks), dim3(256), 0, s, a);
  stage_mark(pl, ST_SPREAD, 1, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || pl.nmulti == 0) return e;
  stage_mark(pl, ST_SPREAD_REDUCE, 0, s);
  hipLaunchKernelGGL(k_spread_reduce<T>, dim3(pl.nmulti), dim3(256), 0, s, pl.d_multi, pl.nmulti, pl.nf[0], pl.nf[1],
                     pl.nf[2], pl.T[0], pl.T[1], pl.nt[1], pl.nt[2], (const C2<T>*)pl.d_partials, (C2<T>*)pl.d_G);
  stage_mark(pl, ST_SPREAD_REDUCE, 1, s);
  return hipGetLastError();
}

hipError_t launch_energy_finalize(const double* parts, int n, double scale, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_finalize, dim3(1), dim3(256), 0, s, parts, n, scale, out);
  return hipGetLastError();
}

template hipError_t launch_spread<double>(const Plan&, hipStream_t);
template hipError_t launch_spread<float>(const Plan&, hipStream_t);

}  // namespace jgb
