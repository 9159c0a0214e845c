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
  const int2* list;
  const WorkItem* items;
  int nitems;
  const C2<T>* uhat;
  const T* wts;
  C2<T>* G;
  C2<T>* partials;
};

constexpr int kWaves = 4;

// Add one node's contribution to the wavefront's tile column.  o is the
// node's first a2 tap relative to the tile origin (uniform); the 16 kernel
// values that land on tile z = 0..15 are the window rec[kRecZ - o + z] of the
// zero-padded record, read with one uniform load, so the update is the same
// 32 multiply-adds for every node with no branch on o.
template <typename T>
__device__ __forceinline__ void add_window(T (&ar)[kTileZ], T (&ai)[kTileZ], const T* rec, int o, T pr, T pi) {
  const T* wz = rec + (kRecZ - o);
#pragma unroll
  for (int z = 0; z < kTileZ; ++z) {
    const T v = wz[z];
    ar[z] += v * pr;
    ai[z] += v * pi;
  }
}

// One block per work item (a tile and a range of its node list).  The four
// wavefronts each take a contiguous quarter of the range and accumulate the
// whole 8 x 8 x kTileZ tile in registers; the partial tiles are then summed
// in LDS in a fixed order and written once.
//
// Nodes are taken B at a time: the scalar loads of a batch (node values and
// z windows) are issued together and the next batch's list entries ride along,
// so one round trip to the scalar cache serves B nodes.
template <typename T, int B>
__global__ void __launch_bounds__(256) k_spread_gather(SpreadArgs<T> a) {
  __shared__ C2<T> red[2][64 * kTileZ];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const WorkItem item = a.items[blockIdx.x];
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

  const int n = item.vend - item.vbegin;
  const int q = (n + kWaves - 1) / kWaves;
  const int kb = item.vbegin + wave * q;
  const int ke = (kb + q < item.vend) ? kb + q : item.vend;
  const int last = ke - 1;

  int2 ent[B];
  if (kb < ke) {
#pragma unroll
    for (int b = 0; b < B; ++b) ent[b] = a.list[kb + b <= last ? kb + b : last];
  }
  for (int k = kb; k < ke; k += B) {
    int2 cur[B];
    C2<T> u[B];
    T wxy[B];
    const T* rec[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      cur[b] = ent[b];
      rec[b] = a.wts + (int64_t)cur[b].x * kRec;
      u[b] = a.uhat[cur[b].x];
      wxy[b] = rec[b][lane & 31];
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int kn = k + B + b;
      ent[b] = a.list[kn <= last ? kn : last];
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (k + b > last) break;
      const int ex = cur[b].y & 1023, ey = (cur[b].y >> 10) & 1023, ez = (cur[b].y >> 20) & 1023;
      int dx = lx - ex;
      if (dx < 0) dx += a.nf0;
      int dy = ly - ey;
      if (dy < 0) dy += a.nf1;
      const bool in = lane_ok && dx < a.w0 && dy < a.w1;
      const T wx = __shfl(wxy[b], dx & 15, 64);
      const T wy = __shfl(wxy[b], 16 + (dy & 15), 64);
      const T p = in ? wx * wy : T(0);
      const T pr = p * u[b].x, pi = p * u[b].y;
      // the footprint starts inside the tile (o = ez) or before it and wraps in
      // (o = ez - nf2 > -w2); on grids narrower than kTileZ + w2 both can hold
      const bool zin = ez < kTileZ;
      const bool zwrap = a.nf2 - ez < a.w2;
      add_window(ar, ai, rec[b], zin ? ez : ez - a.nf2, pr, pi);
      if (zin && zwrap) add_window(ar, ai, rec[b], ez - a.nf2, pr, pi);
    }
  }

  // fixed-order sum of the four partial tiles: (w0 + w2) + (w1 + w3)
  const int base = lane * kTileZ;
  if (wave >= 2) {
#pragma unroll
    for (int z = 0; z < kTileZ; ++z) red[wave - 2][base + z] = C2<T>{ar[z], ai[z]};
  }
  __syncthreads();
  if (wave < 2) {
#pragma unroll
    for (int z = 0; z < kTileZ; ++z) {
      C2<T> o = red[wave][base + z];
      ar[z] += o.x;
      ai[z] += o.y;
    }
  }
  __syncthreads();
  if (wave == 1) {
#pragma unroll
    for (int z = 0; z < kTileZ; ++z) red[0][base + z] = C2<T>{ar[z], ai[z]};
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int z = 0; z < kTileZ; ++z) {
    C2<T> o = red[0][base + z];
    ar[z] += o.x;
    ai[z] += o.y;
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
  a.list = pl.d_list;
  a.items = pl.d_items;
  a.nitems = pl.nitems;
  a.uhat = (const C2<T>*)pl.nodes.uhat;
  a.wts = (const T*)pl.nodes.wts;
  a.G = (C2<T>*)pl.d_G;
  a.partials = (C2<T>*)pl.d_partials;
  unsigned blocks = (unsigned)pl.nitems;
  if (blocks == 0) return hipErrorInvalidConfiguration;
  stage_mark(pl, ST_SPREAD, 0, s);
  constexpr int kBatch = sizeof(T) == 8 ? 2 : 4;
  hipLaunchKernelGGL((k_spread_gather<T, kBatch>), dim3(blocks), dim3(256), 0, s, a);
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
