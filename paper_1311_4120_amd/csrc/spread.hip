// Type-1 front end: spreading of the weighted node values onto the
// oversampled grid (Section 2, eq. 2.6 with the exponential-of-semicircle
// kernel in place of the Gaussian), done as an owner-computes gather:
//
//   G[g] = sum_j uhat_j phi(g0 - s0_j) phi(g1 - s1_j) phi(g2 - s2_j)   (periodic)
//
// A block owns one output tile of T0 x T1 x kGatherZ points (kGatherZ along the
// contiguous axis) and walks the tile's exact node list: every node whose
// footprint touches the tile, with its first tap relative to the tile origin.
// The tile update for a group of nodes is a rank-4 matrix product run on the
// matrix cores (below).  No atomics: every grid point is written once, in a
// fixed summation order, which makes the result deterministic.
//
// Tiles whose candidate list is longer than the chunk cap (the bins near
// k = 0, where every radial shell crowds into a few cells) are split into
// work items that write partial tiles; a second kernel sums them in order.
#include <algorithm>

#include "common.h"

namespace jgb {

namespace {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {  // one 16-byte (fp64) or 8-byte (fp32) access
  T x, y;
};

template <typename T>
struct SpreadArgs {
  int nf0, nf1, nf2;
  int w0, w1, w2;
  int nt1, nt2;
  int width, rstride;  // taps per axis in a node record, values per record
  int lstride;         // values between the LDS copies of two records
  const int2* list;
  const WorkItem* items;
  int nitems;
  const C2<T>* uhat;
  const T* wts;
  C2<T>* G;
  C2<T>* partials;
};

constexpr int kWaves = 4;

// 16x16x4 matrix-core products D += A B: lane 16k + i supplies A[i][k] and
// B[k][i] (so every operand of the gather is an ordinary per-lane load), and
// lane l holds D[row(l, r)][l mod 16] in its result register r, with the row
// mapping of each precision below.
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4v acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the 16x16 result held in register r of lane l (column l % 16)
  static __device__ __forceinline__ int row(int l, int r) { return 4 * r + (l >> 4); }
};
template <>
struct Mfma<float> {
  typedef f4v acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// Load a V at a 32-bit byte offset from a base shared by the wavefront (the
// node tables are far below 4 GB): one address add per load.
template <typename V>
__device__ __forceinline__ V load_at(const void* base, uint32_t byte_off) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + byte_off);
}

// DPP move within rows of 16 lanes: lane i reads lane i - 8 (lanes 0-7 of a
// row read 0).
template <typename T>
__device__ __forceinline__ T row_shr8(T v);
template <>
__device__ __forceinline__ double row_shr8(double v) {
  int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x118, 0xf, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x118, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <>
__device__ __forceinline__ float row_shr8(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, false));
}

// One block per work item (a tile and a range of its node list).  The tile is
// T0 x T1 x kGatherZ points; for four listed nodes its update is
//
//   G[m, (z, part)] += sum_k P[m, k] Q[k, (z, part)],
//   P[m, k] = phi_0(x_m - s_k) phi_1(y_m - s_k),   Q[k, (z, part)] = phi_2(z - s_k) part(uhat_k),
//
// with m the 64 points of the two outer axes in four row blocks of 16 and the
// 16 columns the kGatherZ = 8 points of axis 2 times (real, imaginary): one
// 16x16x4 product per row block, four per group.  Lane 16k + i supplies
// P[16b + i, k] and Q[k, i].  NX and NY are the distinct axis-0 and axis-1
// kernel values a lane needs over its four row blocks (the tile shape makes
// one of them 1); a tap outside the footprint, or a lane past the end of the
// list, reads the zero that ends its node's record, so nothing is masked
// afterwards.  A node's footprint covers 12 of an 8-deep tile's
// z more often than of a 16-deep one, so less of the matrix-core work is spent
// outside footprints.  The wavefronts split the list; their partial tiles are
// summed in LDS in a fixed order and written once.  T1 is the tile extent on
// axis 1 (8 for 3D, 64 for the 1 x 64 tiles of 2D problems).
// NOWRAP: the list's starts are signed, plus kGatherBias, and a tap offset
// is the point minus the start (no reduction modulo nf).
//
// The node data reach the lanes through LDS: for 16 list entries at a time a
// wave copies the 16 node records whole (four lanes per record, 16-byte
// pieces), their weighted values and the entries, and the four groups of four
// then read their kernel values from there.  Scattered 4- or 8-byte loads of
// single kernel values would cost the address unit one cache line per lane
// group and instruction, which is what bounds a gather over tabulated values.
template <typename T>
struct GatherLds {
  static __host__ __device__ int wave_values(int lstride) {  // T values per wave, 16-byte multiple
    return 16 * lstride + 32 + 32 * (int)(sizeof(int2) / sizeof(T));
  }
};

template <typename T, int T1, bool NOWRAP>
__device__ __forceinline__ void gather_body(const SpreadArgs<T>& a, const int blk) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int T0 = 64 / T1;
  constexpr int NX = (T1 == 8) ? 4 : 1;   // distinct x over the row blocks
  constexpr int NY = (T1 == 8) ? 1 : 4;   // distinct y over the row blocks
  extern __shared__ unsigned char smem_raw[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const WorkItem item = a.items[blk];
  if (item.tile < 0) return;  // idle slot of the dispatch order
  const int tile = item.tile;
  const int t2 = tile % a.nt2;
  const int t1 = (tile / a.nt2) % a.nt1;
  const int t0 = tile / (a.nt2 * a.nt1);
  const int o0 = t0 * T0, o1 = t1 * T1, o2 = t2 * kGatherZ;
  const int li = lane & 15, lk = lane >> 4;
  const int zl = li & (kGatherZ - 1);            // tile z of the lane's column
  const int upart = li >= kGatherZ ? 1 : 0;      // imaginary part
  const int W = a.width;
  // the wave's staging area: 16 records, 16 weighted values, 16 entries
  T* recs = reinterpret_cast<T*>(smem_raw) + (size_t)wave * GatherLds<T>::wave_values(a.lstride);
  T* uh = recs + 16 * a.lstride;
  int2* ents = reinterpret_cast<int2*>(uh + 32);

  // the lane's x values (per row block when NX = 4) and y values (per row
  // block when NY = 4); points off the grid never take a value
  // (plus kGatherBias when the starts carry it)
  constexpr int bias = NOWRAP ? kGatherBias : 0;
  int xs[NX], ys[NY];
#pragma unroll
  for (int b = 0; b < NX; ++b) {
    xs[b] = (16 * b + li) / T1 + bias;
    if (o0 + xs[b] - bias >= a.nf0) xs[b] = -(1 << 20);
  }
#pragma unroll
  for (int b = 0; b < NY; ++b) {
    ys[b] = (16 * b + li) % T1 + bias;
    if (o1 + ys[b] - bias >= a.nf1) ys[b] = -(1 << 20);
  }
  const int zb = zl + bias;

  acc_t acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = acc_t{T(0), T(0), T(0), T(0)};

  // short lists use fewer wavefronts (less to sum at the end); the count
  // depends on the list length alone, so the summation order is fixed
  const int n = item.vend - item.vbegin;
  const int nw = (n <= 32) ? 1 : (n <= 128 ? 2 : kWaves);
  const int q = (n + nw - 1) / nw;
  const int kb = wave < nw ? item.vbegin + wave * q : item.vend;
  const int ke = (kb + q < item.vend) ? kb + q : item.vend;

  constexpr int kChunk = 16 / sizeof(T);
  const int nchunk = a.rstride / kChunk;
  const uint32_t rbytes = (uint32_t)(a.rstride * sizeof(T));
  for (int g = kb; g < ke; g += 16) {
    // stage entries g .. g + 15 (lanes past the end copy entry ke - 1, whose
    // kernel values the groups below then never use)
    {
      const int e16 = g + li;
      const int2 ent = load_at<int2>(a.list, (uint32_t)(e16 < ke ? e16 : ke - 1) * 8u);
      const uint32_t rec = (uint32_t)ent.x * rbytes;
      __builtin_amdgcn_wave_barrier();  // the previous batch's reads are done
      for (int c = lk; c < nchunk; c += 4)
        *reinterpret_cast<uint4*>(recs + li * a.lstride + c * kChunk) = load_at<uint4>(a.wts, rec + (uint32_t)c * 16u);
      if (lk == 0) {
        // an entry past the end contributes nothing: its weighted value is zero
        const C2<T> u = load_at<C2<T>>(a.uhat, (uint32_t)ent.x * (uint32_t)sizeof(C2<T>));
        *reinterpret_cast<C2<T>*>(uh + 2 * li) = e16 < ke ? u : C2<T>{T(0), T(0)};
        ents[li] = ent;
      }
      __builtin_amdgcn_wave_barrier();
    }
    // the groups of four that hold entries (the count is uniform over the wave)
    const int ngq = min(4, (ke - g + 3) >> 2);
#pragma unroll
    for (int gq = 0; gq < 4; ++gq) {
      if (gq >= ngq) break;
      const int e = 4 * gq + lk;
      const int2 ent = ents[e];
      const int ex = ent.y & 1023, ey = (ent.y >> 10) & 1023, ez = (ent.y >> 20) & 1023;
      const T* rr = recs + e * a.lstride;
      // tap d = (p - start) mod nf of a point p covers it iff d < w (w <= nf);
      // with signed starts d = p - start, and a negative d is a large unsigned
      // value: min(d, W) points every tap off the footprint at the zero after
      // its axis's values (points off the grid have d < 0)
      auto tap = [&](int d, int axis_nf, int axis) {
        if (!NOWRAP && d < 0) d += axis_nf;
        return rr[axis * (W + 1) + (int)min((uint32_t)d, (uint32_t)W)];
      };
      const T qv = tap(zb - ez, a.nf2, 2) * uh[2 * e + upart];
      T px[NX], py[NY];
#pragma unroll
      for (int b = 0; b < NX; ++b) px[b] = tap(xs[b] - ex, a.nf0, 0);
#pragma unroll
      for (int b = 0; b < NY; ++b) py[b] = tap(ys[b] - ey, a.nf1, 1);
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc[b] = Mfma<T>::mma(px[NX == 4 ? b : 0] * py[NY == 4 ? b : 0], qv, acc[b]);
    }
  }

  // fixed-order sum of the active wavefronts' partial tiles: w0 alone,
  // w0 + w1, or (w0 + w2) + (w1 + w3); the staging area is reused
  __syncthreads();
  T* red0 = reinterpret_cast<T*>(smem_raw);
  T* red1 = red0 + 4 * 4 * 64;
  const int base = lane;  // element (b, r) at base + 64 * (4 b + r)
  if (wave >= 2 && nw == kWaves) {
    T* red = wave == 2 ? red0 : red1;
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[base + 64 * (4 * b + r)] = acc[b][r];
  }
  __syncthreads();
  if (wave < 2 && nw == kWaves) {
    const T* red = wave == 0 ? red0 : red1;
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[b][r] += red[base + 64 * (4 * b + r)];
  }
  __syncthreads();
  if (wave == 1 && nw >= 2) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) red0[base + 64 * (4 * b + r)] = acc[b][r];
  }
  __syncthreads();
  if (wave == 0 && nw >= 2) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[b][r] += red0[base + 64 * (4 * b + r)];
  }
  if (wave != 0) return;
  // column li holds the real part of tile z = li (li < 8) or the imaginary
  // part of z = li - 8: the lanes of the second half of each row of 16 take
  // the real part from 8 lanes down and store the complex value
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const T vi = acc[b][r];
      const T vr = row_shr8(vi);
      if (li >= kGatherZ) {
        const int z = li - kGatherZ;
        const int m = 16 * b + Mfma<T>::row(lane, r);
        const int x = m / T1, y = m % T1;
        if (item.slot < 0) {
          if (o0 + x < a.nf0 && o1 + y < a.nf1 && o2 + z < a.nf2)
            a.G[((int64_t)(o0 + x) * a.nf1 + (o1 + y)) * a.nf2 + o2 + z] = C2<T>{vr, vi};
        } else {
          a.partials[((int64_t)item.slot * 64 + m) * kGatherZ + z] = C2<T>{vr, vi};
        }
      }
    }
}

template <typename T, int T1, bool NOWRAP>
__global__ void __launch_bounds__(256) k_spread_gather(SpreadArgs<T> a) {
  gather_body<T, T1, NOWRAP>(a, blockIdx.x);
}
template <typename T, int T1, bool NOWRAP>
__global__ void __launch_bounds__(256) k_spread_gather_b(const SpreadArgs<T>* __restrict__ tab, const int* __restrict__ bstart, int nm) {
  int m;
  const int blk = batch_block(bstart, nm, blockIdx.x, m);
  if (blk < 0) return;
  gather_body<T, T1, NOWRAP>(tab[m], blk);
}

// Sum the partial tiles of each split tile in slot order and store the tile.
template <typename T>
struct SpreadReduceArgs {
  const int* multi;
  int nmulti, nf0, nf1, nf2, T0, T1, nt1, nt2;
  const C2<T>* partials;
  C2<T>* G;
};

template <typename T>
__device__ __forceinline__ void spread_reduce_body(const SpreadReduceArgs<T>& a, const int blk) {
  const int* multi = a.multi;
  const int nmulti = a.nmulti, nf0 = a.nf0, nf1 = a.nf1, nf2 = a.nf2, T1 = a.T1, nt1 = a.nt1, nt2 = a.nt2;
  const int T0 = a.T0;
  const C2<T>* partials = a.partials;
  C2<T>* G = a.G;
  // two blocks per split tile, one tile point per thread; the slots are
  // summed in slot order, their loads issued several at a time
  const int m = blk >> 1;
  if (m >= nmulti) return;
  const int idx = (blk & 1) * 256 + threadIdx.x;  // < 64 kGatherZ
  const int tile = multi[3 * m], first = multi[3 * m + 1], count = multi[3 * m + 2];
  const int t2 = tile % nt2;
  const int t1 = (tile / nt2) % nt1;
  const int t0 = tile / (nt2 * nt1);
  const int lane = idx / kGatherZ, z = idx % kGatherZ;
  const int g0 = t0 * T0 + lane / T1, g1 = t1 * T1 + lane % T1, g2 = t2 * kGatherZ + z;
  if (g0 >= nf0 || g1 >= nf1 || g2 >= nf2) return;
  const C2<T>* p = partials + (int64_t)first * 64 * kGatherZ + idx;
  // the slots in order, their loads issued eight at a time (a slot past the
  // count loads slot c0 instead, and is dropped): one wait per eight slots
  T sr = T(0), si = T(0);
  for (int c0 = 0; c0 < count; c0 += 8) {
    C2<T> v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = p[(int64_t)(c0 + k < count ? c0 + k : c0) * 64 * kGatherZ];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (c0 + k < count) {
        sr += v[k].x;
        si += v[k].y;
      }
  }
  G[((int64_t)g0 * nf1 + g1) * nf2 + g2] = C2<T>{sr, si};
}

template <typename T>
__global__ void __launch_bounds__(256) k_spread_reduce(SpreadReduceArgs<T> a) { spread_reduce_body<T>(a, blockIdx.x); }
template <typename T>
__global__ void __launch_bounds__(256) k_spread_reduce_b(const SpreadReduceArgs<T>* __restrict__ tab, const int* __restrict__ bstart, int nm) {
  int m;
  const int blk = batch_block(bstart, nm, blockIdx.x, m);
  if (blk < 0) return;
  spread_reduce_body<T>(tab[m], blk);
}

struct FinalizeArgs {
  const double* parts;
  int n;
  double scale;
  const double* extra;
  double* out;
};

__device__ __forceinline__ void finalize_body(const FinalizeArgs& a) {
  const double* parts = a.parts;
  const int n = a.n;
  const double scale = a.scale;
  const double* extra = a.extra;
  double* out = a.out;
  __shared__ double s[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += parts[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = scale * (s[0] + (extra ? *extra : 0.0));
}

__global__ void __launch_bounds__(256) k_energy_finalize(FinalizeArgs a) { finalize_body(a); }
__global__ void __launch_bounds__(256) k_energy_finalize_b(const FinalizeArgs* __restrict__ tab, const int* __restrict__ bstart, int nm) {
  int m;
  if (batch_block(bstart, nm, blockIdx.x, m) < 0) return;
  finalize_body(tab[m]);
}

}  // namespace

// Values between the LDS copies of two node records in the gather: the record
// length plus whole 16-byte steps until four consecutive copies (the four
// entries of a group, read together) start at least eight values apart in the
// 4-byte banks.
template <typename T>
int gather_lds_stride(int rstride) {
  const int step = 16 / (int)sizeof(T);
  for (int s = rstride; s < rstride + 16 * step; s += step) {
    bool ok = true;
    for (int i = 0; i < 4 && ok; ++i)
      for (int k = 0; k < i && ok; ++k) {
        const int span = (int)sizeof(T) / 4;
        const int bi = (i * s * (int)sizeof(T) / 4) % 64, bk = (k * s * (int)sizeof(T) / 4) % 64;
        ok = !(bi < bk + 8 * span && bk < bi + 8 * span);
      }
    if (ok) return s;
  }
  return rstride;
}

template <typename T>
hipError_t launch_spread(const Plan& pl, hipStream_t s) {
  if (pl.ring_spread) return launch_ring_spread<T>(pl, s);
  SpreadArgs<T> a{};
  a.nf0 = pl.nf[0];
  a.nf1 = pl.nf[1];
  a.nf2 = pl.nf[2];
  a.w0 = pl.w[0];
  a.w1 = pl.w[1];
  a.w2 = pl.w[2];
  a.nt1 = pl.gnt[1];
  a.width = pl.width;
  a.rstride = record_stride(pl.width);
  a.lstride = gather_lds_stride<T>(a.rstride);
  a.nt2 = pl.gnt[2];
  a.list = pl.d_list;
  a.items = pl.d_items;
  a.nitems = pl.nitems;
  a.uhat = (const C2<T>*)pl.nodes.uhat;
  a.wts = (const T*)pl.nodes.wts;
  a.G = (C2<T>*)pl.d_G;
  a.partials = (C2<T>*)pl.d_partials;
  unsigned blocks = (unsigned)pl.nitems;
  if (blocks == 0) return hipSuccess;  // no node touches the grid: G stays zero
  stage_mark(pl, ST_SPREAD, 0, s);
  const size_t smem = std::max((size_t)kWaves * GatherLds<T>::wave_values(a.lstride), (size_t)2 * 4 * 4 * 64) * sizeof(T);
  hipError_t e;
  typedef SpreadArgs<T> A;
  if (pl.GT[0] == 8 && pl.GT[1] == 8) {
    if (pl.gather_nowrap)
      e = launch<A, k_spread_gather<T, 8, true>, k_spread_gather_b<T, 8, true>>(a, blocks, 256, smem, s);
    else
      e = launch<A, k_spread_gather<T, 8, false>, k_spread_gather_b<T, 8, false>>(a, blocks, 256, smem, s);
  } else if (pl.GT[0] == 1 && pl.GT[1] == 64) {
    if (pl.gather_nowrap)
      e = launch<A, k_spread_gather<T, 64, true>, k_spread_gather_b<T, 64, true>>(a, blocks, 256, smem, s);
    else
      e = launch<A, k_spread_gather<T, 64, false>, k_spread_gather_b<T, 64, false>>(a, blocks, 256, smem, s);
  } else {
    return hipErrorInvalidValue;
  }
  stage_mark(pl, ST_SPREAD, 1, s);
  if (e != hipSuccess || pl.nmulti == 0) return e;
  stage_mark(pl, ST_SPREAD_REDUCE, 0, s);
  static_assert(64 * kGatherZ == 2 * 256, "two 256-thread blocks per tile");
  const SpreadReduceArgs<T> r{pl.d_multi, pl.nmulti, pl.nf[0], pl.nf[1], pl.nf[2], pl.GT[0], pl.GT[1], pl.gnt[1],
                              pl.gnt[2], (const C2<T>*)pl.d_partials, (C2<T>*)pl.d_G};
  e = launch<SpreadReduceArgs<T>, k_spread_reduce<T>, k_spread_reduce_b<T>>(r, 2 * pl.nmulti, 256, 0, s);
  stage_mark(pl, ST_SPREAD_REDUCE, 1, s);
  return e;
}

hipError_t launch_energy_finalize(const double* parts, int n, double scale, const double* extra, double* out,
                                  hipStream_t s) {
  const FinalizeArgs a{parts, n, scale, extra, out};
  return launch<FinalizeArgs, k_energy_finalize, k_energy_finalize_b>(a, 1, 256, 0, s);
}

template hipError_t launch_spread<double>(const Plan&, hipStream_t);
template hipError_t launch_spread<float>(const Plan&, hipStream_t);

}  // namespace jgb
