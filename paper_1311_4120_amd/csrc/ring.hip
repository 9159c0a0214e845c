// Type-1 spreading factored over the rings of the spherical node set.
//
// The Fourier nodes are the product r_a x theta_b x phi_l (Section 3.1,
// eq. 3.5); the a2 coordinate of a node, r_a cos(theta_b), does not depend
// on its azimuth, so the nodes of one ring (a, b) share their footprint start
// and kernel values along a2.  The spreading sum of eq. 2.6 (with the
// exponential-of-semicircle kernel) then splits into two smaller ones:
//
//   G[x, y, z] = sum_rings phi_2(z - s2_ring) H_ring[x, y],
//   H_ring[x, y] = sum_{j in ring} uhat_j phi_0(x - s0_j) phi_1(y - s1_j),
//
// which costs w^2 per node plus w per ring and grid column instead of w^3 per
// node.  A block owns an output tile of 16 x 8 x 16 points (a0, a1, a2), and
// its four wavefronts share out the tile's ring list: for each ring whose footprint touches the
// tile it builds H_ring over the tile's 16 x 8 (a0, a1) points on the matrix
// cores from the ring's listed nodes (those whose footprint touches the tile,
// four per 16x16x4 product),
//
//   H[x, (y, part)] += sum_{k < 4} phi_0(x - s0_k) (phi_1(y - s1_k) part(uhat_k)),
//
// and then adds phi_2(z - s2) H[x, y] to the a2 points of the tile that the
// ring's footprint covers, on the vector units, with the ring's a2 kernel
// values in scalar registers.  Every grid point is written once per work
// item, in a fixed order: the result is deterministic.  Tiles with long ring
// lists are split into work items that write partial tiles, summed in order
// by a second kernel.
#include <algorithm>

#include "common.h"

namespace jgb {

namespace {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {
  T x, y;
};

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// 16x16x4 products D += A B: lane 16k + i supplies A[i][k] and B[k][i]; lane l
// holds D[row(l, r)][l mod 16] in its result register r.
template <typename T>
struct RingMfma;
template <>
struct RingMfma<double> {
  typedef d4v acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * r + (l >> 4); }
};
template <>
struct RingMfma<float> {
  typedef f4v acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// Exchange a value with the neighbouring lane (lanes 2i and 2i + 1).
template <typename T>
__device__ __forceinline__ T swap_pair(T v);
template <>
__device__ __forceinline__ double swap_pair(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <>
__device__ __forceinline__ float swap_pair(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xf, 0xf, false));
}

// The value lane z holds, in every lane (a scalar register).
template <typename T>
__device__ __forceinline__ T lane_value(T v, int z);
template <>
__device__ __forceinline__ double lane_value(double v, int z) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), z);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), z);
  return __hiloint2double(hi, lo);
}
template <>
__device__ __forceinline__ float lane_value(float v, int z) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), z));
}

template <typename T>
struct RingArgs {
  int nf0, nf1, nf2;
  int nt1, nt2;      // ring tiles along a1 and a2
  int width;         // taps per axis
  int rstride;       // values per node record
  int lstride;       // values between the LDS copies of two records
  const int2* rnodes;  // node entries (node, codes), ring by ring in groups of four
  const RingItem* items;  // tile or partial slot, and the wavefronts' node-entry ranges
  const C2<T>* uhat;
  const T* wts;
  C2<T>* G;
  C2<T>* partials;
};

// LDS of one wavefront: 16 staged records (their a0 and a1 values, and the
// a2 values too for an entry that ends a ring), the 16 nodes' weighted values
// and the 16 entry codes.
template <typename T>
struct RingLds {
  static __host__ __device__ int values(int lstride) {
    // 16 records, 16 complex values, 16 ints; a multiple of 16 bytes
    return 16 * lstride + 32 + 64 / (int)sizeof(T);
  }
};

// NF: 16-byte pieces each lane fetches per batch, ceil(pieces of a record / 4).
template <typename T, int NF>
__device__ __forceinline__ void ring_gather_body(const RingArgs<T>& a, const int blk) {
  typedef RingMfma<T> M;
  typedef typename M::acc_t acc_t;
  constexpr int RX = kRingTile0, RY = kRingTile1, RZ = kRingTile2;
  extern __shared__ unsigned char smem_raw[];
  const RingItem& item = a.items[blk];
  const int tile = item.tile;
  if (tile < 0) return;  // idle slot of the dispatch order
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t2 = tile % a.nt2;
  const int t1 = (tile / a.nt2) % a.nt1;
  const int t0 = tile / (a.nt2 * a.nt1);
  const int o0 = t0 * RX, o1 = t1 * RY, o2 = t2 * RZ;
  const int li = lane & 15, lk = lane >> 4;
  const int W = a.width;
  T* recs = reinterpret_cast<T*>(smem_raw) + (size_t)wave * RingLds<T>::values(a.lstride);
  T* uh = recs + 16 * a.lstride;
  int* codes = reinterpret_cast<int*>(uh + 32);  // entry 4q + k at [4 k + q]

  // operands of the node products: lane 16k + i takes a0 tap x = i of node k
  // (A) and the a1 tap y = i / 2 of node k times part i mod 2 of its weighted
  // value (B); points off the grid never take a value
  const int xa = (o0 + li < a.nf0) ? li + kGatherBias : -(1 << 20);
  const int yb = (o1 + (li >> 1) < a.nf1) ? (li >> 1) + kGatherBias : -(1 << 20);
  const int part = li & 1;

  T g[4][RZ];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int z = 0; z < RZ; ++z) g[r][z] = T(0);

  constexpr int kChunk = 16 / sizeof(T);
  constexpr int kFetch = NF;
  const int nchunk_xy = (2 * (W + 1) + kChunk - 1) / kChunk;  // a record's a0 and a1 values
  const int nchunk_all = (3 * (W + 1) + kChunk - 1) / kChunk;  // and its a2 values
  const uint32_t rbytes = (uint32_t)(a.rstride * sizeof(T));

  // The item's node entries, in batches of 16 (four groups): while one batch
  // is read from LDS the next is on its way into registers -- lane i fetches
  // entry i: the pieces lk, lk + 4, ... of its record and its weighted value
  // -- and the entries of the one after it are loaded.  An entry that ends a
  // ring brings its record's a2 values along.
  const int ebeg = item.e[wave];
  const int ngroups = (item.e[wave + 1] - ebeg) >> 2;
  uint4 pre[kFetch];
  T pur, pui;
#define JGB_RING_FETCH(ent)                                                                                     \
  do {                                                                                                          \
    const uint32_t rec_ = (uint32_t)(ent).x * rbytes;                                                           \
    const int nc_ = ((ent).y >> kRingEndBit) & 1 ? nchunk_all : nchunk_xy;                                      \
    _Pragma("unroll") for (int m = 0; m < kFetch; ++m) {                                                        \
      const int c = lk + 4 * m;                                                                                 \
      pre[m] = c < nc_ ? *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(a.wts) + rec_ +         \
                                                          (uint32_t)c * 16u)                                    \
                       : uint4{0u, 0u, 0u, 0u};                                                                 \
    }                                                                                                           \
    const C2<T> u_ = a.uhat[(ent).x];                                                                           \
    pur = u_.x;                                                                                                 \
    pui = u_.y;                                                                                                 \
  } while (0)
  int2 ent = a.rnodes[ebeg + li];  // the batch being fetched
  if (ngroups > 0) JGB_RING_FETCH(ent);
  int2 ent_next = a.rnodes[ebeg + 16 + li];  // the one after it (the list ends in spare entries)
  acc_t H = acc_t{T(0), T(0), T(0), T(0)};

  for (int gb = 0; gb < ngroups; gb += 4) {
    __builtin_amdgcn_wave_barrier();  // the previous batch's reads are done
    {
      const int nc = (ent.y >> kRingEndBit) & 1 ? nchunk_all : nchunk_xy;
#pragma unroll
      for (int m = 0; m < kFetch; ++m) {
        const int c = lk + 4 * m;
        if (c < nc) *reinterpret_cast<uint4*>(recs + li * a.lstride + c * kChunk) = pre[m];
      }
      if (lk == 0) {
        uh[2 * li] = pur;
        uh[2 * li + 1] = pui;
        codes[4 * (li & 3) + (li >> 2)] = ent.y;
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (gb + 4 < ngroups) {
      ent = ent_next;
      JGB_RING_FETCH(ent);
      ent_next = a.rnodes[ebeg + 4 * (gb + 8) + li];
    }
    // the four groups' operands
    const int4 cq = *reinterpret_cast<const int4*>(codes + 4 * lk);
    const int cv[4] = {cq.x, cq.y, cq.z, cq.w};
    T av[4], bv[4], pz[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int sidx = 4 * q + lk;
      const int ex = cv[q] & 1023, ey = (cv[q] >> 10) & 1023;
      const T* rr = recs + sidx * a.lstride;
      av[q] = rr[min((uint32_t)(xa - ex), (uint32_t)W)];
      bv[q] = rr[(W + 1) + min((uint32_t)(yb - ey), (uint32_t)W)] * uh[2 * sidx + part];
      // the a2 value at tile point z = li of the group's last entry, in case
      // it ends a ring (lanes 48-63 hold that entry's code)
      const int zc = (__builtin_amdgcn_readlane(cv[q], 48) >> kRingZBit) & 1023;
      pz[q] = recs[(4 * q + 3) * a.lstride + 2 * (W + 1) + min((uint32_t)(li + kGatherBias - zc), (uint32_t)W)];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (gb + q >= ngroups) break;
      H = M::mma(av[q], bv[q], H);
      // the group's last entry (lanes 48-63 hold its code) ends a ring: spread
      // the ring sum along a2 over the tile's z points its footprint covers
      const int cl = __builtin_amdgcn_readlane(cv[q], 48);
      if ((cl >> kRingEndBit) & 1) {
        const int zoff = kGatherBias - ((cl >> kRingZBit) & 1023);  // tap of tile point z: z + zoff
#pragma unroll
        for (int z = 0; z < RZ; ++z) {
          if ((unsigned)(z + zoff) < (unsigned)W) {
            const T p = lane_value(pz[q], z);
#pragma unroll
            for (int r = 0; r < 4; ++r) g[r][z] += H[r] * p;
          }
        }
        H = acc_t{T(0), T(0), T(0), T(0)};
      }
    }
  }

#undef JGB_RING_FETCH
  // fixed-order sum of the four wavefronts' tiles, (w0 + w1) + (w2 + w3),
  // through LDS (the staging areas are reused); element (r, z) of lane l at
  // (r RZ + z) 64 + l
  {
    T* red0 = reinterpret_cast<T*>(smem_raw);
    T* red1 = red0 + 64 * 4 * RZ;
    __syncthreads();
    if (wave & 1) {
      T* red = wave == 1 ? red0 : red1;
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int z = 0; z < RZ; ++z) red[(r * RZ + z) * 64 + lane] = g[r][z];
    }
    __syncthreads();
    if (!(wave & 1)) {
      const T* red = wave == 0 ? red0 : red1;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int z = 0; z < RZ; ++z) g[r][z] += red[(r * RZ + z) * 64 + lane];
        __builtin_amdgcn_sched_barrier(0);  // a row at a time: few values in flight
      }
    }
    __syncthreads();
    if (wave == 2) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int z = 0; z < RZ; ++z) red0[(r * RZ + z) * 64 + lane] = g[r][z];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int z = 0; z < RZ; ++z) g[r][z] += red0[(r * RZ + z) * 64 + lane];
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // lane l holds (x = row(l, r), y = (l mod 16) / 2) part l mod 2 of every z:
  // the even lane of a pair stores z < 8 as complex values, the odd one z >= 8
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int x = M::row(lane, r), y = li >> 1;
    const bool inside = o0 + x < a.nf0 && o1 + y < a.nf1;
#pragma unroll
    for (int z = 0; z < RZ / 2; ++z) {
      const T v = part ? g[r][z] : g[r][z + RZ / 2];
      const T o = swap_pair(v);
      const int zz = part ? z + RZ / 2 : z;
      const C2<T> val = part ? C2<T>{o, g[r][z + RZ / 2]} : C2<T>{g[r][z], o};
      if (item.slot < 0) {
        if (inside && o2 + zz < a.nf2) a.G[((int64_t)(o0 + x) * a.nf1 + (o1 + y)) * a.nf2 + o2 + zz] = val;
      } else {
        a.partials[((int64_t)item.slot * (RX * RY) + x * RY + y) * RZ + zz] = val;
      }
    }
  }
}

template <typename T, int NF>
__global__ void __launch_bounds__(256, 2) k_ring_gather(RingArgs<T> a) {
  ring_gather_body<T, NF>(a, blockIdx.x);
}
template <typename T, int NF>
__global__ void __launch_bounds__(256, 2) k_ring_gather_b(const RingArgs<T>* __restrict__ tab, const int* __restrict__ bstart, int nm) {
  int m;
  const int blk = batch_block(bstart, nm, blockIdx.x, m);
  if (blk < 0) return;
  ring_gather_body<T, NF>(tab[m], blk);
}

// Sum the partial tiles of each split ring tile in slot order and store the tile.
template <typename T>
struct RingReduceArgs {
  const int* multi;  // per split tile: tile, first slot, slot count
  int nmulti, nf0, nf1, nf2, nt1, nt2;
  const C2<T>* partials;
  C2<T>* G;
};

constexpr int kRingTilePoints = kRingTile0 * kRingTile1 * kRingTile2;
constexpr int kRingReduceBlocks = kRingTilePoints / 256;

template <typename T>
__device__ __forceinline__ void ring_reduce_body(const RingReduceArgs<T>& a, const int blk) {
  const int m = blk / kRingReduceBlocks;
  if (m >= a.nmulti) return;
  const int idx = (blk % kRingReduceBlocks) * 256 + threadIdx.x;
  const int tile = a.multi[3 * m], first = a.multi[3 * m + 1], count = a.multi[3 * m + 2];
  const int t2 = tile % a.nt2;
  const int t1 = (tile / a.nt2) % a.nt1;
  const int t0 = tile / (a.nt2 * a.nt1);
  const int x = idx / (kRingTile1 * kRingTile2), y = (idx / kRingTile2) % kRingTile1, z = idx % kRingTile2;
  const int g0 = t0 * kRingTile0 + x, g1 = t1 * kRingTile1 + y, g2 = t2 * kRingTile2 + z;
  if (g0 >= a.nf0 || g1 >= a.nf1 || g2 >= a.nf2) return;
  const C2<T>* p = a.partials + (int64_t)first * kRingTilePoints + idx;
  // the slots in order, their loads issued eight at a time (a slot past the
  // count loads slot c0 instead, and is dropped): one wait per eight slots
  T sr = T(0), si = T(0);
  for (int c0 = 0; c0 < count; c0 += 8) {
    C2<T> v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = p[(int64_t)(c0 + k < count ? c0 + k : c0) * kRingTilePoints];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (c0 + k < count) {
        sr += v[k].x;
        si += v[k].y;
      }
  }
  a.G[((int64_t)g0 * a.nf1 + g1) * a.nf2 + g2] = C2<T>{sr, si};
}

template <typename T>
__global__ void __launch_bounds__(256) k_ring_reduce(RingReduceArgs<T> a) { ring_reduce_body<T>(a, blockIdx.x); }
template <typename T>
__global__ void __launch_bounds__(256) k_ring_reduce_b(const RingReduceArgs<T>* __restrict__ tab, const int* __restrict__ bstart, int nm) {
  int m;
  const int blk = batch_block(bstart, nm, blockIdx.x, m);
  if (blk < 0) return;
  ring_reduce_body<T>(tab[m], blk);
}

}  // namespace

// Values between the LDS copies of two staged records: the staged length plus
// whole 16-byte steps until (a) the 16 records a batch writes, one 16-byte
// piece each per instruction, fall on disjoint groups of four 4-byte banks,
// and (b) the four records a product reads together start at least eight
// banks apart.
template <typename T>
int ring_lds_stride(int width) {
  const int step = 16 / (int)sizeof(T);
  const int base = (3 * (width + 1) + step - 1) / step * step;  // a whole record (the a2 values of a ring's end)
  auto bank = [](int i, int s) { return (i * s * (int)sizeof(T) / 4) % 64; };
  for (int s = base; s < base + 16 * step; s += step) {
    bool ok = true;
    for (int i = 0; i < 16 && ok; ++i)
      for (int k = 0; k < i && ok; ++k) ok = !(bank(i, s) < bank(k, s) + 4 && bank(k, s) < bank(i, s) + 4);
    const int span = (int)sizeof(T) / 4;
    for (int i = 0; i < 4 && ok; ++i)
      for (int k = 0; k < i && ok; ++k)
        ok = !(bank(i, s) < bank(k, s) + 8 * span && bank(k, s) < bank(i, s) + 8 * span);
    if (ok) return s;
  }
  return base;
}

template <typename T>
hipError_t launch_ring_spread(const Plan& pl, hipStream_t s) {
  RingArgs<T> a{};
  a.nf0 = pl.nf[0];
  a.nf1 = pl.nf[1];
  a.nf2 = pl.nf[2];
  a.nt1 = pl.rnt[1];
  a.nt2 = pl.rnt[2];
  a.width = pl.width;
  a.rstride = record_stride(pl.width);
  a.lstride = ring_lds_stride<T>(pl.width);
  a.rnodes = pl.d_rnodes;
  a.items = pl.d_ritems;
  a.uhat = (const C2<T>*)pl.nodes.uhat;
  a.wts = (const T*)pl.nodes.wts;
  a.G = (C2<T>*)pl.d_G;
  a.partials = (C2<T>*)pl.d_partials;
  const unsigned blocks = (unsigned)pl.nritems;
  if (blocks == 0) return hipSuccess;  // no node touches the grid: G stays zero
  stage_mark(pl, ST_SPREAD, 0, s);
  const size_t smem =
      std::max((size_t)4 * RingLds<T>::values(a.lstride), (size_t)2 * 64 * 4 * kRingTile2) * sizeof(T);
  // pieces per lane: a whole record in 16-byte pieces over four lanes
  const int nf = ((3 * (pl.width + 1) * (int)sizeof(T) + 15) / 16 + 3) / 4;
  typedef RingArgs<T> A;
  hipError_t e;
  switch (nf) {
    case 1:
    case 2: e = launch<A, k_ring_gather<T, 2>, k_ring_gather_b<T, 2>>(a, blocks, 256, smem, s); break;
    case 3: e = launch<A, k_ring_gather<T, 3>, k_ring_gather_b<T, 3>>(a, blocks, 256, smem, s); break;
    case 4: e = launch<A, k_ring_gather<T, 4>, k_ring_gather_b<T, 4>>(a, blocks, 256, smem, s); break;
    case 5: e = launch<A, k_ring_gather<T, 5>, k_ring_gather_b<T, 5>>(a, blocks, 256, smem, s); break;
    case 6: e = launch<A, k_ring_gather<T, 6>, k_ring_gather_b<T, 6>>(a, blocks, 256, smem, s); break;
    case 7: e = launch<A, k_ring_gather<T, 7>, k_ring_gather_b<T, 7>>(a, blocks, 256, smem, s); break;
    default: return hipErrorInvalidValue;
  }
  stage_mark(pl, ST_SPREAD, 1, s);
  if (e != hipSuccess || pl.nrmulti == 0) return e;
  stage_mark(pl, ST_SPREAD_REDUCE, 0, s);
  const RingReduceArgs<T> r{pl.d_rmulti, pl.nrmulti, pl.nf[0], pl.nf[1], pl.nf[2], pl.rnt[1], pl.rnt[2],
                            (const C2<T>*)pl.d_partials, (C2<T>*)pl.d_G};
  e = launch<RingReduceArgs<T>, k_ring_reduce<T>, k_ring_reduce_b<T>>(r, kRingReduceBlocks * pl.nrmulti, 256, 0, s);
  stage_mark(pl, ST_SPREAD_REDUCE, 1, s);
  return e;
}

template hipError_t launch_ring_spread<double>(const Plan&, hipStream_t);
template hipError_t launch_ring_spread<float>(const Plan&, hipStream_t);

}  // namespace jgb
