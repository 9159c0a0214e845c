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
// One block per sub-bin (or a slice of a crowded one): the block stages the
// grid region every footprint of the sub-bin can touch -- the sub-bin plus
// w - 1 cells on the high side of each axis -- in LDS with coalesced loads,
// then each wavefront interpolates two nodes at a time from LDS, one per half
// of 32 lanes.  Lanes 0..47 first read both nodes' 3 x w tabulated kernel
// values (lane 16a + i holds phi for axis a, tap i) into the wave's LDS copy;
// the lanes of a half then own (b, c) tap pairs of the two inner axes of its
// node and loop over the outer one, and the per-lane sums are reduced within
// each half.
#include "common.h"

namespace jgb {

namespace {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {  // one 16-byte (fp64) or 8-byte (fp32) LDS access
  T x, y;
};

template <typename T>
struct InterpArgs {
  int nf0, nf1, nf2;
  FastDiv dnf0, dnf1, dnf2;
  int w0, w1, w2;
  int T0, T1, T2, S0, S1, S2;
  int nt1, nt2, nsub;
  int E0, E1, E2;   // staged region extents; E2 = W + 16 (padded, see the plan)
  int pstride;      // LDS elements per axis-0 plane of the region
  const Plan::InterpItem* items;
  const int4* hdr;
  const double* coef;
  const int* perm;
  const C2<T>* F;     // rows of hs2 along axis 2
  int hs2;
  int r2c;            // F holds q2 = 0 .. nf2/2 only: F(q) = conj F(-q) beyond
  int mode;
  C2<T>* uhat;
  const T* wts;
  int rstride;      // values per node record (axis a's taps at [a W, a W + W))
  C2<T>* out;
  double* eparts;
};

constexpr int kInterpThreads = 1024;
constexpr int kInterpWaves = kInterpThreads / 64;

// value of lane src, uniform across the wavefront
__device__ __forceinline__ double lane_value(double v, int src) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_value(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// DPP move with row mask RM; lanes without a source (or outside RM) read 0
template <int CTRL, int RM>
__device__ __forceinline__ double dpp(double v) {
  int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, RM, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, RM, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int RM>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, RM, 0xf, false));
}

// Sums over each half of the wavefront: the same scans within rows of 16, then
// the row 0 and 2 totals into rows 1 and 3; lane 31 ends with the sum of lanes
// 0-31 and lane 63 with that of lanes 32-63.
template <typename T>
__device__ __forceinline__ T half_totals(T v) {
  v += dpp<0x111, 0xf>(v);
  v += dpp<0x112, 0xf>(v);
  v += dpp<0x114, 0xf>(v);
  v += dpp<0x118, 0xf>(v);
  v += dpp<0x142, 0xa>(v);
  return v;
}

// D3: three spreading axes; a 2D problem has one tap on axis 0.
template <typename T, int W, bool D3>
__device__ __forceinline__ void interp_body(const InterpArgs<T>& a, const int blk) {
  constexpr int E2 = W + 16;  // staged row length (the plan guarantees a.E2 == E2)
  extern __shared__ unsigned char smem_raw[];
  C2<T>* tile = reinterpret_cast<C2<T>*>(smem_raw);
  __shared__ alignas(16) T wbuf[kInterpWaves][96];
  __shared__ double ws[kInterpWaves];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Plan::InterpItem item = a.items[blk];
  if (item.sub < 0) {  // idle slot of the dispatch order
    if (a.mode != INTERP_TRANSFORM && a.eparts && threadIdx.x == 0) a.eparts[blk] = 0.0;
    return;
  }

  // origin of the sub-bin on the fine grid
  const int bin = item.sub / a.nsub, sub = item.sub % a.nsub;
  const int m1 = a.T1 / a.S1, m2 = a.T2 / a.S2;
  const int s2 = sub % m2, s1 = (sub / m2) % m1, s0 = sub / (m2 * m1);
  const int b2 = bin % a.nt2, b1 = (bin / a.nt2) % a.nt1, b0 = bin / (a.nt2 * a.nt1);
  const int ox = b0 * a.T0 + s0 * a.S0, oy = b1 * a.T1 + s1 * a.S1, oz = b2 * a.T2 + s2 * a.S2;

  // stage the neighbourhood (periodic on the fine grid; the padding columns of
  // the last axis are loaded too and never read).  Thread t copies element
  // i2 = t mod E2 of rows t / E2, t / E2 + rpp, ... (rpp rows per pass); the
  // row's (i0, i1) advances by increments, and the loads go out in batches of
  // kStageBatch before their LDS writes so that they are in flight together.
  {
    constexpr int kStageBatch = 8;
    const int rpp = kInterpThreads / E2;
    const int r0 = threadIdx.x / E2;
    const bool act = r0 < rpp;
    const int i2 = act ? threadIdx.x - r0 * E2 : 0;
    const int g2 = (int)a.dnf2.mod((uint32_t)(oz + i2));
    const bool mirror = a.r2c && 2 * g2 > a.nf2;  // the conjugate mirror of the stored half
    const int m2 = mirror ? a.nf2 - g2 : g2;
    const int d0 = rpp / a.E1, d1 = rpp - d0 * a.E1;
    int i0 = r0 / a.E1, i1 = r0 - (r0 / a.E1) * a.E1;
    const int nrow = a.E0 * a.E1;
    for (int rb = r0; act && rb < nrow; rb += kStageBatch * rpp) {
      T vr[kStageBatch], vi[kStageBatch];
      int dst[kStageBatch];
#pragma unroll
      for (int k = 0; k < kStageBatch; ++k) {
        const int r = rb + k * rpp;
        const bool ok = r < nrow;
        // the region may be wider than the grid on small grids: reduce modulo nf
        int g0 = ok ? (int)a.dnf0.mod((uint32_t)(ox + i0)) : 0;
        int g1 = ok ? (int)a.dnf1.mod((uint32_t)(oy + i1)) : 0;
        if (mirror) {
          g0 = g0 ? a.nf0 - g0 : 0;
          g1 = g1 ? a.nf1 - g1 : 0;
        }
        const C2<T> v = a.F[((int64_t)g0 * a.nf1 + g1) * a.hs2 + m2];
        vr[k] = v.x;
        vi[k] = mirror ? -v.y : v.y;
        dst[k] = ok ? i0 * a.pstride + i1 * E2 + i2 : -1;
        i0 += d0;
        i1 += d1;
        if (i1 >= a.E1) {
          i1 -= a.E1;
          ++i0;
        }
      }
#pragma unroll
      for (int k = 0; k < kStageBatch; ++k)
        if (dst[k] >= 0) tile[dst[k]] = C2<T>{vr[k], vi[k]};
    }
  }
  __syncthreads();

  // Two nodes per wavefront: lanes 0-31 take the wave's node j, lanes 32-63
  // its next one, j + kInterpWaves, so that the reductions and the per-node
  // bookkeeping are shared by two nodes.  Each half reads its node's copy of
  // the record in LDS (48 values: axis a's taps at 16 a), node j's at
  // wbuf[wave][0, 48), the other's at [48, 96).
  constexpr int NP = W * W;             // tap pairs of the two axes a half owns
  constexpr int NQ = (NP + 31) / 32;    // pairs per lane
  constexpr int KW = kInterpWaves;
  const int half = lane >> 5, hl = lane & 31;
  const T* wrow = wbuf[wave] + 48 * half;
  double eacc = 0.0;
  // node data are fetched one pair ahead: the records (lane 16 axis + tap), the
  // footprint starts and the coefficients of the next pair go out before this
  // pair's taps are read from LDS
  const int ax = lane >> 4, tap = lane & 15;
  const bool wlane = ax < 3 && tap < W;
  const int woff = wlane ? ax * (W + 1) + tap : 0;  // inside the node's record for every lane
  auto fetch_w = [&](int jj) { return a.wts[(int64_t)jj * a.rstride + woff]; };
  // a per-lane (vector) load of a value every lane needs, so that it is
  // counted with the other global loads and not with the LDS traffic
  auto vec_index = [](int jj) {
    asm volatile("" : "+v"(jj));
    return jj;
  };
  // the half's node: j, or j + KW (node j when there is none: read, not used)
  int4 h_next{};
  T wa_next = T(0), wb_next = T(0);
  double c_next = 0.0;
  auto fetch = [&](int jj) {
    const bool second = jj + KW < item.end;
    const int jn = vec_index(half && second ? jj + KW : jj);
    h_next = a.hdr[jn];
    wa_next = fetch_w(vec_index(jj));
    wb_next = second ? fetch_w(vec_index(jj + KW)) : T(0);
    if (a.mode != INTERP_TRANSFORM) c_next = a.coef[jn];
  };
  int j = item.begin + wave;
  if (j < item.end) fetch(j);
  for (; j < item.end; j += 2 * KW) {
    const bool second = j + KW < item.end;
    const int4 h = h_next;
    const T wa = wlane ? wa_next : T(0), wb2 = wlane ? wb_next : T(0);
    const double c = c_next;
    if (j + 2 * KW < item.end) fetch(j + 2 * KW);
    const int lx0 = h.x - ox, ly0 = h.y - oy, lz0 = h.z - oz;  // in [0, S)
    if (lane < 48) {
      wbuf[wave][lane] = wa;
      wbuf[wave][48 + lane] = wb2;
    }
    __builtin_amdgcn_wave_barrier();

    // 3D: lane owns tap pair (a, c) of axes 0 and 2 and walks the W taps of
    // axis 1, E2 elements apart (a constant: immediate LDS offsets).  2D: lane
    // owns (b, c) of axes 1 and 2; axis 0 has the single tap 0.
    C2<T> acc[NQ];
    int off[NQ];
    T wyz[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int p = hl + 32 * q;
      const bool ok = p < NP;
      const int pa = ok ? p / W : 0, pc = ok ? p % W : 0;
      if constexpr (D3) {
        wyz[q] = ok ? wrow[pa] * wrow[32 + pc] : T(0);
        off[q] = (lx0 + pa) * a.pstride + ly0 * E2 + lz0 + pc;
      } else {
        wyz[q] = ok ? wrow[16 + pa] * wrow[32 + pc] : T(0);
        off[q] = (ly0 + pa) * E2 + lz0 + pc;
      }
      acc[q] = C2<T>{T(0), T(0)};
    }
    // the loop's weights (the same for every lane of a half) come from the
    // half's copy of the record in LDS, two per broadcast read
#pragma unroll
    for (int ib = 0; ib < (D3 ? W : 1); ib += 2) {
      const C2<T> wpair = *reinterpret_cast<const C2<T>*>(wrow + (D3 ? 16 + ib : 0));
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        if (D3 ? ib + hh < W : hh == 0) {
          const T wbv = hh == 0 ? wpair.x : wpair.y;
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const C2<T> v = tile[off[q] + (ib + hh) * E2];
            acc[q].x += wbv * v.x;
            acc[q].y += wbv * v.y;
          }
        }
      }
    }
    T sr = T(0), si = T(0);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      sr += wyz[q] * acc[q].x;
      si += wyz[q] * acc[q].y;
    }
    // lane 31 ends with the first half's sum, lane 63 with the second's
    sr = half_totals(sr);
    si = half_totals(si);
    const T ar = lane_value(sr, 31), ai = lane_value(si, 31);
    const T br = lane_value(sr, 63), bi = lane_value(si, 63);
    if (lane == 0 || (lane == 32 && second)) {
      const int jj = lane == 0 ? j : j + KW;
      const T vr = lane == 0 ? ar : br, vi = lane == 0 ? ai : bi;
      if (a.mode == INTERP_TRANSFORM) {
        a.out[a.perm[jj]] = C2<T>{vr, vi};
      } else {
        double re = (double)vr, im = (double)vi;
        eacc += c * (re * re + im * im);
        if (a.mode == INTERP_POTENTIAL) a.uhat[jj] = C2<T>{(T)(c * re), (T)(c * im)};
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  // the wave's energy: lane 0's nodes, then lane 32's
  eacc = lane_value(eacc, 0) + lane_value(eacc, 32);

  if (a.mode != INTERP_TRANSFORM && a.eparts) {
    if (lane == 0) ws[wave] = eacc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int i = 0; i < kInterpWaves; ++i) s += ws[i];
      a.eparts[blk] = s;
    }
  }
}

template <typename T, int W, bool D3>
__global__ void __launch_bounds__(kInterpThreads) k_interp(InterpArgs<T> a) {
  interp_body<T, W, D3>(a, blockIdx.x);
}
template <typename T, int W, bool D3>
__global__ void __launch_bounds__(kInterpThreads) k_interp_b(const InterpArgs<T>* __restrict__ tab, const int* __restrict__ bstart, int nm) {
  int m;
  const int blk = batch_block(bstart, nm, blockIdx.x, m);
  if (blk < 0) return;
  interp_body<T, W, D3>(tab[m], blk);
}

// ------------------------------------------------------------------ by tiles
//
// The interpolation as the transpose of the gather's tile product.  For an
// output tile of the gather (8 x 8 x 8 points) and 16 nodes of its list,
//
//   D[(z, part), i] = sum_m B[(z, part), m] P[m, i],
//   B[(z, part), m] = part(F[x_m, y_m, z]),   P[m, i] = phi_0(x_m - s_i) phi_1(y_m - s_i),
//
// over the 64 points m of the tile's two outer axes: sixteen 16x16x4
// matrix-core products, with B (the tile's grid values) loaded once per work
// item and held in registers while the list streams through.  Column i of D
// weighted by phi_2(z - s_i) and summed over z and the two parts is the tile's
// share of node i's transform, stored per list entry; k_interp_reduce adds
// each node's shares in a fixed order.  Lane 16k + j supplies A[j][k] and
// B[k][j], so lane j + 16k holds node j's kernel values; the result register
// r of lane l holds D[row(l, r)][l mod 16], column l mod 16 being the lane's
// own node, so the weighting by phi_2 needs no exchange between lanes.

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T>
struct TileMfma;
template <>
struct TileMfma<double> {
  typedef d4v acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * r + (l >> 4); }
};
template <>
struct TileMfma<float> {
  typedef f4v acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};

template <typename T>
struct TileArgs {
  int nf0, nf1, nf2;
  int w0, w1, w2;
  int nt1, nt2;
  int width, rstride;
  int lstride;        // values between the LDS copies of two records (>= rstride; see the launcher)
  const int2* list;
  const WorkItem* items;
  const T* F;         // oversampled grid, interleaved (re, im), rows of hs2 along axis 2
  int hs2;            // row stride of F along axis 2
  int r2c;            // F holds q2 = 0 .. nf2/2 only: F(q) = conj F(-q) beyond
  const T* wts;
  C2<T>* ipart;
};

template <typename V>
__device__ __forceinline__ V tload(const void* base, uint32_t byte_off) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + byte_off);
}

constexpr int kTileWaves = 4;

// NF: 16-byte pieces of a record each lane fetches, ceil(record pieces / 4).
template <typename T, bool NOWRAP, int NF>
__device__ __forceinline__ void interp_tile_body(const TileArgs<T>& a, const int blk) {
  typedef typename TileMfma<T>::acc_t acc_t;
  extern __shared__ unsigned char smem_raw[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // the wave's copies of its group's 16 node records
  T* recs = reinterpret_cast<T*>(smem_raw) + (size_t)wave * 16 * a.lstride;
  const WorkItem item = a.items[blk];
  if (item.tile < 0) return;  // idle slot of the dispatch order
  const int tile = item.tile;
  const int t2 = tile % a.nt2;
  const int t1 = (tile / a.nt2) % a.nt1;
  const int t0 = tile / (a.nt2 * a.nt1);
  const int o0 = t0 * 8, o1 = t1 * 8, o2 = t2 * 8;
  const int j16 = lane & 15, k4 = lane >> 4;

  // B: the tile's grid values, product t covering points m = 4t .. 4t + 3
  // (x = t / 2, y = 4 (t mod 2) + k) and rows j = (z, part) = (j mod 8, j / 8);
  // points off the grid read zero
  T B[16];
  {
    const int z = j16 & 7, part = j16 >> 3;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      int gx = o0 + (t >> 1), gy = o1 + ((t & 1) << 2) + k4, gz = o2 + z;
      const bool in = gx < a.nf0 && gy < a.nf1 && gz < a.nf2;
      // the Hermitian half: the other half is the conjugate mirror image
      const bool mirror = a.r2c && 2 * gz > a.nf2;
      if (mirror) {
        gx = gx ? a.nf0 - gx : 0;
        gy = gy ? a.nf1 - gy : 0;
        gz = a.nf2 - gz;
      }
      const T v = in ? a.F[2 * (((int64_t)gx * a.nf1 + gy) * a.hs2 + gz) + part] : T(0);
      B[t] = (mirror && part) ? -v : v;
    }
  }
  // the tile z and part of the lane's result registers
  int zr[4], pr[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = TileMfma<T>::row(lane, r);
    zr[r] = row & 7;
    pr[r] = row >> 3;
  }

  constexpr int bias = NOWRAP ? kGatherBias : 0;
  constexpr int kChunk = 16 / sizeof(T);  // values per 16-byte copy
  const int W = a.width;
  const int nchunk = a.rstride / kChunk;  // 16-byte pieces of a record
  const uint32_t rbytes = (uint32_t)(a.rstride * sizeof(T));
  const T* myrec = recs + j16 * a.lstride;
  const int vb = item.vbegin, ve = item.vend;
  // node j16's record reaches the wave's LDS through registers, one group
  // ahead: the four lanes of the node take every fourth 16-byte piece
  // (coalesced runs instead of one scattered load per kernel value) while the
  // group before is computed; the list entries come one group further ahead
  uint4 pre[NF];
  int g0 = vb + 16 * wave;
  int2 entc = tload<int2>(a.list, (uint32_t)min(g0 + j16, ve - 1) * 8u);
#define JGB_TILE_FETCH()                                                                                     \
  do {                                                                                                       \
    const uint32_t rec_ = (uint32_t)entc.x * rbytes;                                                         \
    _Pragma("unroll") for (int m = 0; m < NF; ++m) {                                                         \
      const int c = k4 + 4 * m;                                                                              \
      pre[m] = c < nchunk ? tload<uint4>(a.wts, rec_ + (uint32_t)c * 16u) : uint4{0u, 0u, 0u, 0u};           \
    }                                                                                                        \
  } while (0)
  if (g0 < ve) JGB_TILE_FETCH();
  int2 entn = tload<int2>(a.list, (uint32_t)min(g0 + 16 * kTileWaves + j16, ve - 1) * 8u);
  for (; g0 < ve; g0 += 16 * kTileWaves) {
    const int idx = g0 + j16;
    const bool valid = idx < ve;
    const int2 ent = entc;
    const int ex = ent.y & 1023, ey = (ent.y >> 10) & 1023, ez = (ent.y >> 20) & 1023;
    __builtin_amdgcn_wave_barrier();  // the previous group's reads are done
#pragma unroll
    for (int m = 0; m < NF; ++m) {
      const int c = k4 + 4 * m;
      if (c < nchunk) *reinterpret_cast<uint4*>(recs + j16 * a.lstride + c * kChunk) = pre[m];
    }
    __builtin_amdgcn_wave_barrier();
    if (g0 + 16 * kTileWaves < ve) {
      entc = entn;
      JGB_TILE_FETCH();
      entn = tload<int2>(a.list, (uint32_t)min(g0 + 32 * kTileWaves + j16, ve - 1) * 8u);
    }
    // node j16's kernel values at the tile's 8 x, the lane's 2 y and the z of
    // its result registers; taps outside the footprint read the zero after
    // their axis's values (a lane past the end of the list computes from a
    // copy of the last entry and stores nothing)
    auto tap = [&](int d, int axis_nf, int axis) {
      if (!NOWRAP && d < 0) d += axis_nf;
      return myrec[axis * (W + 1) + (int)min((uint32_t)d, (uint32_t)W)];
    };
    T px[8], py[2], pz[4];
#pragma unroll
    for (int x = 0; x < 8; ++x) px[x] = tap(x + bias - ex, a.nf0, 0);
#pragma unroll
    for (int h = 0; h < 2; ++h) py[h] = tap(k4 + 4 * h + bias - ey, a.nf1, 1);
#pragma unroll
    for (int r = 0; r < 4; ++r) pz[r] = tap(zr[r] + bias - ez, a.nf2, 2);
    acc_t acc = acc_t{T(0), T(0), T(0), T(0)};
    // product t covers the tile points (x = t/2, y = 4 (t mod 2) + 0..3); it
    // is skipped when none of the 16 nodes' footprints reaches them (it would
    // add exact zeros)
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const T pa = px[t >> 1] * py[t & 1];
      if (__ballot(pa != T(0))) acc = TileMfma<T>::mma(B[t], pa, acc);
    }
    T re = T(0), im = T(0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (pr[r] == 0)
        re += acc[r] * pz[r];
      else
        im += acc[r] * pz[r];
    }
    // the other three lane rows hold the node's other z
    re += __shfl_xor(re, 16, 64);
    im += __shfl_xor(im, 16, 64);
    re += __shfl_xor(re, 32, 64);
    im += __shfl_xor(im, 32, 64);
    if (k4 == 0 && valid) a.ipart[idx] = C2<T>{re, im};
  }
#undef JGB_TILE_FETCH
}

template <typename T, bool NOWRAP, int NF>
__global__ void __launch_bounds__(256) k_interp_tile(TileArgs<T> a) {
  interp_tile_body<T, NOWRAP, NF>(a, blockIdx.x);
}
template <typename T, bool NOWRAP, int NF>
__global__ void __launch_bounds__(256) k_interp_tile_b(const TileArgs<T>* __restrict__ tab, const int* __restrict__ bstart, int nm) {
  int m;
  const int blk = batch_block(bstart, nm, blockIdx.x, m);
  if (blk < 0) return;
  interp_tile_body<T, NOWRAP, NF>(tab[m], blk);
}

template <typename T, bool NOWRAP>
hipError_t launch_tile_kernel(const TileArgs<T>& a, unsigned blocks, size_t smem, hipStream_t s) {
  const int nf = (a.rstride * (int)sizeof(T) / 16 + 3) / 4;
  typedef TileArgs<T> A;
  switch (nf) {
    case 1:
    case 2: return launch<A, k_interp_tile<T, NOWRAP, 2>, k_interp_tile_b<T, NOWRAP, 2>>(a, blocks, 256, smem, s);
    case 3: return launch<A, k_interp_tile<T, NOWRAP, 3>, k_interp_tile_b<T, NOWRAP, 3>>(a, blocks, 256, smem, s);
    case 4: return launch<A, k_interp_tile<T, NOWRAP, 4>, k_interp_tile_b<T, NOWRAP, 4>>(a, blocks, 256, smem, s);
    case 5: return launch<A, k_interp_tile<T, NOWRAP, 5>, k_interp_tile_b<T, NOWRAP, 5>>(a, blocks, 256, smem, s);
    case 6: return launch<A, k_interp_tile<T, NOWRAP, 6>, k_interp_tile_b<T, NOWRAP, 6>>(a, blocks, 256, smem, s);
    case 7: return launch<A, k_interp_tile<T, NOWRAP, 7>, k_interp_tile_b<T, NOWRAP, 7>>(a, blocks, 256, smem, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
struct ReduceArgs {
  int Mh;
  const int* nstart;
  const int* npos;
  const C2<T>* ipart;
  const double* coef;
  const int* perm;
  int mode;
  C2<T>* uhat;
  C2<T>* out;
  double* eparts;
};

// Sum each node's tile shares in the order of its list entries (fixed), then
// the epilogue of the interpolation: c_j rho^_j, or the transform itself, and
// the Fourier-side energy partials.
// LPN lanes per node: lane i of a node's LPN sums its entries i, i + LPN,
// ... in that order, then a fixed-order tree sum over the LPN lanes
// (LPN = 1 or 4).  A lane's entries are taken four at a time: their list
// positions are loaded together, then their shares, then summed; the kernel
// waits on that chain of dependent loads, so each lane covers a node's
// usual count in one or two such batches.
template <typename T, int LPN>
__device__ __forceinline__ void interp_reduce_body(const ReduceArgs<T>& a, const int blk) {
  __shared__ double ws[4];
  constexpr int KU = 4;
  const int j = blk * (256 / LPN) + (int)(threadIdx.x / LPN);
  const int li = threadIdx.x % LPN;
  double sr = 0.0, si = 0.0;
  if (j < a.Mh) {
    const int b = a.nstart[j], e = a.nstart[j + 1];
    for (int q0 = b + li; q0 < e; q0 += KU * LPN) {
      int pos[KU];
#pragma unroll
      for (int k = 0; k < KU; ++k) {
        const int q = q0 + k * LPN;
        pos[k] = a.npos[q < e ? q : q0];  // q0 < e: a valid entry stands in
      }
      C2<T> v[KU];
#pragma unroll
      for (int k = 0; k < KU; ++k) v[k] = a.ipart[pos[k]];
#pragma unroll
      for (int k = 0; k < KU; ++k) {
        if (q0 + k * LPN < e) {
          sr += (double)v[k].x;
          si += (double)v[k].y;
        }
      }
    }
  }
  if (LPN == 4) {
    sr += dpp<0xB1, 0xf>(sr);   // quad_perm [1,0,3,2]
    si += dpp<0xB1, 0xf>(si);
    sr += dpp<0x4E, 0xf>(sr);   // quad_perm [2,3,0,1]
    si += dpp<0x4E, 0xf>(si);
  }
  double eacc = 0.0;
  if (j < a.Mh && li == 0) {
    if (a.mode == INTERP_TRANSFORM) {
      a.out[a.perm[j]] = C2<T>{(T)sr, (T)si};
    } else {
      const double c = a.coef[j];
      const double re = (double)(T)sr, im = (double)(T)si;
      if (a.mode == INTERP_ENERGY) eacc = c * (re * re + im * im);
      if (a.mode == INTERP_POTENTIAL) a.uhat[j] = C2<T>{(T)(c * re), (T)(c * im)};
    }
  }
  if (a.mode != INTERP_ENERGY || !a.eparts) return;
  // block sum: shuffles within waves, then the four waves through LDS
  for (int off = 32; off >= 1; off >>= 1) eacc += __shfl_down(eacc, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = eacc;
  __syncthreads();
  if (threadIdx.x == 0) a.eparts[blk] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

template <typename T, int LPN>
__global__ void __launch_bounds__(256) k_interp_reduce(ReduceArgs<T> a) {
  interp_reduce_body<T, LPN>(a, blockIdx.x);
}
template <typename T, int LPN>
__global__ void __launch_bounds__(256) k_interp_reduce_b(const ReduceArgs<T>* __restrict__ tab, const int* __restrict__ bstart, int nm) {
  int m;
  const int blk = batch_block(bstart, nm, blockIdx.x, m);
  if (blk < 0) return;
  interp_reduce_body<T, LPN>(tab[m], blk);
}

template <typename T, int W>
hipError_t launch_w(const InterpArgs<T>& a, bool d3, unsigned blocks, size_t smem, hipStream_t s) {
  if (d3) return launch<InterpArgs<T>, k_interp<T, W, true>, k_interp_b<T, W, true>>(a, blocks, kInterpThreads, smem, s);
  return launch<InterpArgs<T>, k_interp<T, W, false>, k_interp_b<T, W, false>>(a, blocks, kInterpThreads, smem, s);
}

// The largest staged region any plan may use (the attribute is per kernel, so
// it is set to the cap rather than to one plan's size).
template <typename T, int W>
hipError_t allow_lds(size_t smem) {
  const void* ks[4] = {(const void*)k_interp<T, W, true>, (const void*)k_interp<T, W, false>,
                       (const void*)k_interp_b<T, W, true>, (const void*)k_interp_b<T, W, false>};
  for (const void* k : ks) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

// Values between the LDS copies of two node records in k_interp_tile: the
// record length rounded so that copies stay 16-byte aligned, plus whole
// 16-byte steps until the 16 copies of a wave start in 16 distinct pairs of
// 4-byte banks (the lanes of one read touch one value of each copy).
template <typename T>
int tile_lds_stride(int rstride) {
  const int step = 16 / (int)sizeof(T);
  for (int s = rstride; s < rstride + 16 * step; s += step) {
    bool ok = true;
    for (int i = 0; i < 16 && ok; ++i)
      for (int k = 0; k < i && ok; ++k) {
        const int bi = (i * s * (int)sizeof(T) / 4) % 64, bk = (k * s * (int)sizeof(T) / 4) % 64;
        const int span = (int)sizeof(T) / 4;
        ok = !(bi < bk + span && bk < bi + span);
      }
    if (ok) return s;
  }
  return rstride;
}

// lanes per node of the reduction: four from ten list entries per node on
// average (FP64 at 1e-10: about 13), one below (FP32 at 1e-5: about 5); the
// measured optimum at both, since more lanes mean more waves, each waiting on
// the same chain
int reduce_lanes(const Plan& pl) {
  const double mean = pl.Mh > 0 ? (double)pl.nlist / (double)pl.Mh : 0.0;
  return mean >= 10.0 ? 4 : 1;
}

int tile_interp_blocks(const Plan& pl) {
  if (!pl.tile_ok) return 0;
  const int64_t per = 256 / reduce_lanes(pl);
  return (int)((pl.Mh + per - 1) / per);
}

int interp_blocks(const Plan& pl) { return pl.tile_interp ? tile_interp_blocks(pl) : pl.niitems; }

template <typename T>
hipError_t launch_interp_tiles(const Plan& pl, InterpMode mode, void* out, hipStream_t s) {
  TileArgs<T> a{};
  a.nf0 = pl.nf[0];
  a.nf1 = pl.nf[1];
  a.nf2 = pl.nf[2];
  a.w0 = pl.w[0];
  a.w1 = pl.w[1];
  a.w2 = pl.w[2];
  a.nt1 = pl.gnt[1];
  a.nt2 = pl.gnt[2];
  a.width = pl.width;
  a.rstride = record_stride(pl.width);
  a.lstride = tile_lds_stride<T>(a.rstride);
  a.list = pl.d_list;
  a.items = pl.d_items;
  // Algorithm 2: the type-2 spectrum was separated into G's touched tiles
  a.F = (const T*)(pl.split ? pl.d_G : pl.d_F);
  a.hs2 = pl.split ? pl.nf[2] : pl.hs2;
  a.r2c = pl.r2c ? 1 : 0;
  a.wts = (const T*)pl.nodes.wts;
  a.ipart = (C2<T>*)pl.d_ipart;
  stage_mark(pl, ST_INTERP, 0, s);
  if (pl.nitems > 0) {
    const size_t smem = (size_t)kTileWaves * 16 * a.lstride * sizeof(T);
    const hipError_t e = pl.gather_nowrap ? launch_tile_kernel<T, true>(a, (unsigned)pl.nitems, smem, s)
                                          : launch_tile_kernel<T, false>(a, (unsigned)pl.nitems, smem, s);
    if (e != hipSuccess) return e;
  }
  stage_mark(pl, ST_INTERP, 1, s);
  stage_mark(pl, ST_INTERP_REDUCE, 0, s);
  ReduceArgs<T> r{};
  r.Mh = (int)pl.Mh;
  r.nstart = pl.d_nstart;
  r.npos = pl.d_npos;
  r.ipart = (const C2<T>*)pl.d_ipart;
  r.coef = pl.nodes.coef;
  r.perm = pl.nodes.perm;
  r.mode = mode;
  r.uhat = (C2<T>*)pl.nodes.uhat;
  r.out = (C2<T>*)out;
  r.eparts = pl.d_eparts;
  const unsigned rb = (unsigned)interp_blocks(pl);
  hipError_t e = hipSuccess;
  if (rb > 0) {
    const int lpn = reduce_lanes(pl);
    if (lpn == 4)
      e = launch<ReduceArgs<T>, k_interp_reduce<T, 4>, k_interp_reduce_b<T, 4>>(r, rb, 256, 0, s);
    else
      e = launch<ReduceArgs<T>, k_interp_reduce<T, 1>, k_interp_reduce_b<T, 1>>(r, rb, 256, 0, s);
  }
  stage_mark(pl, ST_INTERP_REDUCE, 1, s);
  return e;
}

// Let the plan's interpolation kernel use its staged-region size of LDS
// (called once at plan time, outside any stream capture).
hipError_t interp_prepare(const Plan& pl) {
  switch (pl.width) {
#define JGB_W(W) \
  case W:        \
    return pl.fp64 ? allow_lds<double, W>(kInterpLdsCap) : allow_lds<float, W>(kInterpLdsCap);
    JGB_W(2) JGB_W(3) JGB_W(4) JGB_W(5) JGB_W(6) JGB_W(7) JGB_W(8) JGB_W(9) JGB_W(10) JGB_W(11) JGB_W(12)
    JGB_W(13) JGB_W(14) JGB_W(15) JGB_W(16)
#undef JGB_W
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_interp(const Plan& pl, InterpMode mode, void* out, hipStream_t s) {
  if (pl.tile_interp) return launch_interp_tiles<T>(pl, mode, out, s);
  InterpArgs<T> a{};
  a.nf0 = pl.nf[0];
  a.nf1 = pl.nf[1];
  a.nf2 = pl.nf[2];
  a.dnf0 = FastDiv((uint32_t)pl.nf[0]);
  a.dnf1 = FastDiv((uint32_t)pl.nf[1]);
  a.dnf2 = FastDiv((uint32_t)pl.nf[2]);
  a.w0 = pl.w[0];
  a.w1 = pl.w[1];
  a.w2 = pl.w[2];
  a.T0 = pl.T[0];
  a.T1 = pl.T[1];
  a.T2 = pl.T[2];
  a.S0 = pl.S[0];
  a.S1 = pl.S[1];
  a.S2 = pl.S[2];
  a.nt1 = pl.nt[1];
  a.nt2 = pl.nt[2];
  a.nsub = pl.nsub;
  a.E0 = pl.E[0];
  a.E1 = pl.E[1];
  a.E2 = pl.E[2];
  a.pstride = pl.pstride;
  a.items = pl.d_iitems;
  a.hdr = pl.nodes.hdr;
  a.coef = pl.nodes.coef;
  a.perm = pl.nodes.perm;
  // Algorithm 2: the type-2 spectrum was separated into G's touched tiles
  a.F = (const C2<T>*)(pl.split ? pl.d_G : pl.d_F);
  a.hs2 = pl.split ? pl.nf[2] : pl.hs2;
  a.r2c = pl.r2c ? 1 : 0;
  a.mode = mode;
  a.uhat = (C2<T>*)pl.nodes.uhat;
  a.wts = (const T*)pl.nodes.wts;
  a.rstride = record_stride(pl.width);
  a.out = (C2<T>*)out;
  a.eparts = pl.d_eparts;
  unsigned blocks = (unsigned)pl.niitems;
  if (blocks == 0) return hipSuccess;
  const size_t smem = pl.interp_lds;
  hipError_t e;
  stage_mark(pl, ST_INTERP, 0, s);
  switch (pl.width) {
#define JGB_W(W) \
  case W:        \
    e = launch_w<T, W>(a, pl.dim == 3, blocks, smem, s); \
    break;
    JGB_W(2) JGB_W(3) JGB_W(4) JGB_W(5) JGB_W(6) JGB_W(7) JGB_W(8) JGB_W(9) JGB_W(10) JGB_W(11) JGB_W(12)
    JGB_W(13) JGB_W(14) JGB_W(15) JGB_W(16)
#undef JGB_W
    default:
      e = hipErrorInvalidValue;
  }
  stage_mark(pl, ST_INTERP, 1, s);
  return e;
}

template hipError_t launch_interp<double>(const Plan&, InterpMode, void*, hipStream_t);
template hipError_t launch_interp<float>(const Plan&, InterpMode, void*, hipStream_t);

}  // namespace jgb
