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
  const C2<T>* F;
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
__global__ void __launch_bounds__(kInterpThreads) k_interp(InterpArgs<T> a) {
  constexpr int E2 = W + 16;  // staged row length (the plan guarantees a.E2 == E2)
  extern __shared__ unsigned char smem_raw[];
  C2<T>* tile = reinterpret_cast<C2<T>*>(smem_raw);
  __shared__ alignas(16) T wbuf[kInterpWaves][96];
  __shared__ double ws[kInterpWaves];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Plan::InterpItem item = a.items[blockIdx.x];
  if (item.sub < 0) {  // idle slot of the dispatch order
    if (a.mode != INTERP_TRANSFORM && a.eparts && threadIdx.x == 0) a.eparts[blockIdx.x] = 0.0;
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
        const int g0 = ok ? (int)a.dnf0.mod((uint32_t)(ox + i0)) : 0;
        const int g1 = ok ? (int)a.dnf1.mod((uint32_t)(oy + i1)) : 0;
        const C2<T> v = a.F[((int64_t)g0 * a.nf1 + g1) * a.nf2 + g2];
        vr[k] = v.x;
        vi[k] = v.y;
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
  const int woff = wlane ? ax * W + tap : 0;  // inside the node's record for every lane
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
      a.eparts[blockIdx.x] = s;
    }
  }
}

template <typename T, int W>
hipError_t launch_w(const InterpArgs<T>& a, bool d3, unsigned blocks, size_t smem, hipStream_t s) {
  if (d3)
    hipLaunchKernelGGL((k_interp<T, W, true>), dim3(blocks), dim3(kInterpThreads), smem, s, a);
  else
    hipLaunchKernelGGL((k_interp<T, W, false>), dim3(blocks), dim3(kInterpThreads), smem, s, a);
  return hipGetLastError();
}

template <typename T, int W>
hipError_t allow_lds(size_t smem) {
  hipError_t e = hipFuncSetAttribute((const void*)k_interp<T, W, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)smem);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_interp<T, W, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)smem);
}

}  // namespace

int interp_blocks(const Plan& pl) { return pl.niitems; }

// Let the plan's interpolation kernel use its staged-region size of LDS
// (called once at plan time, outside any stream capture).
hipError_t interp_prepare(const Plan& pl) {
  switch (pl.width) {
#define JGB_W(W) \
  case W:        \
    return pl.fp64 ? allow_lds<double, W>(pl.interp_lds) : allow_lds<float, W>(pl.interp_lds);
    JGB_W(2) JGB_W(3) JGB_W(4) JGB_W(5) JGB_W(6) JGB_W(7) JGB_W(8) JGB_W(9) JGB_W(10) JGB_W(11) JGB_W(12)
    JGB_W(13) JGB_W(14) JGB_W(15) JGB_W(16)
#undef JGB_W
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_interp(const Plan& pl, InterpMode mode, void* out, hipStream_t s) {
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
