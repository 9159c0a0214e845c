// Algorithm 2 (Section 3.3, eq. 3.9): the regular-grid half of the
// partition-of-unity split and the glue that lets both halves share the two
// FFTs of Algorithm 1.
//
// The forward FFT transforms z = rho H / phi^ + i rho H (two real inputs in one
// complex transform), so its output Z holds two spectra:
//   A(q) = (Z(q) + conj Z(-q)) / 2       the type-2 NUFFT's oversampled grid,
//   B(q) = (Z(q) - conj Z(-q)) / (2 i)   rho^(k_q) of eq. 3.2 at k_q = 2 pi q / (2 R_j).
// I1 is the trapezoid rule on that regular frequency grid,
//   I1(x_m) = sum_q M'(q) B(q) e^{i k_q . x_m},  M' = (1 - p) U^ / prod_j (2 R_j),
// a real field; I2 = Re of the type-1 sum of the spreading grid G, which is the
// inverse transform of G's Hermitian part (G(q) + conj G(-q)) / 2.  Both go
// into one spectrum Y = Herm(G) + i M' B, so a single inverse FFT returns
// I2 phi^ in its real part and I1 in its imaginary part.
//
// Index conventions: internal axes (a0, a1, a2), a2 contiguous; the mirror of
// fine index q on an axis of nf points is (nf - q) mod nf, and the signed
// frequency index is q for q < nf/2, q - nf otherwise.
#include <cmath>

#include "common.h"

namespace jgb {

namespace {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {
  T x, y;
};

struct Geom {
  int nf0, nf1, nf2;
  int gs0, gs1, gs2;  // log2 of the gather tile extents
  int gnt1, gnt2;     // gather tiles along axes 1 and 2
};

Geom make_geom(const Plan& pl) {
  Geom g{};
  g.nf0 = pl.nf[0];
  g.nf1 = pl.nf[1];
  g.nf2 = pl.nf[2];
  auto lg = [](int v) {
    int s = 0;
    while ((1 << s) < v) ++s;
    return s;
  };
  g.gs0 = lg(pl.GT[0]);
  g.gs1 = lg(pl.GT[1]);
  g.gs2 = lg(pl.GT[2]);
  g.gnt1 = pl.gnt[1];
  g.gnt2 = pl.gnt[2];
  return g;
}

__device__ inline int mirror(int q, int nf) { return q ? nf - q : 0; }

// One block per gather tile that the interpolation reads: the tile's cells of
// G receive A = (Z(q) + conj Z(-q)) / 2.  The spreading rewrites every such
// tile afterwards, so G's other tiles stay zero.
template <typename T>
__global__ void __launch_bounds__(256) k_split_unmix(Geom g, const int* touched, const C2<T>* __restrict__ Z,
                                                     C2<T>* __restrict__ G) {
  const int tile = touched[blockIdx.x];
  const int t2 = tile % g.gnt2;
  const int r = tile / g.gnt2;
  const int t1 = r % g.gnt1;
  const int t0 = r / g.gnt1;
  const int cells = 1 << (g.gs0 + g.gs1 + g.gs2);
  for (int c = threadIdx.x; c < cells; c += 256) {
    const int c2 = c & ((1 << g.gs2) - 1);
    const int c1 = (c >> g.gs2) & ((1 << g.gs1) - 1);
    const int c0 = c >> (g.gs2 + g.gs1);
    const int i0 = (t0 << g.gs0) + c0, i1 = (t1 << g.gs1) + c1, i2 = (t2 << g.gs2) + c2;
    if (i0 >= g.nf0 || i1 >= g.nf1 || i2 >= g.nf2) continue;
    const int64_t iq = ((int64_t)i0 * g.nf1 + i1) * g.nf2 + i2;
    const int64_t im = ((int64_t)mirror(i0, g.nf0) * g.nf1 + mirror(i1, g.nf1)) * g.nf2 + mirror(i2, g.nf2);
    const C2<T> z = Z[iq], zm = Z[im];
    G[iq] = C2<T>{T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y)};
  }
}

struct SymbolArgs {
  Geom g;
  FastDiv d12, d2;     // nf1 nf2, nf2
  uint32_t npoints;    // (nf0/2 + 1) nf1 nf2: planes q0 = 0 .. nf0/2
  int kernel, dim;
  double a, r0, r1;    // window: a (3D) or R0, R1 (2D)
  double axis[3];      // dipole orientations n and m (physical coordinates)
  double axis2[3];
  double alpha;        // 2.5D dipole constant
  double inv_vol;      // 1 / prod_j (2 R_j)
  const double* kt;    // per axis: k_a(q) for q < nf_a, then exp(-k_a(q)^2 / a)
  int koff[3], eoff[3];
  const unsigned char* tflag;
  const void* G;
  void* F;
  double* eparts;
};

// M'(q) = (1 - p(k_q)) U^(k_q) / prod_j (2 R_j), with its k = 0 limit (1/a for
// the 3D Coulomb kernel; 0 for the dipoles, where 1 - p vanishes and U^ is
// bounded, and for the 2D Coulomb kernel, where 1 - p is below 1e-20 at the
// default scales).  In 2D the physical frequency is (k1, k2) of the internal
// axes (a1, a2).  In 3D the window is the product of per-axis tables, so 1 - p is
// 1 minus that product: at the grid's smallest nonzero |k| the subtraction
// costs under four bits at the default scale a = 2 dk^2.
__device__ inline double split_symbol(const SymbolArgs& s, int q0, int q1, int q2) {
  const double k0 = s.kt[s.koff[0] + q0], k1 = s.kt[s.koff[1] + q1], k2 = s.kt[s.koff[2] + q2];
  const double kk = k0 * k0 + k1 * k1 + k2 * k2;
  if (kk == 0.0) return s.kernel == JGB_COULOMB_3D ? s.inv_vol / s.a : 0.0;
  if (s.dim == 3) {
    const double omp = 1.0 - s.kt[s.eoff[0] + q0] * s.kt[s.eoff[1] + q1] * s.kt[s.eoff[2] + q2];
    if (s.kernel == JGB_COULOMB_3D) return s.inv_vol * omp / kk;
    const double nk = s.axis[0] * k0 + s.axis[1] * k1 + s.axis[2] * k2;
    const double mk = s.axis2[0] * k0 + s.axis2[1] * k1 + s.axis2[2] * k2;
    const double mn = s.axis[0] * s.axis2[0] + s.axis[1] * s.axis2[1] + s.axis[2] * s.axis2[2];
    return s.inv_vol * omp * (3.0 * nk * mk / kk - mn);
  }
  const double kabs = sqrt(kk);
  const double omp = 0.5 * erfc(-12.0 * (kabs - 0.5 * (s.r0 + s.r1)) / (s.r1 - s.r0));
  if (s.kernel == JGB_COULOMB_2D) return s.inv_vol * omp / kabs;
  const double nk = s.axis[0] * k1 + s.axis[1] * k2;
  const double mk = s.axis2[0] * k1 + s.axis2[1] * k2;
  return s.inv_vol * omp * (-s.alpha + 1.5 * (nk * mk - s.axis[2] * s.axis2[2] * kk) / kabs);
}

// Over the pairs {q, -q} (planes q0 <= nf0/2; in the planes that are their
// own mirror, the member with the smaller linear index takes the pair):
//   MODE 0: F(q) <- Herm(G)(q) + M'(q) (Z(q) - conj Z(-q)) / 2, and the same
//           at -q, in place (each pair is read and written by one thread);
//   MODE 1: energy partials sum_q M'(q) |B(q)|^2 per block, nothing written.
template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_split_symbol(SymbolArgs s) {
  const Geom& g = s.g;
  C2<T>* F = (C2<T>*)s.F;
  const C2<T>* G = (const C2<T>*)s.G;
  const uint32_t nf12 = (uint32_t)g.nf1 * g.nf2;
  double eacc = 0.0;
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t t = blockIdx.x * 256u + threadIdx.x; t < s.npoints; t += stride) {
    const int q0 = (int)s.d12.div(t);
    const uint32_t rest = t - (uint32_t)q0 * nf12;
    const int q1 = (int)s.d2.div(rest);
    const int q2 = (int)(rest - (uint32_t)q1 * g.nf2);
    const int m0 = mirror(q0, g.nf0), m1 = mirror(q1, g.nf1), m2 = mirror(q2, g.nf2);
    const int64_t iq = ((int64_t)q0 * g.nf1 + q1) * g.nf2 + q2;
    const int64_t im = ((int64_t)m0 * g.nf1 + m1) * g.nf2 + m2;
    if (m0 == q0 && im < iq) continue;
    const bool self = (im == iq);
    const C2<T> zq = F[iq], zm = F[im];
    // On a Nyquist plane (q_a = nf_a / 2) the grid frequency is its own mirror
    // on that axis, so k(-q) is not -k(q) there and a dipole symbol, which is
    // not a function of |k| alone, differs between q and -q.  I1 is real, so
    // the sum takes the mean of the two (the Hermitian part of M B).
    double M = split_symbol(s, q0, q1, q2);
    if ((s.kernel == JGB_DIPOLE_3D || s.kernel == JGB_DIPOLE_2D) &&
        (2 * q0 == g.nf0 || 2 * q1 == g.nf1 || 2 * q2 == g.nf2))
      M = 0.5 * (M + split_symbol(s, m0, m1, m2));
    // D(q) = Z(q) - conj Z(-q) = 2 i B(q); D(-q) = -conj D(q)
    const T dx = zq.x - zm.x, dy = zq.y + zm.y;
    if constexpr (MODE == 1) {
      eacc += (self ? 0.25 : 0.5) * M * ((double)dx * dx + (double)dy * dy);
    } else {
      C2<T> gq{T(0), T(0)}, gm{T(0), T(0)};
      const int tq = (((q0 >> g.gs0) * g.gnt1) + (q1 >> g.gs1)) * g.gnt2 + (q2 >> g.gs2);
      const int tm = (((m0 >> g.gs0) * g.gnt1) + (m1 >> g.gs1)) * g.gnt2 + (m2 >> g.gs2);
      if (s.tflag[tq]) gq = G[iq];
      if (s.tflag[tm]) gm = G[im];
      const T hm = (T)(0.5 * M);
      F[iq] = C2<T>{T(0.5) * (gq.x + gm.x) + hm * dx, T(0.5) * (gq.y - gm.y) + hm * dy};
      if (!self) F[im] = C2<T>{T(0.5) * (gm.x + gq.x) - hm * dx, T(0.5) * (gm.y - gq.y) + hm * dy};
    }
  }
  if constexpr (MODE == 1) {
    // deterministic block sum: wave shuffle, then the four waves in order
    for (int off = 32; off > 0; off >>= 1) eacc += __shfl_xor(eacc, off, 64);
    __shared__ double wsum[4];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = eacc;
    __syncthreads();
    if (threadIdx.x == 0) s.eparts[blockIdx.x] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
  }
}

}  // namespace

template <typename T>
hipError_t launch_split_unmix(const Plan& pl, hipStream_t s) {
  if (pl.ntouched == 0) return hipSuccess;
  stage_mark(pl, ST_SPLIT_UNMIX, 0, s);
  hipLaunchKernelGGL(k_split_unmix<T>, dim3(pl.ntouched), dim3(256), 0, s, make_geom(pl), pl.d_touched,
                     (const C2<T>*)pl.d_F, (C2<T>*)pl.d_G);
  stage_mark(pl, ST_SPLIT_UNMIX, 1, s);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_split_symbol(const Plan& pl, int energy_mode, int eoff, hipStream_t s) {
  SymbolArgs a{};
  a.g = make_geom(pl);
  a.d12 = FastDiv((uint32_t)pl.nf[1] * pl.nf[2]);
  a.d2 = FastDiv((uint32_t)pl.nf[2]);
  a.npoints = (uint32_t)(pl.nf[0] / 2 + 1) * pl.nf[1] * pl.nf[2];
  a.kernel = pl.p.kernel;
  a.dim = pl.dim;
  a.a = pl.win[0];
  a.r0 = pl.win[0];
  a.r1 = pl.win[1];
  for (int i = 0; i < 3; ++i) a.axis[i] = pl.p.dipole_axis[i];
  for (int i = 0; i < 3; ++i) a.axis2[i] = pl.axis2[i];
  a.alpha = pl.p.alpha;
  double vol = 1.0;
  for (int i = 0; i < 3; ++i)
    if (pl.n[i] > 1) vol *= 2.0 * pl.box[i];
  a.inv_vol = 1.0 / vol;
  a.kt = pl.d_splitk;
  int off = 0;
  for (int i = 0; i < 3; ++i) {
    a.koff[i] = off;
    a.eoff[i] = off + pl.nf[i];
    off += 2 * pl.nf[i];
  }
  a.tflag = pl.d_tflag;
  a.G = pl.d_G;
  a.F = pl.d_F;
  a.eparts = pl.d_eparts + eoff;
  stage_mark(pl, ST_SPLIT_SYMBOL, 0, s);
  if (energy_mode)
    hipLaunchKernelGGL((k_split_symbol<T, 1>), dim3(pl.nsym_blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_split_symbol<T, 0>), dim3(pl.nsym_blocks), dim3(256), 0, s, a);
  stage_mark(pl, ST_SPLIT_SYMBOL, 1, s);
  return hipGetLastError();
}

template hipError_t launch_split_unmix<double>(const Plan&, hipStream_t);
template hipError_t launch_split_unmix<float>(const Plan&, hipStream_t);
template hipError_t launch_split_symbol<double>(const Plan&, int, int, hipStream_t);
template hipError_t launch_split_symbol<float>(const Plan&, int, int, hipStream_t);

}  // namespace jgb
