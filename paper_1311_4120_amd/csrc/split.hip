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
// I2 phi^ in its real part and I1 in its imaginary part; its first pass forms
// Y with each line and its mirror in LDS (fft.hip, k_fft_pair_pass), where the
// potential's path also separates A.  This file holds the separation of A from
// a stored spectrum (the energy-only and transform calls) and the Fourier-side
// energy of I1.
//
// Index conventions: internal axes (a0, a1, a2), a2 contiguous; the mirror of
// fine index q on an axis of nf points is (nf - q) mod nf, and the signed
// frequency index is q for q < nf/2, q - nf otherwise.
#include <cmath>

#include "splitsym.h"

namespace jgb {

namespace {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {
  T x, y;
};

int log2_exact(int v) {
  int s = 0;
  while ((1 << s) < v) ++s;
  return s;
}

// One block per gather tile that the interpolation reads: the tile's cells of
// G receive A = (Z(q) + conj Z(-q)) / 2.  The spreading rewrites every such
// tile afterwards, so G's other tiles stay zero.
template <typename T>
__global__ void __launch_bounds__(256) k_split_unmix(SplitSym g, const int* touched, const C2<T>* __restrict__ Z,
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
    const int64_t im = ((int64_t)split_mirror(i0, g.nf0) * g.nf1 + split_mirror(i1, g.nf1)) * g.nf2 +
                       split_mirror(i2, g.nf2);
    const C2<T> z = Z[iq], zm = Z[im];
    G[iq] = C2<T>{T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y)};
  }
}

// Energy partials of I1 per block, sum_q M'(q) |B(q)|^2 with |B(q)|^2 =
// |Z(q) - conj Z(-q)|^2 / 4, over the pairs {q, -q} (planes q0 <= nf0/2; in
// the planes that are their own mirror, the member with the smaller linear
// index takes the pair, which counts twice unless it is its own mirror).  A
// thread walks its pairs with a stride of the grid, consecutive threads on
// consecutive q2 (the mirrors run backwards, still contiguous).
template <typename T>
__global__ void __launch_bounds__(256) k_split_energy(SplitSym s, FastDiv d12, FastDiv d2, uint32_t npoints,
                                                      const C2<T>* __restrict__ F, double* eparts) {
  const uint32_t nf12 = (uint32_t)s.nf1 * s.nf2;
  double eacc = 0.0;
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t t = blockIdx.x * 256u + threadIdx.x; t < npoints; t += stride) {
    const int q0 = (int)d12.div(t);
    const uint32_t rest = t - (uint32_t)q0 * nf12;
    const int q1 = (int)d2.div(rest);
    const int q2 = (int)(rest - (uint32_t)q1 * s.nf2);
    const int m0 = split_mirror(q0, s.nf0), m1 = split_mirror(q1, s.nf1), m2 = split_mirror(q2, s.nf2);
    const int64_t iq = ((int64_t)q0 * s.nf1 + q1) * s.nf2 + q2;
    const int64_t im = ((int64_t)m0 * s.nf1 + m1) * s.nf2 + m2;
    if (m0 == q0 && im < iq) continue;
    const C2<T> zq = F[iq], zm = F[im];
    const double M = split_symbol_even(s, q0, q1, q2, m0, m1, m2);
    const double dx = (double)zq.x - zm.x, dy = (double)zq.y + zm.y;
    eacc += (im == iq ? 0.25 : 0.5) * M * (dx * dx + dy * dy);
  }
  // deterministic block sum: wave shuffle, then the four waves in order
  for (int off = 32; off > 0; off >>= 1) eacc += __shfl_xor(eacc, off, 64);
  __shared__ double wsum[4];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = eacc;
  __syncthreads();
  if (threadIdx.x == 0) eparts[blockIdx.x] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}

}  // namespace

SplitSym make_split_sym(const Plan& pl) {
  SplitSym a{};
  a.nf0 = pl.nf[0];
  a.nf1 = pl.nf[1];
  a.nf2 = pl.nf[2];
  a.gs0 = log2_exact(pl.GT[0]);
  a.gs1 = log2_exact(pl.GT[1]);
  a.gs2 = log2_exact(pl.GT[2]);
  a.gnt1 = pl.gnt[1];
  a.gnt2 = pl.gnt[2];
  a.kernel = pl.p.kernel;
  a.dim = pl.dim;
  a.a = pl.win[0];
  a.r0 = pl.win[0];
  a.r1 = pl.win[1];
  for (int i = 0; i < 3; ++i) a.axis[i] = pl.p.dipole_axis[i];
  for (int i = 0; i < 3; ++i) a.axis2[i] = pl.axis2[i];
  a.alpha = pl.p.alpha;
  a.mn = a.axis[0] * a.axis2[0] + a.axis[1] * a.axis2[1] + a.axis[2] * a.axis2[2];
  a.n3m3 = a.axis[2] * a.axis2[2];
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
  return a;
}

template <typename T>
hipError_t launch_split_unmix(const Plan& pl, hipStream_t s) {
  if (pl.ntouched == 0) return hipSuccess;
  stage_mark(pl, ST_SPLIT_UNMIX, 0, s);
  hipLaunchKernelGGL(k_split_unmix<T>, dim3(pl.ntouched), dim3(256), 0, s, make_split_sym(pl), pl.d_touched,
                     (const C2<T>*)pl.d_F, (C2<T>*)pl.d_G);
  stage_mark(pl, ST_SPLIT_UNMIX, 1, s);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_split_energy(const Plan& pl, int eoff, hipStream_t s) {
  const uint32_t npoints = (uint32_t)(pl.nf[0] / 2 + 1) * pl.nf[1] * pl.nf[2];
  stage_mark(pl, ST_SPLIT_SYMBOL, 0, s);
  hipLaunchKernelGGL(k_split_energy<T>, dim3(pl.nsym_blocks), dim3(256), 0, s, make_split_sym(pl),
                     FastDiv((uint32_t)pl.nf[1] * pl.nf[2]), FastDiv((uint32_t)pl.nf[2]), npoints,
                     (const C2<T>*)pl.d_F, pl.d_eparts + eoff);
  stage_mark(pl, ST_SPLIT_SYMBOL, 1, s);
  return hipGetLastError();
}

template hipError_t launch_split_unmix<double>(const Plan&, hipStream_t);
template hipError_t launch_split_unmix<float>(const Plan&, hipStream_t);
template hipError_t launch_split_energy<double>(const Plan&, int, hipStream_t);
template hipError_t launch_split_energy<float>(const Plan&, int, hipStream_t);

}  // namespace jgb
