// Algorithm 2's regular-grid spectrum (Section 3.3, eq. 3.9): the symbol of I1
// and the tile geometry, shared by the inverse FFT's first pass (fft.hip),
// which forms the spectrum, and the energy kernel (split.hip).
//
// The forward FFT of rho H / phi^ + i rho H gives Z = A + i B, with
// B(q) = (Z(q) - conj Z(-q)) / (2 i) = rho^(k_q) at k_q = 2 pi q' / (2 R_j)
// (q' the signed index).  The inverse FFT takes
//   Y(q) = (G(q) + conj G(-q)) / 2 + i M'(q) B(q)
//        = (G(q) + conj G(-q)) / 2 + M'(q) (Z(q) - conj Z(-q)) / 2,
// M' = (1 - p) U^ / prod_j (2 R_j), G the spreading grid of I2 (zero outside
// the gather tiles some node touches).  The mirror of fine index q on an axis
// of nf points is (nf - q) mod nf.
#pragma once

#include "common.h"

namespace jgb {

struct SplitSym {
  int nf0, nf1, nf2;
  int gs0, gs1, gs2;   // log2 of the gather tile extents
  int gnt1, gnt2;      // gather tiles along axes 1 and 2
  int kernel, dim;
  double a, r0, r1;    // window: a (3D) or R0, R1 (2D)
  double axis[3];      // dipole orientations n and m (physical coordinates)
  double axis2[3];
  double alpha;        // 2.5D dipole constant
  double mn, n3m3;     // m.n and n_3 m_3
  double inv_vol;      // 1 / prod_j (2 R_j)
  const double* kt;    // per axis: k_a(q) for q < nf_a, then exp(-k_a(q)^2 / a)
  int koff[3], eoff[3];
  const unsigned char* tflag;  // per gather tile: 1 if some node touches it
};

// Host: the plan's symbol parameters (split.hip).
SplitSym make_split_sym(const Plan& pl);

__device__ inline int split_mirror(int q, int nf) { return q ? nf - q : 0; }

// M'(q) with its k = 0 limit (1/a for the 3D Coulomb kernel; 0 for the
// dipoles, where 1 - p vanishes and U^ is bounded, and for the 2D Coulomb and
// Poisson kernels, where 1 - p is below 1e-20 at the default scales and
// (1 - p)/|k|^2 below 1e-17 at the first grid frequency), from
// kk = |k|^2, the 3D window wprod = p(k) (unused in 2D) and n.k, m.k over the
// physical axes (in 2D the in-plane parts).  In 3D the window is the product
// of per-axis tables, so 1 - p is 1 minus that product: at the grid's smallest
// nonzero |k| the subtraction costs under four bits at the default scale
// a = 2 dk^2.
__device__ inline double split_symbol_core(const SplitSym& s, double kk, double wprod, double nk, double mk) {
  if (kk == 0.0) return s.kernel == JGB_COULOMB_3D ? s.inv_vol / s.a : 0.0;
  if (s.dim == 3) {
    const double omp = 1.0 - wprod;
    if (s.kernel == JGB_COULOMB_3D) return s.inv_vol * omp / kk;
    return s.inv_vol * omp * (3.0 * nk * mk / kk - s.mn);
  }
  const double kabs = sqrt(kk);
  const double omp = 0.5 * erfc(-12.0 * (kabs - 0.5 * (s.r0 + s.r1)) / (s.r1 - s.r0));
  if (s.kernel == JGB_COULOMB_2D) return s.inv_vol * omp / kabs;
  if (s.kernel == JGB_POISSON_2D) return s.inv_vol * omp / kk;
  return s.inv_vol * omp * (-s.alpha + 1.5 * (nk * mk - s.n3m3 * kk) / kabs);
}

// M'(q) at fine indices (q0, q1, q2); in 2D the physical frequency is (k1, k2)
// of the internal axes (a1, a2).
__device__ inline double split_symbol(const SplitSym& s, int q0, int q1, int q2) {
  const double k0 = s.kt[s.koff[0] + q0], k1 = s.kt[s.koff[1] + q1], k2 = s.kt[s.koff[2] + q2];
  const double kk = k0 * k0 + k1 * k1 + k2 * k2;
  double nk, mk, w = 0.0;
  if (s.dim == 3) {
    w = s.kt[s.eoff[0] + q0] * s.kt[s.eoff[1] + q1] * s.kt[s.eoff[2] + q2];
    nk = s.axis[0] * k0 + s.axis[1] * k1 + s.axis[2] * k2;
    mk = s.axis2[0] * k0 + s.axis2[1] * k1 + s.axis2[2] * k2;
  } else {
    nk = s.axis[0] * k1 + s.axis[1] * k2;
    mk = s.axis2[0] * k1 + s.axis2[1] * k2;
  }
  return split_symbol_core(s, kk, w, nk, mk);
}

// The symbol the real I1 uses at q.  On a Nyquist plane (q_a = nf_a / 2) the
// grid frequency is its own mirror on that axis, so k(-q) is not -k(q) there
// and a dipole symbol, which is not a function of |k| alone, differs between
// q and -q; I1 is real, so the sum takes the mean of the two (the Hermitian
// part of M B).
__device__ inline double split_symbol_even(const SplitSym& s, int q0, int q1, int q2, int m0, int m1, int m2) {
  double M = split_symbol(s, q0, q1, q2);
  if ((s.kernel == JGB_DIPOLE_3D || s.kernel == JGB_DIPOLE_2D) &&
      (2 * q0 == s.nf0 || 2 * q1 == s.nf1 || 2 * q2 == s.nf2))
    M = 0.5 * (M + split_symbol(s, m0, m1, m2));
  return M;
}

__device__ inline int split_tile(const SplitSym& s, int q0, int q1, int q2) {
  return (((q0 >> s.gs0) * s.gnt1) + (q1 >> s.gs1)) * s.gnt2 + (q2 >> s.gs2);
}

}  // namespace jgb
