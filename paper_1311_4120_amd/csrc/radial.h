// Generalized Gaussian radial rule for band-limited integrands (the remark at
// the end of Section 3.3 and the Conclusions: where polar or spherical
// coordinates leave the radial integrand hard to integrate, a generalized
// Gaussian rule is built for it).  Host code, free of device code.
//
// Along a ray the NUFFT's radial integrand r -> rho^(r e) e^{i r e.x} is
// band-limited (its frequencies are bounded by the box's diameter).  The
// n-node rule of bandwidth c on [-1, 1] of Xiao, Rokhlin and Yarvin (Prolate
// spheroidal wavefunctions, quadrature and interpolation, Inverse Problems 17,
// 2001) integrates e^{i s x}, |s| <= 2c, with fewer nodes than Gauss-Legendre:
// its nodes are the n roots of the prolate spheroidal wave function psi_n^c,
// its weights solve sum_j w_j psi_i^c(x_j) = int psi_i^c, i < n.
//
// psi_i^c = sum_k beta_k sqrt(k + 1/2) P_k: the coefficient vectors are the
// eigenvectors of the symmetric tridiagonal matrices (even k, odd k)
//   A_kk = k (k + 1) + c^2 (2 k (k + 1) - 1) / ((2k + 3)(2k - 1)),
//   A_k,k+2 = c^2 (k + 2)(k + 1) / ((2k + 3) sqrt((2k + 1)(2k + 5))),
// psi_i^c belonging to the i-th smallest eigenvalue overall; here each is found
// by Sturm-sequence bisection and inverse iteration.  The plan's bandwidth for
// n nodes at accuracy eps is c = (pi/2)(n - 2 - 1.8 log10(10/eps) - 0.06 n),
// which keeps the rule's error on e^{i s x}, |s| <= 2c, well below eps;
// below c = 1 the rule is Gauss-Legendre.
#pragma once

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace jgb {
namespace radial {

inline double bandwidth(int n, double eps) {
  const double c = 0.5 * M_PI * (n - 2.0 - 1.8 * std::log10(10.0 / eps) - 0.06 * n);
  return c >= 1.0 ? c : 0.0;
}

// Number of eigenvalues of the symmetric tridiagonal (d, e) below x.
inline int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
  int count = 0;
  double q = 1.0;
  for (size_t i = 0; i < d.size(); ++i) {
    const double off = i ? e[i - 1] * e[i - 1] : 0.0;
    q = d[i] - x - (i ? off / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++count;
  }
  return count;
}

// The m-th smallest eigenvalue (m from 0) of (d, e) and its unit eigenvector.
inline void tridiag_eigenpair(const std::vector<double>& d, const std::vector<double>& e, int m, double& lambda,
                              std::vector<double>& v) {
  const size_t N = d.size();
  double lo = d[0], hi = d[0];
  for (size_t i = 0; i < N; ++i) {
    const double r = (i ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < N ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_count(d, e, mid) > m) hi = mid;
    else lo = mid;
  }
  lambda = 0.5 * (lo + hi);
  // inverse iteration: (A - mu I) y = v, tridiagonal elimination with partial pivoting
  const double mu = lambda + 1e-13 * std::max(1.0, std::fabs(lambda));
  v.assign(N, 1.0 / std::sqrt((double)N));
  std::vector<double> a(N), b(N), c(N), f(N), y(N);
  for (int iter = 0; iter < 4; ++iter) {
    // rows i: sub a[i] (i > 0), diag b[i], super c[i] (i + 1 < N), second super f[i]
    for (size_t i = 0; i < N; ++i) {
      a[i] = i ? e[i - 1] : 0.0;
      b[i] = d[i] - mu;
      c[i] = i + 1 < N ? e[i] : 0.0;
      f[i] = 0.0;
      y[i] = v[i];
    }
    for (size_t i = 0; i + 1 < N; ++i) {
      if (std::fabs(a[i + 1]) > std::fabs(b[i])) {  // swap rows i and i + 1
        std::swap(b[i], a[i + 1]);
        std::swap(c[i], b[i + 1]);
        std::swap(f[i], c[i + 1]);
        std::swap(y[i], y[i + 1]);
      }
      if (b[i] == 0.0) b[i] = 1e-300;
      const double l = a[i + 1] / b[i];
      b[i + 1] -= l * c[i];
      c[i + 1] -= l * f[i];
      y[i + 1] -= l * y[i];
      a[i + 1] = 0.0;
    }
    if (b[N - 1] == 0.0) b[N - 1] = 1e-300;
    for (size_t k = N; k-- > 0;) {
      double s = y[k];
      if (k + 1 < N) s -= c[k] * v[k + 1];
      if (k + 2 < N) s -= f[k] * v[k + 2];
      v[k] = s / b[k];
    }
    double nrm = 0.0;
    for (double x : v) nrm += x * x;
    nrm = std::sqrt(nrm);
    for (double& x : v) x /= nrm;
  }
}

// psi(x) for normalised-Legendre coefficients coef (sum_k coef_k sqrt(k + 1/2) P_k(x)).
inline double prolate_eval(const std::vector<double>& coef, double x) {
  double p0 = 1.0, p1 = x, s = coef[0] * std::sqrt(0.5);
  if (coef.size() > 1) s += coef[1] * std::sqrt(1.5) * p1;
  for (size_t k = 1; k + 1 < coef.size(); ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
    s += coef[k + 1] * std::sqrt(k + 1.5) * p1;
  }
  return s;
}

// The n-node rule of bandwidth c on [-1, 1]: nodes ascending, weights.
inline std::string prolate_rule(double c, int n, std::vector<double>& x, std::vector<double>& w) {
  const int M = 2 * (n + 1) + (int)std::ceil(2.0 * c) + 64;
  std::vector<std::vector<double>> coef(n + 1, std::vector<double>(M, 0.0));
  for (int par = 0; par < 2; ++par) {
    std::vector<double> d, e;
    for (int k = par; k < M; k += 2) {
      const double kk = k;
      d.push_back(kk * (kk + 1) + c * c * (2 * kk * (kk + 1) - 1) / ((2 * kk + 3) * (2 * kk - 1)));
      if (k + 2 < M) e.push_back(c * c * (kk + 2) * (kk + 1) / ((2 * kk + 3) * std::sqrt((2 * kk + 1) * (2 * kk + 5))));
    }
    for (int i = par; i <= n; i += 2) {
      double lambda;
      std::vector<double> v;
      tridiag_eigenpair(d, e, i / 2, lambda, v);
      for (size_t q = 0; q < v.size(); ++q) coef[i][par + 2 * q] = v[q];
    }
  }
  // roots of psi_n: sign changes on a fine Chebyshev grid, then bisection
  const int G = 40 * n + 400;
  x.clear();
  double xa = -1.0, fa = prolate_eval(coef[n], xa);
  for (int g = 1; g <= G; ++g) {
    const double xb = -std::cos(M_PI * g / G), fb = prolate_eval(coef[n], xb);
    if (fa == 0.0) {
      x.push_back(xa);
    } else if (fa * fb < 0.0) {
      double lo = xa, hi = xb, flo = fa;
      for (int it = 0; it < 200 && hi - lo > 1e-16; ++it) {
        const double mid = 0.5 * (lo + hi), fm = prolate_eval(coef[n], mid);
        if ((fm < 0.0) == (flo < 0.0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      x.push_back(0.5 * (lo + hi));
    }
    xa = xb;
    fa = fb;
  }
  if ((int)x.size() != n) return "prolate function has the wrong number of roots";
  // weights: sum_j w_j psi_i(x_j) = int psi_i = sqrt(2) beta_0 (i < n), Gaussian elimination
  std::vector<double> A((size_t)n * (n + 1));
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) A[(size_t)i * (n + 1) + j] = prolate_eval(coef[i], x[j]);
    A[(size_t)i * (n + 1) + n] = std::sqrt(2.0) * coef[i][0];
  }
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * (n + 1) + col]) > std::fabs(A[(size_t)piv * (n + 1) + col])) piv = r;
    if (A[(size_t)piv * (n + 1) + col] == 0.0) return "singular prolate weight system";
    if (piv != col)
      for (int k = 0; k <= n; ++k) std::swap(A[(size_t)piv * (n + 1) + k], A[(size_t)col * (n + 1) + k]);
    for (int r = col + 1; r < n; ++r) {
      const double l = A[(size_t)r * (n + 1) + col] / A[(size_t)col * (n + 1) + col];
      for (int k = col; k <= n; ++k) A[(size_t)r * (n + 1) + k] -= l * A[(size_t)col * (n + 1) + k];
    }
  }
  w.assign(n, 0.0);
  for (int r = n - 1; r >= 0; --r) {
    double s = A[(size_t)r * (n + 1) + n];
    for (int k = r + 1; k < n; ++k) s -= A[(size_t)r * (n + 1) + k] * w[k];
    w[r] = s / A[(size_t)r * (n + 1) + r];
  }
  return "";
}

}  // namespace radial
}  // namespace jgb
