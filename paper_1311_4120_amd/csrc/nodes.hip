// Fourier quadrature nodes and weights (Section 3.1, eqs. 3.5 and 3.7;
// Algorithm 1, step 3), generated on the device in float64.
//
//   radial  : Gauss-Legendre on [0, K]
//   polar   : Gauss-Legendre in theta on [0, pi] with the sin(theta) factor, or
//             Gauss-Legendre in cos(theta) on [-1, 1]
//   azimuth : trapezoidal rule phi_l = 2 pi l / N_phi
//
// The symbol is carried with the Jacobian, S(k) = |k|^{d-1} U^(k), which is
// smooth for every kernel here (Section 3.1 after eq. 3.5): 1 for Coulomb,
// 3 (n.k)(m.k) - (m.n)|k|^2 for the 3D dipole, -alpha |k| + (3/2)
// [(n_p.k)(m_p.k) - n_3 m_3 |k|^2] for the 2.5D dipole (linear along each ray),
// and 1/|k| for the 2D Poisson kernel, whose singular radial integrand is
// completed by the node at k = 0 (plan.hip).
// It is evaluated as written and U^ is never formed.
//
// Only half of the node set is processed downstream: with N_phi even the node
// (r, pi - theta, phi + pi) equals -k, carries the same weight and symbol, and
// its transform is the complex conjugate for real rho.  The half set is
// {phi index l < N_phi/2} and its coefficients carry the factor 2.
//
// For Algorithm 2 (JGB_FLAG_SPLIT) the coefficients also carry the window
// p(k) of I2: exp(-|k|^2 / a) in 3D (eq. 3.10), erfc(12 (|k| - (R0 + R1)/2) /
// (R1 - R0)) / 2 in 2D (eq. 3.12).
#include <cmath>

#include "common.h"

namespace jgb {

namespace {

struct NodeParams {
  int dim, n_r, n_theta, n_phi, rule, kernel, width, rstride;
  int split;       // multiply c_j by the window of Algorithm 2
  double K, beta;
  double win[2];   // 3D: (a, 0); 2D: (R0, R1)
  double axis[3];
  double axis2[3];  // second orientation m (= n unless given)
  double alpha;     // 2.5D dipole constant
  double box[3];  // physical side lengths per internal axis (unit axis: 0)
  int nf[3], w[3], T[3], nt[3], S[3];
  const double* gl_r;
  const double* gl_t;
};

NodeParams make_params(const Plan& pl) {
  NodeParams q{};
  q.dim = pl.dim;
  q.n_r = pl.n_r;
  q.n_theta = pl.n_theta;
  q.n_phi = pl.n_phi;
  q.rule = pl.p.theta_rule;
  q.kernel = pl.p.kernel;
  q.width = pl.width;
  q.rstride = record_stride(pl.width);
  q.K = pl.K;
  q.beta = pl.beta;
  q.split = pl.split ? 1 : 0;
  q.win[0] = pl.win[0];
  q.win[1] = pl.win[1];
  for (int i = 0; i < 3; ++i) q.axis[i] = pl.p.dipole_axis[i];
  for (int i = 0; i < 3; ++i) q.axis2[i] = pl.axis2[i];
  q.alpha = pl.p.alpha;
  for (int i = 0; i < 3; ++i) {
    q.box[i] = (pl.n[i] == 1) ? 0.0 : pl.box[i];
    q.nf[i] = pl.nf[i];
    q.w[i] = pl.w[i];
    q.T[i] = pl.T[i];
    q.nt[i] = pl.nt[i];
    q.S[i] = pl.S[i];
  }
  q.gl_r = pl.d_gl_r;
  q.gl_t = pl.d_gl_t;
  return q;
}

// P_n(x) and P_n'(x) by the three-term recurrence and P'_{k+1} = P'_{k-1} + (2k+1) P_k.
__device__ void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    double d2 = d0 + (2.0 * k + 1.0) * p1;
    p0 = p1;
    p1 = p2;
    d0 = d1;
    d1 = d2;
  }
  p = p1;
  dp = d1;
}

// One thread per root: ascending nodes s_i in out[0..n), weights in out[n..2n).
// Roots of the lower half are found by Newton's method from the classical
// estimate -cos(pi (i + 3/4) / (n + 1/2)); the upper half is their mirror image,
// so the rule is exactly symmetric.
__global__ void k_gl_roots(int n, double* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int j = (i < n - 1 - i) ? i : n - 1 - i;
  double x;
  if (2 * j + 1 == n) {
    x = 0.0;
  } else {
    x = -cos(M_PI * (j + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(n, x, p, dp);
      double dx = p / dp;
      x -= dx;
      if (fabs(dx) <= 1e-16 * fabs(x) + 1e-300) break;
    }
  }
  double p, dp;
  legendre(n, x, p, dp);
  double wgt = 2.0 / ((1.0 - x * x) * dp * dp);
  out[i] = (i == j) ? x : -x;
  out[n + i] = wgt;
}

// Node (a, b, l) of the full set in physical coordinates and its weight.
__device__ void full_node(const NodeParams& q, int a, int b, int l, double k[3], double& W) {
  double s = q.gl_r[a], om = q.gl_r[q.n_r + a];
  double r = 0.5 * q.K * (1.0 + s);
  double wr = 0.5 * q.K * om;
  double sp, cp;
  sincospi(2.0 * l / q.n_phi, &sp, &cp);
  double wphi = 2.0 * M_PI / q.n_phi;
  if (q.dim == 3) {
    double sb = q.gl_t[b], omb = q.gl_t[q.n_theta + b];
    double ct, st, wt;
    if (q.rule == JGB_THETA_GL) {
      // theta = pi (1 + s)/2: cos(theta) = -sin(pi s/2), sin(theta) = cos(pi s/2)
      ct = -sinpi(0.5 * sb);
      st = cospi(0.5 * sb);
      wt = 0.5 * M_PI * omb * st;
    } else {
      ct = sb;
      st = sqrt((1.0 - sb) * (1.0 + sb));
      wt = omb;
    }
    k[0] = r * st * cp;
    k[1] = r * st * sp;
    k[2] = r * ct;
    W = wr * wt * wphi;
  } else {
    k[0] = r * cp;
    k[1] = r * sp;
    k[2] = 0.0;
    W = wr * wphi;
  }
}

// S(k) = |k|^{d-1} U^(k) for the kernels of eq. int3dd handled here (k in
// physical coordinates; 2D nodes have k[2] = 0).
__device__ double symbol(const NodeParams& q, const double k[3]) {
  const double kk = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  if (q.kernel == JGB_DIPOLE_3D) {
    const double nk = q.axis[0] * k[0] + q.axis[1] * k[1] + q.axis[2] * k[2];
    const double mk = q.axis2[0] * k[0] + q.axis2[1] * k[1] + q.axis2[2] * k[2];
    const double mn = q.axis[0] * q.axis2[0] + q.axis[1] * q.axis2[1] + q.axis[2] * q.axis2[2];
    return 3.0 * nk * mk - mn * kk;
  }
  if (q.kernel == JGB_DIPOLE_2D) {
    const double nk = q.axis[0] * k[0] + q.axis[1] * k[1];
    const double mk = q.axis2[0] * k[0] + q.axis2[1] * k[1];
    return -q.alpha * sqrt(kk) + 1.5 * (nk * mk - q.axis[2] * q.axis2[2] * kk);
  }
  if (q.kernel == JGB_POISSON_2D) return 1.0 / sqrt(kk);  // radial nodes are interior: kk > 0
  return 1.0;
}

// The window p(k) of Algorithm 2 (1 without JGB_FLAG_SPLIT).
__device__ double window(const NodeParams& q, const double k[3]) {
  if (!q.split) return 1.0;
  const double kk = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  if (q.dim == 3) return exp(-kk / q.win[0]);
  return 0.5 * erfc(12.0 * (sqrt(kk) - 0.5 * (q.win[0] + q.win[1])) / (q.win[1] - q.win[0]));
}

__device__ void half_node(const NodeParams& q, int64_t h, double k[3], double& W) {
  int nph2 = q.n_phi / 2;
  int l = (int)(h % nph2);
  int64_t rest = h / nph2;
  int a, b;
  if (q.dim == 3) {
    b = (int)(rest % q.n_theta);
    a = (int)(rest / q.n_theta);
  } else {
    b = 0;
    a = (int)rest;
  }
  full_node(q, a, b, l, k, W);
}

// Fine-grid position of the node per internal axis: s = t n_f/(2 pi) with
// t = k h and n_f = 2 N, i.e. s = k R / pi (cells), in (-n_f/2, n_f/2).
__device__ void fine_position(const NodeParams& q, const double k[3], double s[3]) {
  if (q.dim == 3) {
    s[0] = k[0] * q.box[0] / M_PI;
    s[1] = k[1] * q.box[1] / M_PI;
    s[2] = k[2] * q.box[2] / M_PI;
  } else {
    s[0] = 0.0;
    s[1] = k[0] * q.box[1] / M_PI;
    s[2] = k[1] * q.box[2] / M_PI;
  }
}

// First tap of the footprint: ceil(s - w/2), so every tap lies within w/2 of s.
__device__ void footprint(const NodeParams& q, const double s[3], int start[3], double frac[3]) {
  for (int i = 0; i < 3; ++i) {
    double x0 = ceil(s[i] - 0.5 * q.w[i]);
    frac[i] = s[i] - x0;
    long long xi = (long long)x0;
    long long m = xi % q.nf[i];
    if (m < 0) m += q.nf[i];
    start[i] = (int)m;
  }
}

__global__ void k_node_keys(NodeParams q, int64_t Mh, int* keys) {
  int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= Mh) return;
  double k[3], W, s[3], frac[3];
  int st[3];
  half_node(q, h, k, W);
  fine_position(q, k, s);
  footprint(q, s, st, frac);
  int b0 = st[0] / q.T[0], b1 = st[1] / q.T[1], b2 = st[2] / q.T[2];
  int bin = (b0 * q.nt[1] + b1) * q.nt[2] + b2;
  int s0 = (st[0] % q.T[0]) / q.S[0], s1 = (st[1] % q.T[1]) / q.S[1], s2 = (st[2] % q.T[2]) / q.S[2];
  int m1 = q.T[1] / q.S[1], m2 = q.T[2] / q.S[2];
  int nsub = (q.T[0] / q.S[0]) * m1 * m2;
  keys[h] = bin * nsub + (s0 * m1 + s1) * m2 + s2;
}

// Per node: footprint start, fractional offsets, coefficient 2 c_j, and the
// kernel values of the footprint on each axis.  The kernel values depend on
// the node alone, so they are tabulated once here and read by both NUFFT
// directions on every evaluation: axis a's w taps at [a w, a w + w) of the
// node's record (a unit axis: 1 at tap 0, zeros after it).
template <typename T>
__global__ void k_node_setup(NodeParams q, int64_t Mh, const int* perm, int4* hdr, T* f0, T* f1, T* f2,
                             double* coef, T* wts) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Mh) return;
  int64_t h = perm[p];
  double k[3], W, s[3], frac[3];
  int st[3];
  half_node(q, h, k, W);
  fine_position(q, k, s);
  footprint(q, s, st, frac);
  hdr[p] = make_int4(st[0], st[1], st[2], 0);
  f0[p] = (T)frac[0];
  f1[p] = (T)frac[1];
  f2[p] = (T)frac[2];
  double twopi_d = (q.dim == 3) ? 8.0 * M_PI * M_PI * M_PI : 4.0 * M_PI * M_PI;
  // factor 2: the node stands for itself and for -k (conjugate transform, same c)
  coef[p] = 2.0 * W * symbol(q, k) * window(q, k) / twopi_d;
  T* rec = wts + p * q.rstride;
  for (int ax = 0; ax < 3; ++ax) {
    const int w = q.w[ax];
    const T f = (T)frac[ax], tw = (T)(2.0 / w), beta = (T)q.beta;
    T* out = rec + ax * (q.width + 1);
    for (int t = 0; t < q.width; ++t)
      out[t] = (t >= w)  ? T(0)
               : w == 1  ? T(1)
               : q.beta == 0.0 ? gauss_kernel<T>(T(t) - f)
                               : es_kernel<T>(T(t) - f, tw, beta);
  }
}

__global__ void k_node_export(NodeParams q, int64_t M, double* kout, double* wout, double* cout) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  int l = (int)(j % q.n_phi);
  int64_t rest = j / q.n_phi;
  int a, b;
  if (q.dim == 3) {
    b = (int)(rest % q.n_theta);
    a = (int)(rest / q.n_theta);
  } else {
    b = 0;
    a = (int)rest;
  }
  double k[3], W;
  full_node(q, a, b, l, k, W);
  if (kout) {
    for (int i = 0; i < q.dim; ++i) kout[j * q.dim + i] = k[i];
  }
  if (wout) wout[j] = W;
  if (cout) {
    double twopi_d = (q.dim == 3) ? 8.0 * M_PI * M_PI * M_PI : 4.0 * M_PI * M_PI;
    cout[j] = W * symbol(q, k) * window(q, k) / twopi_d;
  }
}

unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hipError_t launch_gl_roots(int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gl_roots, dim3(grid_for(n, 64)), dim3(64), 0, s, n, out);
  return hipGetLastError();
}

hipError_t launch_node_keys(const Plan& pl, int* keys, hipStream_t s) {
  NodeParams q = make_params(pl);
  hipLaunchKernelGGL(k_node_keys, dim3(grid_for(pl.Mh, 256)), dim3(256), 0, s, q, pl.Mh, keys);
  return hipGetLastError();
}

hipError_t launch_node_setup(const Plan& pl, const int* perm, hipStream_t s) {
  NodeParams q = make_params(pl);
  const NodeArrays& a = pl.nodes;
  if (pl.fp64) {
    hipLaunchKernelGGL(k_node_setup<double>, dim3(grid_for(pl.Mh, 256)), dim3(256), 0, s, q, pl.Mh, perm,
                       a.hdr, (double*)a.frac[0], (double*)a.frac[1],
                       (double*)a.frac[2], a.coef, (double*)a.wts);
  } else {
    hipLaunchKernelGGL(k_node_setup<float>, dim3(grid_for(pl.Mh, 256)), dim3(256), 0, s, q, pl.Mh, perm,
                       a.hdr, (float*)a.frac[0], (float*)a.frac[1],
                       (float*)a.frac[2], a.coef, (float*)a.wts);
  }
  return hipGetLastError();
}

hipError_t launch_node_export(const Plan& pl, double* k, double* w, double* c, hipStream_t s) {
  NodeParams q = make_params(pl);
  hipLaunchKernelGGL(k_node_export, dim3(grid_for(pl.M, 256)), dim3(256), 0, s, q, pl.M, k, w, c);
  return hipGetLastError();
}

}  // namespace jgb
