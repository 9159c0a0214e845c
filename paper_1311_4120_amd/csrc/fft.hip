// Oversampled-grid FFTs of the two NUFFTs (Section 2, eqs. 2.5-2.6 and the
// deconvolution step; the type-2 transform runs the type-1 steps in reverse).
//
// Each 3D FFT is three passes of batched 1D transforms, one per axis.  A pass
// stages LB lines of length L in LDS, runs a Stockham autosort FFT with radices
// 8, 4, 2, 3, 5 (also 16 in Algorithm 2's float32 paired passes; twiddles from
// a float64 table rounded to the working type), and writes the lines back.
// Zero padding is never stored: forward passes place the N nonzero inputs of a
// line at fine indices (m mod L), m in [-N/2, N/2), and zero the rest in LDS;
// inverse passes write only those N outputs (the crop to the physical grid).
//
//   forward (type-2 front, sign -1):
//     Z: rho (N0 N1 N2 reals) x H/(phi^0 phi^1 phi^2)  -> A1 [N0][N1][nf2]
//     Y: A1 -> A2 [N0][nf1][nf2]
//     X: A2 -> F  [nf0][nf1][nf2]
//   inverse (type-1 back, sign +1):
//     X: G  -> B2 [N0][nf1][nf2]
//     Y: B2 -> B1 [N0][N1][nf2]
//     Z: B1 -> u = Re(.) / (phi^0 phi^1 phi^2), and partial sums of rho u
//
// Algorithm 2 (JGB_FLAG_SPLIT) changes four things: the forward Z pass also
// places rho H in the imaginary part (two real transforms in one complex
// one); the potential's forward FFT stops before the last axis (X in 3D, Y in
// 2D) and a paired unmix pass along it writes the type-2 grid into the tiles
// the interpolation reads; the inverse's first pass is a fused paired pass that
// transforms the same inputs forward again, forms the combined spectrum of both
// halves and transforms it back (so the full forward spectrum is never
// stored); and the last pass adds the imaginary part (I1) to u.  The
// energy-only and transform calls run the full forward FFT into F.
#include <cmath>

#include "splitsym.h"

namespace jgb {

namespace {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {  // one 16-byte (fp64) or 8-byte (fp32) access
  T x, y;
};

template <typename T>
__device__ inline C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ inline C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ inline C2<T> cmul(C2<T> a, C2<T> b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// multiply by i * s (s = +-1)
template <typename T>
__device__ inline C2<T> cmul_is(C2<T> a, T s) { return {-s * a.y, s * a.x}; }
template <typename T>
__device__ inline C2<T> cscale(C2<T> a, T s) { return {a.x * s, a.y * s}; }

// In-register DFTs of small radix, y_k = sum_n x_n exp(s 2 pi i n k / R).
template <typename T>
__device__ inline void dft2(C2<T>* v, T) {
  C2<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T>
__device__ inline void dft4(C2<T>* v, T s) {
  C2<T> a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  C2<T> c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
  C2<T> isd = cmul_is(d, s);
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, isd);
  v[3] = csub(b, isd);
}

template <typename T>
__device__ inline void dft3(C2<T>* v, T s) {
  const T h = T(0.86602540378443864676);  // sin(2 pi / 3)
  C2<T> t = cadd(v[1], v[2]);
  C2<T> m = {v[0].x - T(0.5) * t.x, v[0].y - T(0.5) * t.y};
  C2<T> d = cmul_is(csub(v[1], v[2]), s * h);
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, d);
  v[2] = csub(m, d);
}

template <typename T>
__device__ inline void dft5(C2<T>* v, T s) {
  const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
  const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
  C2<T> a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
  C2<T> a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
  C2<T> x0 = v[0];
  C2<T> r1 = {x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y};
  C2<T> r2 = {x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y};
  C2<T> q1 = {s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y};
  C2<T> q2 = {s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y};
  C2<T> iq1 = cmul_is(q1, s), iq2 = cmul_is(q2, s);
  v[0] = cadd(x0, cadd(a1, a2));
  v[1] = cadd(r1, iq1);
  v[4] = csub(r1, iq1);
  v[2] = cadd(r2, iq2);
  v[3] = csub(r2, iq2);
}

template <typename T>
__device__ inline void dft8(C2<T>* v, T s) {
  const T r = T(0.70710678118654752440);
  C2<T> e[4] = {v[0], v[2], v[4], v[6]};
  C2<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4(e, s);
  dft4(o, s);
  // twiddles w^k, w = exp(s 2 pi i / 8)
  C2<T> o1 = {r * (o[1].x - s * o[1].y), r * (o[1].y + s * o[1].x)};
  C2<T> o2 = cmul_is(o[2], s);
  C2<T> o3 = {r * (-o[3].x - s * o[3].y), r * (-o[3].y + s * o[3].x)};
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

// Radix 16 as 4 x 4: with n = 4 n1 + n2 and k = k1 + 4 k2,
// y_k = sum_n2 w16^(n2 k1) [sum_n1 x_(4 n1 + n2) w4^(n1 k1)] w4^(n2 k2).
template <typename T>
__device__ inline void dft16(C2<T>* v, T s) {
  const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);  // cos, sin of pi/8
  const T r = T(0.70710678118654752440);
  C2<T> a[4][4];  // a[n2][k1]
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    C2<T> t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
    dft4(t, s);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) a[n2][k1] = t[k1];
  }
  // twiddles w16^m = (cos(2 pi m / 16), s sin(2 pi m / 16)) for m = n2 k1
  const C2<T> w1{c1, s * s1}, w2{r, s * r}, w3{s1, s * c1}, w6{-r, s * r}, w9{-c1, -s * s1};
  a[1][1] = cmul(a[1][1], w1);
  a[1][2] = cmul(a[1][2], w2);
  a[1][3] = cmul(a[1][3], w3);
  a[2][1] = cmul(a[2][1], w2);
  a[2][2] = cmul_is(a[2][2], s);
  a[2][3] = cmul(a[2][3], w6);
  a[3][1] = cmul(a[3][1], w3);
  a[3][2] = cmul(a[3][2], w6);
  a[3][3] = cmul(a[3][3], w9);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    C2<T> t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
    dft4(t, s);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
  }
}

template <typename T, int R>
__device__ inline void dft(C2<T>* v, T s) {
  if constexpr (R == 2) dft2(v, s);
  if constexpr (R == 3) dft3(v, s);
  if constexpr (R == 4) dft4(v, s);
  if constexpr (R == 5) dft5(v, s);
  if constexpr (R == 8) dft8(v, s);
  if constexpr (R == 16) dft16(v, s);
}

// FWD_Z / INV_Z: the oversampled grid's first and last passes (real in or out,
// deconvolution factors); COMPLEX: a complex pass along a strided axis;
// COMPLEX_Z: a complex pass along the contiguous axis (the periodic FFT).
// KINETIC: the GPE driver's kinetic step along one strided axis: the forward
// transform, the multiplier exp(-i h |k|^2 / 2) / N (imaginary time:
// exp(-h |k|^2 / 2) / N), and the inverse transform, in LDS.
// HSYM: the inverse's first pass on a real output, a strided complex pass
// whose input is the Hermitian part of the spreading grid.
enum PassKind { PASS_FWD_Z = 0, PASS_COMPLEX = 1, PASS_INV_Z = 2, PASS_COMPLEX_Z = 3, PASS_KINETIC = 4, PASS_HSYM = 5 };
template <int KIND>
constexpr bool has_factors() { return KIND == PASS_FWD_Z || KIND == PASS_INV_Z; }

template <typename T>
struct PassArgs {
  int L;            // line length
  int64_t nlines;
  int LB;           // lines per block
  int nin;          // inputs per line (L, or N when the input is zero-padded)
  int nout;         // outputs per line (L, or N when the output is cropped)
  int64_t ic;       // lines per outer group; line l = (outer, inner) = (l / ic, l % ic)
  int64_t in_os, in_is, in_es;
  int64_t out_os, out_is, out_es;
  T sign;
  int nrad;
  int rad[12];
  int tws[12];      // twiddle stride of each radix stage, L / (Ns R)
  FastDiv dNs[12];  // Ns of each radix stage (product of the earlier radices)
  FastDiv dLB, dnin, dnout, dic, dn1;
  const C2<T>* tw;  // exp(-2 pi i t / L), t < L
  const void* in;
  void* out;
  // forward Z: deconvolution and cell volume; inverse Z: deconvolution and energy
  const double* dec0;
  const double* dec1;
  const double* dec2;
  double scale;
  int n1, n2;         // physical grid sizes of axes 1 and 2 (Z passes)
  const T* rho;       // inverse Z: density for the energy partial (nullable)
  double* eparts;     // inverse Z: per-block partials of sum rho u
  int split;          // Z passes of Algorithm 2: forward imag = rho H; inverse u += imag
  double* mparts;     // forward Z: per-block sums of rho (the node at k = 0), nullable
  const double* shift;  // inverse Z: constant added to u (the node at k = 0), nullable
  // Hermitian half along the last axis (real input, Algorithm 1): the forward
  // Z pass stores only outputs 0 .. nout - 1 = L/2 (half_out); the inverse Z
  // pass loads those nin = L/2 + 1 values and completes the line by
  // v(L - p) = conj v(p) (half_in); the inverse's first pass (PASS_HSYM)
  // averages each element with the conjugate of its mirror,
  // v(q) = (g(q) + conj g(-q)) / 2, the mirror of line (outer, inner) and
  // element e being (-outer mod sym_no, -inner mod sym_ni, -e mod L)
  int half_out, half_in, sym_no, sym_ni;
  // PASS_HSYM: per input line (outer sym_ni + inner), the circular range
  // {first, span} of elements the spreading can have written; the pass takes
  // the other elements as zero without loading them
  const int2* lext;
  // PASS_COMPLEX (optional): per output line, the circular range {first,
  // span} of elements that are read later; the pass stores no others
  const int2* oext;
  // the paired passes of Algorithm 2 (k_fft_pair_pass): lines are
  // (a, b) of an A x B set, element stride es_in / es_out; P lines and their
  // mirrors per block; nb1 blocks for the rows 0 < a < A/2 (cb per row), then cs
  // per row for the rows that are their own mirror (a = 0 and a = A/2)
  int P, A, B, nb1, cb, cs, dim3;
  FastDiv dP;
  const int* blist;   // the unmix pass's logical blocks
  int64_t es_in, es_out;
  const void* G;
  SplitSym sym;
  // the kinetic pass: k per internal axis in kt (offsets koff), the pass's
  // axis kax (0, or 1 when axis 0 is a unit axis), a line's two other axes
  // (a, b) = (line / nb, line mod nb) with the divisor in dkb
  const double* kt;
  int koff[3];
  int kax;
  FastDiv dkb;
  double kin_h, inv_n;
  int kin_imag;
};

// Byte offset of a pass block's twiddle table in LDS: after LB padded lines
// and, for the Z passes, LB + L deconvolution factors; 16-byte aligned.
template <typename T>
__host__ __device__ inline size_t pass_twiddle_offset(int LB, int L, bool factors) {
  size_t off = (size_t)LB * (L + 1) * sizeof(C2<T>);
  if (factors) off += sizeof(double) * (LB + L);
  return (off + 15) & ~(size_t)15;
}

// Position on the fine grid of physical index i of a line of N: (i - N/2) mod L.
__device__ inline int fine_pos(int i, int N, int L) {
  int m = i - N / 2;
  return m < 0 ? m + L : m;
}

template <typename T, int R, int MAXV>
__device__ inline void stage(C2<T>* lds, int ldl, int L, int LB, int Ns, const FastDiv& dLB, const FastDiv& dNs,
                             int stride_tw, const C2<T>* tw, T sign) {
  const int nbf = L / R;           // butterflies per line
  const int nb = LB * nbf;         // butterflies in the block
  constexpr int MAXB = (MAXV + R - 1) / R;   // butterflies per thread at most
  C2<T> v[MAXB][R];
  int dst[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    int b = threadIdx.x + i * blockDim.x;
    if (b < nb) {
      const int j = (int)dLB.div(b);
      const int l = b - j * LB;
      const int jq = (int)dNs.div(j);
      const int k = j - jq * Ns;
      C2<T>* row = lds + l * ldl;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = row[j + r * nbf];
      if (Ns > 1) {
        // r k stride_tw < R Ns L / (Ns R) = L: no reduction needed
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C2<T> w = tw[r * k * stride_tw];
          w.y *= -sign;  // table holds exp(-2 pi i t/L); sign +1 needs the conjugate
          v[i][r] = cmul(v[i][r], w);
        }
      }
      dft<T, R>(v[i], sign);
      dst[i] = l * ldl + jq * Ns * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    int b = threadIdx.x + i * blockDim.x;
    if (b < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) lds[dst[i] + r * Ns] = v[i][r];
    }
  }
  __syncthreads();
}

// One block transforms LB lines.  Global traffic is issued in bulk: every
// thread computes clamped (always valid) addresses for all of its up to MAXV
// elements and issues the loads back to back, and only then writes LDS, so
// that the loads are in flight together; the store phase reads LDS into
// registers first and then stores.  The pass kind fixes the access order:
// the complex passes run along a strided axis with consecutive threads on
// consecutive lines, the Z passes along the contiguous axis.
template <typename T, int KIND, int MAXV, int NT>
__device__ __forceinline__ void fft_pass_body(const PassArgs<T>& a, const int blk) {
  constexpr bool LINES_FASTEST = (KIND == PASS_COMPLEX || KIND == PASS_KINETIC || KIND == PASS_HSYM);
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int L = a.L;
  const int ldl = L + 1;
  const int LB = a.LB;
  const int line0 = blk * LB;
  // Z passes: deconvolution factors of the block's lines and of the elements,
  // staged after the lines
  double* fline = reinterpret_cast<double*>(smem_raw + (size_t)LB * ldl * sizeof(C2<T>));
  double* felem = fline + LB;
  // the strided passes stage the line's twiddles after the lines (16-byte
  // aligned) and their radix stages read them from LDS; the Z passes, whose
  // blocks are smaller and more numerous per CU, read them from global memory
  constexpr bool TW_LDS = LINES_FASTEST;
  C2<T>* const twl = reinterpret_cast<C2<T>*>(smem_raw + pass_twiddle_offset<T>(LB, L, has_factors<KIND>()));
  const C2<T>* const ltw = TW_LDS ? twl : a.tw;

  // staged while the element loads are in flight (below)
  auto stage_factors = [&]() {
    const int ne = (KIND == PASS_FWD_Z) ? a.nin : a.nout;
    for (int t = threadIdx.x; t < LB + ne; t += NT) {
      if (t < LB) {
        int line = line0 + t;
        if (line >= a.nlines) line = 0;
        const int i0 = (int)a.dn1.div(line), i1 = line - i0 * a.n1;
        fline[t] = (KIND == PASS_FWD_Z ? a.scale : 1.0) * a.dec0[i0] * a.dec1[i1];
      } else {
        felem[t - LB] = a.dec2[t - LB];
      }
    }
  };

  // the output reach of the thread's line (its elements all lie on one line
  // here), read now and used by the stores
  int2 ox{0, L - 1};
  if constexpr (KIND == PASS_COMPLEX) {
    if (a.oext) {
      const int line = line0 + (int)(threadIdx.x - a.dLB.div(threadIdx.x) * LB);
      ox = a.oext[line < a.nlines ? line : 0];
    }
  }

  // zero the padding region of every line when the input is padded
  if (a.nin < L && !a.half_in) {
    const int N = a.nin;
    const int nz = L - N;  // fine positions [N - N/2, L - N/2) stay zero
    for (int idx = threadIdx.x; idx < LB * nz; idx += NT) {
      const int e = (int)a.dLB.div(idx), l = idx - e * LB;
      lds[l * ldl + (N - N / 2) + e] = C2<T>{T(0), T(0)};
    }
  }

  double macc = 0.0;  // forward Z: the block's sum of rho
  // load: every load is issued before any loaded value is used, so that they
  // are in flight together; masked elements load from a valid index instead
  // of branching around the load, and their values are dropped afterwards
  {
    const int total_in = LB * a.nin;
    constexpr bool HSYM = KIND == PASS_HSYM;
    C2<T> buf[MAXV];
    T rbuf[KIND == PASS_FWD_Z ? MAXV : 1];
    C2<T> mir[HSYM ? MAXV : 1];
    int dst[MAXV];
    int le[MAXV];  // Z pass: line (high bits) and element (low 16 bits)
    unsigned keep = 0, keepm = 0;  // bit i: element i's value (its mirror's) is used
    // HSYM: LB divides NT, so all of a thread's elements lie on one line, whose
    // mirror line and reaches are read once, before the element loads
    int hl = 0, hlo = 0, hli = 0, hmo = 0, hmi = 0;
    bool hlok = false;
    int2 xp{0, -1}, xm{0, -1};
    if constexpr (HSYM) {
      hl = threadIdx.x - (int)a.dLB.div(threadIdx.x) * LB;
      const int line = line0 + hl;
      hlok = line < a.nlines;
      const int ln = hlok ? line : 0;
      hlo = (int)a.dic.div(ln);
      hli = ln - hlo * (int)a.ic;
      hmo = hlo ? a.sym_no - hlo : 0;
      hmi = hli ? a.sym_ni - hli : 0;
      xp = a.lext[(int64_t)hlo * a.sym_ni + hli];
      xm = a.lext[(int64_t)hmo * a.sym_ni + hmi];
    }
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      // slots past the block's inputs (padded passes load N of L) issue nothing;
      // the test is uniform across the block.  HSYM takes no such branch:
      // past one, the compiler no longer knows that the line's reaches have
      // arrived and waits for every load in flight before using them; its
      // empty slots are masked lanes instead
      if (!HSYM && i * NT >= total_in) {
        dst[i] = -1;
        le[i] = 0;
        continue;
      }
      const int idx0 = threadIdx.x + i * NT;
      const bool ok = idx0 < total_in;
      const int idx = ok ? idx0 : 0;
      int l, e;
      if constexpr (LINES_FASTEST) {
        e = (int)a.dLB.div(idx);
        l = idx - e * LB;
      } else {
        l = (int)a.dnin.div(idx);
        e = idx - l * a.nin;
      }
      if constexpr (HSYM) {
        // elements beyond their line's reach are zero: not fetched
        const bool lok = ok && hlok;
        const int me = e ? L - e : 0;
        int dp = e - xp.x, dm = me - xm.x;
        dp += dp < 0 ? L : 0;
        dm += dm < 0 ? L : 0;
        const bool in_p = lok && dp <= xp.y, in_m = lok && dm <= xm.y;
        const int64_t base = (int64_t)hlo * a.in_os + (int64_t)hli * a.in_is + (int64_t)e * a.in_es;
        const int64_t mbase = (int64_t)hmo * a.in_os + (int64_t)hmi * a.in_is + (int64_t)me * a.in_es;
        buf[i] = ((const C2<T>*)a.in)[in_p ? base : 0];
        mir[i] = ((const C2<T>*)a.in)[in_m ? mbase : 0];
        keep |= (unsigned)in_p << i;
        keepm |= (unsigned)in_m << i;
        dst[i] = ok ? hl * ldl + e : -1;
        le[i] = 0;
        continue;
      }
      const int line = line0 + l;
      const bool lok = ok && line < a.nlines;
      const int ln = lok ? line : 0;
      const int lo = (int)a.dic.div(ln);
      const int li = ln - lo * (int)a.ic;
      const int64_t base = (int64_t)lo * a.in_os + (int64_t)li * a.in_is + (int64_t)e * a.in_es;
      if constexpr (KIND == PASS_FWD_Z) {
        rbuf[i] = ((const T*)a.in)[base];
        keep |= (unsigned)lok << i;
      } else {
        buf[i] = ((const C2<T>*)a.in)[base];
        keep |= (unsigned)lok << i;
      }
      const int pos = (a.nin < L && !a.half_in) ? fine_pos(e, a.nin, L) : e;
      dst[i] = ok ? l * ldl + pos : -1;
      le[i] = (l << 16) | e;
    }
    // the twiddles or the deconvolution factors, copied while the element
    // loads are in flight
    if constexpr (TW_LDS)
      for (int t = threadIdx.x; t < L; t += NT) twl[t] = a.tw[t];
    if constexpr (has_factors<KIND>()) stage_factors();
    if constexpr (KIND == PASS_FWD_Z) __syncthreads();  // factors staged: the LDS writes below apply them
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      if (dst[i] >= 0) {
        const bool use = (keep >> i) & 1u;
        C2<T> v;
        if constexpr (KIND == PASS_FWD_Z) {
          // deconvolution and cell volume, applied in float64
          const T r = use ? rbuf[i] : T(0);
          const double d = fline[le[i] >> 16] * felem[le[i] & 0xffff];
          macc += (double)r;
          v.y = a.split ? (T)((double)r * a.scale) : T(0);
          v.x = (T)((double)r * d);
        } else if constexpr (HSYM) {
          const bool usem = (keepm >> i) & 1u;
          const T px = use ? buf[i].x : T(0), py = use ? buf[i].y : T(0);
          const T mx = usem ? mir[i].x : T(0), my = usem ? mir[i].y : T(0);
          v = C2<T>{T(0.5) * (px + mx), T(0.5) * (py - my)};
        } else {
          v = use ? buf[i] : C2<T>{T(0), T(0)};
        }
        lds[dst[i]] = v;
      }
    }
  }
  __syncthreads();
  if (a.half_in) {
    // the rest of each line from the Hermitian symmetry of its spectrum
    const int nfill = L - a.nin;
    for (int idx = threadIdx.x; idx < LB * nfill; idx += NT) {
      const int e = (int)a.dLB.div(idx), l = idx - e * LB;
      const int p = a.nin + e;
      const C2<T> v = lds[l * ldl + (L - p)];
      lds[l * ldl + p] = C2<T>{v.x, -v.y};
    }
    __syncthreads();
  }

  // FFT stages
  auto transform = [&](T sign) {
    int Ns = 1;
    for (int st = 0; st < a.nrad; ++st) {
      const int R = a.rad[st];
      const FastDiv& dNs = a.dNs[st];
      const int tws = a.tws[st];
      switch (R) {
        case 8: stage<T, 8, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, ltw, sign); break;
        case 5: stage<T, 5, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, ltw, sign); break;
        case 4: stage<T, 4, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, ltw, sign); break;
        case 3: stage<T, 3, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, ltw, sign); break;
        default: stage<T, 2, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, ltw, sign); break;
      }
      Ns *= R;
    }
  };
  if constexpr (KIND == PASS_KINETIC) {
    transform(T(-1));
    // the multiplier at every element, |k|^2 summed in axis order
    for (int idx = threadIdx.x; idx < LB * L; idx += NT) {
      const int e = (int)a.dLB.div(idx), l = idx - e * LB;
      const int line = line0 + l;
      if (line >= a.nlines) continue;
      const int ia = (int)a.dkb.div(line), ib = line - ia * (int)a.dkb.d;
      const double ke = a.kt[a.koff[a.kax] + e];
      const double kb = a.kt[a.koff[2] + ib];
      const double kx = a.kax == 0 ? ke : a.kt[a.koff[0] + ia];
      const double ky = a.kax == 0 ? a.kt[a.koff[1] + ia] : ke;
      const double ex = 0.5 * a.kin_h * (kx * kx + ky * ky + kb * kb);
      double fr, fi;
      if (a.kin_imag) {
        fr = exp(-ex) * a.inv_n;
        fi = 0.0;
      } else {
        sincos(-ex, &fi, &fr);
        fr *= a.inv_n;
        fi *= a.inv_n;
      }
      C2<T>* pv = lds + l * ldl + e;
      const C2<T> p = *pv;
      const double re = fr * p.x - fi * p.y, im = fr * p.y + fi * p.x;
      *pv = C2<T>{(T)re, (T)im};
    }
    __syncthreads();
    transform(T(1));
  } else {
    transform(a.sign);
  }

  // store: LDS reads first, then the global stores
  double eacc = 0.0;
  double ushift = 0.0;
  if constexpr (KIND == PASS_INV_Z) {
    if (a.shift) ushift = *a.shift;
  }
  {
    const int total_out = LB * a.nout;
    C2<T> buf[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      if (i * NT >= total_out) {  // cropped passes store N of L (uniform test)
        buf[i] = C2<T>{T(0), T(0)};
        continue;
      }
      const int idx0 = threadIdx.x + i * NT;
      const int idx = idx0 < total_out ? idx0 : 0;
      int l, e;
      if constexpr (LINES_FASTEST) {
        e = (int)a.dLB.div(idx);
        l = idx - e * LB;
      } else {
        l = (int)a.dnout.div(idx);
        e = idx - l * a.nout;
      }
      const int pos = (a.nout < L && !a.half_out) ? fine_pos(e, a.nout, L) : e;
      buf[i] = lds[l * ldl + pos];
    }
    T rho_v[KIND == PASS_INV_Z ? MAXV : 1];
    if constexpr (KIND == PASS_INV_Z) {
      // density values for the energy partials, loaded together
#pragma unroll
      for (int i = 0; i < MAXV; ++i) {
        if (i * NT >= total_out) {
          rho_v[i] = T(0);
          continue;
        }
        const int idx0 = threadIdx.x + i * NT;
        const int idx = idx0 < total_out ? idx0 : 0;
        const int l = (int)a.dnout.div(idx), e = idx - l * a.nout;
        int line = line0 + l;
        if (line >= a.nlines) line = 0;
        rho_v[i] = a.rho ? a.rho[(int64_t)line * a.out_os + e] : T(0);
      }
    }
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = threadIdx.x + i * NT;
      if (idx >= total_out) continue;
      int l, e;
      if constexpr (LINES_FASTEST) {
        e = (int)a.dLB.div(idx);
        l = idx - e * LB;
      } else {
        l = (int)a.dnout.div(idx);
        e = idx - l * a.nout;
      }
      const int line = line0 + l;
      if (line >= a.nlines) continue;
      const int lo = (int)a.dic.div(line);
      const int64_t base = (int64_t)lo * a.out_os + (int64_t)(line - lo * (int)a.ic) * a.out_is + (int64_t)e * a.out_es;
      if constexpr (KIND == PASS_COMPLEX) {
        int dp = e - ox.x;
        dp += dp < 0 ? L : 0;
        if (dp > ox.y) continue;  // never read: not stored
      }
      if constexpr (KIND == PASS_INV_Z) {
        double u = (double)buf[i].x * (fline[l] * felem[e]) + ushift;
        if (a.split) u += (double)buf[i].y;
        ((T*)a.out)[base] = (T)u;
        eacc += (double)rho_v[i] * u;
      } else {
        ((C2<T>*)a.out)[base] = buf[i];
      }
    }
  }

  if constexpr (KIND == PASS_FWD_Z) {
    if (a.mparts) {
      // deterministic block sum of rho: wave shuffle, then waves in order
      for (int off = 32; off > 0; off >>= 1) macc += __shfl_xor(macc, off, 64);
      __shared__ double msum[NT / 64];
      __syncthreads();
      if ((threadIdx.x & 63) == 0) msum[threadIdx.x >> 6] = macc;
      __syncthreads();
      if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += msum[i];
        a.mparts[blk] = s;
      }
    }
  }
  if constexpr (KIND == PASS_INV_Z) {
    if (a.eparts) {
      // deterministic block sum: wave shuffle, then waves in order
      for (int off = 32; off > 0; off >>= 1) eacc += __shfl_xor(eacc, off, 64);
      __shared__ double wsum[NT / 64];
      __syncthreads();
      if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = eacc;
      __syncthreads();
      if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += wsum[i];
        a.eparts[blk] = s;
      }
    }
  }
}

template <typename T, int KIND, int MAXV, int NT>
__global__ void __launch_bounds__(NT) k_fft_pass(PassArgs<T> a) {
  fft_pass_body<T, KIND, MAXV, NT>(a, blockIdx.x);
}
template <typename T, int KIND, int MAXV, int NT>
__global__ void __launch_bounds__(NT) k_fft_pass_b(const PassArgs<T>* __restrict__ tab, const int* __restrict__ bstart, int nm) {
  int m;
  const int blk = batch_block(bstart, nm, blockIdx.x, m);
  if (blk < 0) return;
  fft_pass_body<T, KIND, MAXV, NT>(tab[m], blk);
}

// Algorithm 2's paired passes along the last forward / first inverse axis.  A
// block takes P lines (a, b) of one row a and their mirrors
// ((A - a) mod A, (B - b) mod B), loads the lines' N inputs from the output of
// the forward pass before (the other axes already transformed), zero-pads them
// to L in LDS and runs the forward transform there, so that Z(q) and Z(-q)
// (element (L - e) mod L of the mirror line) sit in the block's LDS together.
//   PAIR_UNMIX: writes A = (Z(q) + conj Z(-q)) / 2 into the gather tiles of G
//     that the interpolation reads (only blocks with such a tile run);
//   PAIR_FUSED: forms the inverse transform's spectrum
//       Y(q) = (G(q) + conj G(-q)) / 2 + M'(q) (Z(q) - conj Z(-q)) / 2  (splitsym.h),
//     each thread writing Y at q and at -q, transforms both lines back and
//     stores the cropped outputs.
// Z is never stored: the unmix pass touches a few lines, and the fused pass
// reads the N-point inputs instead of the L-point spectrum.  Every line is
// owned by one block; a line that is its own mirror sits in two rows of its
// block, which end up equal.  Registers are capped at 128 (four waves per SIMD).
enum PairMode { PAIR_UNMIX = 0, PAIR_FUSED = 1 };

template <typename T, int MODE, int MAXV, int NT>
__global__ void __launch_bounds__(NT, 4) k_fft_pair_pass(PassArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);
  const int L = a.L;
  const int ldl = L + 1;
  const int P = a.P;
  const int LB = 2 * P;
  // The logical block.  Unmix: from the plan's list.  Fused: workgroups are
  // dealt round robin to the eight XCDs, so workgroup w runs on XCD w mod 8;
  // the logical ids are dealt out in runs, one run per XCD, so that
  // neighbouring chunks share an L2 (a chunk's mirror run is misaligned by one
  // element and shares its edge segments with the next chunk's).
  int bid;
  if constexpr (MODE == PAIR_UNMIX) {
    bid = a.blist[blockIdx.x];
  } else {
    const int nb = (int)gridDim.x, w = (int)blockIdx.x;
    const int x = w & 7, q = nb >> 3, r = nb & 7;
    bid = x * q + (x < r ? x : r) + (w >> 3);
  }
  // the block's row and chunk
  int ar, c;
  bool self;
  if (bid < a.nb1) {
    ar = 1 + bid / a.cb;
    c = bid % a.cb;
    self = false;
  } else {
    const int sb = bid - a.nb1;
    ar = (sb / a.cs == 0) ? 0 : a.A / 2;
    c = sb % a.cs;
    self = true;
  }
  // line slot l < P: own line (ar, c P + l); l >= P: the mirror of slot l - P
  // (ar <= A/2 and bq < B, so the mirror indices need no division)
  auto line_of = [&](int l, int& la, int& lb) {
    const int j = (l < P) ? l : l - P;
    int bq = c * P + j;
    const bool valid = self ? (bq <= a.B / 2) : (bq < a.B);
    if (!valid) bq = 0;
    if (l < P) {
      la = ar;
      lb = bq;
    } else {
      la = ar ? a.A - ar : 0;
      lb = bq ? a.B - bq : 0;
    }
    return valid;
  };
  const C2<T>* X = (const C2<T>*)a.in;
  const SplitSym& sy = a.sym;
  // tables after the lines: the element axis's frequencies and window values,
  // per line slot the constant parts of |k|^2, p, n.k and m.k, and the line's
  // row of gather-tile flags along the element axis
  const int ea = a.dim3 ? 0 : 1;                              // the element axis
  const int gse = a.dim3 ? sy.gs0 : sy.gs1;                    // its tile shift
  const int ngte = (L + (1 << gse) - 1) >> gse;                // its tiles
  double* sk = reinterpret_cast<double*>(smem_raw + (size_t)LB * ldl * sizeof(C2<T>));
  double* se = sk + L;
  double* lkk = se + L;
  double* lw = lkk + LB;
  double* lnk = lw + LB;
  double* lmk = lnk + LB;
  unsigned char* ltf = reinterpret_cast<unsigned char*>(lmk + LB);  // LB x ngte
  const int N = a.nin;
  // zero the padding of every line: fine positions [N - N/2, L - N/2)
  for (int idx = threadIdx.x; idx < LB * (L - N); idx += NT) {
    const int e = (int)a.dLB.div(idx), l = idx - e * LB;
    lds[l * ldl + (N - N / 2) + e] = C2<T>{T(0), T(0)};
  }
  // load the N inputs of both line sets, all loads issued before the LDS writes
  {
    const int total_in = LB * N;
    C2<T> buf[MAXV];
    int dst[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      if (i * NT >= total_in) {  // uniform: the inputs are N of L per line
        buf[i] = C2<T>{T(0), T(0)};
        dst[i] = -1;
        continue;
      }
      const int idx0 = threadIdx.x + i * NT;
      const bool ok = idx0 < total_in;
      const int idx = ok ? idx0 : 0;
      const int e = (int)a.dLB.div(idx);
      const int l = idx - e * LB;
      int la, lb;
      const bool valid = line_of(l, la, lb) && ok;
      const C2<T> v = X[(int64_t)e * a.es_in + (int64_t)la * a.B + lb];
      buf[i] = valid ? v : C2<T>{T(0), T(0)};
      dst[i] = ok ? l * ldl + fine_pos(e, N, L) : -1;
    }
    for (int t = threadIdx.x; t < L + LB + LB * ngte; t += NT) {
      if (t < L) {
        sk[t] = sy.kt[sy.koff[ea] + t];
        se[t] = sy.kt[sy.eoff[ea] + t];
      } else if (t < L + LB) {
        const int l = t - L;
        int la, lb;
        line_of(l, la, lb);
        const double k2 = sy.kt[sy.koff[2] + lb];
        double k1 = 0.0, w = 1.0;
        if (a.dim3) {
          k1 = sy.kt[sy.koff[1] + la];
          w = sy.kt[sy.eoff[1] + la] * sy.kt[sy.eoff[2] + lb];
        }
        lkk[l] = k1 * k1 + k2 * k2;
        lw[l] = w;
        // n.k over the physical axes: 3D (x1, x2, x3) = (a0, a1, a2), the
        // element carrying n_1; 2D (x1, x2) = (a1, a2), the element again n_1
        lnk[l] = a.dim3 ? sy.axis[1] * k1 + sy.axis[2] * k2 : sy.axis[1] * k2;
        lmk[l] = a.dim3 ? sy.axis2[1] * k1 + sy.axis2[2] * k2 : sy.axis2[1] * k2;
      } else {
        const int r = t - L - LB;
        const int l = r / ngte, te = r - l * ngte;
        int la, lb;
        line_of(l, la, lb);
        const int tile = a.dim3 ? ((te * sy.gnt1 + (la >> sy.gs1)) * sy.gnt2 + (lb >> sy.gs2))
                                : (te * sy.gnt2 + (lb >> sy.gs2));
        ltf[l * ngte + te] = sy.tflag[tile];
      }
    }
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
      if (dst[i] >= 0) lds[dst[i]] = buf[i];
  }
  __syncthreads();
  // forward transform of the 2P lines (sign -1): Z
  {
    int Ns = 1;
    for (int st = 0; st < a.nrad; ++st) {
      const int R = a.rad[st];
      const FastDiv& dNs = a.dNs[st];
      const int tws = a.tws[st];
      switch (R) {
        case 16:
          // float32 only: the radix-16 stage's registers would cost the float64
          // kernels occupancy (the plan never gives them radix 16)
          if constexpr (sizeof(T) == 4) stage<T, 16, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, a.tw, T(-1));
          break;
        case 8: stage<T, 8, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, a.tw, T(-1)); break;
        case 5: stage<T, 5, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, a.tw, T(-1)); break;
        case 4: stage<T, 4, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, a.tw, T(-1)); break;
        case 3: stage<T, 3, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, a.tw, T(-1)); break;
        default: stage<T, 2, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, a.tw, T(-1)); break;
      }
      Ns *= R;
    }
  }
  C2<T>* G = (C2<T>*)a.G;
  if constexpr (MODE == PAIR_UNMIX) {
    // A at every element pair (own line l, element e) <-> (mirror slot l + P,
    // (L - e) mod L) whose gather tile the interpolation reads; A(-q) = conj A(q)
    for (int idx = threadIdx.x; idx < P * L; idx += NT) {
      const int e = (int)a.dP.div(idx);
      const int l = idx - e * P;
      int la, lb;
      if (!line_of(l, la, lb)) continue;
      const int em = e ? L - e : 0;
      const int lm = l + P;
      const C2<T> zq = lds[l * ldl + e], zm = lds[lm * ldl + em];
      const C2<T> aq{T(0.5) * (zq.x + zm.x), T(0.5) * (zq.y - zm.y)};
      if (ltf[l * ngte + (e >> gse)]) {
        const int q0 = a.dim3 ? e : 0, q1 = a.dim3 ? la : e;
        G[((int64_t)q0 * sy.nf1 + q1) * sy.nf2 + lb] = aq;
      }
      if (ltf[lm * ngte + (em >> gse)]) {
        int ma, mb;
        line_of(lm, ma, mb);
        const int m0 = a.dim3 ? em : 0, m1 = a.dim3 ? ma : em;
        G[((int64_t)m0 * sy.nf1 + m1) * sy.nf2 + mb] = C2<T>{aq.x, -aq.y};
      }
    }
    return;
  }
  // form Y at every element pair (own line l, element e) <-> (mirror slot l + P, (L - e) mod L)
  {
    const bool dip = sy.kernel == JGB_DIPOLE_3D || sy.kernel == JGB_DIPOLE_2D;
    for (int idx = threadIdx.x; idx < P * L; idx += NT) {
      const int e = (int)a.dP.div(idx);
      const int l = idx - e * P;
      int la, lb;
      if (!line_of(l, la, lb)) continue;
      const int em = e ? L - e : 0;
      const int lm = l + P;
      const double ke = sk[e];
      double M = split_symbol_core(sy, ke * ke + lkk[l], se[e] * lw[l], sy.axis[0] * ke + lnk[l],
                                   sy.axis2[0] * ke + lmk[l]);
      if (dip && (2 * e == L || 2 * lb == a.B || (a.dim3 && 2 * la == a.A))) {
        // on a Nyquist plane, the mean with the mirror's symbol; off them the
        // mirror's k is exactly -k (the frequencies are 2 pi q' / (2 R) with
        // q' a signed integer) and its symbol equals M bit for bit
        const double km = sk[em];
        M = 0.5 * (M + split_symbol_core(sy, km * km + lkk[lm], se[em] * lw[lm], sy.axis[0] * km + lnk[lm],
                                         sy.axis2[0] * km + lmk[lm]));
      }
      C2<T>* pq = lds + l * ldl + e;
      C2<T>* pm = lds + lm * ldl + em;
      const C2<T> zq = *pq, zm = *pm;
      const T hm = (T)(0.5 * M);
      // D(q) = Z(q) - conj Z(-q) = 2 i B(q); D(-q) = -conj D(q)
      const T dx = zq.x - zm.x, dy = zq.y + zm.y;
      C2<T> gq{T(0), T(0)}, gm{T(0), T(0)};
      if (ltf[l * ngte + (e >> gse)]) {
        const int q0 = a.dim3 ? e : 0, q1 = a.dim3 ? la : e;
        gq = G[((int64_t)q0 * sy.nf1 + q1) * sy.nf2 + lb];
      }
      if (ltf[lm * ngte + (em >> gse)]) {
        int ma, mb;
        line_of(lm, ma, mb);
        const int m0 = a.dim3 ? em : 0, m1 = a.dim3 ? ma : em;
        gm = G[((int64_t)m0 * sy.nf1 + m1) * sy.nf2 + mb];
      }
      *pq = C2<T>{T(0.5) * (gq.x + gm.x) + hm * dx, T(0.5) * (gq.y - gm.y) + hm * dy};
      *pm = C2<T>{T(0.5) * (gm.x + gq.x) - hm * dx, T(0.5) * (gm.y - gq.y) + hm * dy};
    }
  }
  __syncthreads();
  // inverse transform of the 2P lines (sign +1)
  {
    int Ns = 1;
    for (int st = 0; st < a.nrad; ++st) {
      const int R = a.rad[st];
      const FastDiv& dNs = a.dNs[st];
      const int tws = a.tws[st];
      switch (R) {
        case 16:
          // float32 only: the radix-16 stage's registers would cost the float64
          // kernels occupancy (the plan never gives them radix 16)
          if constexpr (sizeof(T) == 4) stage<T, 16, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, a.tw, T(1));
          break;
        case 8: stage<T, 8, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, a.tw, T(1)); break;
        case 5: stage<T, 5, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, a.tw, T(1)); break;
        case 4: stage<T, 4, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, a.tw, T(1)); break;
        case 3: stage<T, 3, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, a.tw, T(1)); break;
        default: stage<T, 2, MAXV>(lds, ldl, L, LB, Ns, a.dLB, dNs, tws, a.tw, T(1)); break;
      }
      Ns *= R;
    }
  }
  // store the cropped outputs of both line sets
  {
    const int total_out = LB * a.nout;
    C2<T> buf[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      if (i * NT >= total_out) {
        buf[i] = C2<T>{T(0), T(0)};
        continue;
      }
      const int idx0 = threadIdx.x + i * NT;
      const int idx = idx0 < total_out ? idx0 : 0;
      const int e = (int)a.dLB.div(idx);
      const int l = idx - e * LB;
      buf[i] = lds[l * ldl + fine_pos(e, a.nout, L)];
    }
    C2<T>* out = (C2<T>*)a.out;
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = threadIdx.x + i * NT;
      if (idx >= total_out) continue;
      const int e = (int)a.dLB.div(idx);
      const int l = idx - e * LB;
      int la, lb;
      if (!line_of(l, la, lb)) continue;
      out[(int64_t)e * a.es_out + (int64_t)la * a.B + lb] = buf[i];
    }
  }
}

void factor(int L, int* rad, int& nrad, bool radix16 = false) {
  nrad = 0;
  int m = L;
  while (radix16 && m % 16 == 0) {
    rad[nrad++] = 16;
    m /= 16;
  }
  while (m % 8 == 0) {
    rad[nrad++] = 8;
    m /= 8;
  }
  while (m % 4 == 0) {
    rad[nrad++] = 4;
    m /= 4;
  }
  while (m % 2 == 0) {
    rad[nrad++] = 2;
    m /= 2;
  }
  while (m % 3 == 0) {
    rad[nrad++] = 3;
    m /= 3;
  }
  while (m % 5 == 0) {
    rad[nrad++] = 5;
    m /= 5;
  }
}

// Block shapes (threads x complex elements per thread; the staged elements
// cap / L give the lines per block).  Measured on the 256-point lines of the
// 128^3 grids: the strided passes keep every row of a block at 128 contiguous
// bytes (8 fp64 or 16 fp32 lines) with four or more blocks per CU, the Z
// passes stage 2048 elements per block, and the paired pass of Algorithm 2
// runs 256 threads (4 fp64 or 8 fp32 line pairs).  Every cap holds a whole
// line of the largest grid (nf = 1024), the paired pass's a line and its
// mirror.
constexpr int PASS_PAIR = 9;
template <typename T, int KIND = PASS_PAIR>
constexpr int pass_threads() {
  if (KIND == PASS_COMPLEX || KIND == PASS_KINETIC || KIND == PASS_HSYM) return sizeof(T) == 8 ? 256 : 512;
  if (KIND == PASS_FWD_Z || KIND == PASS_INV_Z) return 256;
  if (KIND == PASS_PAIR) return 256;
  return 512;
}
template <typename T, int KIND = PASS_PAIR>
constexpr int pass_elems() {
  if (KIND == PASS_COMPLEX || KIND == PASS_KINETIC || KIND == PASS_HSYM || KIND == PASS_FWD_Z || KIND == PASS_INV_Z)
    return 8;
  return sizeof(T) == 8 ? 8 : 16;
}
template <typename T, int KIND>
constexpr int pass_cap() { return pass_threads<T, KIND>() * pass_elems<T, KIND>(); }
static_assert(pass_cap<double, PASS_COMPLEX>() >= 1024 && pass_cap<float, PASS_COMPLEX>() >= 1024 &&
                  pass_cap<double, PASS_FWD_Z>() >= 1024 && pass_cap<float, PASS_FWD_Z>() >= 1024 &&
                  pass_cap<double, PASS_COMPLEX_Z>() >= 1024 && pass_cap<double, PASS_PAIR>() >= 2048 &&
                  pass_cap<float, PASS_PAIR>() >= 2048,
              "a block must stage at least one line of nf = 1024 points");
// The first forward and last inverse passes run the same lines with the same
// shape: their per-block partial sums (d_mparts, d_eparts) are counted once,
// by fft_inverse_z_blocks.
static_assert(pass_cap<double, PASS_FWD_Z>() == pass_cap<double, PASS_INV_Z>() &&
                  pass_cap<float, PASS_FWD_Z>() == pass_cap<float, PASS_INV_Z>(),
              "the Z passes share their block shape");

template <typename T, int KIND = PASS_PAIR>
int lines_per_block(int L) {
  const int cap = pass_elems<T, KIND>() * pass_threads<T, KIND>();  // complex elements staged per block
  const int maxlb = sizeof(T) == 8 ? 16 : 32;
  int lb = cap / L;
  if (lb > maxlb) lb = maxlb;
  if (lb < 1) lb = 1;
  if (KIND == PASS_HSYM)  // a power of two, dividing the block's threads
    while (lb & (lb - 1)) lb &= lb - 1;
  return lb;
}

template <typename T, int KIND>
hipError_t run_pass(const Plan& pl, int stage, PassArgs<T> a, hipStream_t s) {
  factor(a.L, a.rad, a.nrad);
  a.LB = lines_per_block<T, KIND>(a.L);
  // with an output reach per line, a thread's elements must lie on one line:
  // the lines per block divide the thread count
  if (KIND == PASS_COMPLEX && a.oext)
    while (pass_threads<T, KIND>() % a.LB != 0) --a.LB;
  {
    int Ns = 1;
    for (int st = 0; st < a.nrad; ++st) {
      a.dNs[st] = FastDiv((uint32_t)Ns);
      a.tws[st] = a.L / (Ns * a.rad[st]);
      Ns *= a.rad[st];
    }
  }
  if (a.nlines >= (1 << 30) || (int64_t)a.LB * a.L >= (1 << 30)) return hipErrorInvalidValue;
  // whole lines, with reaches; a thread's elements on one line
  if (KIND == PASS_HSYM && (a.nin != a.L || !a.lext || pass_threads<T, KIND>() % a.LB != 0)) return hipErrorInvalidValue;
  // an output reach per line, the thread's elements on one whole line
  if (a.oext && (KIND != PASS_COMPLEX || a.nout != a.L || pass_threads<T, KIND>() % a.LB != 0))
    return hipErrorInvalidValue;
  a.dLB = FastDiv((uint32_t)a.LB);
  a.dnin = FastDiv((uint32_t)a.nin);
  a.dnout = FastDiv((uint32_t)a.nout);
  a.dic = FastDiv((uint32_t)a.ic);
  a.dn1 = FastDiv((uint32_t)(a.n1 > 0 ? a.n1 : 1));
  unsigned blocks = (unsigned)((a.nlines + a.LB - 1) / a.LB);
  // lines, deconvolution factors (Z passes), twiddles (strided passes)
  constexpr bool TW_LDS = KIND == PASS_COMPLEX || KIND == PASS_KINETIC || KIND == PASS_HSYM;
  const size_t smem = pass_twiddle_offset<T>(a.LB, a.L, has_factors<KIND>()) + (TW_LDS ? (size_t)a.L * sizeof(C2<T>) : 0);
  constexpr int NT = pass_threads<T, KIND>();
  constexpr int MAXV = pass_elems<T, KIND>();
  stage_mark(pl, stage, 0, s);
  const hipError_t e =
      launch<PassArgs<T>, k_fft_pass<T, KIND, MAXV, NT>, k_fft_pass_b<T, KIND, MAXV, NT>>(a, blocks, NT, smem, s);
  stage_mark(pl, stage, 1, s);
  return e;
}

// The paired passes of Algorithm 2 along the internal axis `axis` (0 in 3D:
// lines (q1, q2); 1 in 2D: lines q2): block geometry, shared with the plan's
// list of unmix blocks.
template <typename T>
unsigned pair_geometry(PassArgs<T>& a) {
  // float32: radix 16 (two stages for L = 256 instead of three; the pass runs
  // two transforms per line, and fewer LDS round trips pay there)
  factor(a.L, a.rad, a.nrad, sizeof(T) == 4);
  {
    int Ns = 1;
    for (int st = 0; st < a.nrad; ++st) {
      a.dNs[st] = FastDiv((uint32_t)Ns);
      a.tws[st] = a.L / (Ns * a.rad[st]);
      Ns *= a.rad[st];
    }
  }
  const int lb = lines_per_block<T>(a.L);
  a.P = lb / 2 > 0 ? lb / 2 : 1;
  a.LB = 2 * a.P;
  a.dLB = FastDiv((uint32_t)a.LB);
  a.dP = FastDiv((uint32_t)a.P);
  a.cb = (a.B + a.P - 1) / a.P;
  a.cs = (a.B / 2 + 1 + a.P - 1) / a.P;
  a.nb1 = (a.A > 1) ? (a.A / 2 - 1) * a.cb : 0;
  return (unsigned)(a.nb1 + (a.A > 1 ? 2 : 1) * a.cs);
}

template <typename T, int MODE>
hipError_t run_pair_pass(const Plan& pl, int stage, PassArgs<T> a, hipStream_t s) {
  unsigned blocks = pair_geometry<T>(a);
  if (MODE == PAIR_UNMIX) {
    blocks = (unsigned)pl.nublocks;
    a.blist = pl.d_ublocks;
    if (blocks == 0) return hipSuccess;
  }
  const int gse = a.dim3 ? a.sym.gs0 : a.sym.gs1;
  const int ngte = (a.L + (1 << gse) - 1) >> gse;
  const size_t smem = (size_t)a.LB * (a.L + 1) * sizeof(C2<T>) + sizeof(double) * (2 * a.L + 4 * a.LB) +
                      (size_t)a.LB * ngte;
  constexpr int NT = pass_threads<T>();
  constexpr int MAXV = pass_elems<T>();
  stage_mark(pl, stage, 0, s);
  hipLaunchKernelGGL((k_fft_pair_pass<T, MODE, MAXV, NT>), dim3(blocks), dim3(NT), smem, s, a);
  stage_mark(pl, stage, 1, s);
  return hipGetLastError();
}

template <typename T>
PassArgs<T> base_args(const Plan& pl, int axis, T sign) {
  PassArgs<T> a{};
  a.L = pl.nf[axis];
  a.sign = sign;
  a.tw = (const C2<T>*)pl.d_tw[axis];
  a.n1 = pl.n[1];
  a.n2 = pl.n[2];
  return a;
}

// Algorithm 2's paired passes run along the last forward axis (a0 in 3D, a1 in
// 2D) on the output of the forward pass before it, which sits in W: 3D
// [n0][f1][f2], 2D [1][n1][f2].
template <typename T>
PassArgs<T> split_pair_args(const Plan& pl, int axis) {
  const bool has_x = pl.nf[0] > 1;
  PassArgs<T> a = base_args<T>(pl, axis, T(1));
  a.nin = (int)pl.n[axis];
  a.nout = (int)pl.n[axis];
  a.A = has_x ? (int)pl.nf[1] : 1;
  a.B = (int)pl.nf[2];
  a.es_in = has_x ? (int64_t)pl.nf[1] * pl.nf[2] : pl.nf[2];
  a.es_out = a.es_in;
  a.dim3 = has_x ? 1 : 0;
  a.in = pl.d_W;
  a.G = pl.d_G;
  a.sym = make_split_sym(pl);
  return a;
}

// The forward passes; with last = false the pass along the last axis (a0 in
// 3D, a1 in 2D) is left to Algorithm 2's paired passes.
template <typename T>
hipError_t forward_passes(const Plan& pl, const T* rho, hipStream_t s, bool last) {
  const int64_t n0 = pl.n[0], n1 = pl.n[1], n2 = pl.n[2];
  const int64_t f0 = pl.nf[0], f1 = pl.nf[1], f2 = pl.nf[2];
  const bool has_x = f0 > 1;
  // lines along axis 2 that the later passes keep (the Hermitian half
  // 0 .. f2/2 for a real input; all f2 otherwise) and their row stride
  const int64_t c2 = pl.r2c ? pl.h2 : f2, r2 = pl.r2c ? pl.hs2 : f2;
  // G belongs to the spreading: the intermediates use F and W
  void* A1 = has_x ? pl.d_F : pl.d_W;
  void* A2 = has_x ? pl.d_W : pl.d_F;
  hipError_t e;
  {  // Z: rho -> A1 [n0][n1][r2]
    PassArgs<T> a = base_args<T>(pl, 2, T(-1));
    a.nlines = n0 * n1;
    a.nin = (int)n2;
    a.nout = (int)c2;
    a.half_out = pl.r2c ? 1 : 0;
    a.ic = 1;
    a.in_os = n2;
    a.in_is = 0;
    a.in_es = 1;
    a.out_os = r2;
    a.out_is = 0;
    a.out_es = 1;
    a.in = rho;
    a.out = A1;
    a.dec0 = pl.d_deconv[0];
    a.dec1 = pl.d_deconv[1];
    a.dec2 = pl.d_deconv[2];
    a.scale = pl.H;
    a.split = pl.split ? 1 : 0;
    a.mparts = (pl.c0 != 0.0) ? pl.d_mparts : nullptr;
    if ((e = run_pass<T, PASS_FWD_Z>(pl, ST_FWD_Z, a, s)) != hipSuccess) return e;
  }
  if (has_x || last) {  // Y: A1 -> A2 [n0][f1][r2]
    PassArgs<T> a = base_args<T>(pl, 1, T(-1));
    a.nlines = n0 * c2;
    a.nin = (int)n1;
    a.nout = (int)f1;
    a.ic = c2;
    a.in_os = n1 * r2;
    a.in_is = 1;
    a.in_es = r2;
    a.out_os = f1 * r2;
    a.out_is = 1;
    a.out_es = r2;
    a.in = A1;
    a.out = A2;
    if ((e = run_pass<T, PASS_COMPLEX>(pl, ST_FWD_Y, a, s)) != hipSuccess) return e;
  }
  if (has_x && last) {  // X: A2 -> F [f0][f1][r2]
    PassArgs<T> a = base_args<T>(pl, 0, T(-1));
    a.nlines = f1 * c2;
    a.nin = (int)n0;
    a.nout = (int)f0;
    a.ic = c2;
    a.in_os = r2;
    a.in_is = 1;
    a.in_es = f1 * r2;
    a.out_os = r2;
    a.out_is = 1;
    a.out_es = f1 * r2;
    a.in = A2;
    a.out = pl.d_F;
    // Algorithm 1: the interpolation by tiles reads F only within each
    // line's reach (Algorithm 2's unmixing and Fourier-side energy read all
    // of F)
    a.oext = pl.tile_interp && !pl.split ? pl.d_fext : nullptr;
    if ((e = run_pass<T, PASS_COMPLEX>(pl, ST_FWD_X, a, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

template <typename T>
hipError_t launch_fft_forward(const Plan& pl, const T* rho, hipStream_t s) {
  return forward_passes<T>(pl, rho, s, true);
}

template <typename T>
hipError_t launch_split_forward(const Plan& pl, const T* rho, hipStream_t s) {
  hipError_t e = forward_passes<T>(pl, rho, s, false);
  if (e != hipSuccess) return e;
  return run_pair_pass<T, PAIR_UNMIX>(pl, ST_SPLIT_UNMIX, split_pair_args<T>(pl, pl.nf[0] > 1 ? 0 : 1), s);
}

std::vector<int> split_unmix_blocks(const Plan& pl, const std::vector<unsigned char>& tf) {
  const int axis = pl.nf[0] > 1 ? 0 : 1;
  PassArgs<double> a = base_args<double>(pl, axis, 1.0);
  const SplitSym sy = make_split_sym(pl);
  a.A = pl.nf[0] > 1 ? (int)pl.nf[1] : 1;
  a.B = (int)pl.nf[2];
  a.dim3 = pl.nf[0] > 1 ? 1 : 0;
  unsigned nblocks;
  if (pl.fp64) {
    nblocks = pair_geometry<double>(a);
  } else {
    PassArgs<float> b{};
    b.L = a.L;
    b.A = a.A;
    b.B = a.B;
    nblocks = pair_geometry<float>(b);
    a.P = b.P;
    a.cb = b.cb;
    a.cs = b.cs;
    a.nb1 = b.nb1;
  }
  const int gse = a.dim3 ? sy.gs0 : sy.gs1;
  const int ngte = (a.L + (1 << gse) - 1) >> gse;
  std::vector<int> out;
  for (int bid = 0; bid < (int)nblocks; ++bid) {
    int ar, c;
    bool self;
    if (bid < a.nb1) {
      ar = 1 + bid / a.cb;
      c = bid % a.cb;
      self = false;
    } else {
      const int sb = bid - a.nb1;
      ar = (sb / a.cs == 0) ? 0 : a.A / 2;
      c = sb % a.cs;
      self = true;
    }
    bool any = false;
    for (int l = 0; l < 2 * a.P && !any; ++l) {
      const int j = l < a.P ? l : l - a.P;
      const int bq = c * a.P + j;
      if (!(self ? (bq <= a.B / 2) : (bq < a.B))) continue;
      const int la = l < a.P ? ar : (ar ? a.A - ar : 0);
      const int lb = l < a.P ? bq : (bq ? a.B - bq : 0);
      for (int te = 0; te < ngte && !any; ++te) {
        const int tile = a.dim3 ? ((te * sy.gnt1 + (la >> sy.gs1)) * sy.gnt2 + (lb >> sy.gs2))
                                : (te * sy.gnt2 + (lb >> sy.gs2));
        any = tf[tile] != 0;
      }
    }
    if (any) out.push_back(bid);
  }
  return out;
}

template <typename T>
hipError_t launch_fft_inverse(const Plan& pl, T* u, const T* rho_for_energy, hipStream_t s) {
  const int64_t n0 = pl.n[0], n1 = pl.n[1], n2 = pl.n[2];
  const int64_t f0 = pl.nf[0], f1 = pl.nf[1], f2 = pl.nf[2];
  const bool has_x = f0 > 1;
  // the input spectrum: the spreading grid; Algorithm 2's first pass instead
  // forms its spectrum from the forward passes' output in W and from G, line
  // pairs at a time (k_fft_pair_pass), and in 2D runs in place on W (each
  // block reads all of its lines before it writes them back, and no two blocks
  // share a line)
  void* src = pl.d_G;
  void* B2 = has_x ? pl.d_F : src;  // (2D: the input grid itself)
  void* B1 = pl.d_W;
  // a real output needs only the Hermitian part of the spectrum,
  // (G(q) + conj G(-q)) / 2, at the lines 0 .. f2/2 of axis 2: the first pass
  // forms it from G and G's mirror (rows of r2), the last completes each line
  const int64_t c2 = pl.r2c ? pl.h2 : f2, r2 = pl.r2c ? pl.hs2 : f2;
  hipError_t e;
  if (has_x) {  // X: src -> B2 [n0][f1][r2]
    PassArgs<T> a = base_args<T>(pl, 0, T(1));
    a.nlines = f1 * c2;
    a.nin = (int)f0;
    a.nout = (int)n0;
    a.ic = c2;
    a.in_os = f2;
    a.in_is = 1;
    a.in_es = f1 * f2;
    a.out_os = r2;
    a.out_is = 1;
    a.out_es = f1 * r2;
    a.sym_no = (int)f1;
    a.sym_ni = (int)f2;
    a.lext = pl.d_gext;
    a.in = src;
    a.out = B2;
    if (pl.split) {
      PassArgs<T> b = split_pair_args<T>(pl, 0);
      b.out = B2;
      e = run_pair_pass<T, PAIR_FUSED>(pl, ST_INV_X, b, s);
    } else {
      e = run_pass<T, PASS_HSYM>(pl, ST_INV_X, a, s);  // r2c: Algorithm 1
    }
    if (e != hipSuccess) return e;
  }
  if (pl.split && !has_x) {  // 2D Algorithm 2: Y: W -> B1 = W [1][n1][f2], paired
    PassArgs<T> b = split_pair_args<T>(pl, 1);
    b.out = B1;
    if ((e = run_pair_pass<T, PAIR_FUSED>(pl, ST_INV_Y, b, s)) != hipSuccess) return e;
  } else {  // Y: B2 -> B1 [n0][n1][r2]; in 2D the first pass, reading G [1][f1][f2]
    PassArgs<T> a = base_args<T>(pl, 1, T(1));
    const int64_t rin = has_x ? r2 : f2;
    a.nlines = n0 * c2;
    a.nin = (int)f1;
    a.nout = (int)n1;
    a.ic = c2;
    a.in_os = f1 * rin;
    a.in_is = 1;
    a.in_es = rin;
    a.out_os = n1 * r2;
    a.out_is = 1;
    a.out_es = r2;
    a.sym_no = 1;
    a.sym_ni = (int)f2;
    a.lext = pl.d_gext;
    a.in = B2;
    a.out = B1;
    // in 2D the first pass (Algorithm 1, real output), else a plain strided pass
    e = has_x ? run_pass<T, PASS_COMPLEX>(pl, ST_INV_Y, a, s) : run_pass<T, PASS_HSYM>(pl, ST_INV_Y, a, s);
    if (e != hipSuccess) return e;
  }
  {  // Z: B1 -> u [n0][n1][n2], real part, deconvolution, energy partials
    PassArgs<T> a = base_args<T>(pl, 2, T(1));
    a.nlines = n0 * n1;
    a.nin = (int)c2;
    a.half_in = pl.r2c ? 1 : 0;
    a.nout = (int)n2;
    a.ic = 1;
    a.in_os = r2;
    a.in_is = 0;
    a.in_es = 1;
    a.out_os = n2;
    a.out_is = 0;
    a.out_es = 1;
    a.in = B1;
    a.out = u;
    a.dec0 = pl.d_deconv[0];
    a.dec1 = pl.d_deconv[1];
    a.dec2 = pl.d_deconv[2];
    a.rho = rho_for_energy;
    a.eparts = rho_for_energy ? pl.d_eparts : nullptr;
    a.split = pl.split ? 1 : 0;
    a.shift = (pl.c0 != 0.0) ? pl.d_origin : nullptr;
    if ((e = run_pass<T, PASS_INV_Z>(pl, ST_INV_Z, a, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Periodic complex FFT of a grid of n0 x n1 x n2 points in place (no padding,
// no crop): the GPE driver's kinetic step.  tw[a]: exp(-2 pi i t / n_a), t < n_a.
template <typename T>
hipError_t launch_fft_periodic(const Plan& pl, void* const tw[3], void* data, int sign, hipStream_t s) {
  const int64_t n0 = pl.n[0], n1 = pl.n[1], n2 = pl.n[2];
  const T sg = (T)sign;
  hipError_t e;
  auto common = [&](int axis) {
    PassArgs<T> a{};
    a.L = pl.n[axis];
    a.nin = a.nout = a.L;
    a.sign = sg;
    a.tw = (const C2<T>*)tw[axis];
    a.n1 = (int)n1;
    a.n2 = (int)n2;
    a.in = data;
    a.out = data;
    return a;
  };
  {  // axis 2, contiguous: lines [n0][n1]
    PassArgs<T> a = common(2);
    a.nlines = n0 * n1;
    a.ic = 1;
    a.in_os = a.out_os = n2;
    a.in_is = a.out_is = 0;
    a.in_es = a.out_es = 1;
    if ((e = run_pass<T, PASS_COMPLEX_Z>(pl, -1, a, s)) != hipSuccess) return e;
  }
  {  // axis 1: lines [n0][n2]
    PassArgs<T> a = common(1);
    a.nlines = n0 * n2;
    a.ic = n2;
    a.in_os = a.out_os = n1 * n2;
    a.in_is = a.out_is = 1;
    a.in_es = a.out_es = n2;
    if ((e = run_pass<T, PASS_COMPLEX>(pl, -1, a, s)) != hipSuccess) return e;
  }
  if (n0 > 1) {  // axis 0: lines [n1 n2]
    PassArgs<T> a = common(0);
    a.nlines = n1 * n2;
    a.ic = n1 * n2;
    a.in_os = a.out_os = 0;
    a.in_is = a.out_is = 1;
    a.in_es = a.out_es = n1 * n2;
    if ((e = run_pass<T, PASS_COMPLEX>(pl, -1, a, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_fft_periodic<double>(const Plan&, void* const[3], void*, int, hipStream_t);
template hipError_t launch_fft_periodic<float>(const Plan&, void* const[3], void*, int, hipStream_t);

// The GPE kinetic step in place: forward passes along a2 (and a1 in 3D), one
// kinetic pass along the last axis (a0, or a1 when a0 is a unit axis) that
// transforms forward, multiplies and transforms back, then the inverse passes
// in reverse order.  kt: k per internal axis at offsets koff.
template <typename T>
hipError_t launch_fft_periodic_kinetic(const Plan& pl, void* const tw[3], void* data, const double* kt,
                                       const int koff[3], double h, int imaginary, double inv_n, hipStream_t s) {
  const int64_t n0 = pl.n[0], n1 = pl.n[1], n2 = pl.n[2];
  const bool has_x = n0 > 1;
  auto common = [&](int axis, T sg) {
    PassArgs<T> a{};
    a.L = pl.n[axis];
    a.nin = a.nout = a.L;
    a.sign = sg;
    a.tw = (const C2<T>*)tw[axis];
    a.n1 = (int)n1;
    a.n2 = (int)n2;
    a.in = data;
    a.out = data;
    a.kt = kt;
    for (int i = 0; i < 3; ++i) a.koff[i] = koff[i];
    a.kin_h = h;
    a.inv_n = inv_n;
    a.kin_imag = imaginary;
    a.dkb = FastDiv((uint32_t)n2);  // a line's other two axes: (line / n2, line mod n2)
    return a;
  };
  auto pass_z = [&](T sg) {  // axis 2, contiguous: lines [n0][n1]
    PassArgs<T> a = common(2, sg);
    a.nlines = n0 * n1;
    a.ic = 1;
    a.in_os = a.out_os = n2;
    a.in_is = a.out_is = 0;
    a.in_es = a.out_es = 1;
    return run_pass<T, PASS_COMPLEX_Z>(pl, -1, a, s);
  };
  auto pass_y = [&](T sg, bool kinetic) {  // axis 1: lines [n0][n2], line = i0 n2 + i2
    PassArgs<T> a = common(1, sg);
    a.nlines = n0 * n2;
    a.ic = n2;
    a.in_os = a.out_os = n1 * n2;
    a.in_is = a.out_is = 1;
    a.in_es = a.out_es = n2;
    a.kax = 1;
    return kinetic ? run_pass<T, PASS_KINETIC>(pl, -1, a, s) : run_pass<T, PASS_COMPLEX>(pl, -1, a, s);
  };
  auto pass_x_kinetic = [&]() {  // axis 0: lines [n1 n2], line = i1 n2 + i2
    PassArgs<T> a = common(0, T(-1));
    a.nlines = n1 * n2;
    a.ic = n1 * n2;
    a.in_os = a.out_os = 0;
    a.in_is = a.out_is = 1;
    a.in_es = a.out_es = n1 * n2;
    a.kax = 0;
    return run_pass<T, PASS_KINETIC>(pl, -1, a, s);
  };
  hipError_t e;
  if ((e = pass_z(T(-1))) != hipSuccess) return e;
  if (has_x) {
    if ((e = pass_y(T(-1), false)) != hipSuccess) return e;
    if ((e = pass_x_kinetic()) != hipSuccess) return e;
    if ((e = pass_y(T(1), false)) != hipSuccess) return e;
  } else {
    if ((e = pass_y(T(-1), true)) != hipSuccess) return e;
  }
  return pass_z(T(1));
}

template hipError_t launch_fft_periodic_kinetic<double>(const Plan&, void* const[3], void*, const double*,
                                                        const int[3], double, int, double, hipStream_t);
template hipError_t launch_fft_periodic_kinetic<float>(const Plan&, void* const[3], void*, const double*,
                                                       const int[3], double, int, double, hipStream_t);

// d_origin = {c0 H sum rho, c0 (H sum rho)^2} from the first forward pass's
// per-block sums (one block, fixed order).
struct OriginArgs {
  const double* parts;
  int n;
  double H, c0;
  double* out;
};

__device__ __forceinline__ void origin_body(const OriginArgs& a) {
  const double* parts = a.parts;
  const int n = a.n;
  const double H = a.H, c0 = a.c0;
  double* out = a.out;
  __shared__ double s[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += parts[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double r0 = H * s[0];
    out[0] = c0 * r0;
    out[1] = c0 * r0 * r0;
  }
}

__global__ void __launch_bounds__(256) k_origin(OriginArgs a) { origin_body(a); }
__global__ void __launch_bounds__(256) k_origin_b(const OriginArgs* __restrict__ tab, const int* __restrict__ bstart, int nm) {
  int m;
  if (batch_block(bstart, nm, blockIdx.x, m) < 0) return;
  origin_body(tab[m]);
}

hipError_t launch_origin(const Plan& pl, hipStream_t s) {
  const OriginArgs a{pl.d_mparts, fft_inverse_z_blocks(pl), pl.H, pl.c0, pl.d_origin};
  return launch<OriginArgs, k_origin, k_origin_b>(a, 1, 256, 0, s);
}

int fft_inverse_z_blocks(const Plan& pl) {
  int lb = pl.fp64 ? lines_per_block<double, PASS_INV_Z>(pl.nf[2]) : lines_per_block<float, PASS_INV_Z>(pl.nf[2]);
  int64_t nl = (int64_t)pl.n[0] * pl.n[1];
  return (int)((nl + lb - 1) / lb);
}

template hipError_t launch_fft_forward<double>(const Plan&, const double*, hipStream_t);
template hipError_t launch_split_forward<double>(const Plan&, const double*, hipStream_t);
template hipError_t launch_split_forward<float>(const Plan&, const float*, hipStream_t);
template hipError_t launch_fft_forward<float>(const Plan&, const float*, hipStream_t);
template hipError_t launch_fft_inverse<double>(const Plan&, double*, const double*, hipStream_t);
template hipError_t launch_fft_inverse<float>(const Plan&, float*, const float*, hipStream_t);

}  // namespace jgb
