/*
 * jgb.h -- C ABI of the MI355X library for free-space Coulomb and dipole-dipole
 * convolutions by the Fourier-quadrature + NUFFT method of Jiang, Greengard and
 * Bao (arXiv:1311.4120).
 *
 * What is computed (Section 3, Algorithm 1 and the energy remark after
 * Algorithm 2).  On the uniform grid x_n = -R_j/2 + n_j h_j, h_j = R_j/N_j,
 * n_j = 0..N_j-1 (eq. 3.2), with H = prod_j h_j:
 *
 *   rho^_j = H sum_n rho_n exp(-i k_j . x_n)                    (eq. 3.2)
 *   u_n    = Re sum_j c_j rho^_j exp(+i k_j . x_n)               (eq. 3.7)
 *   E      = (lambda/2) H sum_n rho_n u_n                        (eq. gpe2)
 *
 * where k_j and W_j are the Fourier quadrature nodes and weights of eq. 3.7
 * (Gauss-Legendre in r on [0,K], Gauss-Legendre in theta, trapezoidal in phi)
 * and c_j = (2 pi)^{-d} W_j |k_j|^{d-1} U^(k_j) with the kernel's transform
 * U^ from eq. int3dd.  The type-2 and type-1 sums are evaluated by NUFFTs on
 * the GPU to the requested tolerance; the result matches the direct sums to
 * eps in relative L2 norm.
 *
 * Conventions shared by every call.
 *   - Arrays are C-order (N_1, N_2[, N_3]): the last axis is contiguous; axis j
 *     of the array is coordinate x_j.  Element [i_1,i_2,i_3] sits at
 *     (-R_1/2 + i_1 h_1, ...).
 *   - rho, u and gradients are device pointers of float64 (JGB_FP64) or
 *     float32 (JGB_MIXED).  Energies are always one float64 in device memory.
 *   - The caller owns every array it passes.  A plan owns its node tables,
 *     bins and workspace: allocated in jgb_plan, freed in jgb_destroy.
 *   - Compute calls only enqueue work on the plan's stream and return; they
 *     never synchronise, so they may be captured in a HIP graph.  A launch
 *     failure returns JGB_ERR_DEVICE; an asynchronous fault surfaces at the
 *     caller's next synchronisation.
 *   - A plan is not thread-safe; distinct plans are independent.  Two calls
 *     on one plan that overlap in time (different streams) race on its
 *     workspace.
 *   - Every call returns a jgb_status and never throws.  jgb_last_error()
 *     gives a message for the last failure on the calling thread.
 */
#ifndef JGB_H
#define JGB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  JGB_OK = 0,
  JGB_ERR_INVALID_ARG = 1,   /* a parameter or pointer violates its contract */
  JGB_ERR_UNSUPPORTED = 2,   /* valid request this library does not implement */
  JGB_ERR_OUT_OF_MEMORY = 3, /* device or host allocation failed; nothing leaked */
  JGB_ERR_DEVICE = 4         /* a HIP runtime call or kernel launch failed     */
} jgb_status;

/* The interaction kernels of eq. int3dd handled by this library, with n the
 * dipole axis and m the second orientation (m = n unless dipole_axis2 is set):
 *   JGB_COULOMB_3D : U = 1/(4 pi |x|),  U^ = 1/|k|^2             (eq. Cou3D)
 *   JGB_COULOMB_2D : U = 1/(2 pi |x|) in the plane, U^ = 1/|k|    (eq. Cou2D)
 *   JGB_DIPOLE_3D  : U = (3/4pi)(m.n - 3 (x.n)(x.m)/|x|^2)/|x|^3,
 *                    U^ = -(m.n) + 3 (n.k)(m.k)/|k|^2
 *                    (eqs. dipkernel, dipkernelF; dipkerneld, dipkerneldF)
 *   JGB_DIPOLE_2D  : the 2.5D dipole in the plane, n and m unit 3-vectors with
 *                    in-plane parts n_p, m_p and normal parts n_3, m_3,
 *                    U^ = -alpha + 3 [(n_p.k)(m_p.k) - n_3 m_3 |k|^2] / (2|k|)
 *                    (eqs. dipkernel2d, dipkernelF2d; dipkernel2dd, dipkernelF2dd)
 *   JGB_POISSON_2D : U = -(1/2pi) log|x| in the plane, U^ = 1/|k|^2, the example
 *                    of a symbol the Jacobian does not cancel (end of Section 4).
 *                    The radial integrand g(r)/r is not integrable at 0; the log
 *                    kernel fixes its finite part, and the radial rule is the
 *                    Gauss-Legendre one with a node at k = 0 of coefficient
 *                    c_0 = (log K - sum_a w_a / r_a + gamma - log 2) / (2 pi)
 *                    (jgb_info.origin_coef): u gains c_0 rho^(0), rho^(0) = H sum rho,
 *                    exact for g polynomial of degree <= 2 n_r. */
typedef enum {
  JGB_COULOMB_3D = 0, JGB_COULOMB_2D = 1, JGB_DIPOLE_3D = 2, JGB_DIPOLE_2D = 3, JGB_POISSON_2D = 4
} jgb_kernel;

/* JGB_FP64: every step in float64.
 * JGB_MIXED: grids, FFTs and kernel taps in float32; nodes, weights, symbol,
 *            deconvolution factors and energies in float64; requires eps >= 1e-6. */
typedef enum { JGB_FP64 = 0, JGB_MIXED = 1 } jgb_precision;

/* Gauss-Legendre rule for the polar angle (3D only).
 *   JGB_THETA_GL   : GL nodes in theta on [0, pi], weight includes sin(theta)
 *                    (the literal reading of eq. 3.7).
 *   JGB_COSTHETA_GL: GL nodes in cos(theta) on [-1, 1] (the same integral). */
typedef enum { JGB_THETA_GL = 0, JGB_COSTHETA_GL = 1 } jgb_theta_rule;

/* flags */
#define JGB_FLAG_NONE 0u
/* Time the candidate work-item sizes of the interpolation and spreading
 * kernels on the device at plan time and keep the fastest.  When the
 * environment variable JGB_AUTOTUNE_CACHE names a file, results are read from
 * and written to it (a JSON object keyed by grid, node counts, cutoff, width
 * and precision), so later plans of the same shape skip the timing. */
#define JGB_FLAG_AUTOTUNE 1u
/* Evaluate u by the partition-of-unity split of Algorithm 2 (Section 3.3,
 * eq. 3.9) instead of Algorithm 1.  A smooth window p (eq. 3.10 in 3D,
 * eq. 3.12 in 2D) splits the Fourier integral into
 *   I1 = (2 pi)^{-d} int (1 - p) U^ rho^ e^{ik.x} dk,
 * whose integrand is smooth, taken by the trapezoid rule on the regular
 * frequency grid k_q = 2 pi q / (2 R_j) (the oversampled grid of step 3): a
 * periodic convolution of the zero-padded density, by FFT, exact up to
 * rounding; and
 *   I2 = (2 pi)^{-d} int p U^ rho^ e^{ik.x} dk,
 * Algorithm 1 on the plan's node set with c_j multiplied by p(k_j).  Because p
 * decays on the scale of the box's Fourier spacing dk = 2 pi / max_j R_j, I2
 * needs few nodes whatever N is.  The result matches the same discrete sums
 * evaluated directly to eps (relative L2 of u, relative E).  See
 * jgb_params.window and jgb_params.kmax for the scales. */
#define JGB_FLAG_SPLIT 2u
/* Interpolate by tiles on the matrix cores (3D only, else UNSUPPORTED): the
 * type-2 back end runs as the transpose of the spreading's tile products --
 * for each output tile of the spreading and 16 of its listed nodes at a time,
 * 16x16x4 products of the tile's grid values with the nodes' kernel values --
 * and each node's shares of its tiles are summed in a fixed order.  Without
 * this flag the interpolation stages each sub-bin's neighbourhood in LDS; with
 * JGB_FLAG_AUTOTUNE alone the plan times both and keeps the faster.  Results
 * agree to rounding.  Costs one complex value and one index per list entry of
 * device memory. */
#define JGB_FLAG_INTERP_TILES 4u
/* Spread by rings (3D only, else UNSUPPORTED; also UNSUPPORTED when an
 * oversampled side is shorter than its tile plus the width less one: 16 + w - 1
 * on a0 and a2, 8 + w - 1 on a1).  The node set is the product r_a x theta_b
 * x phi_l (Section 3.1), and the a2 coordinate r_a cos(theta_b) of a node does
 * not depend on its azimuth: the type-1 front end first sums each ring's
 * nodes over the two other axes on the matrix cores, then spreads each such
 * ring sum along a2 once.  Without this flag the spreading sums every node
 * over all three axes; with JGB_FLAG_AUTOTUNE alone the plan times both and
 * keeps the faster.  Results agree to rounding.  Costs two index tables of
 * about one entry per node and touched tile of device memory. */
#define JGB_FLAG_SPREAD_RINGS 8u
/* Radial nodes by a generalized Gaussian rule for band-limited integrands
 * (Section 3.3's last remark; Conclusions) instead of Gauss-Legendre: along a
 * ray the radial integrand rho^(r e) e^{i r e.x} is band-limited by the box's
 * diameter, and the rule of Xiao, Rokhlin and Yarvin (nodes at the roots of a
 * prolate spheroidal wave function psi_{n_r}^c, weights exact on psi_0 ..
 * psi_{n_r - 1}) integrates such functions with fewer nodes.  The bandwidth is
 * c = (pi/2)(n_r - 2 - 1.8 log10(10/eps) - 0.06 n_r) on [-1, 1] (jgb_info.
 * radial_c; Gauss-Legendre when c < 1).  Any kernel; for JGB_POISSON_2D the
 * node at k = 0 takes the rule's own weights.  UNSUPPORTED if the rule cannot
 * be built (n_r > 2048). */
#define JGB_FLAG_RADIAL_GGQ 16u
/* The paper's own spreading kernel (Section 2, the heat kernel g_tau and the
 * deconvolution sqrt(pi/tau) e^{k^2 tau}) instead of the exponential of a
 * semicircle: with the oversampled grid of 2N points per axis and
 * tau = 6/N^2, a Gaussian over the nearest 12 points, exp(-pi^2 d^2 / 24) at
 * a distance of d fine cells, for about six digits.  The paper's 24-point,
 * twelve-digit setting exceeds the 16-tap node records: with this flag eps
 * below 1e-6 is UNSUPPORTED.  Both algorithms; jgb_info.width reports 12 and
 * jgb_info.beta 0. */
#define JGB_FLAG_GAUSSIAN_KERNEL 32u

typedef struct jgb_plan_s* jgb_plan_t;

typedef struct {
  uint32_t struct_size;    /* = sizeof(jgb_params); guards against ABI drift */
  int32_t dim;             /* 2 or 3 */
  int64_t n[3];            /* N_j: even, 8 <= N_j <= 512, 2 N_j of the form 2^a 3^b 5^c;
                              n[2] ignored when dim == 2 */
  double box[3];           /* R_j > 0, full side lengths of B = prod [-R_j/2, R_j/2) */
  int32_t kernel;          /* jgb_kernel; JGB_COULOMB_2D, JGB_DIPOLE_2D and JGB_POISSON_2D need
                              dim == 2, the others dim == 3 */
  double dipole_axis[3];   /* unit vector n (| |n| - 1 | <= 1e-12); ignored for Coulomb */
  double lambda;           /* interaction constant of eq. gpe2, finite */
  double eps;              /* requested relative L2 accuracy of u (and relative accuracy of E)
                              against the direct sums: [1e-13, 1e-2]; JGB_MIXED needs >= 1e-6 */
  int32_t precision;       /* jgb_precision */
  int32_t n_r;             /* radial GL nodes, >= 1 */
  int32_t n_theta;         /* polar GL nodes (3D), >= 1; ignored when dim == 2 */
  int32_t n_phi;           /* azimuthal trapezoid nodes: even, >= 2 (k -> -k closure) */
  int32_t theta_rule;      /* jgb_theta_rule */
  double kmax;             /* radius K of the Fourier ball; 0 -> pi / max_j h_j; must be
                              in (0, pi / max_j h_j] otherwise.  With JGB_FLAG_SPLIT it is
                              the radius of I2's ball, and 0 means min(pi / max_j h_j,
                              sqrt(40 a)) in 3D (p < 5e-18 beyond) or min(pi / max_j h_j, R1)
                              in 2D (p < 1.1e-17 beyond) */
  int32_t device;          /* HIP device ordinal the plan lives on */
  void* stream;            /* hipStream_t for all work of this plan (NULL = default stream) */
  uint32_t flags;          /* JGB_FLAG_* (any other bit -> INVALID_ARG) */
  double window[2];        /* JGB_FLAG_SPLIT only (both 0 otherwise): the window of Algorithm 2,
                              with dk = 2 pi / max_j R_j.
                              3D: window[0] = a of p(k) = exp(-|k|^2 / a) (eq. 3.10),
                                  0 -> 2 dk^2; window[1] = 0.
                              2D: window = {R0, R1} of p(k) = erfc(12 (|k| - (R0 + R1)/2)
                                  / (R1 - R0)) / 2 (eq. 3.12), {0, 0} -> {0.8 dk, 10 dk};
                                  otherwise 0 < R0 < R1.
                              Values must be finite. */
  double dipole_axis2[3];  /* second dipole orientation m: all zero -> m = n; otherwise a unit
                              vector like dipole_axis.  Ignored for Coulomb. */
  double alpha;            /* JGB_DIPOLE_2D: the constant of the -alpha delta term; finite.
                              Ignored for the other kernels (must still be finite). */
} jgb_params;

/* Plan facts, for diagnostics and for sizing caller buffers. */
typedef struct {
  uint32_t struct_size;    /* = sizeof(jgb_info) */
  int32_t dim;
  int64_t n[3];            /* grid (dim == 2: n[2] = 1) */
  int64_t nf[3];           /* oversampled FFT grid (2 N_j) */
  int64_t n_nodes;         /* M = n_r n_theta n_phi (3D) or n_r n_phi (2D) */
  int64_t n_half;          /* nodes processed on the device: M / 2 (k and -k paired) */
  int32_t width;           /* spreading kernel width in fine-grid cells per axis */
  double beta;             /* exponential-of-semicircle kernel shape parameter (0: the Gaussian) */
  double kmax;             /* K actually used */
  int64_t workspace_bytes; /* device memory owned by the plan */
  int32_t interp_chunk;    /* nodes per interpolation block at most; 0: the autotuner chose the
                              interpolation by tiles on the matrix cores */
  int32_t spread_chunk;    /* list entries per spreading block at most; negative: the spreading
                              by rings (JGB_FLAG_SPREAD_RINGS, or the autotuner's choice) with
                              -spread_chunk node entries per block at most */
  uint32_t flags;          /* the plan's JGB_FLAG_* */
  double window[2];        /* JGB_FLAG_SPLIT: the window scales used (a, 0) or (R0, R1); else 0 */
  double origin_coef;      /* c_0 of the node at k = 0 (JGB_POISSON_2D; 0 for the others) */
  double radial_c;         /* JGB_FLAG_RADIAL_GGQ: the radial rule's bandwidth c (0: Gauss-Legendre) */
} jgb_info;

/* Build a plan: validates the parameters, generates the Fourier nodes and
 * weights on the device (Algorithm 1, step 3), bin-sorts them, tabulates the
 * deconvolution factors and allocates the workspace.  Synchronises the plan's
 * stream before returning.  On success *out owns all plan memory.
 * Errors: INVALID_ARG (NULL pointers, any rule in jgb_params broken),
 * UNSUPPORTED (valid but outside this library's limits), OUT_OF_MEMORY, DEVICE. */
jgb_status jgb_plan(const jgb_params* params, jgb_plan_t* out);

/* u = U*rho on the grid (Algorithm 1, steps 4-5; with JGB_FLAG_SPLIT,
 * Algorithm 2: u = I1 + I2) and, if energy != NULL,
 * E = (lambda/2) H sum rho u (physical-side trapezoid sum, energy remark).
 * rho, u: device arrays of prod N_j elements of the plan's dtype;
 * energy: device float64 or NULL.  rho and u must not overlap.
 * Enqueue only (asynchronous on the plan's stream). */
jgb_status jgb_potential(jgb_plan_t plan, const void* rho, void* u, double* energy);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as jgb_potential, bit for bit, with every per-call buffer (the
 * oversampled grids, the FFT pass intermediate, the gather's partial tiles,
 * the weighted node values and the partial sums) taken from one file-scope
 * device array of JGB_NOALLOC_SCRATCH_BYTES per GPU, held from library load
 * until the process ends, instead of the plan's workspace.  The call
 * allocates nothing; the plan (made beforehand by jgb_plan) supplies its node
 * tables and lists.  Arguments and layout as jgb_potential.
 * Errors: INVALID_ARG as jgb_potential; UNSUPPORTED when the plan's per-call
 * buffers exceed the array (for cubic grids about 64^3 in float64, 80^3 in
 * mixed precision; jgb_info.workspace_bytes is an upper bound); DEVICE.
 * Every call on one GPU shares that GPU's array and overwrites it: two calls
 * that overlap in time on one GPU (different streams, threads or plans) race
 * and give wrong results.  Enqueue only. */
#define JGB_NOALLOC_SCRATCH_BYTES (128u << 20)
jgb_status jgb_potential_noalloc(jgb_plan_t plan, const void* rho, void* u, double* energy);

/* E only, via the Fourier-side sum E = (lambda/2) sum_j c_j |rho^_j|^2, which
 * equals the physical-side sum exactly for real rho (substitute eq. 3.2 into
 * the energy).  Runs only the type-2 half of the pipeline.  With
 * JGB_FLAG_SPLIT the sum gains the regular-grid part of I1,
 * (lambda/2) (prod_j 2 R_j)^{-1} sum_q (1 - p(k_q)) U^(k_q) |rho^(k_q)|^2.
 * rho: device array; energy: device float64.  Enqueue only. */
jgb_status jgb_energy(jgb_plan_t plan, const void* rho, double* energy);

/* Vector-Jacobian product of jgb_potential with respect to rho:
 * grad_rho = A^T grad_u, where u = A rho and A_{nl} = H Re sum_j c_j
 * exp(i k_j.(x_n - x_l)) is symmetric, so this applies A to grad_u (the type-2
 * NUFFT is the adjoint of the type-1, end of Section 2).  Device arrays of the
 * plan's dtype; must not overlap.  Enqueue only. */
jgb_status jgb_potential_backward(jgb_plan_t plan, const void* grad_u, void* grad_rho);

/* Density of a wave function, rho = |psi|^2 (the introduction, after eq.
 * gpe2).  psi: device complex array (interleaved re, im) of prod N_j elements
 * of the plan's real dtype; rho: device real array.  Must not overlap.
 * Enqueue only. */
jgb_status jgb_density(jgb_plan_t plan, const void* psi, void* rho);

/* Gradient of the interaction energy E(|psi|^2) = (lambda/2) H sum |psi|^2 u
 * (eq. gpe2) with respect to conj(psi): since u = A rho with A symmetric,
 * dE/drho = lambda H u and dE/dpsi* = lambda H u psi.  Writes
 *   grad = factor * g * lambda * H * u * psi,
 * where g = *gscale (a device float64, e.g. the upstream gradient of a
 * scalar loss; NULL means 1) and factor is a host constant (2 gives PyTorch's
 * convention for complex inputs, grad = dL/dRe + i dL/dIm = 2 dL/dpsi*).
 * psi, grad: device complex arrays; u: device real array from jgb_potential
 * of rho = |psi|^2.  grad must not overlap u.  Enqueue only. */
jgb_status jgb_psi_gradient(jgb_plan_t plan, const void* psi, const void* u, const double* gscale, double factor,
                            void* grad);

/* Type-2 stage alone (Algorithm 1, step 4), for diagnostics: rho^_j at the
 * device's half node set (k_j with phi index l < n_phi/2; the other half is
 * conj(rho^) at -k_j), in natural node order (radial index slowest, then
 * theta, then phi).  rhohat: device complex array of n_half elements
 * (interleaved re, im) of the plan's dtype.  Enqueue only. */
jgb_status jgb_transform(jgb_plan_t plan, const void* rho, void* rhohat);

/* Fourier nodes of the plan for diagnostics (Algorithm 1, step 3): all M
 * nodes in natural order.  k: device float64 array (M, dim); w: device float64
 * array of the quadrature weights W_j (measure dr dtheta dphi with sin(theta),
 * or dr dphi); c: device float64 array of c_j = (2pi)^{-d} W_j |k_j|^{d-1} U^(k_j)
 * (times p(k_j) with JGB_FLAG_SPLIT).
 * Any of the three may be NULL.  Enqueue only. */
jgb_status jgb_nodes(jgb_plan_t plan, double* k, double* w, double* c);

/* Stage timing for measurement.  While enabled, every compute call records a
 * HIP event on the plan's stream before and after each kernel launch (the
 * first max_calls calls only); nothing synchronises until jgb_timing_end,
 * which waits for the stream and writes the average duration in milliseconds
 * of each stage over the recorded calls that ran it (0 for stages that never
 * ran) into stage_ms[JGB_NUM_STAGES], and the number of recorded calls into
 * *calls.  Stage order:
 *   0 forward FFT pass on axis 3 with deconvolution and padding
 *   1 forward FFT pass on axis 2          2 forward FFT pass on axis 1
 *   3 interpolation + weight x symbol + Fourier-side energy terms
 *   4 spreading (gather)                  5 sum of split spreading tiles
 *   6 inverse FFT pass on axis 1          7 inverse FFT pass on axis 2
 *   8 inverse FFT pass on axis 3 with crop, deconvolution and energy terms
 *   9 energy reduction
 *  10 JGB_FLAG_SPLIT: separation of the two real transforms on the tiles
 *     the interpolation reads
 *  11 JGB_FLAG_SPLIT: I1's symbol (or its energy sum) over the regular grid
 *  12 interpolation by tiles: sum of each node's tile shares, weight x symbol
 *     and Fourier-side energy terms (stage 3 is then the tile products alone)
 * (2D problems run no pass on a third axis: stages 2 and 6 stay 0.)
 * Errors: INVALID_ARG (NULL plan, max_calls < 1 or > 100000, NULL outputs),
 * OUT_OF_MEMORY (event creation), DEVICE. */
#define JGB_NUM_STAGES 13
jgb_status jgb_timing_begin(jgb_plan_t plan, int max_calls);
jgb_status jgb_timing_end(jgb_plan_t plan, double* stage_ms, int* calls);

/* ---------------------------------------------------------------- batches
 * Many independent densities evaluated together, as in the repeated
 * evaluations of a time-splitting or ground-state solver (Section 1: u is
 * needed on the grid many times for different rho).  A batch owns one plan
 * per member; binding device buffers captures the whole batch into one HIP
 * graph, and each evaluation of the batch is one graph launch:
 *   nstreams == 1: one kernel launch per pipeline site (forward FFT passes,
 *     interpolation, spreading, inverse FFT passes, energy) over all members,
 *     its blocks the members' blocks in turn, each block taking its member's
 *     arguments from a table (members by Algorithm 2 fall back to the next
 *     form);
 *   nstreams > 1: every member's own pipeline, the members spread over
 *     nstreams concurrent branches (longest first, each to the least loaded
 *     branch), so that different members' kernels overlap.
 * Each member's results are bitwise those of its own plan either way. */
typedef struct jgb_batch_s* jgb_batch_t;

/* Create the member plans (as jgb_plan each; all params must name
 * params[0].device and params[0].stream) and nstreams streams of the batch's
 * own at default priority (the graph is captured on them, so params[0].stream
 * may be the NULL stream).  count in [1, 65536], nstreams in [1, 8].
 * Errors as jgb_plan (the message names the failing member). */
jgb_status jgb_batch_create(const jgb_params* params, int count, int nstreams, jgb_batch_t* out);

/* Bind member i to the device arrays rho[i] -> u[i] (its grid and dtype) and,
 * if energies != NULL, its energy to energies[i] (device float64 array of
 * count).  The host arrays rho and u are read during the call only.
 * Synchronises the batch stream, then captures and instantiates the graph
 * (replacing a previous one).  Member plans must not have timing enabled. */
jgb_status jgb_batch_bind(jgb_batch_t batch, const void* const* rho, void* const* u, double* energies);

/* Evaluate every member: the graph runs on a stream owned by the batch,
 * ordered after the work already enqueued on params[0].stream, and later work
 * on params[0].stream is ordered after it.  Enqueue only.  INVALID_ARG if
 * nothing is bound. */
jgb_status jgb_batch_run(jgb_batch_t batch);

/* Kernel launches one jgb_batch_run replays (after jgb_batch_bind): one per
 * pipeline site over all members when the members' pipelines merge (every
 * member by Algorithm 1), else the members' own launches on the batch's
 * streams.  *launches must not be NULL. */
jgb_status jgb_batch_launches(jgb_batch_t batch, int* launches);

/* Member plan i (owned by the batch: do not destroy it). */
jgb_status jgb_batch_plan(jgb_batch_t batch, int i, jgb_plan_t* plan);

/* Synchronise, then free the graph, streams, events and member plans. */
jgb_status jgb_batch_destroy(jgb_batch_t batch);

/* ---------------------------------------------------------------- GPE driver
 * Time splitting for the Gross-Pitaevskii (or Schroedinger-Poisson) equation
 *   i psi_t = [-1/2 Lap + V + beta |psi|^2 + lambda Phi] psi,   Phi = U * |psi|^2,
 * the application that evaluates the potential of eq. gpe many times for a
 * changing rho = |psi|^2 (Section 1).  One step of length dt is Strang
 * splitting: N(dt/2), K(dt), N(dt/2) with
 *   N(h): psi <- exp(-i h (V + beta |psi|^2 + lambda Phi)) psi
 *   K(h): psi <- IDFT(exp(-i h |k|^2 / 2) DFT(psi)),  k_j = 2 pi q_j / R_j
 * (the Laplacian periodic on the box: psi must be negligible at its edges).
 * N keeps |psi|, so Phi is evaluated once per step (plus once per call).  In
 * imaginary time (the ground-state flow) the factors are exp(-h ...) and
 * exp(-h |k|^2 / 2), Phi is evaluated before each half-step, and psi is
 * renormalised to H sum |psi|^2 = 1 after every step.  psi is a device complex
 * array (interleaved re, im) of the plan's real dtype on the grid. */
typedef struct jgb_gpe_s* jgb_gpe_t;

typedef struct {
  uint32_t struct_size;    /* = sizeof(jgb_gpe_params) */
  jgb_params potential;    /* the plan of Phi: grid, box, kernel, nodes, accuracy, precision,
                              flags (JGB_FLAG_SPLIT allowed); its lambda is the lambda above;
                              its device and stream are the driver's */
  double trap[3];          /* V = (1/2) sum_j trap_j^2 x_j^2 when V is NULL (2D: trap[0..1]) */
  const void* V;           /* optional device real array of V on the grid (plan's dtype);
                              caller-owned, read at every step; NULL -> the harmonic trap */
  double beta;             /* local interaction constant, finite */
  double dt;               /* time step (imaginary time: d tau), finite, nonzero (negative runs
                              real time backward) */
  int32_t imaginary;       /* 0: real time; 1: imaginary time with renormalisation */
} jgb_gpe_params;

/* Create the driver: its own stream (default priority), the potential's plan on
 * it, and workspace for rho, Phi and the energy sums.  Errors as jgb_plan, plus
 * INVALID_ARG for the driver's own fields. */
jgb_status jgb_gpe_create(const jgb_gpe_params* params, jgb_gpe_t* out);

/* Advance psi in place by nsteps steps (nsteps >= 0).  use_graph = 1 captures
 * one step into a HIP graph on the first call for this psi and replays it
 * (one launch per step); 0 enqueues every kernel directly (same result).
 * Ordered after earlier work on params.potential.stream, and later work on
 * that stream is ordered after it.  Enqueue only. */
jgb_status jgb_gpe_step(jgb_gpe_t gpe, void* psi, int nsteps, int use_graph);

/* Energies of psi into out (device float64[7]):
 *   {norm, kinetic, trap, local, nonlocal, total, mu}
 * norm = H sum |psi|^2, kinetic = (H / (2 N)) sum_q |k_q|^2 |DFT(psi)_q|^2,
 * trap = H sum V |psi|^2, local = (beta/2) H sum |psi|^4,
 * nonlocal = (lambda/2) H sum Phi |psi|^2 (eq. gpe2), total = their sum,
 * mu = (kinetic + trap + 2 local + 2 nonlocal) / norm.  Enqueue only. */
jgb_status jgb_gpe_energy(jgb_gpe_t gpe, const void* psi, double* out);

/* Synchronise and free the driver (and its plan).  NULL is accepted. */
jgb_status jgb_gpe_destroy(jgb_gpe_t gpe);

/* Copy plan facts into *info (host memory, info->struct_size must be set). */
jgb_status jgb_plan_info(jgb_plan_t plan, jgb_info* info);

/* Synchronise the plan's stream, then free everything the plan owns.
 * NULL is accepted and ignored. */
jgb_status jgb_destroy(jgb_plan_t plan);

/* Message for the last non-OK status returned on the calling thread ("" if
 * none).  The pointer stays valid until the next jgb_* call on this thread. */
const char* jgb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* JGB_H */
