// Internal declarations of the jgb library: the plan object, the spreading
// kernel, and the launchers of every device kernel.
//
// Internal geometry.  Every problem is handled as three axes (a0, a1, a2),
// a2 contiguous in memory.  A 3D problem maps physical axes (x1, x2, x3) to
// (a0, a1, a2); a 2D problem maps (x1, x2) to (a1, a2) and leaves a0 with one
// grid point, one fine-grid point and a spreading width of one.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fastdiv.h"
#include "jgb.h"

namespace jgb {

// Largest spreading width supported (taps per axis).
constexpr int kMaxWidth = 16;
// Largest staged interpolation region, bytes of LDS (of 160 KB per CU, beside
// the kernel's static LDS).
constexpr size_t kInterpLdsCap = 144 * 1024;
// Largest FFT line length (oversampled grid points on one axis).
constexpr int kMaxLine = 1024;
// Output tile of the type-1 gather kernel: TX x TY lanes, TZ points per lane.
constexpr int kTileZ = 16;
// Output tile of the type-1 gather along axis 2 (the bins above stay kTileZ).
constexpr int kGatherZ = 8;
// Offset added to the signed tile-relative footprint starts of the gather lists
// (when the plan's grid needs no wrap-around, Plan::gather_nowrap).
constexpr int kGatherBias = 512;
// Output tile of the ring-factored gather (3D): a0 x a1 x a2 points.
constexpr int kRingTile0 = 16;
constexpr int kRingTile1 = 8;
constexpr int kRingTile2 = 16;
// Bits of a ring node entry's code beside its a0 and a1 start codes (10 bits
// each): the entry is its ring's last in the tile, and then the a2 start code.
constexpr int kRingEndBit = 20;
constexpr int kRingZBit = 21;
// Spare entries at the end of the ring node list (read by the prefetch of the
// batch after the last).
constexpr int kRingSpare = 32;
// Per-node kernel values, tabulated at plan time: for each internal axis a,
// the w values of its taps at [a (w + 1), a (w + 1) + w) of the node's record
// followed by a zero (a unit axis has the single value 1 at tap 0 and zeros
// after it), so that tap d of axis a is read at a (w + 1) + min(d, w) for any
// d taken as unsigned -- a tap off the footprint on either side reads the
// zero, with no mask.  Records are record_stride values apart, 3 (w + 1)
// rounded up to a multiple of 4.
inline int record_stride(int width) { return (3 * (width + 1) + 3) / 4 * 4; }

// ----------------------------------------------------------------- errors

void set_error(const std::string& msg);
const char* get_error();

struct Status {
  jgb_status code = JGB_OK;
  std::string msg;
  static Status ok() { return {}; }
};

// ----------------------------------------------------------------- plan

template <typename T>
struct cplx {
  T re, im;
};

struct NodeArrays {
  // Half node set in bin-sorted order.
  int4* hdr = nullptr;                         // first tap per axis (x, y, z), wrapped into [0, nf); w unused
  void* frac[3] = {nullptr, nullptr, nullptr};  // s - start in fine cells, T
  double* coef = nullptr;                      // 2 c_j (pair k, -k folded in)
  int* perm = nullptr;                         // sorted position -> natural half index
  void* uhat = nullptr;                        // c_j rho^_j, complex T
  void* wts = nullptr;                         // per node record_stride(width) kernel values, T
};

struct WorkItem {
  int tile;    // linear tile index (t0 * nt1 + t1) * nt2 + t2
  int vbegin;  // range of the node list d_list handled by this item
  int vend;
  int slot;    // -1: write the tile to the grid; >= 0: write partial slot
};

// A work item of the spreading by rings: a tile (slot -1) or one of its
// partial tiles (slot >= 0), and the node-entry ranges [e[w], e[w + 1]) of
// the block's four wavefronts, each holding whole rings.
struct RingItem {
  int tile;
  int slot;
  int e[5];
};

enum Stage {
  ST_FWD_Z = 0, ST_FWD_Y, ST_FWD_X, ST_INTERP, ST_SPREAD, ST_SPREAD_REDUCE,
  ST_INV_X, ST_INV_Y, ST_INV_Z, ST_ENERGY, ST_SPLIT_UNMIX, ST_SPLIT_SYMBOL, ST_INTERP_REDUCE, ST_COUNT
};

// Event ring for per-stage timing (see jgb_timing_begin).
struct Timing {
  bool on = false;
  int max_calls = 0;
  int calls = 0;
  std::vector<hipEvent_t> ev;   // max_calls * ST_COUNT * 2
  std::vector<char> used;       // max_calls * ST_COUNT
};

struct Plan {
  jgb_params p{};
  mutable Timing timing;
  int device = 0;
  hipStream_t stream = nullptr;
  int dim = 3;
  bool fp64 = true;
  size_t real_bytes = 8;

  int n[3] = {1, 1, 1};    // grid points per internal axis
  int nf[3] = {1, 1, 1};   // oversampled grid per internal axis
  int w[3] = {1, 1, 1};    // taps per internal axis
  double h[3] = {1, 1, 1}; // physical spacing per internal axis (1 for the unit axis)
  double box[3] = {1, 1, 1};
  double H = 1.0;          // cell volume prod h_j over physical axes
  double K = 0.0;          // radius of the Fourier ball
  double radial_c = 0.0;   // bandwidth of the generalized Gaussian radial rule (0: Gauss-Legendre)
  double axis2[3] = {0, 0, 0};  // second dipole orientation m (= the dipole axis n unless given)
  int width = 0;
  double beta = 0.0;
  int64_t M = 0, Mh = 0;
  int n_r = 0, n_theta = 1, n_phi = 0;

  // 1D quadrature rules on the device (float64)
  double* d_gl_r = nullptr;   // radial GL nodes s and weights on [-1,1]: 2*n_r
  double* d_gl_t = nullptr;   // theta GL nodes and weights: 2*n_theta

  NodeArrays nodes;

  // bins == output tiles of the gather; each bin splits into nsub sub-bins of
  // extent S, the unit whose oversampled-grid neighbourhood the interpolation
  // stages in LDS
  int T[3] = {1, 1, 1};      // tile / bin extent per axis
  int S[3] = {1, 1, 1};      // sub-bin extent per axis (divides T)
  int E[3] = {1, 1, 1};      // staged interpolation region per axis (E[2] padded)
  int pstride = 1;           // LDS elements per axis-0 plane of the staged region (>= E1 E2)
  int nsub = 1;
  struct InterpItem {
    int sub;    // key of the sub-bin: bin * nsub + sub-bin index
    int begin;  // range of bin-sorted nodes
    int end;
  };
  InterpItem* d_iitems = nullptr;
  int niitems = 0;
  int iitems_cap = 0;
  int interp_chunk = 512;      // nodes per interpolation block at most (tunable)
  int spread_chunk = 4096;     // list entries per gather block at most (tunable)
  int items_cap = 0, multi_cap = 0, slots_cap = 0;
  std::vector<int> h_sub_start;      // host copy: sorted-node offsets per sub-bin key
  std::vector<int64_t> h_tcount;     // host copy: list offsets per tile
  size_t interp_lds = 0;     // bytes of the staged grid region
  int nt[3] = {1, 1, 1};     // tiles per axis
  int ntiles = 0;
  int GT[3] = {1, 1, 1};     // gather output tile per axis (axis 2: kGatherZ)
  int gnt[3] = {1, 1, 1};    // gather tiles per axis
  int ngtiles = 0;
  int* d_bin_start = nullptr;  // ntiles + 1 offsets into the sorted node list
  int2* d_list = nullptr;      // per tile, the nodes whose footprint touches it (concatenated):
                               // (node, first tap relative to the tile per axis, 10 bits each)
  int64_t nlist = 0;
  bool gather_nowrap = false;  // list starts are signed, plus kGatherBias (else modulo nf)
  WorkItem* d_items = nullptr;
  int nitems = 0;
  int nslots = 0;
  int* d_multi = nullptr;      // per multi-chunk tile: tile index, first slot, slot count (3 ints)
  int nmulti = 0;
  void* d_partials = nullptr;  // nslots tiles of complex T

  // Interpolation by tiles (3D): the gather's tiles, lists and work items
  // drive a matrix-core contraction of each tile's grid values with the
  // kernel values of 16 listed nodes at a time; every list entry yields the
  // node's partial sum over that tile (d_ipart, in list order), and a second
  // kernel sums each node's partials in a fixed order through the node-major
  // index d_nstart / d_npos (node j's entries are d_npos[d_nstart[j] ..
  // d_nstart[j + 1])).
  bool tile_ok = false;        // the tables below are built (autotuned 3D plans)
  bool tile_interp = false;    // and the interpolation uses them

  // Spreading by rings (3D): the nodes of one ring (r_a, theta_b) share their
  // a2 footprint, so each tile of kRingTile0 x kRingTile1 x kRingTile2 points
  // lists, ring by ring, the ring's nodes that touch the tile (d_rnodes: node
  // and code = a0 start | a1 start << 10, each ring padded to whole groups of
  // four with entries whose a0 values all vanish; the ring's last entry also
  // carries kRingEndBit and its a2 start at kRingZBit; kRingSpare spare
  // entries at the end).  Work items run over ranges of a tile's entries that
  // hold whole rings; split tiles write partial tiles (d_partials) that
  // d_rmulti sums.  The host keeps per tile its ring ranges (h_rcount into
  // h_rcost, each ring's entry count, h_rfirst its first entry).
  bool ring_ok = false;        // the ring tables are built
  bool ring_spread = false;    // and the spreading uses them
  int rnt[3] = {1, 1, 1};      // ring tiles per axis
  int nrtiles = 0;
  int2* d_rnodes = nullptr;
  int64_t nrings_ent = 0, nrnodes = 0;
  std::vector<int64_t> h_rcount;  // host: ring offsets per ring tile
  std::vector<int> h_rcost;       // host: per ring of a tile, its node entries
  std::vector<int> h_rfirst;      // host: per ring of a tile, its first node entry
  RingItem* d_ritems = nullptr;
  int nritems = 0, nrslots = 0, nrmulti = 0;
  int* d_rmulti = nullptr;
  int ritems_cap = 0, rmulti_cap = 0, rslots_cap = 0;
  int ring_chunk = 8192;       // node entries per ring work item at most (tunable)

  // Hermitian half of the oversampled spectrum (Algorithm 1: rho and u are
  // real).  The forward FFT keeps only the lines q2 = 0 .. nf2/2 of axis 2
  // (h2 of them, rows of hs2 >= h2 elements: F is [nf0][nf1][hs2]); the
  // interpolation reads F(q) for q2 > nf2/2 as conj F(-q); the inverse's
  // first pass forms (G(q) + conj G(-q)) / 2 on those lines and its last
  // completes each line by symmetry.
  bool r2c = false;
  int h2 = 0, hs2 = 0;
  // per line of G along the inverse's first axis (lines q1 nf2 + q2 in 3D,
  // q2 in 2D): the circular range {first, span} the spreading can write;
  // the first inverse pass reads zero outside it (Algorithm 1)
  int2* d_gext = nullptr;
  // per line of the spectrum F along the forward's last axis (lines q1 c2 +
  // q2 over the kept q2 < c2, 3D plans with the tile tables): the circular
  // range {first, span} the interpolation by tiles reads; the forward's last
  // pass stores nothing outside it when the interpolation runs by tiles and
  // nothing else reads F (Algorithm 1)
  int2* d_fext = nullptr;
  int* d_nstart = nullptr;     // Mh + 1 offsets into d_npos
  int* d_npos = nullptr;       // nlist list positions, node-major
  void* d_ipart = nullptr;     // nlist complex T: per list entry, the tile's share of the node's value

  // FFT tables
  void* d_tw[3] = {nullptr, nullptr, nullptr};      // exp(-2 pi i t / nf) for t < nf, complex T
  double* d_deconv[3] = {nullptr, nullptr, nullptr};// 1 / phi^(m) for m in [-n/2, n/2)

  // grids
  void* d_F = nullptr;  // nf0*nf1*nf2 complex T
  void* d_G = nullptr;  // same size; written only by the spreading (tiles no node touches stay zero)
  void* d_W = nullptr;  // FFT pass intermediate, n0*nf1*nf2 complex T
  double* d_eparts = nullptr;  // energy partials
  int neparts = 0;

  // the node at k = 0 of the 2D Poisson kernel: u += c0 H sum rho.  The first
  // forward pass writes per-block sums of rho (d_mparts, as many as the last
  // inverse pass has blocks); d_origin = {c0 H sum rho, c0 (H sum rho)^2}.
  double c0 = 0.0;
  double* d_mparts = nullptr;
  double* d_origin = nullptr;

  // Algorithm 2 (JGB_FLAG_SPLIT).  The forward FFT transforms rho H / phi^ +
  // i rho H in one go; G's touched tiles first receive the part the
  // interpolation needs, then the spreading result; the inverse FFT's first
  // pass forms the combined spectrum, which it turns into Re = I2 phi^ and
  // Im = I1.  The energy-only and transform calls keep the whole forward
  // spectrum in F (the Fourier-side energy of I1 sums over all of it).
  bool split = false;
  double win[2] = {0.0, 0.0};      // 3D: (a, 0); 2D: (R0, R1)
  int* d_touched = nullptr;        // gather tiles some node touches
  int ntouched = 0;
  unsigned char* d_tflag = nullptr;  // per gather tile: 1 if touched
  int* d_ublocks = nullptr;        // logical blocks of the unmix pass (fft.hip)
  int nublocks = 0;
  double* d_splitk = nullptr;      // per internal axis a: k_a(q) for q < nf_a, then exp(-k_a(q)^2 / a)
  int nsym_blocks = 0;             // blocks of the symbol kernel (also its energy partials)

  size_t workspace_bytes = 0;
  std::vector<void*> allocations;

  // Bytes of each per-call buffer the compute calls write besides the
  // caller's outputs, as allocated: F, G, W, the gather's partial tiles, the
  // weighted node values, and the energy, origin-sum and origin partials.
  enum { WS_F = 0, WS_G, WS_W, WS_PARTIALS, WS_UHAT, WS_EPARTS, WS_MPARTS, WS_ORIGIN, WS_IPART, WS_COUNT };
  size_t ws_bytes[WS_COUNT] = {};
};

// ----------------------------------------------------------------- kernel shape

// Exponential of semicircle, phi(x) = exp(beta (sqrt(1 - (2x/w)^2) - 1)) for
// |x| <= w/2: the spreading kernel (a substitute for the Gaussian of the
// Section 2 NUFFT, chosen for its smaller width at equal accuracy).
template <typename T>
__host__ __device__ inline T es_kernel(T x, T two_over_w, T beta) {
  T z = x * two_over_w;
  T q = T(1) - z * z;
  if (q <= T(0)) return T(0);
  return exp(beta * (sqrt(q) - T(1)));
}

// The paper's spreading kernel (Section 2): the heat kernel with tau = 6/N^2
// on the grid of 2N points per axis, exp(-pi^2 x^2 / 24) at a distance of x
// fine cells, over the nearest 12 points.
template <typename T>
__host__ __device__ inline T gauss_kernel(T x) {
  return exp(T(-M_PI * M_PI / 24.0) * x * x);
}

// ----------------------------------------------------------------- batches
//
// A batch (jgb_batch_*) evaluates many plans with one launch per pipeline
// site over all of its members.  While a launch record is open on the calling
// thread (launch_record()), the launchers append each kernel launch -- its
// argument block, grid, block and LDS size, and the function that launches
// the kernel's batched form -- instead of issuing it.  The batch then merges
// its members' records site by site and issues, for each site, one launch
// whose blocks are the members' blocks in turn: block b belongs to the member
// m with bstart[m] <= b < bstart[m + 1] and runs as that member's block
// b - bstart[m] (see batch_block), with the member's argument block from a
// device table.

typedef hipError_t (*BatchLaunch)(const void* table, const int* bstart, int nmembers, unsigned blocks,
                                  unsigned threads, size_t smem, hipStream_t s);
struct LaunchRecord {
  BatchLaunch launch;
  std::vector<unsigned char> args;  // the kernel's argument block
  unsigned blocks = 0, threads = 0;
  size_t smem = 0;
};
// the calling thread's open record (null: launches are issued)
std::vector<LaunchRecord>*& launch_record();

// The member m of a batched launch that block b belongs to, and b's block
// within the member, or -1 for a padding block.  bstart holds the members'
// first blocks (nm + 1 offsets, each a multiple of eight, so that every
// member's blocks keep their place in the dispatch order across the eight
// XCDs) and then the members' block counts.
__device__ __forceinline__ int batch_block(const int* bstart, int nm, int b, int& m) {
  int lo = 0, hi = nm - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bstart[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  m = lo;
  const int blk = b - bstart[lo];
  return blk < bstart[nm + 1 + lo] ? blk : -1;
}

template <typename A, void (*KB)(const A*, const int*, int)>
hipError_t batch_launch(const void* table, const int* bstart, int nm, unsigned blocks, unsigned threads, size_t smem,
                        hipStream_t s) {
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(KB, dim3(blocks), dim3(threads), smem, s, static_cast<const A*>(table), bstart, nm);
  return hipGetLastError();
}

// Launch kernel K (argument block a) or, with a record open, record it with
// its batched form KB.
template <typename A, void (*K)(A), void (*KB)(const A*, const int*, int)>
hipError_t launch(const A& a, unsigned blocks, unsigned threads, size_t smem, hipStream_t s) {
  if (std::vector<LaunchRecord>* rec = launch_record()) {
    LaunchRecord r;
    r.launch = &batch_launch<A, KB>;
    r.args.assign(reinterpret_cast<const unsigned char*>(&a), reinterpret_cast<const unsigned char*>(&a) + sizeof(A));
    r.blocks = blocks;
    r.threads = threads;
    r.smem = smem;
    rec->push_back(std::move(r));
    return hipSuccess;
  }
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(K, dim3(blocks), dim3(threads), smem, s, a);
  return hipGetLastError();
}

// ----------------------------------------------------------------- launchers

// Record the stage's start / end event of the current call when timing is on.
inline void stage_mark(const Plan& pl, int stage, int which, hipStream_t s) {
  Timing& t = pl.timing;
  if (stage < 0 || !t.on || t.calls >= t.max_calls) return;
  size_t i = (size_t)t.calls * ST_COUNT + stage;
  (void)hipEventRecord(t.ev[2 * i + which], s);
  if (which == 1) t.used[i] = 1;
}
inline void call_done(const Plan& pl) {
  Timing& t = pl.timing;
  if (t.on && t.calls < t.max_calls) t.calls++;
}

hipError_t launch_gl_roots(int n, double* out, hipStream_t s);
hipError_t launch_node_keys(const Plan& pl, int* keys, hipStream_t s);
hipError_t launch_node_setup(const Plan& pl, const int* perm_dev, hipStream_t s);
hipError_t launch_node_export(const Plan& pl, double* k, double* w, double* c, hipStream_t s);

// mode of the interpolation pass
enum InterpMode { INTERP_POTENTIAL = 0, INTERP_ENERGY = 1, INTERP_TRANSFORM = 2 };

template <typename T>
hipError_t launch_fft_forward(const Plan& pl, const T* rho, hipStream_t s);
template <typename T>
hipError_t launch_fft_inverse(const Plan& pl, T* u, const T* rho_for_energy, hipStream_t s);
// Algorithm 2's potential: the forward passes but the last, then the paired
// unmix pass along the last axis, which writes A into G's touched tiles (the
// inverse's first pass recomputes Z from the same input, so Z is not stored)
template <typename T>
hipError_t launch_split_forward(const Plan& pl, const T* rho, hipStream_t s);
// the unmix pass's logical blocks for the touched-tile flags tf
std::vector<int> split_unmix_blocks(const Plan& pl, const std::vector<unsigned char>& tf);
template <typename T>
hipError_t launch_interp(const Plan& pl, InterpMode mode, void* out, hipStream_t s);
template <typename T>
hipError_t launch_spread(const Plan& pl, hipStream_t s);
template <typename T>
hipError_t launch_ring_spread(const Plan& pl, hipStream_t s);
template <typename T>
hipError_t launch_density(const Plan& pl, const void* psi, void* rho, hipStream_t s);
template <typename T>
hipError_t launch_psi_gradient(const Plan& pl, const void* psi, const void* u, const double* gscale, double factor,
                               void* grad, hipStream_t s);
// Algorithm 2: the tiles of G the interpolation reads get the transform of
// rho H / phi^ alone; I1's Fourier-side energy partials go to d_eparts + eoff
// (the inverse FFT's first pass forms its own spectrum)
template <typename T>
hipError_t launch_split_unmix(const Plan& pl, hipStream_t s);
template <typename T>
hipError_t launch_split_energy(const Plan& pl, int eoff, hipStream_t s);
// periodic complex FFT of the plan's N grid in place (sign -1 or +1)
template <typename T>
hipError_t launch_fft_periodic(const Plan& pl, void* const tw[3], void* data, int sign, hipStream_t s);
// the GPE kinetic step in place: forward FFT, multiplier exp(-i h |k|^2 / 2) / N
// (imaginary: exp(-h |k|^2 / 2) / N), inverse FFT, with the last forward and
// the first inverse pass fused; kt: k per internal axis at offsets koff
template <typename T>
hipError_t launch_fft_periodic_kinetic(const Plan& pl, void* const tw[3], void* data, const double* kt,
                                       const int koff[3], double h, int imaginary, double inv_n, hipStream_t s);
// u = U*rho (and E) by the plan's pipeline, enqueued on stream st
jgb_status potential_pipeline(Plan& pl, const void* rho, void* u, double* energy, hipStream_t st);
int fft_inverse_z_blocks(const Plan& pl);
int interp_blocks(const Plan& pl);
// energy partials the interpolation by tiles writes (0 without its tables)
int tile_interp_blocks(const Plan& pl);
hipError_t interp_prepare(const Plan& pl);
// out = scale (sum of the n parts + *extra); extra may be null
hipError_t launch_energy_finalize(const double* parts, int n, double scale, const double* extra, double* out,
                                  hipStream_t s);
// d_origin from d_mparts (the node at k = 0)
hipError_t launch_origin(const Plan& pl, hipStream_t s);

}  // namespace jgb

// The opaque plan handle of the C ABI.
struct jgb_plan_s {
  jgb::Plan pl;
};
