// Plan construction: parameter checks, NUFFT accuracy parameters, device node
// generation and bin sort, FFT and deconvolution tables, gather work lists and
// workspace.  Everything here runs once per plan; the compute calls only read
// what the plan holds.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <string>
#include <thread>

#include "common.h"
#include "lists.h"
#include "radial.h"

namespace jgb {

namespace {

// candidate work-item sizes; the first of each is the smallest and sizes the buffers
constexpr int kInterpChunks[] = {256, 512, 1024, 2048};
constexpr int kSpreadChunks[] = {256, 512, 1024, 2048, 4096, 8192};
// the autotuner's record of the interpolation by tiles in place of a chunk size
constexpr int kTileInterp = -1;
// node entries per work item of the ring-factored spreading (a ring entry
// counts as kRingEntryCost node entries)
constexpr int kRingChunks[] = {512, 1024, 2048, 4096, 8192, 16384};
constexpr int kRingEntryCost = 8;
// The chunks below 1024 (2048 by rings) are tried only for small node sets
// (such as Algorithm 2's I2), where a few long items would leave most CUs
// idle; for large sets their partial tiles would not pay.
constexpr int64_t kSmallNodeSet = 65536;
int min_spread_chunk(int64_t Mh) { return Mh <= kSmallNodeSet ? 256 : 1024; }
int min_ring_chunk(int64_t Mh) { return Mh <= kSmallNodeSet ? 512 : 2048; }
constexpr size_t kInterpLdsMax = kInterpLdsCap;

bool is_235(int64_t n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

Status fail(jgb_status c, const std::string& m) { return Status{c, m}; }

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on the
// three-term recurrence (host copy for the deconvolution quadrature).
void host_gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    if (2 * i + 1 == n) z = 0.0;
    double p1 = 1, dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0;
      p1 = z;
      double d0 = 0.0, d1 = 1.0;
      for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        double d2 = d0 + (2.0 * k + 1.0) * p1;
        p0 = p1;
        p1 = p2;
        d0 = d1;
        d1 = d2;
      }
      dp = d1;
      if (2 * i + 1 == n) break;
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    x[n - 1 - i] = -z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Fourier transform of the spreading kernel, phi^(xi) = int phi(x) cos(xi x) dx
// over |x| <= w/2, by Gauss-Legendre quadrature in float64; for the paper's
// Gaussian exp(-pi^2 x^2 / 24) (beta = 0) its closed form over the whole line,
// sqrt(24 / pi) exp(-6 xi^2 / pi^2), the deconvolution of Section 2.
std::vector<double> kernel_ft(int w, double beta, const std::vector<double>& xi) {
  if (beta == 0.0) {
    std::vector<double> out(xi.size());
    for (size_t k = 0; k < xi.size(); ++k) out[k] = std::sqrt(24.0 / M_PI) * std::exp(-6.0 * xi[k] * xi[k] / (M_PI * M_PI));
    return out;
  }
  std::vector<double> z, om;
  int nq = std::max(200, 8 * w + 40);
  host_gauss_legendre(nq, z, om);
  std::vector<double> out(xi.size(), 0.0);
  double half = 0.5 * w;
  for (size_t k = 0; k < xi.size(); ++k) {
    double s = 0.0;
    for (int q = 0; q < nq; ++q) {
      double phi = std::exp(beta * (std::sqrt((1.0 - z[q]) * (1.0 + z[q])) - 1.0));
      s += om[q] * phi * std::cos(xi[k] * half * z[q]);
    }
    out[k] = half * s;
  }
  return out;
}

// Failure injection for tests of the out-of-memory path: with the environment
// variable JGB_FAULT=alloc:K, the K-th device allocation of every plan fails
// as if the device were out of memory (K >= 1).
int injected_alloc_failure() {
  const char* f = getenv("JGB_FAULT");
  if (!f || strncmp(f, "alloc:", 6) != 0) return 0;
  return atoi(f + 6);
}

template <typename Tp>
Status dev_alloc(Plan& pl, Tp** ptr, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 16;
  const int fault = injected_alloc_failure();
  if (fault > 0 && (int)pl.allocations.size() + 1 == fault)
    return fail(JGB_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed (injected)");
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(JGB_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  pl.allocations.push_back(p);
  pl.workspace_bytes += bytes;
  *ptr = (Tp*)p;
  return Status::ok();
}

Status upload(Plan& pl, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return Status::ok();
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, pl.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(pl.stream);
  if (e != hipSuccess) return fail(JGB_ERR_DEVICE, std::string("upload: ") + hipGetErrorString(e));
  return Status::ok();
}

#define TRY(x)                       \
  do {                               \
    Status st_ = (x);                \
    if (st_.code != JGB_OK) return st_; \
  } while (0)

#define TRY_HIP(x, what)                                                              \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) return fail(JGB_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)


// Dispatch order of work items.  Items are grouped into cost classes a factor
// 1.5 apart and the classes go largest first, so that the long items (tiles
// and sub-bins near k = 0, up to a thousand times the median) start early and
// do not form the tail.  Within a class the items keep their spatial order
// and are cut into eight contiguous runs, one per XCD (the hardware hands
// block p to XCD p mod 8, each XCD with its own L2), so that neighbouring
// items -- which read the same node records and grid halos -- share an L2.
// Each class is padded to a multiple of eight with idle items.  The spatial
// order is that of `key` (the Morton code of the tile's or bin's coordinates),
// so that the items a CU group has in flight at once form a compact 3D block
// rather than a thin slab, and a node's neighbouring tiles meet in one L2.
template <typename Item, typename Cost, typename Key>
std::vector<Item> dispatch_order(const std::vector<Item>& items, Cost cost, const Item& idle, Key key) {
  constexpr int kXcd = 8;
  auto cls = [&](const Item& it) { return (int)std::floor(std::log(1.0 + cost(it)) / std::log(1.5)); };
  std::vector<Item> o = items;
  std::stable_sort(o.begin(), o.end(), [&](const Item& x, const Item& y) {
    const int cx = cls(x), cy = cls(y);
    return cx != cy ? cx > cy : key(x) < key(y);
  });
  std::vector<Item> out;
  size_t b = 0;
  while (b < o.size()) {
    size_t e = b;
    while (e < o.size() && cls(o[e]) == cls(o[b])) ++e;
    const size_t m = e - b, q = (m + kXcd - 1) / kXcd;
    const size_t p0 = out.size();
    out.resize(p0 + kXcd * q, idle);
    for (int x = 0; x < kXcd; ++x)
      for (size_t i = 0; i < q; ++i) {
        const size_t src = b + x * q + i;
        if (src < e) out[p0 + kXcd * i + x] = o[src];
      }
    b = e;
  }
  return out;
}

// Morton code of three 10-bit coordinates (bits interleaved, a2 lowest).
uint64_t morton3(uint32_t a0, uint32_t a1, uint32_t a2) {
  uint64_t m = 0;
  for (int b = 0; b < 10; ++b)
    m |= ((uint64_t)((a2 >> b) & 1) << (3 * b)) | ((uint64_t)((a1 >> b) & 1) << (3 * b + 1)) |
         ((uint64_t)((a0 >> b) & 1) << (3 * b + 2));
  return m;
}

// Interpolation work items: nonempty sub-bins, split into runs of at most
// chunk nodes.
std::vector<Plan::InterpItem> interp_items(const Plan& pl, int chunk) {
  std::vector<Plan::InterpItem> iit;
  const std::vector<int>& ss = pl.h_sub_start;
  for (size_t k = 0; k + 1 < ss.size(); ++k)
    for (int b = ss[k]; b < ss[k + 1]; b += chunk) iit.push_back(Plan::InterpItem{(int)k, b, std::min(ss[k + 1], b + chunk)});
  const int nsub = pl.nsub, n12 = pl.nt[1] * pl.nt[2];
  auto key = [&](const Plan::InterpItem& it) {
    const int bin = it.sub / nsub;
    const int b0 = bin / n12, r = bin - b0 * n12, b1 = r / pl.nt[2], b2 = r - b1 * pl.nt[2];
    return (morton3(b0, b1, b2) << 8) | (uint64_t)(it.sub - bin * nsub);
  };
  return dispatch_order(iit, [](const Plan::InterpItem& it) { return (double)(it.end - it.begin); },
                        Plan::InterpItem{-1, 0, 0}, key);
}

// Gather work items: one block per tile, tiles with longer lists split into
// chunks whose partial tiles are summed afterwards.
void spread_items(const Plan& pl, int chunk, std::vector<WorkItem>& items, std::vector<int>& multi, int& nslots) {
  items.clear();
  multi.clear();
  nslots = 0;
  const std::vector<int64_t>& tc = pl.h_tcount;
  for (int tile = 0; tile < pl.ngtiles; ++tile) {
    const int64_t b = tc[tile], e = tc[tile + 1], L = e - b;
    if (L == 0) continue;  // stays zero (cleared at plan time)
    if (L <= chunk) {
      items.push_back(WorkItem{tile, (int)b, (int)e, -1});
    } else {
      int k = (int)((L + chunk - 1) / chunk);
      multi.push_back(tile);
      multi.push_back(nslots);
      multi.push_back(k);
      for (int c = 0; c < k; ++c) {
        int64_t vb = b + (int64_t)c * chunk;
        int64_t ve = std::min<int64_t>(e, vb + chunk);
        items.push_back(WorkItem{tile, (int)vb, (int)ve, nslots + c});
      }
      nslots += k;
    }
  }
  const int n12 = pl.gnt[1] * pl.gnt[2];
  auto key = [&](const WorkItem& it) {
    const int t0 = it.tile / n12, r = it.tile - t0 * n12, t1 = r / pl.gnt[2], t2 = r - t1 * pl.gnt[2];
    return morton3(t0, t1, t2);
  };
  items = dispatch_order(items, [](const WorkItem& it) { return (double)(it.vend - it.vbegin); },
                         WorkItem{-1, 0, 0, -1}, key);
}

// Work items of the spreading by rings: one per ring tile, tiles whose rings
// cost more than chunk split at ring boundaries into items that write
// partial tiles (cost: node entries plus kRingEntryCost per ring); each item's
// rings are shared out among the block's four wavefronts in contiguous runs
// of about equal cost.
void ring_items(const Plan& pl, int chunk, std::vector<RingItem>& items, std::vector<int>& multi, int& nslots) {
  items.clear();
  multi.clear();
  nslots = 0;
  const std::vector<int64_t>& rc = pl.h_rcount;
  std::vector<double> cum(pl.h_rcost.size() + 1, 0.0);
  for (size_t i = 0; i < pl.h_rcost.size(); ++i) cum[i + 1] = cum[i] + pl.h_rcost[i] + kRingEntryCost;
  auto entry = [&](int64_t r) {  // first node entry of ring r (r may be one past a tile's last)
    return r < (int64_t)pl.h_rfirst.size() ? pl.h_rfirst[r] : pl.h_rfirst.back() + pl.h_rcost.back();
  };
  auto make = [&](int tile, int slot, int64_t s, int64_t t) {
    RingItem it{tile, slot, {0, 0, 0, 0, 0}};
    const double total = cum[t] - cum[s];
    int64_t r = s;
    it.e[0] = entry(s);
    for (int w = 1; w < 4; ++w) {
      while (r < t && cum[r] - cum[s] < w * total / 4) ++r;
      it.e[w] = (r < t) ? entry(r) : pl.h_rfirst[t - 1] + pl.h_rcost[t - 1];
    }
    it.e[4] = pl.h_rfirst[t - 1] + pl.h_rcost[t - 1];
    items.push_back(it);
  };
  for (int tile = 0; tile < pl.nrtiles; ++tile) {
    const int64_t b = rc[tile], e = rc[tile + 1];
    if (b == e) continue;  // stays zero (cleared at plan time)
    if (cum[e] - cum[b] <= chunk) {
      make(tile, -1, b, e);
      continue;
    }
    const int first = nslots;
    int64_t s = b;
    while (s < e) {
      int64_t t = s + 1;
      while (t < e && cum[t + 1] - cum[s] <= chunk) ++t;
      make(tile, nslots++, s, t);
      s = t;
    }
    multi.push_back(tile);
    multi.push_back(first);
    multi.push_back(nslots - first);
  }
  const int n12 = pl.rnt[1] * pl.rnt[2];
  auto key = [&](const RingItem& it) {
    const int t0 = it.tile / n12, r = it.tile - t0 * n12, t1 = r / pl.rnt[2], t2 = r - t1 * pl.rnt[2];
    return morton3(t0, t1, t2);
  };
  items = dispatch_order(items, [&](const RingItem& it) { return (double)(it.e[4] - it.e[0]); },
                         RingItem{-1, -1, {0, 0, 0, 0, 0}}, key);
}

Status apply_ring_chunk(Plan& pl, int chunk) {
  std::vector<RingItem> items;
  std::vector<int> multi;
  int nslots = 0;
  ring_items(pl, chunk, items, multi, nslots);
  if ((int)items.size() > pl.ritems_cap || (int)multi.size() > pl.rmulti_cap || nslots > pl.rslots_cap)
    return fail(JGB_ERR_DEVICE, "ring items exceed capacity");
  TRY(upload(pl, pl.d_ritems, items.data(), sizeof(RingItem) * items.size()));
  if (!multi.empty()) TRY(upload(pl, pl.d_rmulti, multi.data(), sizeof(int) * multi.size()));
  pl.nritems = (int)items.size();
  pl.nrslots = nslots;
  pl.nrmulti = (int)multi.size() / 3;
  pl.ring_chunk = chunk;
  return Status::ok();
}

// Host threads for the list construction: the hardware's, at most 16.
int host_threads() {
  const unsigned hw = std::thread::hardware_concurrency();
  return (int)std::min(16u, std::max(1u, hw));
}

// Node entries of the spreading by rings (Plan::d_rnodes) from the
// bin-sorted nodes' natural half indices (perm) and footprint starts (hdr):
// per ring tile, the rings that touch it in ring order, and per ring its
// nodes that touch the tile, in sorted order.
Status build_ring_lists(Plan& pl, const std::vector<int>& perm, const std::vector<lists::Start>& hdr) {
  const int RT[3] = {kRingTile0, kRingTile1, kRingTile2};
  lists::Geometry g{};
  for (int a = 0; a < 3; ++a) {
    pl.rnt[a] = (pl.nf[a] + RT[a] - 1) / RT[a];
    g.nf[a] = pl.nf[a];
    g.T[a] = RT[a];
    g.nt[a] = pl.rnt[a];
    g.w[a] = pl.w[a];
  }
  pl.nrtiles = pl.rnt[0] * pl.rnt[1] * pl.rnt[2];
  std::vector<lists::Entry> rnodes;
  const std::string err = lists::ring_lists(g, kGatherBias, pl.n_phi / 2, pl.n_r * pl.n_theta, perm, hdr, kRingEndBit,
                                            kRingZBit, kRingSpare, rnodes, pl.h_rcount, pl.h_rcost, pl.h_rfirst,
                                            host_threads());
  if (!err.empty()) return fail(JGB_ERR_UNSUPPORTED, err);
  pl.nrings_ent = (int64_t)pl.h_rcost.size();
  pl.nrnodes = (int64_t)rnodes.size();
  static_assert(sizeof(lists::Entry) == sizeof(int2), "list entries are int2 on the device");
  TRY(dev_alloc(pl, &pl.d_rnodes, sizeof(lists::Entry) * rnodes.size()));
  TRY(upload(pl, pl.d_rnodes, rnodes.data(), sizeof(lists::Entry) * rnodes.size()));
  // item tables large enough for every chunk candidate
  std::vector<RingItem> items;
  std::vector<int> multi;
  int nslots = 0;
  pl.ritems_cap = pl.rmulti_cap = pl.rslots_cap = 0;
  for (int c : kRingChunks) {
    if (c < min_ring_chunk(pl.Mh)) continue;
    ring_items(pl, c, items, multi, nslots);
    pl.ritems_cap = std::max(pl.ritems_cap, (int)items.size());
    pl.rmulti_cap = std::max(pl.rmulti_cap, (int)multi.size());
    pl.rslots_cap = std::max(pl.rslots_cap, nslots);
  }
  TRY(dev_alloc(pl, &pl.d_ritems, sizeof(RingItem) * std::max(pl.ritems_cap, 1)));
  TRY(dev_alloc(pl, &pl.d_rmulti, sizeof(int) * std::max(pl.rmulti_cap, 1)));
  return Status::ok();
}

Status apply_interp_chunk(Plan& pl, int chunk) {
  std::vector<Plan::InterpItem> iit = interp_items(pl, chunk);
  if ((int)iit.size() > pl.iitems_cap) return fail(JGB_ERR_DEVICE, "interpolation items exceed capacity");
  TRY(upload(pl, pl.d_iitems, iit.data(), sizeof(Plan::InterpItem) * iit.size()));
  pl.niitems = (int)iit.size();
  pl.interp_chunk = chunk;
  return Status::ok();
}

Status apply_spread_chunk(Plan& pl, int chunk) {
  std::vector<WorkItem> items;
  std::vector<int> multi;
  int nslots = 0;
  spread_items(pl, chunk, items, multi, nslots);
  if ((int)items.size() > pl.items_cap || (int)multi.size() > pl.multi_cap || nslots > pl.slots_cap)
    return fail(JGB_ERR_DEVICE, "gather items exceed capacity");
  TRY(upload(pl, pl.d_items, items.data(), sizeof(WorkItem) * items.size()));
  TRY(upload(pl, pl.d_multi, multi.data(), sizeof(int) * multi.size()));
  pl.nitems = (int)items.size();
  pl.nslots = nslots;
  pl.nmulti = (int)multi.size() / 3;
  pl.spread_chunk = chunk;
  return Status::ok();
}

// ------------------------------------------------------------ autotuning
//
// The work-item sizes of the two tap kernels trade load balance against
// per-item overhead, and the best values depend on the node distribution
// (grid, node counts, cutoff), the width and the precision.  With
// JGB_FLAG_AUTOTUNE the plan times every candidate on the device and keeps
// the fastest; results are cached in the JSON file named by the environment
// variable JGB_AUTOTUNE_CACHE (an object mapping a key string to
// {"interp_chunk": i, "spread_chunk": s}).

std::string tune_key(const Plan& pl) {
  char buf[256];
  double kh = pl.K * std::max(pl.h[0] * (pl.n[0] > 1), std::max(pl.h[1], pl.h[2])) / M_PI;
  snprintf(buf, sizeof(buf), "gfx950 d%d n%dx%dx%d nodes%dx%dx%d rule%d kh%.6f w%d%s %s", pl.dim, pl.n[0], pl.n[1],
           pl.n[2], pl.n_r, pl.n_theta, pl.n_phi, pl.p.theta_rule, kh, pl.width, pl.beta == 0.0 ? " gauss" : "",
           pl.fp64 ? "fp64" : "mixed");
  return buf;
}

bool cache_lookup(const std::string& path, const std::string& key, int& ic, int& sc) {
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return false;
  std::string text;
  char chunk[4096];
  size_t got;
  while ((got = fread(chunk, 1, sizeof(chunk), f)) > 0) text.append(chunk, got);
  fclose(f);
  size_t at = text.find("\"" + key + "\"");
  if (at == std::string::npos) return false;
  size_t i1 = text.find("\"interp_chunk\":", at), i2 = text.find("\"spread_chunk\":", at);
  if (i1 == std::string::npos || i2 == std::string::npos) return false;
  if (sscanf(text.c_str() + i1, "\"interp_chunk\": %d", &ic) != 1) return false;
  if (sscanf(text.c_str() + i2, "\"spread_chunk\": %d", &sc) != 1) return false;
  bool ok_i = false, ok_s = false;
  for (int c : kInterpChunks) ok_i |= (c == ic);
  ok_i |= ic == kTileInterp;
  for (int c : kSpreadChunks) ok_s |= (c == sc);
  for (int c : kRingChunks) ok_s |= (-c == sc);  // spreading by rings
  return ok_i && ok_s;
}

void cache_store(const std::string& path, const std::string& key, int ic, int sc, double ms_i, double ms_s) {
  std::string text;
  if (FILE* f = fopen(path.c_str(), "r")) {
    char chunk[4096];
    size_t got;
    while ((got = fread(chunk, 1, sizeof(chunk), f)) > 0) text.append(chunk, got);
    fclose(f);
  }
  size_t close = text.rfind('}');
  char entry[512];
  snprintf(entry, sizeof(entry), "\"%s\": {\"interp_chunk\": %d, \"spread_chunk\": %d, \"interp_ms\": %.4f, \"spread_ms\": %.4f}",
           key.c_str(), ic, sc, ms_i, ms_s);
  std::string out;
  if (close == std::string::npos || text.find('{') == std::string::npos) {
    out = std::string("{\n  ") + entry + "\n}\n";
  } else {
    std::string head = text.substr(0, close);
    while (!head.empty() && (head.back() == '\n' || head.back() == ' ')) head.pop_back();
    bool empty = head.find_last_not_of("{ \n") == std::string::npos;
    out = head + (empty ? "\n  " : ",\n  ") + entry + "\n}\n";
  }
  if (FILE* f = fopen(path.c_str(), "w")) {
    fwrite(out.data(), 1, out.size(), f);
    fclose(f);
  }
}

template <typename T>
Status time_stage(Plan& pl, bool interp, double& best_ms) {
  hipEvent_t e0, e1;
  TRY_HIP(hipEventCreate(&e0), "event");
  TRY_HIP(hipEventCreate(&e1), "event");
  best_ms = 1e30;
  hipError_t err = hipSuccess;
  for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
    err = hipEventRecord(e0, pl.stream);
    if (err == hipSuccess)
      err = interp ? launch_interp<T>(pl, INTERP_POTENTIAL, nullptr, pl.stream) : launch_spread<T>(pl, pl.stream);
    if (err == hipSuccess) err = hipEventRecord(e1, pl.stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0 && err == hipSuccess) best_ms = std::min(best_ms, (double)ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  TRY_HIP(err, "autotune timing");
  return Status::ok();
}

Status autotune(Plan& pl) {
  const char* path = getenv("JGB_AUTOTUNE_CACHE");
  const std::string key = tune_key(pl);
  int ic = 0, sc = 0;
  const bool forced = (pl.p.flags & JGB_FLAG_INTERP_TILES) != 0;
  const bool forced_rings = (pl.p.flags & JGB_FLAG_SPREAD_RINGS) != 0;
  if (path && cache_lookup(path, key, ic, sc) && (ic != kTileInterp || pl.tile_ok) && (sc > 0 || pl.ring_ok) &&
      !(forced_rings && sc > 0)) {
    pl.tile_interp = forced || ic == kTileInterp;
    if (!pl.tile_interp) TRY(apply_interp_chunk(pl, ic));
    pl.ring_spread = sc < 0;
    if (sc > 0) TRY(apply_spread_chunk(pl, sc));
    else TRY(apply_ring_chunk(pl, -sc));
    return Status::ok();
  }
  // ordinary values on the grid: time on an all-zero oversampled grid
  size_t ngrid = (size_t)pl.nf[0] * pl.nf[1] * pl.nf[2];
  TRY_HIP(hipMemsetAsync(pl.d_F, 0, ngrid * 2 * pl.real_bytes, pl.stream), "autotune clear");
  double best_i = 1e30, best_s = 1e30;
  for (int c : kInterpChunks) {
    TRY(apply_interp_chunk(pl, c));
    double ms;
    TRY(pl.fp64 ? time_stage<double>(pl, true, ms) : time_stage<float>(pl, true, ms));
    if (ms < best_i) {
      best_i = ms;
      ic = c;
    }
  }
  TRY(apply_interp_chunk(pl, ic));
  if (pl.tile_ok && !(pl.p.flags & JGB_FLAG_INTERP_TILES)) {
    // the interpolation by tiles on the matrix cores, against the best chunk
    pl.tile_interp = true;
    double ms;
    TRY(pl.fp64 ? time_stage<double>(pl, true, ms) : time_stage<float>(pl, true, ms));
    if (ms < best_i) {
      best_i = ms;
      ic = kTileInterp;
    } else {
      pl.tile_interp = false;
    }
  }
  double ms0;
  TRY(pl.fp64 ? time_stage<double>(pl, true, ms0) : time_stage<float>(pl, true, ms0));  // node values for spreading
  pl.ring_spread = false;
  if (!forced_rings) {
    for (int c : kSpreadChunks) {
      if (c < min_spread_chunk(pl.Mh)) continue;
      TRY(apply_spread_chunk(pl, c));
      double ms;
      TRY(pl.fp64 ? time_stage<double>(pl, false, ms) : time_stage<float>(pl, false, ms));
      if (ms < best_s) {
        best_s = ms;
        sc = c;
      }
    }
    TRY(apply_spread_chunk(pl, sc));
  }
  if (pl.ring_ok) {
    // the spreading by rings, each chunk, against the best of the above
    pl.ring_spread = true;
    int rc = 0;
    double best_r = 1e30;
    for (int c : kRingChunks) {
      if (c < min_ring_chunk(pl.Mh)) continue;
      TRY(apply_ring_chunk(pl, c));
      double ms;
      TRY(pl.fp64 ? time_stage<double>(pl, false, ms) : time_stage<float>(pl, false, ms));
      if (ms < best_r) {
        best_r = ms;
        rc = c;
      }
    }
    TRY(apply_ring_chunk(pl, rc));
    if (best_r < best_s || forced_rings) {
      best_s = best_r;
      sc = -rc;
    } else {
      pl.ring_spread = false;
    }
  }
  if (path) cache_store(path, key, ic, sc, best_i, best_s);
  return Status::ok();
}

}  // namespace

void accuracy_parameters(double eps, bool gaussian, int& w, double& beta);

Status validate(const jgb_params* p) {
  if (!p) return fail(JGB_ERR_INVALID_ARG, "params is NULL");
  if (p->struct_size != sizeof(jgb_params)) return fail(JGB_ERR_INVALID_ARG, "params.struct_size != sizeof(jgb_params)");
  if (p->dim != 2 && p->dim != 3) return fail(JGB_ERR_INVALID_ARG, "dim must be 2 or 3");
  for (int j = 0; j < p->dim; ++j) {
    int64_t n = p->n[j];
    if (n < 8 || n > 512 || n % 2) return fail(JGB_ERR_INVALID_ARG, "n[j] must be even and in [8, 512]");
    if (!is_235(2 * n)) return fail(JGB_ERR_UNSUPPORTED, "2 n[j] must factor into 2, 3 and 5");
    if (!(std::isfinite(p->box[j]) && p->box[j] > 0)) return fail(JGB_ERR_INVALID_ARG, "box[j] must be finite and > 0");
  }
  if (p->kernel == JGB_COULOMB_2D || p->kernel == JGB_DIPOLE_2D || p->kernel == JGB_POISSON_2D) {
    if (p->dim != 2) return fail(JGB_ERR_INVALID_ARG, "2D kernels need dim == 2");
  } else if (p->kernel == JGB_COULOMB_3D || p->kernel == JGB_DIPOLE_3D) {
    if (p->dim != 3) return fail(JGB_ERR_INVALID_ARG, "3D kernels need dim == 3");
  } else {
    return fail(JGB_ERR_INVALID_ARG, "unknown kernel");
  }
  if (p->kernel == JGB_DIPOLE_3D || p->kernel == JGB_DIPOLE_2D) {
    double nn = 0, mm = 0;
    for (int i = 0; i < 3; ++i) {
      if (!std::isfinite(p->dipole_axis[i])) return fail(JGB_ERR_INVALID_ARG, "dipole_axis not finite");
      if (!std::isfinite(p->dipole_axis2[i])) return fail(JGB_ERR_INVALID_ARG, "dipole_axis2 not finite");
      nn += p->dipole_axis[i] * p->dipole_axis[i];
      mm += p->dipole_axis2[i] * p->dipole_axis2[i];
    }
    if (std::fabs(std::sqrt(nn) - 1.0) > 1e-12) return fail(JGB_ERR_INVALID_ARG, "dipole_axis must be a unit vector");
    if (mm != 0.0 && std::fabs(std::sqrt(mm) - 1.0) > 1e-12)
      return fail(JGB_ERR_INVALID_ARG, "dipole_axis2 must be zero or a unit vector");
  }
  if (!std::isfinite(p->alpha)) return fail(JGB_ERR_INVALID_ARG, "alpha must be finite");
  if (!std::isfinite(p->lambda)) return fail(JGB_ERR_INVALID_ARG, "lambda must be finite");
  if (!(p->eps >= 1e-13 && p->eps <= 1e-2)) return fail(JGB_ERR_INVALID_ARG, "eps must be in [1e-13, 1e-2]");
  if (p->precision != JGB_FP64 && p->precision != JGB_MIXED) return fail(JGB_ERR_INVALID_ARG, "unknown precision");
  if (p->precision == JGB_MIXED && p->eps < 1e-6) return fail(JGB_ERR_INVALID_ARG, "JGB_MIXED needs eps >= 1e-6");
  if (p->n_r < 1) return fail(JGB_ERR_INVALID_ARG, "n_r must be >= 1");
  if (p->dim == 3 && p->n_theta < 1) return fail(JGB_ERR_INVALID_ARG, "n_theta must be >= 1");
  if (p->n_phi < 2 || p->n_phi % 2) return fail(JGB_ERR_INVALID_ARG, "n_phi must be even and >= 2");
  if (p->theta_rule != JGB_THETA_GL && p->theta_rule != JGB_COSTHETA_GL) return fail(JGB_ERR_INVALID_ARG, "unknown theta_rule");
  double hmax = 0;
  for (int j = 0; j < p->dim; ++j) hmax = std::max(hmax, p->box[j] / (double)p->n[j]);
  double kn = M_PI / hmax;
  if (!(std::isfinite(p->kmax) && p->kmax >= 0)) return fail(JGB_ERR_INVALID_ARG, "kmax must be finite and >= 0");
  if (p->kmax > kn * (1 + 1e-12)) return fail(JGB_ERR_INVALID_ARG, "kmax must not exceed pi / max_j h_j");
  if (p->flags & ~(JGB_FLAG_AUTOTUNE | JGB_FLAG_SPLIT | JGB_FLAG_INTERP_TILES | JGB_FLAG_SPREAD_RINGS |
                   JGB_FLAG_RADIAL_GGQ | JGB_FLAG_GAUSSIAN_KERNEL))
    return fail(JGB_ERR_INVALID_ARG, "unknown flags");
  if ((p->flags & JGB_FLAG_RADIAL_GGQ) && p->n_r > 2048)
    return fail(JGB_ERR_UNSUPPORTED, "JGB_FLAG_RADIAL_GGQ needs n_r <= 2048");
  if ((p->flags & JGB_FLAG_GAUSSIAN_KERNEL) && p->eps < 1e-6)
    return fail(JGB_ERR_UNSUPPORTED, "JGB_FLAG_GAUSSIAN_KERNEL gives about six digits: eps >= 1e-6");
  if ((p->flags & JGB_FLAG_INTERP_TILES) && p->dim != 3)
    return fail(JGB_ERR_UNSUPPORTED, "JGB_FLAG_INTERP_TILES needs dim == 3");
  if ((p->flags & JGB_FLAG_SPREAD_RINGS) && p->dim != 3)
    return fail(JGB_ERR_UNSUPPORTED, "JGB_FLAG_SPREAD_RINGS needs dim == 3");
  for (int i = 0; i < 2; ++i)
    if (!std::isfinite(p->window[i])) return fail(JGB_ERR_INVALID_ARG, "window must be finite");
  if (!(p->flags & JGB_FLAG_SPLIT)) {
    if (p->window[0] != 0.0 || p->window[1] != 0.0) return fail(JGB_ERR_INVALID_ARG, "window needs JGB_FLAG_SPLIT");
  } else if (p->dim == 3) {
    if (p->window[0] < 0.0 || p->window[1] != 0.0)
      return fail(JGB_ERR_INVALID_ARG, "3D window: window[0] = a >= 0 (0: default), window[1] = 0");
  } else {
    const bool dflt = p->window[0] == 0.0 && p->window[1] == 0.0;
    if (!dflt && !(p->window[0] > 0.0 && p->window[1] > p->window[0]))
      return fail(JGB_ERR_INVALID_ARG, "2D window: {R0, R1} with 0 < R0 < R1, or {0, 0}");
  }
  int64_t M = (int64_t)p->n_r * p->n_phi * (p->dim == 3 ? p->n_theta : 1);
  if (M / 2 > (int64_t)std::numeric_limits<int>::max() / 2) return fail(JGB_ERR_UNSUPPORTED, "too many nodes");
  {
    // the spreading kernel addresses the per-node tables (kernel-value records
    // and weighted values of the half node set) by 32-bit byte offsets
    int w;
    double beta;
    accuracy_parameters(p->eps, (p->flags & JGB_FLAG_GAUSSIAN_KERNEL) != 0, w, beta);
    const uint64_t rb = p->precision == JGB_FP64 ? 8 : 4, Mh = (uint64_t)(M / 2);
    if (Mh * (uint64_t)record_stride(w) * rb >= (1ull << 32) || Mh * 2 * rb >= (1ull << 32))
      return fail(JGB_ERR_UNSUPPORTED, "node tables of 4 GiB or more (too many nodes for this eps and precision)");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(JGB_ERR_DEVICE, "no HIP device");
  }
  if (p->device < 0 || p->device >= ndev) return fail(JGB_ERR_INVALID_ARG, "device ordinal out of range");
  return Status::ok();
}

// Spreading width and shape for a requested accuracy at oversampling 2: the
// kernel's aliasing error falls by about a decade per extra tap.  The paper's
// Gaussian (Section 2, about six digits) always spreads to 12 points; beta 0
// marks it.
void accuracy_parameters(double eps, bool gaussian, int& w, double& beta) {
  if (gaussian) {
    w = 12;
    beta = 0.0;
    return;
  }
  w = (int)std::ceil(std::log10(10.0 / eps)) + 1;
  w = std::max(2, std::min(kMaxWidth, w));
  beta = 2.30 * w;
}

Status build_plan(Plan& pl, const jgb_params* p) {
  // wall time of the plan's phases, for JGB_LOG
  const auto t_start = std::chrono::steady_clock::now();
  double t_phase[5] = {0, 0, 0, 0, 0};  // nodes and sort, gather lists, ring lists, tables and grids, tuning
  auto since = [](std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  pl.p = *p;
  pl.device = p->device;
  pl.stream = (hipStream_t)p->stream;
  pl.dim = p->dim;
  pl.fp64 = p->precision == JGB_FP64;
  pl.real_bytes = pl.fp64 ? 8 : 4;
  TRY_HIP(hipSetDevice(pl.device), "hipSetDevice");

  // internal axes
  if (pl.dim == 3) {
    for (int i = 0; i < 3; ++i) {
      pl.n[i] = (int)p->n[i];
      pl.box[i] = p->box[i];
    }
  } else {
    pl.n[0] = 1;
    pl.box[0] = 1.0;
    pl.n[1] = (int)p->n[0];
    pl.n[2] = (int)p->n[1];
    pl.box[1] = p->box[0];
    pl.box[2] = p->box[1];
  }
  double hmax = 0;
  pl.H = 1.0;
  for (int i = 0; i < 3; ++i) {
    if (pl.n[i] == 1) {
      pl.nf[i] = 1;
      pl.h[i] = 1.0;
      continue;
    }
    pl.nf[i] = 2 * pl.n[i];
    pl.h[i] = pl.box[i] / pl.n[i];
    pl.H *= pl.h[i];
    hmax = std::max(hmax, pl.h[i]);
  }
  pl.K = (p->kmax > 0) ? p->kmax : M_PI / hmax;
  // Algorithm 1 on a real density keeps the Hermitian half of the spectrum
  // (Algorithm 2 packs a second real transform into the imaginary part)
  pl.split = (p->flags & JGB_FLAG_SPLIT) != 0;
  pl.r2c = !pl.split;
  pl.h2 = pl.nf[2] / 2 + 1;
  pl.hs2 = pl.r2c ? (pl.h2 + 7) / 8 * 8 : pl.nf[2];
  {
    // the second dipole orientation: m = n unless given
    double mm = 0;
    for (int i = 0; i < 3; ++i) mm += p->dipole_axis2[i] * p->dipole_axis2[i];
    for (int i = 0; i < 3; ++i) pl.axis2[i] = (mm != 0.0) ? p->dipole_axis2[i] : p->dipole_axis[i];
  }
  pl.split = (p->flags & JGB_FLAG_SPLIT) != 0;
  if (pl.split) {
    // Algorithm 2's window in units of the box's Fourier spacing dk = 2 pi /
    // max_j R_j (remarks after eqs. 3.10 and 3.12), and I2's ball: up to where
    // the window is below 5e-18 (3D: exp(-40)) or 1.1e-17 (2D: erfc(6)/2)
    double rmax = 0;
    for (int i = 0; i < 3; ++i)
      if (pl.n[i] > 1) rmax = std::max(rmax, pl.box[i]);
    const double dk = 2.0 * M_PI / rmax;
    if (pl.dim == 3) {
      pl.win[0] = (p->window[0] > 0) ? p->window[0] : 2.0 * dk * dk;
      pl.win[1] = 0.0;
      if (p->kmax <= 0) pl.K = std::min(M_PI / hmax, std::sqrt(40.0 * pl.win[0]));
    } else {
      const bool dflt = p->window[0] == 0.0 && p->window[1] == 0.0;
      pl.win[0] = dflt ? 0.8 * dk : p->window[0];
      pl.win[1] = dflt ? 10.0 * dk : p->window[1];
      if (p->kmax <= 0) pl.K = std::min(M_PI / hmax, pl.win[1]);
    }
  }
  accuracy_parameters(p->eps, (p->flags & JGB_FLAG_GAUSSIAN_KERNEL) != 0, pl.width, pl.beta);
  for (int i = 0; i < 3; ++i) pl.w[i] = (pl.n[i] == 1) ? 1 : pl.width;
  pl.n_r = p->n_r;
  pl.n_theta = (pl.dim == 3) ? p->n_theta : 1;
  pl.n_phi = p->n_phi;
  pl.M = (int64_t)pl.n_r * pl.n_theta * pl.n_phi;
  pl.Mh = pl.M / 2;

  // tiles (== bins)
  pl.T[2] = kTileZ;
  if (pl.dim == 3) {
    pl.T[0] = 8;
    pl.T[1] = 8;
  } else {
    pl.T[0] = 1;
    pl.T[1] = 64;
  }
  pl.ntiles = 1;
  for (int i = 0; i < 3; ++i) {
    pl.nt[i] = (pl.nf[i] + pl.T[i] - 1) / pl.T[i];
    pl.ntiles *= pl.nt[i];
  }
  // the gather's output tiles: the bins' (a0, a1) extent, kGatherZ along a2
  pl.GT[0] = pl.T[0];
  pl.GT[1] = pl.T[1];
  pl.GT[2] = kGatherZ;
  pl.ngtiles = 1;
  for (int i = 0; i < 3; ++i) {
    pl.gnt[i] = (pl.nf[i] + pl.GT[i] - 1) / pl.GT[i];
    pl.ngtiles *= pl.gnt[i];
  }
  // sub-bins: the power-of-two sub-tile whose staged neighbourhood fits the LDS
  // budget with the fewest staged cells per sub-bin cell.  LDS layout of the
  // neighbourhood: rows of E2 = w2 + 16 elements along axis 2 (S2 >= 2 keeps
  // E2 fixed at that value, which the kernel takes as a compile-time stride),
  // planes of `pstride` >= E1 E2 elements along axis 0, with pstride = w (mod 16).
  // The 3D kernel's lanes read tap pairs (a, c) at a pstride + c: consecutive
  // lanes p hit p (mod 16), distinct banks for every 16 lanes, which the LDS
  // (64 banks of 4 bytes) serves together for 16-byte reads; the 2D kernel's
  // lanes read pairs (b, c) at b E2 + c = p (mod 16) likewise.
  {
    const int per_row = 16;
    auto extents = [&](const int S[3], int E[3], int& pstride) {
      for (int i = 0; i < 3; ++i) E[i] = S[i] + pl.w[i] - 1;
      E[2] = pl.w[2] + per_row * ((S[2] - 1 + per_row - 1) / per_row);
      pstride = E[1] * E[2];
      pstride += ((pl.width - pstride) % 16 + 16) % 16;
      return (size_t)E[0] * pstride * 2 * pl.real_bytes;
    };
    double best = 0.0;
    bool found = false;
    for (int s0 = pl.T[0]; s0 >= 1; s0 /= 2)
      for (int s1 = pl.T[1]; s1 >= 1; s1 /= 2)
        for (int s2 = pl.T[2]; s2 >= 2; s2 /= 2) {
          const int S[3] = {s0, s1, s2};
          int E[3], ps;
          const size_t bytes = extents(S, E, ps);
          if (bytes > kInterpLdsMax) continue;
          const double amp = (double)E[0] * E[1] * E[2] / ((double)s0 * s1 * s2);
          if (!found || amp < best * (1.0 - 1e-12)) {
            found = true;
            best = amp;
            for (int i = 0; i < 3; ++i) {
              pl.S[i] = S[i];
              pl.E[i] = E[i];
            }
            pl.pstride = ps;
            pl.interp_lds = bytes;
          }
        }
    if (!found) return fail(JGB_ERR_UNSUPPORTED, "interpolation neighbourhood exceeds LDS");
    if (pl.E[2] != pl.width + 16) return fail(JGB_ERR_UNSUPPORTED, "interpolation row length");
  }
  pl.nsub = (pl.T[0] / pl.S[0]) * (pl.T[1] / pl.S[1]) * (pl.T[2] / pl.S[2]);

  // 1D rules on the device
  TRY(dev_alloc(pl, &pl.d_gl_r, 2 * sizeof(double) * pl.n_r));
  TRY(dev_alloc(pl, &pl.d_gl_t, 2 * sizeof(double) * pl.n_theta));
  pl.radial_c = (p->flags & JGB_FLAG_RADIAL_GGQ) ? radial::bandwidth(pl.n_r, p->eps) : 0.0;
  if (pl.radial_c > 0.0) {
    // the generalized Gaussian rule on [-1, 1], built on the host
    std::vector<double> x, w;
    const std::string err = radial::prolate_rule(pl.radial_c, pl.n_r, x, w);
    if (!err.empty()) return fail(JGB_ERR_UNSUPPORTED, "radial rule: " + err);
    x.insert(x.end(), w.begin(), w.end());
    TRY(upload(pl, pl.d_gl_r, x.data(), sizeof(double) * 2 * pl.n_r));
  } else {
    TRY_HIP(launch_gl_roots(pl.n_r, pl.d_gl_r, pl.stream), "gl roots");
  }
  TRY_HIP(launch_gl_roots(pl.n_theta, pl.d_gl_t, pl.stream), "gl roots");
  if (p->kernel == JGB_POISSON_2D) {
    // the node at k = 0 of the finite-part radial rule: with r_a = K (1 + s_a)/2
    // and w_a = K omega_a / 2, sum_a w_a / r_a = sum_a omega_a / (1 + s_a)
    std::vector<double> gl(2 * pl.n_r);
    TRY_HIP(hipMemcpyAsync(gl.data(), pl.d_gl_r, sizeof(double) * 2 * pl.n_r, hipMemcpyDeviceToHost, pl.stream),
            "gl copy");
    TRY_HIP(hipStreamSynchronize(pl.stream), "gl sync");
    double swr = 0.0;
    for (int a = 0; a < pl.n_r; ++a) swr += gl[pl.n_r + a] / (1.0 + gl[a]);
    const double euler_gamma = 0.57721566490153286061;
    pl.c0 = (std::log(pl.K) - swr + euler_gamma - std::log(2.0)) / (2.0 * M_PI);
  }

  // two work items per CU fill a launch
  int ncu = 0;
  TRY_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, pl.device), "CU count");
  const int fill_items = 2 * std::max(ncu, 1);

  // bin keys of the half node set, stable counting sort on the host
  const int64_t Mh = pl.Mh;
  int* d_keys = nullptr;
  TRY(dev_alloc(pl, &d_keys, sizeof(int) * Mh));
  TRY_HIP(launch_node_keys(pl, d_keys, pl.stream), "node keys");
  std::vector<int> keys(Mh);
  TRY_HIP(hipMemcpyAsync(keys.data(), d_keys, sizeof(int) * Mh, hipMemcpyDeviceToHost, pl.stream), "keys copy");
  TRY_HIP(hipStreamSynchronize(pl.stream), "keys sync");
  const int nkeys = pl.ntiles * pl.nsub;
  std::vector<int> sub_start(nkeys + 1, 0);
  for (int64_t h = 0; h < Mh; ++h) sub_start[keys[h] + 1]++;
  for (int b = 0; b < nkeys; ++b) sub_start[b + 1] += sub_start[b];
  std::vector<int> perm(Mh);
  {
    std::vector<int> fill(sub_start.begin(), sub_start.end() - 1);
    for (int64_t h = 0; h < Mh; ++h) perm[fill[keys[h]]++] = (int)h;
  }
  std::vector<int> bin_start(pl.ntiles + 1, 0);
  for (int b = 0; b <= pl.ntiles; ++b) bin_start[b] = sub_start[(size_t)b * pl.nsub];
  pl.h_sub_start = sub_start;
  {
    pl.iitems_cap = 0;
    for (int c : kInterpChunks) pl.iitems_cap = std::max(pl.iitems_cap, (int)interp_items(pl, c).size());
    // the untuned chunk: the default, halved while a launch would have fewer
    // than two work items per CU (small node sets, such as I2's)
    while (pl.interp_chunk > kInterpChunks[0] && (int)interp_items(pl, pl.interp_chunk).size() < fill_items)
      pl.interp_chunk /= 2;
    TRY(dev_alloc(pl, &pl.d_iitems, sizeof(Plan::InterpItem) * std::max(pl.iitems_cap, 1)));
    TRY(apply_interp_chunk(pl, pl.interp_chunk));
  }
  TRY(dev_alloc(pl, &pl.nodes.perm, sizeof(int) * Mh));
  TRY(upload(pl, pl.nodes.perm, perm.data(), sizeof(int) * Mh));
  TRY(dev_alloc(pl, &pl.nodes.hdr, sizeof(int4) * Mh));
  for (int i = 0; i < 3; ++i) TRY(dev_alloc(pl, &pl.nodes.frac[i], pl.real_bytes * Mh));
  TRY(dev_alloc(pl, &pl.nodes.coef, sizeof(double) * Mh));
  pl.ws_bytes[Plan::WS_UHAT] = 2 * pl.real_bytes * Mh;
  TRY(dev_alloc(pl, &pl.nodes.uhat, pl.ws_bytes[Plan::WS_UHAT]));
  TRY(dev_alloc(pl, &pl.nodes.wts, (size_t)record_stride(pl.width) * pl.real_bytes * Mh));
  TRY_HIP(hipMemsetAsync(pl.nodes.wts, 0, (size_t)record_stride(pl.width) * pl.real_bytes * Mh, pl.stream),
          "clear kernel values");
  TRY_HIP(launch_node_setup(pl, pl.nodes.perm, pl.stream), "node setup");
  TRY(dev_alloc(pl, &pl.d_bin_start, sizeof(int) * (pl.ntiles + 1)));
  TRY(upload(pl, pl.d_bin_start, bin_start.data(), sizeof(int) * (pl.ntiles + 1)));

  TRY_HIP(hipStreamSynchronize(pl.stream), "node setup sync");
  t_phase[0] = since(t_start);
  const auto t_lists = std::chrono::steady_clock::now();
  // exact per-tile node lists: node j (bin-sorted order) is listed under every
  // output tile its w^3 footprint touches, so the gather never visits a node
  // that misses its tile
  static_assert(sizeof(lists::Start) == sizeof(int4), "node headers are int4 on the device");
  std::vector<lists::Start> hdr(Mh);
  TRY_HIP(hipMemcpyAsync(hdr.data(), pl.nodes.hdr, sizeof(int4) * Mh, hipMemcpyDeviceToHost, pl.stream), "hdr copy");
  TRY_HIP(hipStreamSynchronize(pl.stream), "hdr sync");
  // entry: node index and its first tap relative to the tile origin on each
  // axis (10 bits each).  When every axis has nf >= T + w - 1 the start of a
  // footprint that touches the tile has exactly one representative in
  // [-(w - 1), T - 1], stored plus kGatherBias, and the gather needs no
  // reduction modulo nf; otherwise it is stored modulo nf (nf <= 1024).
  pl.gather_nowrap = true;
  for (int a = 0; a < 3; ++a) pl.gather_nowrap &= pl.nf[a] >= pl.GT[a] + pl.w[a] - 1;
  // the node-major index of the list, for the tile interpolation (built only
  // for autotuned plans: the tuner times it against the staged interpolation
  // and keeps the faster)
  pl.tile_ok = pl.dim == 3 && pl.GT[0] == 8 && pl.GT[1] == 8 && pl.GT[2] == 8 &&
               (p->flags & (JGB_FLAG_AUTOTUNE | JGB_FLAG_INTERP_TILES));
  pl.tile_interp = pl.tile_ok && (p->flags & JGB_FLAG_INTERP_TILES);
  std::vector<int64_t> tcount;
  std::vector<lists::Entry> list;
  std::vector<int> nstart, npos;
  {
    lists::Geometry g{};
    for (int a = 0; a < 3; ++a) {
      g.nf[a] = pl.nf[a];
      g.T[a] = pl.GT[a];
      g.nt[a] = pl.gnt[a];
      g.w[a] = pl.w[a];
    }
    const std::string err =
        lists::gather_lists(g, pl.gather_nowrap, kGatherBias, hdr, tcount, list, pl.tile_ok, nstart, npos, host_threads());
    if (!err.empty()) return fail(JGB_ERR_UNSUPPORTED, err);
  }
  const int64_t nlist = tcount[pl.ngtiles];
  if (pl.tile_ok) {
    TRY(dev_alloc(pl, &pl.d_nstart, sizeof(int) * (Mh + 1)));
    TRY(upload(pl, pl.d_nstart, nstart.data(), sizeof(int) * (Mh + 1)));
    TRY(dev_alloc(pl, &pl.d_npos, sizeof(int) * std::max<int64_t>(nlist, 1)));
    if (nlist) TRY(upload(pl, pl.d_npos, npos.data(), sizeof(int) * nlist));
    pl.ws_bytes[Plan::WS_IPART] = (size_t)std::max<int64_t>(nlist, 1) * 2 * pl.real_bytes;
    TRY(dev_alloc(pl, &pl.d_ipart, pl.ws_bytes[Plan::WS_IPART]));
  }
  TRY(dev_alloc(pl, &pl.d_list, sizeof(lists::Entry) * list.size()));
  TRY(upload(pl, pl.d_list, list.data(), sizeof(lists::Entry) * list.size()));
  pl.nlist = nlist;

  pl.h_tcount = tcount;
  if (pl.r2c) {
    // the spreading grid's reach per line of the inverse's first pass (axis
    // 0 in 3D, axis 1 in 2D): that pass reads zero beyond it
    lists::Geometry g{};
    for (int a = 0; a < 3; ++a) {
      g.nf[a] = pl.nf[a];
      g.T[a] = 1;
      g.nt[a] = pl.nf[a];
      g.w[a] = pl.w[a];
    }
    std::vector<lists::Extent> ext;
    const std::string err = lists::line_extents(g, pl.nf[0] > 1 ? 0 : 1, hdr, ext, host_threads());
    if (!err.empty()) return fail(JGB_ERR_UNSUPPORTED, err);
    static_assert(sizeof(lists::Extent) == sizeof(int2), "line extents are int2 on the device");
    TRY(dev_alloc(pl, &pl.d_gext, sizeof(int2) * ext.size()));
    TRY(upload(pl, pl.d_gext, ext.data(), sizeof(int2) * ext.size()));
  }
  if (pl.tile_ok) {
    // the spectrum's reach per line of the forward transform's last pass,
    // from the tiles the interpolation by tiles reads: that pass stores
    // nothing beyond it when the interpolation runs by tiles
    lists::Geometry g{};
    for (int a = 0; a < 3; ++a) {
      g.nf[a] = pl.nf[a];
      g.T[a] = pl.GT[a];
      g.nt[a] = pl.gnt[a];
      g.w[a] = pl.w[a];
    }
    std::vector<lists::Extent> ext;
    const std::string err = lists::tile_read_extents(g, tcount, pl.r2c, ext, host_threads());
    if (!err.empty()) return fail(JGB_ERR_UNSUPPORTED, err);
    TRY(dev_alloc(pl, &pl.d_fext, sizeof(int2) * ext.size()));
    TRY(upload(pl, pl.d_fext, ext.data(), sizeof(int2) * ext.size()));
  }
  t_phase[1] = since(t_lists);
  const auto t_rings = std::chrono::steady_clock::now();
  // the ring tables (3D; built when forced or for the tuner to time)
  {
    const bool forced = (p->flags & JGB_FLAG_SPREAD_RINGS) != 0;
    bool fits = pl.dim == 3;
    const int RT[3] = {kRingTile0, kRingTile1, kRingTile2};
    for (int a = 0; a < 3; ++a) fits &= pl.nf[a] >= RT[a] + pl.w[a] - 1;
    if (forced && !fits)
      return fail(JGB_ERR_UNSUPPORTED, "JGB_FLAG_SPREAD_RINGS needs every oversampled side >= tile + width - 1");
    pl.ring_ok = fits && (p->flags & (JGB_FLAG_AUTOTUNE | JGB_FLAG_SPREAD_RINGS));
    if (pl.ring_ok) TRY(build_ring_lists(pl, perm, hdr));
  }
  {
    std::vector<WorkItem> items;
    std::vector<int> multi;
    int nslots = 0;
    pl.items_cap = pl.multi_cap = pl.slots_cap = 0;
    for (int c : kSpreadChunks) {
      if (c < min_spread_chunk(pl.Mh)) continue;
      spread_items(pl, c, items, multi, nslots);
      pl.items_cap = std::max(pl.items_cap, (int)items.size());
      pl.multi_cap = std::max(pl.multi_cap, (int)multi.size());
      pl.slots_cap = std::max(pl.slots_cap, nslots);
    }
    while (pl.spread_chunk > min_spread_chunk(pl.Mh)) {
      spread_items(pl, pl.spread_chunk, items, multi, nslots);
      if ((int)items.size() >= fill_items) break;
      pl.spread_chunk /= 2;
    }
    TRY(dev_alloc(pl, &pl.d_items, sizeof(WorkItem) * std::max(pl.items_cap, 1)));
    TRY(dev_alloc(pl, &pl.d_multi, sizeof(int) * std::max(pl.multi_cap, 1)));
    pl.ws_bytes[Plan::WS_PARTIALS] = std::max((size_t)std::max(pl.slots_cap, 1) * 64 * kGatherZ,
                                              (size_t)pl.rslots_cap * kRingTile0 * kRingTile1 * kRingTile2) *
                                     2 * pl.real_bytes;
    TRY(dev_alloc(pl, &pl.d_partials, pl.ws_bytes[Plan::WS_PARTIALS]));
    TRY(apply_spread_chunk(pl, pl.spread_chunk));
    if (pl.ring_ok) {
      // the untuned ring chunk: halved while a launch would have fewer than
      // two work items per CU
      std::vector<RingItem> ritems;
      while (pl.ring_chunk > min_ring_chunk(pl.Mh)) {
        ring_items(pl, pl.ring_chunk, ritems, multi, nslots);
        if ((int)ritems.size() >= fill_items) break;
        pl.ring_chunk /= 2;
      }
      TRY(apply_ring_chunk(pl, pl.ring_chunk));
      pl.ring_spread = (p->flags & JGB_FLAG_SPREAD_RINGS) != 0;
    }
  }

  t_phase[2] = since(t_rings);
  const auto t_tables = std::chrono::steady_clock::now();
  // FFT twiddles and deconvolution factors per axis
  for (int a = 0; a < 3; ++a) {
    const int L = pl.nf[a];
    std::vector<double> twd(2 * L);
    for (int t = 0; t < L; ++t) {
      twd[2 * t] = std::cos(2.0 * M_PI * t / L);
      twd[2 * t + 1] = -std::sin(2.0 * M_PI * t / L);
    }
    if (pl.fp64) {
      TRY(dev_alloc(pl, &pl.d_tw[a], sizeof(double) * 2 * L));
      TRY(upload(pl, pl.d_tw[a], twd.data(), sizeof(double) * 2 * L));
    } else {
      std::vector<float> twf(twd.begin(), twd.end());
      TRY(dev_alloc(pl, &pl.d_tw[a], sizeof(float) * 2 * L));
      TRY(upload(pl, pl.d_tw[a], twf.data(), sizeof(float) * 2 * L));
    }
    const int N = pl.n[a];
    std::vector<double> dec(N, 1.0);
    if (N > 1) {
      std::vector<double> xi(N);
      for (int i = 0; i < N; ++i) xi[i] = 2.0 * M_PI * (i - N / 2) / (double)L;
      std::vector<double> ph = kernel_ft(pl.w[a], pl.beta, xi);
      for (int i = 0; i < N; ++i) dec[i] = 1.0 / ph[i];
    }
    TRY(dev_alloc(pl, &pl.d_deconv[a], sizeof(double) * N));
    TRY(upload(pl, pl.d_deconv[a], dec.data(), sizeof(double) * N));
  }

  // grids and energy partials
  size_t ngrid = (size_t)pl.nf[0] * pl.nf[1] * pl.nf[2];
  pl.ws_bytes[Plan::WS_F] = pl.ws_bytes[Plan::WS_G] = ngrid * 2 * pl.real_bytes;
  pl.ws_bytes[Plan::WS_W] = (size_t)pl.n[0] * pl.nf[1] * pl.nf[2] * 2 * pl.real_bytes;
  TRY(dev_alloc(pl, &pl.d_F, pl.ws_bytes[Plan::WS_F]));
  TRY(dev_alloc(pl, &pl.d_G, pl.ws_bytes[Plan::WS_G]));
  TRY(dev_alloc(pl, &pl.d_W, pl.ws_bytes[Plan::WS_W]));
  // only the spreading writes G, and only tiles some node touches: the others
  // are cleared here once
  TRY_HIP(hipMemsetAsync(pl.d_G, 0, ngrid * 2 * pl.real_bytes, pl.stream), "clear spreading grid");
  if (pl.split) {
    // gather tiles some node touches: the interpolation reads only these, the
    // spreading writes only these
    std::vector<int> tl;
    std::vector<unsigned char> tf(pl.ngtiles, 0);
    for (int t = 0; t < pl.ngtiles; ++t)
      if (pl.h_tcount[t + 1] > pl.h_tcount[t]) {
        tl.push_back(t);
        tf[t] = 1;
      }
    pl.ntouched = (int)tl.size();
    TRY(dev_alloc(pl, &pl.d_touched, sizeof(int) * std::max<size_t>(tl.size(), 1)));
    if (!tl.empty()) TRY(upload(pl, pl.d_touched, tl.data(), sizeof(int) * tl.size()));
    TRY(dev_alloc(pl, &pl.d_tflag, (size_t)pl.ngtiles));
    TRY(upload(pl, pl.d_tflag, tf.data(), (size_t)pl.ngtiles));
    // the unmix pass's blocks: those whose line pairs cross a touched tile
    {
      std::vector<int> ub = split_unmix_blocks(pl, tf);
      pl.nublocks = (int)ub.size();
      TRY(dev_alloc(pl, &pl.d_ublocks, sizeof(int) * std::max<size_t>(ub.size(), 1)));
      if (!ub.empty()) TRY(upload(pl, pl.d_ublocks, ub.data(), sizeof(int) * ub.size()));
    }
    // per axis: the regular grid's frequencies k_q = 2 pi q' / (2 R), q' the
    // signed index, and exp(-k_q^2 / a) (3D; 1 in 2D)
    std::vector<double> kt;
    for (int a = 0; a < 3; ++a) {
      const int L = pl.nf[a];
      std::vector<double> kv(L, 0.0), ev(L, 1.0);
      if (pl.n[a] > 1)
        for (int q = 0; q < L; ++q) {
          const int sq = (q < L / 2) ? q : q - L;
          kv[q] = 2.0 * M_PI * sq / (2.0 * pl.box[a]);
          if (pl.dim == 3) ev[q] = std::exp(-kv[q] * kv[q] / pl.win[0]);
        }
      kt.insert(kt.end(), kv.begin(), kv.end());
      kt.insert(kt.end(), ev.begin(), ev.end());
    }
    TRY(dev_alloc(pl, &pl.d_splitk, sizeof(double) * kt.size()));
    TRY(upload(pl, pl.d_splitk, kt.data(), sizeof(double) * kt.size()));
    const int64_t npts = (int64_t)(pl.nf[0] / 2 + 1) * pl.nf[1] * pl.nf[2];
    pl.nsym_blocks = (int)std::min<int64_t>((npts + 255) / 256, 4096);
  }
  if (pl.c0 != 0.0) {
    pl.ws_bytes[Plan::WS_MPARTS] = sizeof(double) * std::max(fft_inverse_z_blocks(pl), 1);
    pl.ws_bytes[Plan::WS_ORIGIN] = sizeof(double) * 2;
    TRY(dev_alloc(pl, &pl.d_mparts, pl.ws_bytes[Plan::WS_MPARTS]));
    TRY(dev_alloc(pl, &pl.d_origin, pl.ws_bytes[Plan::WS_ORIGIN]));
  }
  pl.neparts = std::max(fft_inverse_z_blocks(pl), std::max(pl.iitems_cap, tile_interp_blocks(pl)) + pl.nsym_blocks);
  pl.neparts = std::max(pl.neparts, 1);
  pl.ws_bytes[Plan::WS_EPARTS] = sizeof(double) * pl.neparts;
  TRY(dev_alloc(pl, &pl.d_eparts, pl.ws_bytes[Plan::WS_EPARTS]));
  TRY_HIP(interp_prepare(pl), "interpolation LDS limit");
  TRY_HIP(hipStreamSynchronize(pl.stream), "tables sync");
  t_phase[3] = since(t_tables);
  const auto t_tune = std::chrono::steady_clock::now();
  if (p->flags & JGB_FLAG_AUTOTUNE) TRY(autotune(pl));
  t_phase[4] = since(t_tune);
  // JGB_LOG=1: one line per plan on stderr with the shape the plan chose
  if (const char* lg = getenv("JGB_LOG")) {
    if (lg[0] && lg[0] != '0')
      fprintf(stderr,
              "jgb plan: dim %d n %dx%dx%d nf %dx%dx%d nodes %lld (half %lld) width %d %s %s%s interp %s chunk %d "
              "spread chunk %d tiles %d items %d list entries %lld workspace %.1f MB; seconds: nodes %.3f lists %.3f "
              "rings %.3f tables %.3f tuning %.3f\n",
              pl.dim, pl.n[0], pl.n[1], pl.n[2], pl.nf[0], pl.nf[1], pl.nf[2], (long long)pl.M, (long long)pl.Mh,
              pl.width, pl.fp64 ? "fp64" : "mixed", pl.split ? "algorithm 2" : "algorithm 1",
              pl.r2c ? " (half spectrum)" : "", pl.tile_interp ? "by tiles" : "staged", pl.interp_chunk,
              pl.ring_spread ? -pl.ring_chunk : pl.spread_chunk, pl.ring_spread ? pl.nrtiles : pl.ngtiles,
              pl.ring_spread ? pl.nritems : pl.nitems, (long long)(pl.ring_spread ? pl.nrnodes : pl.nlist),
              pl.workspace_bytes / 1e6, t_phase[0], t_phase[1], t_phase[2], t_phase[3], t_phase[4]);
  }
  TRY_HIP(hipStreamSynchronize(pl.stream), "plan sync");
  TRY_HIP(hipGetLastError(), "plan kernels");
  return Status::ok();
}

void free_plan(Plan& pl) {
  for (void* p : pl.allocations) (void)hipFree(p);
  pl.allocations.clear();
}

}  // namespace jgb
