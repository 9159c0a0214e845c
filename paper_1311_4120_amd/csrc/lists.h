// Host construction of the tap kernels' node lists, free of device code so
// that a CPU build can run it under the address and undefined-behaviour
// sanitizers (the plan calls the same functions).
//
//   gather_lists: for every output tile of the three-axis gather, the nodes
//     whose w^3 footprint touches it (Section 2: the spreading sum of eq. 2.6
//     restricted to the tile), each with its first tap relative to the tile
//     origin on every axis, 10 bits each; optionally the node-major index of
//     the same list (the interpolation by tiles sums a node's entries).
//   ring_lists: for every tile of the spreading by rings, ring by ring (the
//     rings (r_a, theta_b) of the node set of Section 3.1, whose nodes share
//     their a2 footprint), the ring's nodes that touch the tile, each ring
//     padded to whole groups of four, its last entry flagged and carrying the
//     ring's a2 start.
//   line_extents: for every line of the spreading grid along the inverse
//     transform's first axis, the range of positions the nodes' footprints
//     can reach (the grid is zero elsewhere).
//   tile_read_extents: for every line of the forward transform's spectrum
//     along its last axis, the range of positions the interpolation by tiles
//     reads (the rest need not be stored).
//
// Starts are the nodes' first taps wrapped into [0, nf).  A tile-relative
// start is stored, when every axis has nf >= T + w - 1, as its one
// representative in [-(w - 1), T - 1] plus a bias ("nowrap"); otherwise modulo
// nf.  Either way it must fit in 10 bits: the functions return an error
// message instead of a list that would not.
//
// Both run on `threads` host threads over contiguous ranges of nodes (or
// rings, or tiles): per-thread counts per tile give every thread its own
// write positions, so the lists come out identical to a serial build.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

namespace jgb {
namespace lists {

struct Start {  // the layout of the plan's int4 node header
  int x, y, z, unused;
};
struct Entry {  // the layout of an int2 list entry
  int node, code;
};

struct Geometry {
  int nf[3];  // oversampled grid per axis
  int T[3];   // tile extent per axis
  int nt[3];  // tiles per axis
  int w[3];   // taps per axis
};

constexpr int kMaxTaps = 16;

// The distinct tiles (extent T, nf points per axis) that w taps from x0 touch,
// in tap order; returns their number.
inline int touched(int x0, int nf, int T, int w, int* out) {
  int n = 0;
  for (int t = 0; t < w; ++t) {
    const int tile = ((x0 + t) % nf) / T;
    bool seen = false;
    for (int i = 0; i < n; ++i) seen |= (out[i] == tile);
    if (!seen) out[n++] = tile;
  }
  return n;
}

// A footprint start relative to a tile origin, as stored in a list entry.
inline int start_code(int rel, int nf, int T, bool nowrap, int bias) {
  int e = ((rel % nf) + nf) % nf;
  if (!nowrap) return e;
  if (e > T - 1) e -= nf;
  return e + bias;
}

inline bool code_fits(int c) { return c >= 0 && c <= 1023; }

// f(begin, end, thread) over `threads` contiguous ranges of [0, n).
template <typename F>
void parallel_ranges(int64_t n, int threads, F f) {
  threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, n));
  if (threads == 1) {
    f((int64_t)0, n, 0);
    return;
  }
  std::vector<std::thread> pool;
  pool.reserve(threads);
  for (int t = 0; t < threads; ++t) pool.emplace_back(f, n * t / threads, n * (t + 1) / threads, t);
  for (std::thread& th : pool) th.join();
}

// Threads worth starting: one per 4096 nodes at most, and per-thread counts
// per tile within 256 MB.
inline int usable_threads(int threads, int64_t nodes, int64_t ntiles) {
  const int64_t by_mem = ((int64_t)256 << 20) / std::max<int64_t>(1, ntiles * (int64_t)sizeof(int64_t));
  return (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)threads, nodes / 4096 + 1, by_mem}));
}

// Turns per-thread counts per tile (cnt[t][tile]) into per-thread write
// positions (in place) and tile offsets (offs, ntiles + 1).
inline void count_offsets(std::vector<std::vector<int64_t>>& cnt, int64_t ntiles, std::vector<int64_t>& offs) {
  offs.assign(ntiles + 1, 0);
  int64_t run = 0;
  for (int64_t tile = 0; tile < ntiles; ++tile) {
    offs[tile] = run;
    for (std::vector<int64_t>& c : cnt) {
      const int64_t k = c[tile];
      c[tile] = run;
      run += k;
    }
  }
  offs[ntiles] = run;
}

// The three-axis gather's lists (see above): tcount gets ntiles + 1 offsets
// into list; list gets the entries tile by tile, nodes in their order, then
// one spare entry.  With node_major, nstart (Mh + 1 offsets) and npos (list
// positions) index each node's entries in the order of its tiles.
inline std::string gather_lists(const Geometry& g, bool nowrap, int bias, const std::vector<Start>& hdr,
                                std::vector<int64_t>& tcount, std::vector<Entry>& list, bool node_major,
                                std::vector<int>& nstart, std::vector<int>& npos, int threads = 1) {
  for (int a = 0; a < 3; ++a)
    if (g.w[a] < 1 || g.w[a] > kMaxTaps || g.w[a] > g.nf[a]) return "width out of range";
  const int64_t Mh = (int64_t)hdr.size();
  const int64_t ntiles = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];
  threads = usable_threads(threads, Mh, ntiles);
  // visit(j, f): f(tile, code) for node j's tiles in tap order
  auto visit = [&](int64_t j, auto&& f) {
    int tx[kMaxTaps], ty[kMaxTaps], tz[kMaxTaps];
    const int nx = touched(hdr[j].x, g.nf[0], g.T[0], g.w[0], tx);
    const int ny = touched(hdr[j].y, g.nf[1], g.T[1], g.w[1], ty);
    const int nz = touched(hdr[j].z, g.nf[2], g.T[2], g.w[2], tz);
    for (int a0 = 0; a0 < nx; ++a0)
      for (int a1 = 0; a1 < ny; ++a1)
        for (int a2 = 0; a2 < nz; ++a2) {
          const int64_t tile = ((int64_t)tx[a0] * g.nt[1] + ty[a1]) * g.nt[2] + tz[a2];
          const int ex = start_code(hdr[j].x - tx[a0] * g.T[0], g.nf[0], g.T[0], nowrap, bias);
          const int ey = start_code(hdr[j].y - ty[a1] * g.T[1], g.nf[1], g.T[1], nowrap, bias);
          const int ez = start_code(hdr[j].z - tz[a2] * g.T[2], g.nf[2], g.T[2], nowrap, bias);
          f(tile, ex, ey, ez);
        }
  };
  std::vector<std::vector<int64_t>> cnt(threads, std::vector<int64_t>(ntiles, 0));
  std::vector<int64_t> per_node(node_major ? Mh + 1 : 0, 0);
  std::atomic<bool> bad{false};
  parallel_ranges(Mh, threads, [&](int64_t b, int64_t e, int t) {
    std::vector<int64_t>& c = cnt[t];
    for (int64_t j = b; j < e; ++j)
      visit(j, [&](int64_t tile, int ex, int ey, int ez) {
        c[tile]++;
        if (node_major) per_node[j + 1]++;
        if (!code_fits(ex) || !code_fits(ey) || !code_fits(ez)) bad = true;
      });
  });
  if (bad) return "gather list start out of range";
  count_offsets(cnt, ntiles, tcount);
  const int64_t nlist = tcount[ntiles];
  // the kernels address the list by 32-bit byte offsets (8 bytes per entry)
  // and the node-major index by 32-bit positions
  if ((nlist + 1) * 8 >= ((int64_t)1 << 32)) return "gather lists too long";
  list.assign(nlist + 1, Entry{0, 0});
  nstart.clear();
  npos.clear();
  if (node_major) {
    nstart.assign(Mh + 1, 0);
    for (int64_t j = 0; j < Mh; ++j) nstart[j + 1] = nstart[j] + (int)per_node[j + 1];
    npos.assign(nlist, 0);
  }
  parallel_ranges(Mh, threads, [&](int64_t b, int64_t e, int t) {
    std::vector<int64_t>& at = cnt[t];
    for (int64_t j = b; j < e; ++j) {
      int k = 0;
      visit(j, [&](int64_t tile, int ex, int ey, int ez) {
        if (node_major) npos[nstart[j] + k++] = (int)at[tile];
        list[at[tile]++] = Entry{(int)j, ex | (ey << 10) | (ez << 20)};
      });
    }
  });
  return "";
}

// The ring lists (see above).  perm[j] is node j's natural half index
// ((a n_theta + b) nph2 + l); nrings = n_r n_theta.  rnodes gets the entries
// (each ring's last carries 1 << end_bit and its a2 start code << z_bit;
// padding entries repeat the ring's first node with the a0 and a1 codes 1023,
// which leave every a0 tap off the tile), then `spare` spare entries; per tile,
// rcount gets the offsets of its rings into rcost (each ring's entries) and
// rfirst (each ring's first entry).
inline std::string ring_lists(const Geometry& g, int bias, int nph2, int nrings, const std::vector<int>& perm,
                              const std::vector<Start>& hdr, int end_bit, int z_bit, int spare,
                              std::vector<Entry>& rnodes, std::vector<int64_t>& rcount, std::vector<int>& rcost,
                              std::vector<int>& rfirst, int threads = 1) {
  for (int a = 0; a < 3; ++a)
    if (g.nf[a] < g.T[a] + g.w[a] - 1 || g.w[a] < 1 || g.w[a] > kMaxTaps) return "grid too small for ring tiles";
  const int64_t Mh = (int64_t)hdr.size();
  if ((int64_t)perm.size() != Mh || nph2 < 1 || nrings < 1 || (int64_t)nrings * nph2 != Mh)
    return "node set is not a product of rings";
  const int64_t ntiles = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];
  threads = usable_threads(threads, Mh, ntiles);
  // the nodes ring by ring
  std::vector<int64_t> rstart(nrings + 1, 0);
  for (int64_t j = 0; j < Mh; ++j) {
    if (perm[j] < 0 || perm[j] >= Mh) return "node index out of range";
    rstart[perm[j] / nph2 + 1]++;
  }
  for (int r = 0; r < nrings; ++r) rstart[r + 1] += rstart[r];
  std::vector<int> byring(Mh);
  {
    std::vector<int64_t> fill(rstart.begin(), rstart.end() - 1);
    for (int64_t j = 0; j < Mh; ++j) byring[fill[perm[j] / nph2]++] = (int)j;
  }
  auto visit = [&](int j, auto&& f) {
    int tx[kMaxTaps], ty[kMaxTaps], tz[kMaxTaps];
    const int nx = touched(hdr[j].x, g.nf[0], g.T[0], g.w[0], tx);
    const int ny = touched(hdr[j].y, g.nf[1], g.T[1], g.w[1], ty);
    const int nz = touched(hdr[j].z, g.nf[2], g.T[2], g.w[2], tz);
    for (int a0 = 0; a0 < nx; ++a0)
      for (int a1 = 0; a1 < ny; ++a1)
        for (int a2 = 0; a2 < nz; ++a2) {
          const int64_t tile = ((int64_t)tx[a0] * g.nt[1] + ty[a1]) * g.nt[2] + tz[a2];
          const int ex = start_code(hdr[j].x - tx[a0] * g.T[0], g.nf[0], g.T[0], true, bias);
          const int ey = start_code(hdr[j].y - ty[a1] * g.T[1], g.nf[1], g.T[1], true, bias);
          f(tile, ex, ey);
        }
  };
  // per tile, its entries in ring order (threads over contiguous rings)
  std::vector<std::vector<int64_t>> cnt(threads, std::vector<int64_t>(ntiles, 0));
  std::atomic<bool> bad{false};
  parallel_ranges(nrings, threads, [&](int64_t rb, int64_t re, int t) {
    std::vector<int64_t>& c = cnt[t];
    for (int64_t q = rstart[rb]; q < rstart[re]; ++q)
      visit(byring[q], [&](int64_t tile, int ex, int ey) {
        c[tile]++;
        if (!code_fits(ex) || !code_fits(ey)) bad = true;
      });
  });
  if (bad) return "ring list start out of range";
  std::vector<int64_t> tcnt;
  count_offsets(cnt, ntiles, tcnt);
  const int64_t nent = tcnt[ntiles];
  std::vector<int> enode(nent), ering(nent), ecode(nent);
  parallel_ranges(nrings, threads, [&](int64_t rb, int64_t re, int t) {
    std::vector<int64_t>& at = cnt[t];
    for (int64_t r = rb; r < re; ++r)
      for (int64_t q = rstart[r]; q < rstart[r + 1]; ++q) {
        const int j = byring[q];
        visit(j, [&](int64_t tile, int ex, int ey) {
          const int64_t k = at[tile]++;
          enode[k] = j;
          ering[k] = (int)r;
          ecode[k] = ex | (ey << 10);
        });
      }
  });
  // each tile's rings, padded to whole groups of four: sizes first (threads
  // over contiguous tiles), then the entries at their offsets
  const int kPad = 1023 | (1023 << 10);
  std::vector<int64_t> tsize(ntiles + 1, 0), tring(ntiles + 1, 0);
  parallel_ranges(ntiles, threads, [&](int64_t b, int64_t e, int) {
    for (int64_t t = b; t < e; ++t)
      for (int64_t i = tcnt[t]; i < tcnt[t + 1];) {
        int64_t k = i;
        while (k < tcnt[t + 1] && ering[k] == ering[i]) ++k;
        tsize[t + 1] += (k - i + 3) / 4 * 4;
        tring[t + 1]++;
        i = k;
      }
  });
  for (int64_t t = 0; t < ntiles; ++t) {
    tsize[t + 1] += tsize[t];
    tring[t + 1] += tring[t];
  }
  if (tsize[ntiles] + spare >= ((int64_t)1 << 31)) return "ring node lists too long";
  rnodes.assign(tsize[ntiles] + spare, Entry{0, kPad});  // the spare entries are read by the last prefetch
  rcost.assign(tring[ntiles], 0);
  rfirst.assign(tring[ntiles], 0);
  rcount = tring;
  parallel_ranges(ntiles, threads, [&](int64_t b, int64_t e, int) {
    for (int64_t t = b; t < e; ++t) {
      const int tz0 = (int)(t % g.nt[2]);
      int64_t at = tsize[t], ring = tring[t];
      for (int64_t i = tcnt[t]; i < tcnt[t + 1];) {
        int64_t k = i;
        while (k < tcnt[t + 1] && ering[k] == ering[i]) ++k;
        const int j0 = enode[i];
        const int64_t nb = at;
        for (int64_t q = i; q < k; ++q) rnodes[at++] = Entry{enode[q], ecode[q]};
        while ((at - nb) % 4) rnodes[at++] = Entry{j0, kPad};
        const int ez = start_code(hdr[j0].z - tz0 * g.T[2], g.nf[2], g.T[2], true, bias);
        if (!code_fits(ez)) bad = true;
        rnodes[at - 1].code |= (1 << end_bit) | ((ez & 1023) << z_bit);
        rfirst[ring] = (int)nb;
        rcost[ring] = (int)(at - nb);
        ++ring;
        i = k;
      }
    }
  });
  if (bad) return "ring list start out of range";
  return "";
}

struct Extent {  // the layout of an int2 line extent
  int first, span;
};

// The spreading writes kernel values only inside the nodes' footprints, so a
// line of the spreading grid along axis ax (0, or 1 when axis 0 is a unit
// axis) is zero outside the footprints that cross it.  Per line (index
// q_a nf[2] + q2 over the two other axes a, 2), ext gets the circular range
// {first, span} of positions first .. first + span (mod nf[ax]) that holds
// every footprint crossing the line: span -1 for a line none crosses, span
// nf[ax] - 1 for the whole line.  Each footprint is taken at its start's
// representative in (-nf/2, nf/2], and the range is the hull of those in
// unwrapped positions.
inline std::string line_extents(const Geometry& g, int ax, const std::vector<Start>& hdr, std::vector<Extent>& ext,
                                int threads = 1) {
  if (ax != 0 && ax != 1) return "line axis must be 0 or 1";
  for (int a = 0; a < 3; ++a)
    if (g.w[a] < 1 || g.w[a] > kMaxTaps || g.w[a] > g.nf[a]) return "width out of range";
  const int oa = ax == 0 ? 1 : 0;  // the other axis besides 2
  const int nf = g.nf[ax], w = g.w[ax];
  const int64_t nlines = (int64_t)g.nf[oa] * g.nf[2];
  const int64_t Mh = (int64_t)hdr.size();
  threads = usable_threads(threads, Mh, 2 * nlines);
  // per thread: the lowest and highest unwrapped position per line
  std::vector<std::vector<int>> lo(threads), hi(threads);
  parallel_ranges(Mh, threads, [&](int64_t j0, int64_t j1, int t) {
    std::vector<int>& L = lo[t];
    std::vector<int>& H = hi[t];
    L.assign(nlines, INT32_MAX);
    H.assign(nlines, INT32_MIN);
    for (int64_t j = j0; j < j1; ++j) {
      const int st[3] = {hdr[j].x, hdr[j].y, hdr[j].z};
      const int s = 2 * st[ax] > nf ? st[ax] - nf : st[ax];
      for (int da = 0; da < g.w[oa]; ++da) {
        const int qa = (st[oa] + da) % g.nf[oa];
        for (int d2 = 0; d2 < g.w[2]; ++d2) {
          const int64_t line = (int64_t)qa * g.nf[2] + (st[2] + d2) % g.nf[2];
          L[line] = std::min(L[line], s);
          H[line] = std::max(H[line], s + w - 1);
        }
      }
    }
  });
  ext.assign(nlines, Extent{0, -1});
  for (int64_t line = 0; line < nlines; ++line) {
    int l = INT32_MAX, h = INT32_MIN;
    for (int t = 0; t < threads; ++t) {
      if (lo[t].empty()) continue;
      l = std::min(l, lo[t][line]);
      h = std::max(h, hi[t][line]);
    }
    if (l > h) continue;
    if (h - l >= nf - 1)
      ext[line] = Extent{0, nf - 1};
    else
      ext[line] = Extent{((l % nf) + nf) % nf, h - l};
  }
  return "";
}

// The smallest circular range {first, span} (as in line_extents) that holds
// every set position of a line's bitmap (nw words over nf positions).
inline Extent bitmap_hull(const uint64_t* b, int nw, int nf) {
  // the largest run of unset positions between two set ones, or around the
  // end of the line, is the part left out
  int first = -1, prev = -1, gap = -1, gap_end = 0;
  for (int k = 0; k < nw; ++k)
    for (uint64_t v = b[k]; v; v &= v - 1) {
      const int q = k * 64 + __builtin_ctzll(v);
      if (first < 0)
        first = q;
      else if (q - prev - 1 > gap) {
        gap = q - prev - 1;
        gap_end = q;
      }
      prev = q;
    }
  if (first < 0) return Extent{0, -1};
  if (nf - 1 - prev + first >= gap) return Extent{first, prev - first};
  return Extent{gap_end, nf - 1 - gap};
}

// The interpolation by tiles reads the forward transform's spectrum only in
// the gather tiles that hold list entries: all their points on the grid and,
// when the spectrum is the Hermitian half (mirror), the conjugate mirror
// image (-q0, -q1, nf2 - q2) in place of each point with 2 q2 > nf2.  Per line
// of the spectrum along axis 0 (index q1 c2 + q2 over the lines kept, c2 =
// nf2 / 2 + 1 with mirror, nf2 without), ext gets the smallest circular range
// {first, span} (as in line_extents) that holds every position read on it;
// the transform's last pass need not store the rest.
inline std::string tile_read_extents(const Geometry& g, const std::vector<int64_t>& tcount, bool mirror,
                                     std::vector<Extent>& ext, int threads = 1) {
  const int nf0 = g.nf[0], nf1 = g.nf[1], nf2 = g.nf[2];
  const int64_t ntiles = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];
  if ((int64_t)tcount.size() != ntiles + 1) return "tile offsets do not match the tiles";
  const int c2 = mirror ? nf2 / 2 + 1 : nf2;
  const int nw = (nf0 + 63) / 64;
  const int64_t nlines = (int64_t)nf1 * c2;
  std::vector<uint64_t> bits((size_t)(nlines * nw), 0);
  // per tile column (t1, t2): the axis-0 positions of its listed tiles (X) and
  // their mirror images (Xm), then or-ed into the column's lines
  std::vector<uint64_t> X(nw), Xm(nw);
  for (int t1 = 0; t1 < g.nt[1]; ++t1)
    for (int t2 = 0; t2 < g.nt[2]; ++t2) {
      std::fill(X.begin(), X.end(), 0);
      std::fill(Xm.begin(), Xm.end(), 0);
      bool any = false;
      for (int t0 = 0; t0 < g.nt[0]; ++t0) {
        const int64_t tile = ((int64_t)t0 * g.nt[1] + t1) * g.nt[2] + t2;
        if (tcount[tile + 1] == tcount[tile]) continue;
        any = true;
        for (int x = t0 * g.T[0]; x < std::min((t0 + 1) * g.T[0], nf0); ++x) {
          const int xm = x ? nf0 - x : 0;
          X[x >> 6] |= 1ull << (x & 63);
          Xm[xm >> 6] |= 1ull << (xm & 63);
        }
      }
      if (!any) continue;
      for (int y = t1 * g.T[1]; y < std::min((t1 + 1) * g.T[1], nf1); ++y)
        for (int z = t2 * g.T[2]; z < std::min((t2 + 1) * g.T[2], nf2); ++z) {
          const bool m = mirror && 2 * z > nf2;
          const int64_t line = m ? (int64_t)(y ? nf1 - y : 0) * c2 + (nf2 - z) : (int64_t)y * c2 + z;
          uint64_t* b = &bits[(size_t)(line * nw)];
          const std::vector<uint64_t>& src = m ? Xm : X;
          for (int k = 0; k < nw; ++k) b[k] |= src[k];
        }
    }
  ext.assign(nlines, Extent{0, -1});
  const int nth = (int)std::max<int64_t>(1, std::min<int64_t>(threads, nlines / 4096 + 1));
  parallel_ranges(nlines, nth, [&](int64_t l0, int64_t l1, int) {
    for (int64_t line = l0; line < l1; ++line) ext[line] = bitmap_hull(&bits[(size_t)(line * nw)], nw, nf0);
  });
  return "";
}

}  // namespace lists
}  // namespace jgb
