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
//
// Starts are the nodes' first taps wrapped into [0, nf).  A tile-relative
// start is stored, when every axis has nf >= T + w - 1, as its one
// representative in [-(w - 1), T - 1] plus a bias ("nowrap"); otherwise modulo
// nf.  Either way it must fit in 10 bits: the functions return an error
// message instead of a list that would not.
#pragma once

#include <cstdint>
#include <string>
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

// The three-axis gather's lists (see above): tcount gets ntiles + 1 offsets
// into list; list gets the entries tile by tile, nodes in their order, then
// one spare entry.  With node_major, nstart (Mh + 1 offsets) and npos (list
// positions) index each node's entries in the order of its tiles.
inline std::string gather_lists(const Geometry& g, bool nowrap, int bias, const std::vector<Start>& hdr,
                                std::vector<int64_t>& tcount, std::vector<Entry>& list, bool node_major,
                                std::vector<int>& nstart, std::vector<int>& npos) {
  for (int a = 0; a < 3; ++a)
    if (g.w[a] < 1 || g.w[a] > kMaxTaps || g.w[a] > g.nf[a]) return "width out of range";
  const int64_t Mh = (int64_t)hdr.size();
  const int64_t ntiles = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];
  tcount.assign(ntiles + 1, 0);
  int tx[kMaxTaps], ty[kMaxTaps], tz[kMaxTaps];
  for (int64_t j = 0; j < Mh; ++j) {
    const int nx = touched(hdr[j].x, g.nf[0], g.T[0], g.w[0], tx);
    const int ny = touched(hdr[j].y, g.nf[1], g.T[1], g.w[1], ty);
    const int nz = touched(hdr[j].z, g.nf[2], g.T[2], g.w[2], tz);
    for (int a0 = 0; a0 < nx; ++a0)
      for (int a1 = 0; a1 < ny; ++a1)
        for (int a2 = 0; a2 < nz; ++a2) tcount[((int64_t)tx[a0] * g.nt[1] + ty[a1]) * g.nt[2] + tz[a2] + 1]++;
  }
  for (int64_t t = 0; t < ntiles; ++t) tcount[t + 1] += tcount[t];
  const int64_t nlist = tcount[ntiles];
  // the kernels address the list by 32-bit byte offsets (8 bytes per entry)
  // and the node-major index by 32-bit positions
  if ((nlist + 1) * 8 >= ((int64_t)1 << 32)) return "gather lists too long";
  list.assign(nlist + 1, Entry{0, 0});
  nstart.clear();
  npos.clear();
  if (node_major) {
    nstart.assign(Mh + 1, 0);
    npos.reserve(nlist);
  }
  std::vector<int64_t> fill(tcount.begin(), tcount.end() - 1);
  for (int64_t j = 0; j < Mh; ++j) {
    if (node_major) nstart[j] = (int)npos.size();
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
          if (!code_fits(ex) || !code_fits(ey) || !code_fits(ez)) return "gather list start out of range";
          if (node_major) npos.push_back((int)fill[tile]);
          list[fill[tile]++] = Entry{(int)j, ex | (ey << 10) | (ez << 20)};
        }
  }
  if (node_major) nstart[Mh] = (int)npos.size();
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
                              std::vector<int>& rfirst) {
  for (int a = 0; a < 3; ++a)
    if (g.nf[a] < g.T[a] + g.w[a] - 1 || g.w[a] < 1 || g.w[a] > kMaxTaps) return "grid too small for ring tiles";
  const int64_t Mh = (int64_t)hdr.size();
  if ((int64_t)perm.size() != Mh || nph2 < 1 || nrings < 1 || (int64_t)nrings * nph2 != Mh)
    return "node set is not a product of rings";
  const int64_t ntiles = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];
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
  std::vector<int64_t> tcnt(ntiles + 1, 0);
  int tx[kMaxTaps], ty[kMaxTaps], tz[kMaxTaps];
  for (int64_t j = 0; j < Mh; ++j) {
    const int nx = touched(hdr[j].x, g.nf[0], g.T[0], g.w[0], tx);
    const int ny = touched(hdr[j].y, g.nf[1], g.T[1], g.w[1], ty);
    const int nz = touched(hdr[j].z, g.nf[2], g.T[2], g.w[2], tz);
    for (int a0 = 0; a0 < nx; ++a0)
      for (int a1 = 0; a1 < ny; ++a1)
        for (int a2 = 0; a2 < nz; ++a2) tcnt[((int64_t)tx[a0] * g.nt[1] + ty[a1]) * g.nt[2] + tz[a2] + 1]++;
  }
  for (int64_t t = 0; t < ntiles; ++t) tcnt[t + 1] += tcnt[t];
  const int64_t nent = tcnt[ntiles];
  // per tile, its entries in ring order
  std::vector<int> enode(nent), ering(nent), ecode(nent);
  {
    std::vector<int64_t> fill(tcnt.begin(), tcnt.end() - 1);
    for (int r = 0; r < nrings; ++r)
      for (int64_t q = rstart[r]; q < rstart[r + 1]; ++q) {
        const int j = byring[q];
        const int nx = touched(hdr[j].x, g.nf[0], g.T[0], g.w[0], tx);
        const int ny = touched(hdr[j].y, g.nf[1], g.T[1], g.w[1], ty);
        const int nz = touched(hdr[j].z, g.nf[2], g.T[2], g.w[2], tz);
        for (int a0 = 0; a0 < nx; ++a0)
          for (int a1 = 0; a1 < ny; ++a1)
            for (int a2 = 0; a2 < nz; ++a2) {
              const int64_t tile = ((int64_t)tx[a0] * g.nt[1] + ty[a1]) * g.nt[2] + tz[a2];
              const int ex = start_code(hdr[j].x - tx[a0] * g.T[0], g.nf[0], g.T[0], true, bias);
              const int ey = start_code(hdr[j].y - ty[a1] * g.T[1], g.nf[1], g.T[1], true, bias);
              if (!code_fits(ex) || !code_fits(ey)) return "ring list start out of range";
              const int64_t at = fill[tile]++;
              enode[at] = j;
              ering[at] = r;
              ecode[at] = ex | (ey << 10);
            }
      }
  }
  const int kPad = 1023 | (1023 << 10);
  rnodes.clear();
  rnodes.reserve(nent + nent / 4 + spare);
  rcount.assign(ntiles + 1, 0);
  rcost.clear();
  rfirst.clear();
  for (int64_t t = 0; t < ntiles; ++t) {
    const int tz0 = (int)(t % g.nt[2]);
    for (int64_t i = tcnt[t]; i < tcnt[t + 1];) {
      int64_t e = i;
      while (e < tcnt[t + 1] && ering[e] == ering[i]) ++e;
      const int j0 = enode[i];
      const int64_t nb = (int64_t)rnodes.size();
      for (int64_t q = i; q < e; ++q) rnodes.push_back(Entry{enode[q], ecode[q]});
      while ((rnodes.size() - nb) % 4) rnodes.push_back(Entry{j0, kPad});
      const int ez = start_code(hdr[j0].z - tz0 * g.T[2], g.nf[2], g.T[2], true, bias);
      if (!code_fits(ez)) return "ring list start out of range";
      rnodes.back().code |= (1 << end_bit) | (ez << z_bit);
      if ((int64_t)rnodes.size() + spare >= ((int64_t)1 << 31)) return "ring node lists too long";
      rfirst.push_back((int)nb);
      rcost.push_back((int)(rnodes.size() - nb));
      i = e;
    }
    rcount[t + 1] = (int64_t)rcost.size();
  }
  for (int i = 0; i < spare; ++i) rnodes.push_back(Entry{0, kPad});  // read by the last prefetch
  return "";
}

}  // namespace lists
}  // namespace jgb
