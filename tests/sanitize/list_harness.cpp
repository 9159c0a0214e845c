// CPU harness for the host list construction (paper_1311_4120_amd/csrc/lists.h),
// built with the address and undefined-behaviour sanitizers by
// tests/test_list_sanitizers.py.  It builds the gather and ring lists for
// product node sets r_a x theta_b x phi_l on oversampled grids up to 1024 points
// per axis (N = 512, where the 10-bit start codes are tightest) and checks every
// entry against a brute-force enumeration of the (node, tile) pairs whose
// footprints meet.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "lists.h"
#include "radial.h"

using namespace jgb::lists;

static int failures = 0;
#define CHECK(cond, ...)                         \
  do {                                           \
    if (!(cond)) {                               \
      if (failures++ < 20) {                     \
        fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
        fprintf(stderr, __VA_ARGS__);            \
        fprintf(stderr, "\n");                   \
      }                                          \
    }                                            \
  } while (0)

struct Case {
  const char* name;
  int dim;          // 3, or 2 (a0 a unit axis)
  int nf[3];
  int w;
  int n_r, n_theta, n_phi;
  int T[3];         // tile extent
  bool ring;        // also build the ring lists (3D)
};

static int mod(int a, int n) { return ((a % n) + n) % n; }

// first taps of the half node set (l < n_phi / 2), natural order
static std::vector<Start> node_starts(const Case& c, std::vector<int>& natural) {
  std::vector<Start> h;
  const double kmax = 0.999;  // fraction of the alias-free radius nf / 2 cells
  for (int a = 0; a < c.n_r; ++a)
    for (int b = 0; b < (c.dim == 3 ? c.n_theta : 1); ++b)
      for (int l = 0; l < c.n_phi / 2; ++l) {
        const double r = kmax * (a + 0.5) / c.n_r;
        const double th = M_PI * (b + 0.5) / c.n_theta;
        const double ph = 2 * M_PI * l / c.n_phi;
        double k[3];
        if (c.dim == 3) {
          k[0] = r * std::sin(th) * std::cos(ph);
          k[1] = r * std::sin(th) * std::sin(ph);
          k[2] = r * std::cos(th);
        } else {
          k[0] = 0.0;
          k[1] = r * std::cos(ph);
          k[2] = r * std::sin(ph);
        }
        Start s{0, 0, 0, 0};
        int* out[3] = {&s.x, &s.y, &s.z};
        for (int ax = 0; ax < 3; ++ax) {
          const int w = (c.nf[ax] == 1) ? 1 : c.w;
          const double pos = k[ax] * c.nf[ax] / 2;  // fine-grid position in cells
          *out[ax] = mod((int)std::ceil(pos - 0.5 * w), c.nf[ax]);
        }
        natural.push_back((int)h.size());
        h.push_back(s);
      }
  return h;
}

static bool touches(int start, int nf, int w, int tile, int T) {
  for (int t = 0; t < w; ++t)
    if (((start + t) % nf) / T == tile) return true;
  return false;
}

// relative start of node start s against a tile origin o, as a code decodes it
static int decoded(int code, bool nowrap, int bias) { return nowrap ? code - bias : code; }

static void run(const Case& c, bool nowrap_gather) {
  std::vector<int> natural;
  std::vector<Start> hdr = node_starts(c, natural);
  const int64_t Mh = (int64_t)hdr.size();
  Geometry g{};
  for (int a = 0; a < 3; ++a) {
    g.nf[a] = c.nf[a];
    g.T[a] = c.T[a];
    g.nt[a] = (c.nf[a] + c.T[a] - 1) / c.T[a];
    g.w[a] = (c.nf[a] == 1) ? 1 : c.w;
  }
  const int bias = 512;
  bool nowrap = nowrap_gather;
  for (int a = 0; a < 3; ++a) nowrap &= g.nf[a] >= g.T[a] + g.w[a] - 1;
  // a permutation of the nodes, as the plan's bin sort produces one
  std::vector<int> perm(Mh);
  for (int64_t j = 0; j < Mh; ++j) perm[j] = (int)((j * 7919 + 13) % Mh);
  std::set<int> seen(perm.begin(), perm.end());
  if ((int64_t)seen.size() != Mh) {  // 7919 shares a factor with Mh: use the identity
    for (int64_t j = 0; j < Mh; ++j) perm[j] = (int)j;
  }
  std::vector<Start> sorted(Mh);
  for (int64_t j = 0; j < Mh; ++j) sorted[j] = hdr[perm[j]];

  // brute force: every (node, tile) pair whose footprints meet
  std::map<int64_t, std::vector<int>> pairs;  // tile -> nodes (sorted index)
  for (int64_t j = 0; j < Mh; ++j) {
    int tl[3][kMaxTaps], nt[3];
    const int st[3] = {sorted[j].x, sorted[j].y, sorted[j].z};
    for (int a = 0; a < 3; ++a) nt[a] = touched(st[a], g.nf[a], g.T[a], g.w[a], tl[a]);
    for (int i0 = 0; i0 < nt[0]; ++i0)
      for (int i1 = 0; i1 < nt[1]; ++i1)
        for (int i2 = 0; i2 < nt[2]; ++i2) {
          const int64_t t = ((int64_t)tl[0][i0] * g.nt[1] + tl[1][i1]) * g.nt[2] + tl[2][i2];
          pairs[t].push_back((int)j);
        }
  }

  // line extents along the inverse transform's first axis: every footprint
  // cell lies in its line's range, lines no footprint crosses are empty, and
  // the threaded build equals the serial one
  {
    const int ax = c.dim == 3 ? 0 : 1, oa = ax == 0 ? 1 : 0;
    std::vector<Extent> ext, ext1;
    std::string e8 = line_extents(g, ax, sorted, ext, 8);
    CHECK(e8.empty(), "%s: line_extents: %s", c.name, e8.c_str());
    CHECK(line_extents(g, ax, sorted, ext1, 1).empty(), "%s: serial line extents", c.name);
    const int64_t nlines = (int64_t)g.nf[oa] * g.nf[2];
    CHECK((int64_t)ext.size() == nlines && ext1.size() == ext.size(), "%s: line extent count", c.name);
    bool same = ext.size() == ext1.size();
    for (size_t i = 0; same && i < ext.size(); ++i) same = ext[i].first == ext1[i].first && ext[i].span == ext1[i].span;
    CHECK(same, "%s: threaded line extents differ from the serial build", c.name);
    std::vector<char> crossed(nlines, 0);
    int64_t outside = 0;
    for (int64_t j = 0; j < Mh; ++j) {
      const int st[3] = {sorted[j].x, sorted[j].y, sorted[j].z};
      for (int da = 0; da < g.w[oa]; ++da)
        for (int d2 = 0; d2 < g.w[2]; ++d2) {
          const int64_t line = (int64_t)((st[oa] + da) % g.nf[oa]) * g.nf[2] + (st[2] + d2) % g.nf[2];
          crossed[line] = 1;
          const Extent e = ext[line];
          for (int dx = 0; dx < g.w[ax]; ++dx) {
            const int q = (st[ax] + dx) % g.nf[ax];
            if (e.span < 0 || mod(q - e.first, g.nf[ax]) > e.span) ++outside;
          }
        }
    }
    CHECK(outside == 0, "%s: %lld footprint cells outside their line's extent", c.name, (long long)outside);
    int64_t covered = 0;
    for (int64_t line = 0; line < nlines; ++line) {
      const Extent e = ext[line];
      if (!crossed[line]) {
        CHECK(e.span == -1, "%s: line %lld has an extent but no footprint crosses it", c.name, (long long)line);
        continue;
      }
      CHECK(e.first >= 0 && e.first < g.nf[ax] && e.span >= 0 && e.span < g.nf[ax], "%s: extent range", c.name);
      covered += e.span + 1;
    }
    // the half node set of a ball fills about 30% of the large grids: the
    // extents must not degenerate to whole lines there
    if (g.nf[ax] >= 512)
      CHECK(covered < (int64_t)(0.45 * nlines * g.nf[ax]), "%s: extents cover %.2f of the grid", c.name,
            (double)covered / ((double)nlines * g.nf[ax]));
  }

  // gather lists
  std::vector<int64_t> tcount;
  std::vector<Entry> list;
  std::vector<int> nstart, npos;
  std::string err = gather_lists(g, nowrap, bias, sorted, tcount, list, true, nstart, npos, 8);
  CHECK(err.empty(), "%s: gather_lists: %s", c.name, err.c_str());
  if (!err.empty()) return;
  {
    // the threaded build equals the serial one
    std::vector<int64_t> tc1;
    std::vector<Entry> l1;
    std::vector<int> ns1, np1;
    CHECK(gather_lists(g, nowrap, bias, sorted, tc1, l1, true, ns1, np1, 1).empty(), "%s: serial build", c.name);
    bool same = tc1 == tcount && ns1 == nstart && np1 == npos && l1.size() == list.size();
    for (size_t i = 0; same && i < l1.size(); ++i) same = l1[i].node == list[i].node && l1[i].code == list[i].code;
    CHECK(same, "%s: threaded gather lists differ from the serial build", c.name);
  }
  const int64_t ntiles = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];

  // the spectrum's reach per line for the interpolation by tiles: every point
  // it reads (all points of the listed tiles, mirrored past nf2 / 2 for the
  // Hermitian half) lies in its line's range, both ends of a range are points
  // it reads, lines it reads nothing of are empty, and the threaded build
  // equals the serial one
  if (c.dim == 3 && !c.ring)
    for (int mirror = 0; mirror < 2; ++mirror) {
      std::vector<Extent> fx, fx1;
      CHECK(tile_read_extents(g, tcount, mirror, fx, 8).empty(), "%s: tile_read_extents", c.name);
      CHECK(tile_read_extents(g, tcount, mirror, fx1, 1).empty(), "%s: serial tile read extents", c.name);
      bool same = fx.size() == fx1.size();
      for (size_t i = 0; same && i < fx.size(); ++i) same = fx[i].first == fx1[i].first && fx[i].span == fx1[i].span;
      CHECK(same, "%s: threaded tile read extents differ from the serial build", c.name);
      const int nf0 = g.nf[0], nf1 = g.nf[1], nf2 = g.nf[2];
      const int c2 = mirror ? nf2 / 2 + 1 : nf2;
      const int64_t nl = (int64_t)nf1 * c2;
      CHECK((int64_t)fx.size() == nl, "%s: one reach per spectrum line", c.name);
      if ((int64_t)fx.size() != nl) continue;
      std::vector<char> any(nl, 0), at_first(nl, 0), at_last(nl, 0);
      int64_t outside = 0;
      for (int64_t t = 0; t < ntiles; ++t) {
        if (tcount[t + 1] == tcount[t]) continue;
        const int t0 = (int)(t / ((int64_t)g.nt[1] * g.nt[2])), t1 = (int)((t / g.nt[2]) % g.nt[1]),
                  t2 = (int)(t % g.nt[2]);
        for (int x = t0 * g.T[0]; x < std::min((t0 + 1) * g.T[0], nf0); ++x)
          for (int y = t1 * g.T[1]; y < std::min((t1 + 1) * g.T[1], nf1); ++y)
            for (int z = t2 * g.T[2]; z < std::min((t2 + 1) * g.T[2], nf2); ++z) {
              const bool m = mirror && 2 * z > nf2;
              const int qx = m ? mod(-x, nf0) : x, qy = m ? mod(-y, nf1) : y, qz = m ? nf2 - z : z;
              const int64_t line = (int64_t)qy * c2 + qz;
              const Extent e = fx[line];
              any[line] = 1;
              if (e.span < 0 || mod(qx - e.first, nf0) > e.span) ++outside;
              if (qx == e.first) at_first[line] = 1;
              if (qx == mod(e.first + e.span, nf0)) at_last[line] = 1;
            }
      }
      CHECK(outside == 0, "%s: %lld points read outside their line's reach (mirror %d)", c.name, (long long)outside,
            mirror);
      int64_t loose = 0, stray = 0;
      for (int64_t line = 0; line < nl; ++line) {
        if (!any[line]) stray += fx[line].span != -1;
        else loose += !(at_first[line] && at_last[line]);
      }
      CHECK(stray == 0, "%s: %lld unread lines with a reach", c.name, (long long)stray);
      CHECK(loose == 0, "%s: %lld reaches not ending at read points", c.name, (long long)loose);
    }
  int64_t total = 0;
  for (int64_t t = 0; t < ntiles; ++t) {
    const int t0 = (int)(t / ((int64_t)g.nt[1] * g.nt[2])), t1 = (int)((t / g.nt[2]) % g.nt[1]), t2 = (int)(t % g.nt[2]);
    const int org[3] = {t0 * g.T[0], t1 * g.T[1], t2 * g.T[2]};
    const std::vector<int>& want = pairs.count(t) ? pairs[t] : std::vector<int>();
    CHECK((int64_t)want.size() == tcount[t + 1] - tcount[t], "%s: tile %lld lists %lld nodes, %zu touch it", c.name,
          (long long)t, (long long)(tcount[t + 1] - tcount[t]), want.size());
    for (int64_t e = tcount[t]; e < tcount[t + 1]; ++e) {
      const Entry en = list[e];
      CHECK(en.node >= 0 && en.node < Mh, "%s: node index", c.name);
      if (en.node < 0 || en.node >= Mh) continue;
      const int codes[3] = {en.code & 1023, (en.code >> 10) & 1023, (en.code >> 20) & 1023};
      const int st[3] = {sorted[en.node].x, sorted[en.node].y, sorted[en.node].z};
      for (int a = 0; a < 3; ++a) {
        const int rel = decoded(codes[a], nowrap, bias);
        CHECK(mod(rel - (st[a] - org[a]), g.nf[a]) == 0, "%s: axis %d start code %d of node %d in tile %lld", c.name,
              a, codes[a], en.node, (long long)t);
        if (nowrap) CHECK(rel >= -(g.w[a] - 1) && rel <= g.T[a] - 1, "%s: nowrap code range", c.name);
        CHECK(touches(st[a], g.nf[a], g.w[a], org[a] / g.T[a], g.T[a]), "%s: listed node misses the tile", c.name);
      }
      if (e > tcount[t]) CHECK(list[e - 1].node < en.node, "%s: entries of a tile in node order", c.name);
    }
    total += tcount[t + 1] - tcount[t];
  }
  CHECK((int64_t)list.size() == total + 1, "%s: one spare entry", c.name);
  // node-major index
  CHECK((int64_t)nstart.size() == Mh + 1 && nstart[Mh] == (int)npos.size() && (int64_t)npos.size() == total,
        "%s: node-major index sizes", c.name);
  for (int64_t j = 0; j < Mh; ++j)
    for (int q = nstart[j]; q < nstart[j + 1]; ++q)
      CHECK(npos[q] >= 0 && npos[q] < total && list[npos[q]].node == (int)j, "%s: node-major position", c.name);

  if (!c.ring) return;
  // ring lists (natural index = (a n_theta + b) nph2 + l)
  const int nph2 = c.n_phi / 2;
  std::vector<Entry> rnodes;
  std::vector<int64_t> rcount;
  std::vector<int> rcost, rfirst;
  const int end_bit = 20, z_bit = 21, spare = 32;
  err = ring_lists(g, bias, nph2, c.n_r * c.n_theta, perm, sorted, end_bit, z_bit, spare, rnodes, rcount, rcost, rfirst,
                   8);
  CHECK(err.empty(), "%s: ring_lists: %s", c.name, err.c_str());
  if (!err.empty()) return;
  {
    std::vector<Entry> r1;
    std::vector<int64_t> rc1;
    std::vector<int> cost1, first1;
    CHECK(ring_lists(g, bias, nph2, c.n_r * c.n_theta, perm, sorted, end_bit, z_bit, spare, r1, rc1, cost1, first1, 1)
              .empty(),
          "%s: serial ring build", c.name);
    bool same = rc1 == rcount && cost1 == rcost && first1 == rfirst && r1.size() == rnodes.size();
    for (size_t i = 0; same && i < r1.size(); ++i) same = r1[i].node == rnodes[i].node && r1[i].code == rnodes[i].code;
    CHECK(same, "%s: threaded ring lists differ from the serial build", c.name);
  }
  int64_t listed = 0;
  for (int64_t t = 0; t < ntiles; ++t) {
    const int t0 = (int)(t / ((int64_t)g.nt[1] * g.nt[2])), t1 = (int)((t / g.nt[2]) % g.nt[1]), t2 = (int)(t % g.nt[2]);
    const int org[3] = {t0 * g.T[0], t1 * g.T[1], t2 * g.T[2]};
    std::multiset<int> want;
    if (pairs.count(t)) want.insert(pairs[t].begin(), pairs[t].end());
    std::multiset<int> got;
    std::set<int> rings_seen;
    for (int64_t r = rcount[t]; r < rcount[t + 1]; ++r) {
      CHECK(rcost[r] > 0 && rcost[r] % 4 == 0, "%s: ring padded to groups of four", c.name);
      const int ring = perm[rnodes[rfirst[r]].node] / nph2;
      CHECK(!rings_seen.count(ring), "%s: a ring listed twice in a tile", c.name);
      rings_seen.insert(ring);
      for (int q = 0; q < rcost[r]; ++q) {
        const Entry en = rnodes[rfirst[r] + q];
        const bool last = q == rcost[r] - 1;
        CHECK(((en.code >> end_bit) & 1) == (last ? 1 : 0), "%s: ring end flag", c.name);
        CHECK(perm[en.node] / nph2 == ring, "%s: entry of another ring", c.name);
        const int cx = en.code & 1023, cy = (en.code >> 10) & 1023;
        if (cx == 1023 && cy == 1023) continue;  // padding
        got.insert(en.node);
        const int st[2] = {sorted[en.node].x, sorted[en.node].y};
        CHECK(mod(cx - bias - (st[0] - org[0]), g.nf[0]) == 0 && mod(cy - bias - (st[1] - org[1]), g.nf[1]) == 0,
              "%s: ring entry start codes", c.name);
        if (last) {
          const int cz = (en.code >> z_bit) & 1023;
          CHECK(mod(cz - bias - (sorted[en.node].z - org[2]), g.nf[2]) == 0, "%s: ring a2 start code", c.name);
        }
      }
      const Entry lastent = rnodes[rfirst[r] + rcost[r] - 1];
      const int cz = (lastent.code >> z_bit) & 1023;
      CHECK(mod(cz - bias - (sorted[lastent.node].z - org[2]), g.nf[2]) == 0, "%s: ring a2 start code", c.name);
      listed += rcost[r];
    }
    CHECK(got == want, "%s: tile %lld: ring lists hold %zu nodes, %zu touch it", c.name, (long long)t, got.size(),
          want.size());
  }
  CHECK((int64_t)rnodes.size() == listed + spare, "%s: spare ring entries", c.name);
}

int main(int argc, char** argv) {
  if (argc == 4 && std::string(argv[1]) == "radial") {
    // the plan's generalized Gaussian radial rule of bandwidth c with n nodes
    std::vector<double> x, w;
    const std::string err = jgb::radial::prolate_rule(atof(argv[2]), atoi(argv[3]), x, w);
    if (!err.empty()) {
      fprintf(stderr, "%s\n", err.c_str());
      return 1;
    }
    for (size_t i = 0; i < x.size(); ++i) printf("%.17g %.17g\n", x[i], w[i]);
    return 0;
  }
  {
    // the circular hull of a line's read positions: empty, one point, all,
    // a range around the end of the line, the largest of two gaps left out
    // (ties to the gap around the end), across 64-bit words
    auto hull = [](std::initializer_list<int> set, int nf) {
      std::vector<uint64_t> b((nf + 63) / 64, 0);
      for (int q : set) b[q >> 6] |= 1ull << (q & 63);
      return bitmap_hull(b.data(), (int)b.size(), nf);
    };
    auto is = [](Extent e, int first, int span) { return e.first == first && e.span == span; };
    CHECK(is(hull({}, 100), 0, -1), "hull: empty line");
    CHECK(is(hull({37}, 100), 37, 0), "hull: one point");
    std::initializer_list<int> all = {0, 1, 2, 3, 4, 5, 6, 7};
    CHECK(is(hull(all, 8), 0, 7), "hull: whole line");
    CHECK(is(hull({0, 1, 2, 97, 98, 99}, 100), 97, 5), "hull: range around the end");
    CHECK(is(hull({10, 20, 90}, 100), 90, 30), "hull: wrap gap smaller than the inner one");
    CHECK(is(hull({10, 60, 70}, 100), 60, 50), "hull: inner gap (49) larger than the one around the end (39)");
    CHECK(is(hull({10, 30, 40}, 100), 10, 30), "hull: gap around the end largest");
    CHECK(is(hull({0, 50}, 100), 0, 50), "hull: equal gaps keep the first range");
    CHECK(is(hull({5, 63, 64, 200}, 256), 200, 120), "hull: across words, the 64..200 gap left out");
    CHECK(is(hull({1, 255}, 256), 255, 2), "hull: two points straddling the end");
  }
  const Case cases[] = {
      // N = 512: the oversampled side 1024, the largest the 10-bit codes allow
      {"3d_512_w12", 3, {1024, 1024, 1024}, 12, 24, 16, 32, {8, 8, 8}, false},
      {"3d_512_w16_rings", 3, {1024, 1024, 1024}, 16, 24, 16, 32, {16, 8, 16}, true},
      {"3d_ragged_w12_rings", 3, {40, 48, 60}, 12, 10, 8, 12, {16, 8, 16}, true},
      {"3d_small_wrap_w12", 3, {16, 16, 24}, 12, 6, 4, 8, {8, 8, 8}, false},
      {"2d_512_w12", 2, {1, 1024, 1024}, 12, 64, 1, 96, {1, 64, 8}, false},
  };
  for (const Case& c : cases) {
    run(c, true);
    if (c.dim == 3 && !c.ring) run(c, false);  // modulo-nf start codes (what small grids store)
    fprintf(stderr, "case %s done\n", c.name);
  }
  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("ok\n");
  return 0;
}
