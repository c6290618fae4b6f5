// Host-only checks of libsfm's geometry code (topology.cpp), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitized.py; no GPU and no HIP runtime calls.
//
// * TileGeometry: for every 6m up to the 256-row limit and every stored word size, the word map
//   of one block covers each entry of the upper triangle of the P16 x P16 block exactly once,
//   except the pairs at distance 8 inside a diagonal tile (the half-diagonal, stored twice); every
//   tile, the tail and the block start on a 128-byte line; padding words sit outside the block.
// * Topology: equal and uneven box splits; neighbour tables are symmetric across faces; strict
//   owners are -1 exactly on box planes and otherwise hold the node inside; non-strict owners are
//   the lowest-index box that holds the node; bad configurations are rejected with a message.
// Exit status 0 when every check passes; the first failure is printed.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <string>
#include <vector>

#include "sfm_internal.h"

namespace {

int failures = 0;

void check(bool ok, const std::string& what) {
  if (!ok && failures++ < 20) std::fprintf(stderr, "FAIL: %s\n", what.c_str());
}

void check_tiles(int p, int elem) {
  sfm::TileGeometry g;
  g.init(p, elem);
  std::vector<int32_t> rows, cols;
  g.word_map(rows, cols, elem);
  const std::string tag = "p=" + std::to_string(p) + " elem=" + std::to_string(elem);
  check((int64_t)rows.size() == g.words_per_block, tag + ": word count");
  check(g.P16 % 16 == 0 && g.P16 >= p && g.P16 < p + 16, tag + ": P16");
  check((g.words_per_block * elem) % sfm::kLineBytes == 0, tag + ": block length on a line");
  check(((int64_t)g.tail_off * elem) % sfm::kLineBytes == 0, tag + ": tail on a line");
  for (int q = 0; q < g.npairs; ++q) check(((int64_t)g.job_off[q] * elem) % sfm::kLineBytes == 0, tag + ": job on a line");
  std::vector<int> count((size_t)g.P16 * g.P16, 0);
  for (size_t w = 0; w < rows.size(); ++w) {
    const int r = rows[w], c = cols[w];
    if (r == g.P16 && c == g.P16) {
      check(w >= (size_t)g.tail_off, tag + ": padding before the tail");
      continue;
    }
    if (r < 0 || c < 0 || r >= g.P16 || c >= g.P16) {
      check(false, tag + ": word outside the block");
      continue;
    }
    const int lo = std::min(r, c), hi = std::max(r, c);
    ++count[(size_t)lo * g.P16 + hi];
  }
  for (int r = 0; r < g.P16; ++r)
    for (int c = r; c < g.P16; ++c) {
      const bool half = (r / 16 == c / 16) && (c - r == 8);
      check(count[(size_t)r * g.P16 + c] == (half ? 2 : 1),
            tag + ": entry (" + std::to_string(r) + "," + std::to_string(c) + ") stored " +
                std::to_string(count[(size_t)r * g.P16 + c]) + " times");
    }
}

sfm_config config(int nx, int ny, int nz, int sx, int sy, int sz, int m, int k) {
  sfm_config c{};
  c.ncell[0] = nx; c.ncell[1] = ny; c.ncell[2] = nz;
  c.sub_cells[0] = sx; c.sub_cells[1] = sy; c.sub_cells[2] = sz;
  c.h = 10.0;
  c.m = m;
  c.k = k;
  c.precision = SFM_PREC_FP32;
  return c;
}

void check_topology(const sfm::Topology& t, const std::string& tag) {
  for (int s = 0; s < t.S; ++s)
    for (int f = 0; f < 6; ++f) {
      const int nb = t.nbr[(size_t)s * 6 + f];
      if (nb >= 0) {
        check(nb < t.S && t.nbr[(size_t)nb * 6 + (f ^ 1)] == s, tag + ": neighbour table not symmetric");
        int o[3], on[3], w[3], wn[3];
        t.origin(s, o);
        t.origin(nb, on);
        t.cells(s, w);
        t.cells(nb, wn);
        const int d = f / 2;
        check((f & 1) ? on[d] == o[d] + w[d] : on[d] + wn[d] == o[d], tag + ": neighbour does not touch the face");
        for (int e = 0; e < 3; ++e)
          if (e != d) check(on[e] == o[e] && wn[e] == w[e], tag + ": neighbour does not share the whole face");
      }
    }
  for (int l = 0; l <= t.ncell[2]; ++l)
    for (int j = 0; j <= t.ncell[1]; ++j)
      for (int i = 0; i <= t.ncell[0]; ++i) {
        const int g[3] = {i, j, l};
        bool plane = false;
        for (int d = 0; d < 3; ++d)
          for (int v : t.cut[d]) plane = plane || g[d] == v;
        const int ss = t.owner(i, j, l, true);
        check((ss < 0) == plane, tag + ": strict owner on a plane");
        auto holds = [&](int s, bool strict) {
          int o[3], w[3];
          t.origin(s, o);
          t.cells(s, w);
          for (int d = 0; d < 3; ++d) {
            const int r = g[d] - o[d];
            if (strict ? (r <= 0 || r >= w[d]) : (r < 0 || r > w[d])) return false;
          }
          return true;
        };
        if (ss >= 0) check(holds(ss, true), tag + ": strict owner does not hold the node");
        const int sn = t.owner(i, j, l, false);
        int lowest = -1;
        for (int s = 0; s < t.S && lowest < 0; ++s)
          if (holds(s, false)) lowest = s;
        check(sn == lowest, tag + ": owner is not the lowest-index box holding the node");
      }
  check(t.owner(-1, 0, 0, false) == -1 && t.owner(0, 0, t.ncell[2] + 1, true) == -1, tag + ": outside the grid");
}

}  // namespace

int main() {
  for (int m = 1; 6 * m <= 256; ++m)
    for (int elem : {2, 4, 8}) check_tiles(6 * m, elem);

  {
    sfm::Topology t;
    check(t.init(config(32, 32, 32, 16, 16, 16, 4, 8)).empty(), "equal boxes accepted");
    check(t.S == 8 && t.p == 24 && t.m1 == 2 && t.m2 == 2, "equal boxes: sizes");
    check_topology(t, "32^3 / 16^3");
  }
  {
    sfm::Topology t;
    check(t.init(config(30, 20, 24, 10, 10, 12, 3, 5)).empty(), "ragged accepted");
    check(t.m1 == 3 && t.m2 == 1, "m = 3 factorisation");
    check_topology(t, "ragged");
  }
  std::mt19937 rng(7);
  for (int trial = 0; trial < 40; ++trial) {
    int32_t nbox[3], cells[32];
    int used = 0;
    int ncell[3];
    for (int d = 0; d < 3; ++d) {
      nbox[d] = 1 + (int)(rng() % 4);
      ncell[d] = 0;
      for (int b = 0; b < nbox[d]; ++b) {
        cells[used + b] = 4 + (int)(rng() % 9);
        ncell[d] += cells[used + b];
      }
      used += nbox[d];
    }
    sfm::Topology t;
    const std::string err = t.init(config(ncell[0], ncell[1], ncell[2], 2, 2, 2, 2, 2), nbox, cells);
    check(err.empty(), "uneven boxes accepted: " + err);
    if (err.empty()) check_topology(t, "uneven trial " + std::to_string(trial));
  }
  {
    sfm::Topology t;
    check(!t.init(config(32, 32, 30, 16, 16, 16, 4, 8)).empty(), "ncell not a multiple of sub_cells rejected");
    check(!t.init(config(32, 32, 32, 16, 16, 1, 4, 8)).empty(), "one-cell boxes rejected");
    check(!t.init(config(32, 32, 32, 16, 16, 16, 4, 1)).empty(), "k = 1 rejected");
    check(!t.init(config(8, 8, 8, 4, 4, 4, 25, 2)).empty(), "too many patches rejected");
    check(!t.init(config(32, 32, 32, 16, 16, 16, 4, 300)).empty(), "ROM larger than the subdomain rejected");
    check(!t.init(config(32, 32, 32, 16, 16, 16, 50, 2)).empty(), "6m above 256 rejected");
    const int32_t nb[3] = {2, 1, 1}, bad[4] = {12, 17, 28, 28};
    check(!t.init(config(28, 28, 28, 2, 2, 2, 1, 2), nb, bad).empty(), "box sizes not adding up rejected");
  }
  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("geometry checks passed\n");
  return 0;
}
