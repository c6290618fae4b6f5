// Host-side geometry: subdomain decomposition, faces, and the tile layout of the
// coefficient stream.
//
// Decomposition (Introduction; Stage 1 section): the box of ncell cells is split into a
// tensor product of box subdomains (per axis, equal boxes of sub_cells cells or a list of box
// sizes) that share their interface nodes; neighbours across a face share the whole face.
// Faces are ordered x-, x+, y-, y+, z-, z+; face f of subdomain s is an interface
// when a neighbour box exists (nbr >= 0) and outer otherwise.  Boundary entry
// q = f * m + patch of the boundary layer U_1 is shared with entry (f ^ 1) * m + patch
// of the neighbour across face f.
#include <algorithm>
#include <cstdio>

#include "sfm_internal.h"

namespace sfm {

void TileGeometry::init(int p_, int elem_bytes) {
  p = p_;
  P16 = (p + kTile - 1) / kTile * kTile;
  nt = P16 / kTile;
  npairs = (nt + 1) / 2;
  nslots = nt + nt * (nt - 1) / 2;
  auto strip_words = [&](int I) { return (int64_t)kDiagWords + (int64_t)kOffWords * (nt - 1 - I); };
  int64_t off = 0;
  for (int g = 0; g < npairs; ++g) {
    job_off[g] = (int32_t)off;
    off += strip_words(g);
    if (g != nt - 1 - g) off += strip_words(nt - 1 - g);
  }
  tail_off = (int32_t)off;
  const int64_t line = kLineBytes / elem_bytes;
  words_per_block = off + ((int64_t)kHalfDiagWords * nt + line - 1) / line * line;
}

// Lane and diagonal index (t) of word w of a tile in the stored order: every load
// instruction of a 16-lane row reads 16 bytes per lane, i.e. e = 16 / elem_bytes
// consecutive t of one lane; word w = (v * 16 + lane) * e + (t - v * e).
static void tile_word(int w, int elem_bytes, int& lane, int& t) {
  const int e = 16 / elem_bytes;
  const int v = w / (16 * e), rem = w % (16 * e);
  lane = rem / e;
  t = e * v + rem % e;
}

void TileGeometry::word_map(std::vector<int32_t>& rows, std::vector<int32_t>& cols, int elem_bytes) const {
  rows.clear();
  cols.clear();
  rows.reserve(words_per_block);
  cols.reserve(words_per_block);
  for (int g = 0; g < npairs; ++g) {
    const int strips[2] = {g, nt - 1 - g};
    const int ns = strips[0] == strips[1] ? 1 : 2;
    for (int si = 0; si < ns; ++si) {
      const int I = strips[si];
      for (int w = 0; w < kDiagWords; ++w) {
        int lane, t;
        tile_word(w, elem_bytes, lane, t);
        rows.push_back(kTile * I + lane);
        cols.push_back(kTile * I + (lane + t) % kTile);
      }
      for (int J = I + 1; J < nt; ++J) {
        for (int w = 0; w < kOffWords; ++w) {
          int lane, t;
          tile_word(w, elem_bytes, lane, t);
          rows.push_back(kTile * I + lane);
          cols.push_back(kTile * J + (lane + t) % kTile);
        }
      }
    }
  }
  for (int I = 0; I < nt; ++I)
    for (int lane = 0; lane < kTile; ++lane) {
      rows.push_back(kTile * I + lane);
      cols.push_back(kTile * I + (lane + 8) % kTile);
    }
  while ((int64_t)rows.size() < words_per_block) {   // padding: outside the block, stored as 0
    rows.push_back(P16);
    cols.push_back(P16);
  }
}

static std::string fmt(const char* f, long a = 0, long b = 0, long c = 0) {
  char buf[256];
  std::snprintf(buf, sizeof buf, f, a, b, c);
  return buf;
}

std::string Topology::init(const sfm_config& cfg, const int32_t* nbox, const int32_t* box_cells) {
  if ((nbox == nullptr) != (box_cells == nullptr)) return "nbox and box_cells go together";
  int64_t used = 0;
  for (int d = 0; d < 3; ++d) {
    if (cfg.ncell[d] < 1) return fmt("ncell[%ld] = %ld must be positive", d, cfg.ncell[d]);
    ncell[d] = cfg.ncell[d];
    cut[d].assign(1, 0);
    if (!box_cells) {
      if (cfg.sub_cells[d] < 2) return fmt("sub_cells[%ld] = %ld must be at least 2", d, cfg.sub_cells[d]);
      if (cfg.ncell[d] % cfg.sub_cells[d] != 0)
        return fmt("ncell[%ld] = %ld is not a multiple of sub_cells = %ld", d, cfg.ncell[d], cfg.sub_cells[d]);
      for (int b = 0; b < cfg.ncell[d] / cfg.sub_cells[d]; ++b) cut[d].push_back(cut[d].back() + cfg.sub_cells[d]);
    } else {
      if (nbox[d] < 1 || nbox[d] > cfg.ncell[d]) return fmt("nbox[%ld] = %ld out of range", d, nbox[d]);
      for (int b = 0; b < nbox[d]; ++b) {
        const int32_t w = box_cells[used + b];
        if (w < 2) return fmt("box %ld along axis %ld has %ld cells; at least 2 are needed", b, d, w);
        if ((int64_t)cut[d].back() + w > cfg.ncell[d])
          return fmt("box sizes along axis %ld add up to more than ncell = %ld", d, cfg.ncell[d]);
        cut[d].push_back(cut[d].back() + w);
      }
      if (cut[d].back() != cfg.ncell[d])
        return fmt("box sizes along axis %ld add up to %ld, not ncell = %ld", d, cut[d].back(), cfg.ncell[d]);
      used += nbox[d];
    }
    nsub[d] = (int)cut[d].size() - 1;
  }
  if (!(cfg.h > 0.0)) return "h must be positive";
  if (cfg.m < 1) return "m must be at least 1";
  if (cfg.k < 2) return "k must be at least 2";
  if (cfg.precision != SFM_PREC_FP32 && cfg.precision != SFM_PREC_BF16_FP32ACC && cfg.precision != SFM_PREC_FP64)
    return "unknown precision";
  if (cfg.build_batch < 0) return "build_batch must be >= 0";
  m = cfg.m;
  k = cfg.k;
  p = 6 * m;
  if (p > kTile * kMaxNt) return fmt("6m = %ld exceeds the supported maximum %ld", p, kTile * kMaxNt);
  // m = m1 * m2, m1 >= m2, m1 - m2 minimal
  m1 = m;
  m2 = 1;
  for (int d = 1; d * d <= m; ++d)
    if (m % d == 0) { m2 = d; m1 = m / d; }
  int wmin[3], wmax[3];
  for (int d = 0; d < 3; ++d) {
    wmin[d] = ncell[d];
    wmax[d] = 0;
    for (int b = 0; b < nsub[d]; ++b) {
      wmin[d] = std::min(wmin[d], cut[d][b + 1] - cut[d][b]);
      wmax[d] = std::max(wmax[d], cut[d][b + 1] - cut[d][b]);
    }
  }
  const int smin = std::min(wmin[0], std::min(wmin[1], wmin[2]));
  if (m1 >= smin)
    return fmt("patch count %ld along a face edge needs more than %ld cells per subdomain edge", m1, m1);
  const int64_t nmin = (int64_t)(wmin[0] + 1) * (wmin[1] + 1) * (wmin[2] + 1);
  N_max = (int64_t)(wmax[0] + 1) * (wmax[1] + 1) * (wmax[2] + 1);
  if ((int64_t)p * k > nmin)
    return fmt("ROM size 6mk = %ld exceeds the %ld nodes of the smallest subdomain", (long)p * k, (long)nmin);
  const int64_t S64 = (int64_t)nsub[0] * nsub[1] * nsub[2];
  if (S64 > (1 << 24)) return "too many subdomains";
  S = (int)S64;
  nbr.assign((size_t)S * 6, -1);
  for (int bz = 0; bz < nsub[2]; ++bz)
    for (int by = 0; by < nsub[1]; ++by)
      for (int bx = 0; bx < nsub[0]; ++bx) {
        const int s = index(bx, by, bz);
        const int b[3] = {bx, by, bz};
        for (int f = 0; f < 6; ++f) {
          int nb[3] = {b[0], b[1], b[2]};
          const int d = f / 2;
          nb[d] += (f % 2) ? 1 : -1;
          if (nb[d] >= 0 && nb[d] < nsub[d]) nbr[(size_t)s * 6 + f] = index(nb[0], nb[1], nb[2]);
        }
      }
  return "";
}

void Topology::box_of(int s, int b[3]) const {
  b[0] = s % nsub[0];
  b[1] = (s / nsub[0]) % nsub[1];
  b[2] = s / (nsub[0] * nsub[1]);
}

int Topology::owner(int i, int j, int l, bool strict) const {
  const int g[3] = {i, j, l};
  int b[3];
  for (int d = 0; d < 3; ++d) {
    if (g[d] < 0 || g[d] > ncell[d]) return -1;
    // q: the box with cut[q] <= g < cut[q + 1] (the last box for g = ncell)
    int q = (int)(std::upper_bound(cut[d].begin(), cut[d].end(), g[d]) - cut[d].begin()) - 1;
    q = std::min(q, nsub[d] - 1);
    const bool on_plane = g[d] == cut[d][q] || g[d] == cut[d][q + 1];
    if (strict) {
      if (on_plane) return -1;   // on a subdomain plane (interface or outer boundary)
      b[d] = q;
    } else {
      b[d] = (g[d] == cut[d][q] && q > 0) ? q - 1 : q;   // lowest box holding the node
    }
  }
  return index(b[0], b[1], b[2]);
}

void Topology::origin(int s, int o[3]) const {
  int b[3];
  box_of(s, b);
  for (int d = 0; d < 3; ++d) o[d] = cut[d][b[d]];
}

void Topology::cells(int s, int c[3]) const {
  int b[3];
  box_of(s, b);
  for (int d = 0; d < 3; ++d) c[d] = cut[d][b[d] + 1] - cut[d][b[d]];
}

}  // namespace sfm
