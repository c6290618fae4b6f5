// C ABI of libsfm: context management, ROM installation, stepping, state and checks.
//
// Algorithm 1 of the paper: Stage 1 (ROM construction) lives in build.hip; Stage 2
// (the leapfrog of the coupled ROMs) is driven from here with the kernels of
// step_kernels.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "sfm_internal.h"

using sfm::kTile;

namespace {
thread_local std::string g_create_error;

#define SFM_TRY_HIP(ctx, call)                                                              \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return (ctx)->fail(SFM_EHIP, std::string(#call) + " failed: " + hipGetErrorString(e_)); \
  } while (0)

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

__global__ void reset_state_kernel(float* U, float* D, const float* U0, const float* V0, float dt, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    U[i] = U0 ? U0[i] : 0.f;
    D[i] = V0 ? dt * V0[i] : 0.f;
  }
}

// Levels j >= k_of[s] of a [S][k][row] state are outside subdomain s's ROM: hold them at zero.
__global__ void zero_levels_kernel(float* X, const int32_t* k_of, int k, int64_t row, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sj = i / row;
    if ((int)(sj % k) >= k_of[sj / k]) X[i] = 0.f;
  }
}

}  // namespace

hipError_t sfm::clear_extra_levels(sfm_ctx c, float* X, int cols, hipStream_t st) {
  if (!c->k_of_d || !X) return hipSuccess;
  const sfm::Topology& t = c->topo;
  const int64_t row = (int64_t)c->geo.P16 * cols;
  hipLaunchKernelGGL(zero_levels_kernel, dim3(1024), dim3(256), 0, st, X, c->k_of_d, t.k, row, (int64_t)t.S * t.k * row);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------- context helpers
// *e is written only on failure, so a run of allocations sharing one status reports the first
// failure even when later ones succeed (callers initialise it to hipSuccess).
void* sfm_ctx_s::dalloc(size_t bytes, hipError_t* e) {
  void* p = nullptr;
  const hipError_t r = hipMalloc(&p, std::max<size_t>(bytes, 16));
  if (r != hipSuccess) {
    *e = r;
    return nullptr;
  }
  owned.push_back(p);
  return p;
}

void sfm_ctx_s::dfree(void* p) {
  if (!p) return;
  auto it = std::find(owned.begin(), owned.end(), p);
  if (it != owned.end()) {
    (void)hipFree(p);
    owned.erase(it);
  }
}

void sfm_ctx_s::dfree_all() {
  for (void* p : owned) (void)hipFree(p);
  owned.clear();
}

namespace sfm {

// Drop every ROM-dependent buffer (before a new build or load).
void release_roms(sfm_ctx c) {
  release_shots(c);
  c->dfree(c->wmap_d);
  c->wmap_d = nullptr;
  void* bufs[] = {c->tiles_d, c->coef64_d, c->src_vec_d, c->src_vec64_d, c->src_off_d, c->src_ids_d,
                  c->sw_off_d, c->sw_q_d, c->sw_src_d, c->sw_w_d, c->rec_sub_d, c->rec_rows_d,
                  c->rec_rows64_d, c->U0_d, c->V0_d, c->rec_perm_d, c->rs_off_d, c->hist_slot_d,
                  c->hist_d, c->plain_blocks_d};
  for (void* b : bufs) c->dfree(b);
  c->tiles_d = nullptr; c->coef64_d = nullptr; c->src_vec_d = nullptr; c->src_vec64_d = nullptr;
  c->src_off_d = nullptr; c->src_ids_d = nullptr; c->sw_off_d = nullptr; c->sw_q_d = nullptr;
  c->sw_src_d = nullptr; c->sw_w_d = nullptr; c->rec_sub_d = nullptr; c->rec_rows_d = nullptr;
  c->rec_rows64_d = nullptr; c->U0_d = nullptr; c->V0_d = nullptr; c->rec_perm_d = nullptr;
  c->rs_off_d = nullptr; c->hist_slot_d = nullptr; c->hist_d = nullptr; c->plain_blocks_d = nullptr;
  c->dfree(c->k_of_d);
  c->k_of_d = nullptr;
  c->dfree(c->order_d);
  c->order_d = nullptr;
  c->k_of.clear();
  c->n_rs = 0;
  c->rs_max = 0;
  c->has_roms = false;
  c->nsrc = c->nrec = 0;
  c->src_sub.clear();
  c->dt_max = -1.0;
}

template <typename T>
static T* alloc_copy(sfm_ctx c, const std::vector<T>& v, hipError_t* e) {
  T* d = static_cast<T*>(c->dalloc(v.size() * sizeof(T), e));
  if (!d) return nullptr;
  if (!v.empty()) {
    const hipError_t r = hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (r != hipSuccess) *e = r;
  }
  return d;
}

// Resolve source / receiver nodes to subdomains; host arrays of ijk triples.
sfm_status locate_points(sfm_ctx c, int32_t nsrc, const int32_t* src_ijk, int32_t nrec, const int32_t* rec_ijk,
                         std::vector<int32_t>& src_sub, std::vector<int32_t>& src_local,
                         std::vector<int32_t>& rec_sub, std::vector<int32_t>& rec_local) {
  const Topology& t = c->topo;
  if (nsrc < 0 || nrec < 0) return c->fail(SFM_EINVAL, "negative source or receiver count");
  if ((nsrc > 0 && !src_ijk) || (nrec > 0 && !rec_ijk)) return c->fail(SFM_EINVAL, "missing node array");
  auto local = [&](int s, const int32_t* g) {
    int o[3], w[3];
    t.origin(s, o);
    t.cells(s, w);
    return ((g[2] - o[2]) * (w[1] + 1) + (g[1] - o[1])) * (w[0] + 1) + (g[0] - o[0]);
  };
  src_sub.resize(nsrc);
  src_local.resize(nsrc);
  for (int i = 0; i < nsrc; ++i) {
    const int32_t* g = src_ijk + 3 * i;
    const int s = t.owner(g[0], g[1], g[2], true);
    if (s < 0)
      return c->fail(SFM_EINVAL, "source " + std::to_string(i) + " at (" + std::to_string(g[0]) + "," +
                                     std::to_string(g[1]) + "," + std::to_string(g[2]) +
                                     ") is not strictly inside a subdomain");
    src_sub[i] = s;
    src_local[i] = local(s, g);
  }
  rec_sub.resize(nrec);
  rec_local.resize(nrec);
  for (int i = 0; i < nrec; ++i) {
    const int32_t* g = rec_ijk + 3 * i;
    const int s = t.owner(g[0], g[1], g[2], false);
    if (s < 0) return c->fail(SFM_EINVAL, "receiver " + std::to_string(i) + " is outside the grid");
    rec_sub[i] = s;
    rec_local[i] = local(s, g);
  }
  return SFM_OK;
}

// Install ROMs whose FP64 coefficients already sit in c->coef64_d ([S][2][k][p][p]),
// given the boundary face masses H = diag(Gamma-hat_1) (host, [S][p]) and FP64 source
// vectors / receiver rows on the device.  Builds the streamed tiles, the combined face
// masses C_f = (sum over sides of 1/H)^{-1} (eq. "bdrytstep"), the boundary-layer source
// weights w_f = C_f sum over sides of H^{-1} s_1, and resets the state.
sfm_status finalize_roms(sfm_ctx c, const std::vector<double>& H, const std::vector<int32_t>& src_sub,
                         const std::vector<double>& src_vec_host, const std::vector<int32_t>& rec_sub,
                         hipStream_t st) {
  const Topology& t = c->topo;
  const TileGeometry& g = c->geo;
  const int S = t.S, k = t.k, p = t.p, P16 = g.P16, m = t.m;
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < H.size(); ++i)
    if (!(H[i] > 0.0)) return c->fail(SFM_EBREAKDOWN, "non-positive face mass diag(Gamma-hat_1)");

  // streamed tiles
  std::vector<int32_t> wrow, wcol;
  c->tile_elem = tile_elem_bytes(c->cfg.precision);
  g.word_map(wrow, wcol, (int)c->tile_elem);
  int32_t* wrow_d = alloc_copy(c, wrow, &e);
  if (e != hipSuccess) return c->fail(SFM_ENOMEM, "word map allocation failed");
  int32_t* wcol_d = alloc_copy(c, wcol, &e);
  if (e != hipSuccess) return c->fail(SFM_ENOMEM, "word map allocation failed");
  {
    std::vector<uint32_t> wmap(wrow.size());
    for (size_t i = 0; i < wrow.size(); ++i) wmap[i] = ((uint32_t)wrow[i] << 16) | (uint32_t)wcol[i];
    c->dfree(c->wmap_d);
    c->wmap_d = alloc_copy(c, wmap, &e);
    if (e != hipSuccess) return c->fail(SFM_ENOMEM, "word map allocation failed");
  }
  const size_t tile_bytes = (size_t)S * (2 * k - 1) * g.words_per_block * c->tile_elem;
  c->tiles_d = c->dalloc(tile_bytes, &e);
  if (!c->tiles_d) return c->fail(SFM_ENOMEM, "coefficient tiles: out of device memory");
  SFM_TRY_HIP(c, launch_pack(c->coef64_d, 0, 0, k, p, g, wrow_d, wcol_d, c->tiles_d, c->cfg.precision, S, st));

  // combined face masses
  std::vector<float> C((size_t)S * P16, 0.f);
  for (int s = 0; s < S; ++s)
    for (int q = 0; q < p; ++q) {
      const int f = q / m, pat = q % m;
      const int nb = t.nbr[(size_t)s * 6 + f];
      double inv = 1.0 / H[(size_t)s * p + q];
      if (nb >= 0) inv += 1.0 / H[(size_t)nb * p + (f ^ 1) * m + pat];
      C[(size_t)s * P16 + q] = (float)(1.0 / inv);
    }
  SFM_TRY_HIP(c, hipMemcpyAsync(c->C_d, C.data(), C.size() * sizeof(float), hipMemcpyHostToDevice, st));

  // sources: interior CSR and boundary-layer weights
  const int nsrc = (int)src_sub.size();
  c->nsrc = nsrc;
  c->src_sub = src_sub;
  if (nsrc > 0) {
    std::vector<int32_t> off(S + 1, 0), ids(nsrc);
    for (int i = 0; i < nsrc; ++i) off[src_sub[i] + 1]++;
    for (int s = 0; s < S; ++s) off[s + 1] += off[s];
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int i = 0; i < nsrc; ++i) ids[fill[src_sub[i]]++] = i;
    c->src_off_d = alloc_copy(c, off, &e);
    c->src_ids_d = alloc_copy(c, ids, &e);
    struct W { int s, q, src; float w; };
    std::vector<W> ws;
    for (int i = 0; i < nsrc; ++i) {
      const int a = src_sub[i];
      for (int q = 0; q < p; ++q) {
        const double s1 = src_vec_host[(size_t)i * k * p + q];
        if (s1 == 0.0) continue;
        const float w = (float)((double)C[(size_t)a * P16 + q] * s1 / H[(size_t)a * p + q]);
        ws.push_back({a, q, i, w});
        const int f = q / m, pat = q % m;
        const int nb = t.nbr[(size_t)a * 6 + f];
        if (nb >= 0) ws.push_back({nb, (f ^ 1) * m + pat, i, w});
      }
    }
    std::stable_sort(ws.begin(), ws.end(), [](const W& x, const W& y) { return x.s < y.s; });
    std::vector<int32_t> swoff(S + 1, 0), swq(ws.size()), swsrc(ws.size());
    std::vector<float> sww(ws.size());
    for (size_t i = 0; i < ws.size(); ++i) {
      swoff[ws[i].s + 1]++;
      swq[i] = ws[i].q;
      swsrc[i] = ws[i].src;
      sww[i] = ws[i].w;
    }
    for (int s = 0; s < S; ++s) swoff[s + 1] += swoff[s];
    c->sw_off_d = alloc_copy(c, swoff, &e);
    c->sw_q_d = alloc_copy(c, swq, &e);
    c->sw_src_d = alloc_copy(c, swsrc, &e);
    c->sw_w_d = alloc_copy(c, sww, &e);
    c->src_vec_d = static_cast<float*>(c->dalloc((size_t)nsrc * k * P16 * sizeof(float), &e));
    if (e != hipSuccess) return c->fail(SFM_ENOMEM, "source buffers: out of device memory");
    SFM_TRY_HIP(c, launch_pad_rows(c->src_vec64_d, (int64_t)nsrc * k, p, P16, c->src_vec_d, st));
  }
  // receivers, sorted by subdomain (stable), with the per-subdomain history ring
  const int nrec = (int)rec_sub.size();
  c->nrec = nrec;
  if (nrec > 0) {
    std::vector<int32_t> perm(nrec);
    for (int i = 0; i < nrec; ++i) perm[i] = i;
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return rec_sub[a] < rec_sub[b]; });
    std::vector<int32_t> sub_sorted(nrec), slot_of(S, -1), rs_off;
    for (int i = 0; i < nrec; ++i) {
      const int s = rec_sub[perm[i]];
      sub_sorted[i] = s;
      if (slot_of[s] < 0) {
        slot_of[s] = (int)rs_off.size();
        rs_off.push_back(i);
      }
    }
    rs_off.push_back(nrec);
    c->n_rs = (int)rs_off.size() - 1;
    for (int q = 0; q < c->n_rs; ++q) c->rs_max = std::max(c->rs_max, rs_off[q + 1] - rs_off[q]);
    c->rec_sub_d = alloc_copy(c, sub_sorted, &e);
    c->rec_perm_d = alloc_copy(c, perm, &e);
    c->rs_off_d = alloc_copy(c, rs_off, &e);
    c->hist_slot_d = alloc_copy(c, slot_of, &e);
    const size_t hist_bytes = (size_t)kHistWindow * c->n_rs * k * P16 * sizeof(float);
    c->hist_d = static_cast<float*>(c->dalloc(hist_bytes, &e));
    c->rec_rows_d = static_cast<float*>(c->dalloc((size_t)nrec * k * P16 * sizeof(float), &e));
    if (e != hipSuccess) return c->fail(SFM_ENOMEM, "receiver buffers: out of device memory");
    SFM_TRY_HIP(c, hipMemsetAsync(c->hist_d, 0, hist_bytes, st));   // padding entries stay zero
    // FP64 rows (caller order) -> FP32 padded rows (sorted order)
    std::vector<int32_t> inv(nrec);
    for (int i = 0; i < nrec; ++i) inv[i] = perm[i];
    int32_t* gather_d = alloc_copy(c, inv, &e);
    double* tmp = static_cast<double*>(c->dalloc((size_t)nrec * k * p * sizeof(double), &e));
    if (e != hipSuccess) return c->fail(SFM_ENOMEM, "receiver buffers: out of device memory");
    SFM_TRY_HIP(c, launch_gather_rows(c->rec_rows64_d, gather_d, nrec, (int64_t)k * p, tmp, st));
    SFM_TRY_HIP(c, launch_pad_rows(tmp, (int64_t)nrec * k, p, P16, c->rec_rows_d, st));
    SFM_TRY_HIP(c, hipStreamSynchronize(st));
    c->dfree(tmp);
    c->dfree(gather_d);
  }
  const int64_t nstate = (int64_t)S * k * P16;
  SFM_TRY_HIP(c, hipMemsetAsync(c->exch_d, 0, (size_t)S * P16 * sizeof(float), st));
  hipLaunchKernelGGL(reset_state_kernel, dim3(1024), dim3(256), 0, st, c->U_d, c->D_d, c->U0_d, nullptr, 0.f, nstate);
  SFM_TRY_HIP(c, hipGetLastError());
  SFM_TRY_HIP(c, hipStreamSynchronize(st));
  c->dfree(wrow_d);
  c->dfree(wcol_d);
  c->n = 0;
  c->has_roms = true;
  return SFM_OK;
}

}  // namespace sfm

using namespace sfm;

namespace sfm {
sfm_status drain_events(sfm_ctx c, std::vector<hipEvent_t>& ev, double* ms3, int64_t* steps) {
  if (ev.empty()) return SFM_OK;
  const hipError_t sync = hipEventSynchronize(ev.back());
  for (size_t s = 0; sync == hipSuccess && s + 4 <= ev.size(); s += 4) {
    // A step that failed part-way left some of its events unrecorded: it is not counted, and
    // the error the query leaves behind is cleared so that no later launch check reports it.
    float ms[3];
    bool ok = true;
    for (int q = 0; q < 3 && ok; ++q) ok = hipEventElapsedTime(&ms[q], ev[s + q], ev[s + q + 1]) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      continue;
    }
    for (int q = 0; q < 3; ++q) ms3[q] += ms[q];
    ++*steps;
  }
  c->ev_pool.insert(c->ev_pool.end(), ev.begin(), ev.end());
  ev.clear();
  if (sync != hipSuccess) return c->fail(SFM_EHIP, std::string("hipEventSynchronize failed: ") + hipGetErrorString(sync));
  return SFM_OK;
}

static sfm_status drain_timing(sfm_ctx c) { return drain_events(c, c->ev, c->timed_ms, &c->timed_steps); }
}  // namespace sfm

// ----------------------------------------------------------------------------- ABI
extern "C" {

sfm_status sfm_create(const sfm_config* cfg, sfm_ctx* out) { return sfm_create_boxes(cfg, nullptr, nullptr, out); }

sfm_status sfm_create_boxes(const sfm_config* cfg, const int32_t* nbox, const int32_t* box_cells, sfm_ctx* out) {
  if (!out) {
    g_create_error = "out is NULL";
    return SFM_EINVAL;
  }
  *out = nullptr;
  if (!cfg) {
    g_create_error = "cfg is NULL";
    return SFM_EINVAL;
  }
  Topology topo;
  const std::string msg = topo.init(*cfg, nbox, box_cells);
  if (!msg.empty()) {
    g_create_error = msg;
    return SFM_EINVAL;
  }
  {
    TileGeometry g;
    g.init(topo.p, tile_elem_bytes(cfg->precision));
    const size_t acc = cfg->precision == SFM_PREC_FP64 ? sizeof(double) : sizeof(float);
    const size_t lds = acc * ((size_t)2 * topo.k * g.P16 + (size_t)topo.k * g.nslots * kTile);
    if (lds > kMaxLdsBytes) {
      g_create_error = "k = " + std::to_string(topo.k) + " and p = " + std::to_string(topo.p) + " need " +
                       std::to_string(lds) + " bytes of LDS per subdomain work-group, above the " +
                       std::to_string(kMaxLdsBytes) + " of a CU";
      return SFM_EINVAL;
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    g_create_error = "no HIP device available";
    return SFM_EHIP;
  }
  sfm_ctx c = new (std::nothrow) sfm_ctx_s();
  if (!c) {
    g_create_error = "host allocation failed";
    return SFM_ENOMEM;
  }
  c->cfg = *cfg;
  c->topo = topo;
  c->geo.init(topo.p, tile_elem_bytes(cfg->precision));
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    g_create_error = "hipGetDevice failed";
    return SFM_EHIP;
  }
  hipError_t e = hipSuccess;
  const int64_t nstate = (int64_t)topo.S * topo.k * c->geo.P16;
  c->nbr_d = alloc_copy(c, topo.nbr, &e);
  if (e == hipSuccess) c->C_d = static_cast<float*>(c->dalloc((size_t)topo.S * c->geo.P16 * sizeof(float), &e));
  if (e == hipSuccess) c->U_d = static_cast<float*>(c->dalloc(nstate * sizeof(float), &e));
  if (e == hipSuccess) c->D_d = static_cast<float*>(c->dalloc(nstate * sizeof(float), &e));
  if (e == hipSuccess) c->exch_d = static_cast<float*>(c->dalloc((size_t)topo.S * c->geo.P16 * sizeof(float), &e));
  if (e == hipSuccess) c->red_d = static_cast<double*>(c->dalloc((kNormScratch0 + 1024) * sizeof(double), &e));
  if (e == hipSuccess) c->work_a_d = static_cast<float*>(c->dalloc(nstate * sizeof(float), &e));
  if (e == hipSuccess) c->work_b_d = static_cast<float*>(c->dalloc(nstate * sizeof(float), &e));
  if (e == hipSuccess) e = hipMemset(c->U_d, 0, nstate * sizeof(float));
  if (e == hipSuccess) e = hipMemset(c->D_d, 0, nstate * sizeof(float));
  if (e == hipSuccess) e = hipMemset(c->C_d, 0, (size_t)topo.S * c->geo.P16 * sizeof(float));
  if (e != hipSuccess) {
    g_create_error = std::string("device allocation failed: ") + hipGetErrorString(e);
    c->dfree_all();
    delete c;
    return SFM_ENOMEM;
  }
  *out = c;
  return SFM_OK;
}

void sfm_destroy(sfm_ctx c) {
  if (!c) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->shot_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  sfm::drop_shot_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  c->dfree_all();
  (void)hipSetDevice(cur);
  delete c;
}

const char* sfm_last_error(sfm_ctx c) { return c ? c->err.c_str() : g_create_error.c_str(); }

extern "C" sfm_status sfm_set_timing(sfm_ctx c, int32_t enable) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  SFM_TRY_HIP(c, hipSetDevice(c->device));
  sfm_status rc = drain_timing(c);
  if (rc != SFM_OK) return rc;
  if (enable < 0) return c->fail(SFM_EINVAL, "sfm_set_timing: enable must be >= 0");
  c->timing = enable != 0;
  if (c->timing) {
    c->timing_every = enable;
    c->timing_seen = 0;
    c->timed_steps = 0;
    c->timed_ms[0] = c->timed_ms[1] = c->timed_ms[2] = 0.0;
  }
  return SFM_OK;
}

extern "C" sfm_status sfm_query(sfm_ctx c, sfm_info* out) {
  if (!c || !out) return SFM_EINVAL;
  if (c->timing || !c->ev.empty()) {
    sfm_status rc = drain_timing(c);
    if (rc != SFM_OK) return rc;
  }
  out->timed_steps = c->timed_steps;
  out->timed_main_ms = c->timed_ms[0];
  out->timed_face_ms = c->timed_ms[1];
  out->timed_record_ms = c->timed_ms[2];
  const Topology& t = c->topo;
  out->n_subdomains = t.S;
  out->p = t.p;
  out->k = t.k;
  out->nsrc = c->nsrc;
  out->nrec = c->nrec;
  out->has_roms = c->has_roms ? 1 : 0;
  out->steps_done = c->n;
  const int64_t elem = tile_elem_bytes(c->cfg.precision);
  out->coef_bytes = (int64_t)t.S * (2 * t.k - 1) * c->geo.words_per_block * elem;
  out->coef_bytes_algorithmic = (int64_t)t.S * (2 * t.k - 1) * ((int64_t)t.p * (t.p + 1) / 2) * elem;
  out->state_bytes = (int64_t)t.S * t.k * t.p * 4;
  out->build_seconds = c->build_seconds;
  out->rho_estimate = c->rho_est;
  out->rho_bound = c->rho_bound;
  out->watchdog_checks = c->wd_checks;
  return SFM_OK;
}

sfm_status sfm_load_roms(sfm_ctx c, const double* gamma, const double* gamma_hat, int32_t nsrc,
                         const int32_t* src_ijk, const double* src_vec, int32_t nrec, const int32_t* rec_ijk,
                         const double* rec_rows) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!gamma || !gamma_hat) return c->fail(SFM_EINVAL, "gamma and gamma_hat are required");
  if ((nsrc > 0 && !src_vec) || (nrec > 0 && !rec_rows)) return c->fail(SFM_EINVAL, "missing projections");
  SFM_TRY_HIP(c, hipSetDevice(c->device));
  const Topology& t = c->topo;
  const int S = t.S, k = t.k, p = t.p;
  std::vector<int32_t> src_sub, src_local, rec_sub, rec_local;
  sfm_status rc = locate_points(c, nsrc, src_ijk, nrec, rec_ijk, src_sub, src_local, rec_sub, rec_local);
  if (rc != SFM_OK) return rc;
  // Gamma-hat_1 must be diagonal (non-overlapping boundary functions).
  std::vector<double> H((size_t)S * p);
  const size_t blk = (size_t)p * p;
  for (int s = 0; s < S; ++s) {
    const double* g1 = gamma_hat + (size_t)s * k * blk;
    double dmax = 0.0, omax = 0.0;
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j) {
        const double v = std::fabs(g1[(size_t)i * p + j]);
        if (i == j) dmax = std::max(dmax, v); else omax = std::max(omax, v);
      }
    if (omax > 1e-10 * dmax)
      return c->fail(SFM_EINVAL, "gamma_hat[" + std::to_string(s) + "][0] is not diagonal");
    for (int i = 0; i < p; ++i) H[(size_t)s * p + i] = g1[(size_t)i * p + i];
  }
  release_roms(c);
  hipError_t e = hipSuccess;
  c->coef64_d = static_cast<double*>(c->dalloc((size_t)S * 2 * k * blk * sizeof(double), &e));
  if (!c->coef64_d) return c->fail(SFM_ENOMEM, "FP64 coefficients: out of device memory");
  for (int s = 0; s < S; ++s) {
    SFM_TRY_HIP(c, hipMemcpy(c->coef64_d + (size_t)s * 2 * k * blk, gamma + (size_t)s * k * blk,
                             k * blk * sizeof(double), hipMemcpyHostToDevice));
    SFM_TRY_HIP(c, hipMemcpy(c->coef64_d + ((size_t)s * 2 + 1) * k * blk, gamma_hat + (size_t)s * k * blk,
                             k * blk * sizeof(double), hipMemcpyHostToDevice));
  }
  std::vector<double> sv;
  if (nsrc > 0) {
    sv.assign(src_vec, src_vec + (size_t)nsrc * k * p);
    c->src_vec64_d = alloc_copy(c, sv, &e);
  }
  if (nrec > 0) {
    std::vector<double> rr(rec_rows, rec_rows + (size_t)nrec * k * p);
    c->rec_rows64_d = alloc_copy(c, rr, &e);
  }
  if (e != hipSuccess) return c->fail(SFM_ENOMEM, "projection buffers: out of device memory");
  c->build_seconds = 0.0;
  return finalize_roms(c, H, src_sub, sv, rec_sub, nullptr);
}

sfm_status sfm_export_roms(sfm_ctx c, double* gamma, double* gamma_hat) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs: call sfm_build_roms or sfm_load_roms first");
  const Topology& t = c->topo;
  const size_t chunk = (size_t)t.k * t.p * t.p * sizeof(double);
  SFM_TRY_HIP(c, hipSetDevice(c->device));
  SFM_TRY_HIP(c, hipDeviceSynchronize());
  if (gamma)
    SFM_TRY_HIP(c, hipMemcpy2D(gamma, chunk, c->coef64_d, 2 * chunk, chunk, t.S, hipMemcpyDeviceToHost));
  if (gamma_hat)
    SFM_TRY_HIP(c, hipMemcpy2D(gamma_hat, chunk, reinterpret_cast<const char*>(c->coef64_d) + chunk, 2 * chunk,
                               chunk, t.S, hipMemcpyDeviceToHost));
  return SFM_OK;
}

sfm_status sfm_export_projections(sfm_ctx c, double* src_vec, double* rec_rows) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs");
  const Topology& t = c->topo;
  SFM_TRY_HIP(c, hipSetDevice(c->device));
  SFM_TRY_HIP(c, hipDeviceSynchronize());
  if (src_vec && c->nsrc > 0)
    SFM_TRY_HIP(c, hipMemcpy(src_vec, c->src_vec64_d, (size_t)c->nsrc * t.k * t.p * sizeof(double),
                             hipMemcpyDeviceToHost));
  if (rec_rows && c->nrec > 0)
    SFM_TRY_HIP(c, hipMemcpy(rec_rows, c->rec_rows64_d, (size_t)c->nrec * t.k * t.p * sizeof(double),
                             hipMemcpyDeviceToHost));
  return SFM_OK;
}

}  // extern "C"

namespace sfm {

static StepParams make_step_params(sfm_ctx c) {
  StepParams prm{};
  const TileGeometry& g = c->geo;
  prm.tiles = c->tiles_d;
  prm.words_per_block = g.words_per_block;
  prm.words_per_sub = (int64_t)(2 * c->topo.k - 1) * g.words_per_block;
  std::memcpy(prm.job_off, g.job_off, sizeof(prm.job_off));
  prm.tail_off = g.tail_off;
  prm.S = c->topo.S;
  prm.k = c->topo.k;
  prm.k_of = c->k_of_d;
  prm.order = c->order_d;
  prm.P16 = g.P16;
  prm.nt = g.nt;
  prm.npairs = g.npairs;
  prm.nslots = g.nslots;
  prm.U = c->U_d;
  prm.D = c->D_d;
  prm.exch = c->exch_d;
  return prm;
}

static FaceParams make_face_params(sfm_ctx c) {
  FaceParams f{};
  f.S = c->topo.S;
  f.k = c->topo.k;
  f.P16 = c->geo.P16;
  f.p = c->topo.p;
  f.m = c->topo.m;
  f.nbr = c->nbr_d;
  f.C = c->C_d;
  f.exch = c->exch_d;
  f.U = c->U_d;
  f.D = c->D_d;
  return f;
}

// a = a(u) of the coupled scheme without forcing (both kernels in operator mode).
hipError_t apply_operator(sfm_ctx c, const float* u, float* a, hipStream_t st) {
  StepParams prm = make_step_params(c);
  prm.mode = 1;
  prm.Uin = u;
  prm.Aout = a;
  hipError_t e = launch_step_main(prm, c->cfg.precision, st);
  if (e != hipSuccess) return e;
  FaceParams f = make_face_params(c);
  f.mode = 1;
  f.Aout = a;
  return launch_step_face(f, st);
}

// One leapfrog step of the single-shot state (no receivers): wavelet_row = this step's source
// amplitudes [nsrc]; kx_out (optional) receives the interior flux differences of the step and
// u_out (optional) the state the step starts from.
sfm_status forward_step(sfm_ctx c, double dt, const float* wavelet_row, float* kx_out, float* u_out,
                        hipStream_t st) {
  StepParams prm = make_step_params(c);
  FaceParams f = make_face_params(c);
  prm.mode = 0;
  f.mode = 0;
  prm.dt2 = (float)(dt * dt);
  f.dt2 = prm.dt2;
  prm.nsrc = f.nsrc = c->nsrc;
  prm.wavelet = f.wavelet = wavelet_row;
  prm.step = f.step = 0;
  if (c->nsrc > 0) {
    prm.src_off = c->src_off_d;
    prm.src_ids = c->src_ids_d;
    prm.src_vec = c->src_vec_d;
    f.sw_off = c->sw_off_d;
    f.sw_q = c->sw_q_d;
    f.sw_src = c->sw_src_d;
    f.sw_w = c->sw_w_d;
  }
  prm.kx_out = kx_out;
  prm.u_out = u_out;
  SFM_TRY_HIP(c, launch_step_main(prm, c->cfg.precision, st));
  SFM_TRY_HIP(c, launch_step_face(f, st));
  return SFM_OK;
}

StepParams step_params(sfm_ctx c) { return make_step_params(c); }

}  // namespace sfm

extern "C" {

sfm_status sfm_step(sfm_ctx c, int32_t nsteps, double dt, const float* wavelet_dev, float* traces_dev, int64_t ld,
                    void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs: call sfm_build_roms or sfm_load_roms first");
  if (nsteps < 0) return c->fail(SFM_EINVAL, "nsteps must be >= 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return c->fail(SFM_EINVAL, "dt must be positive and finite");
  if (c->nsrc > 0 && nsteps > 0 && !wavelet_dev) return c->fail(SFM_EINVAL, "wavelet_dev is required with sources");
  if (traces_dev && ld < nsteps) return c->fail(SFM_EINVAL, "ld must be >= nsteps");
  if (c->dt_max > 0.0 && dt > c->dt_max)
    return c->fail(SFM_EUNSTABLE, "dt = " + std::to_string(dt) + " exceeds the stability limit " +
                                      std::to_string(c->dt_max));
  SFM_TRY_HIP(c, hipSetDevice(c->device));
  hipStream_t st = as_stream(stream);
  StepParams prm = make_step_params(c);
  FaceParams f = make_face_params(c);
  prm.mode = 0;
  f.mode = 0;
  prm.dt2 = (float)(dt * dt);
  f.dt2 = prm.dt2;
  prm.nsrc = f.nsrc = c->nsrc;
  prm.wavelet = f.wavelet = wavelet_dev;
  if (c->nsrc > 0) {
    prm.src_off = c->src_off_d;
    prm.src_ids = c->src_ids_d;
    prm.src_vec = c->src_vec_d;
    f.sw_off = c->sw_off_d;
    f.sw_q = c->sw_q_d;
    f.sw_src = c->sw_src_d;
    f.sw_w = c->sw_w_d;
  }
  RecWindowParams r{};
  r.n_rs = c->n_rs;
  r.k = c->topo.k;
  r.P16 = c->geo.P16;
  r.rs_off = c->rs_off_d;
  r.perm = c->rec_perm_d;
  r.rows = c->rec_rows_d;
  r.hist = c->hist_d;
  r.traces = traces_dev;
  r.ld = ld;
  const bool recording = traces_dev && c->nrec > 0;
  if (recording) {
    prm.hist = f.hist = c->hist_d;
    prm.hist_slot = f.hist_slot = c->hist_slot_d;
  }
  const int64_t slot_stride = (int64_t)c->n_rs * c->topo.k * c->geo.P16;
  for (int32_t i = 0; i < nsteps; ++i) {
    prm.step = f.step = i;
    const int t = i % kHistWindow;
    prm.hist_off = f.hist_off = t * slot_stride;
    const bool rec = recording && (t == kHistWindow - 1 || i + 1 == nsteps);
    hipEvent_t* e = nullptr;
    if (c->time_this_step()) {
      SFM_TRY_HIP(c, c->take_events(c->ev));
      e = &c->ev[c->ev.size() - 4];
      SFM_TRY_HIP(c, hipEventRecord(e[0], st));
    }
    SFM_TRY_HIP(c, launch_step_main(prm, c->cfg.precision, st));
    if (e) SFM_TRY_HIP(c, hipEventRecord(e[1], st));
    SFM_TRY_HIP(c, launch_step_face(f, st));
    if (e) SFM_TRY_HIP(c, hipEventRecord(e[2], st));
    if (rec) {
      r.w = t + 1;
      r.col0 = i - t;
      SFM_TRY_HIP(c, launch_record_window(r, st, c->rs_max));
    }
    if (e) SFM_TRY_HIP(c, hipEventRecord(e[3], st));
    if (c->wd_every > 0 && ((i + 1) % c->wd_every == 0 || i + 1 == nsteps)) {
      const int64_t n = (int64_t)c->topo.S * c->topo.k * c->geo.P16;
      double nrm2 = 0.0;
      SFM_TRY_HIP(c, launch_norm2(c->U_d, n, c->red_d, st));
      SFM_TRY_HIP(c, hipMemcpyAsync(&nrm2, c->red_d, sizeof(double), hipMemcpyDeviceToHost, st));
      SFM_TRY_HIP(c, hipStreamSynchronize(st));
      ++c->wd_checks;
      const double nrm = std::sqrt(nrm2);
      if (!std::isfinite(nrm) || nrm > c->wd_max_norm) {
        c->n += i + 1;
        return c->fail(SFM_EUNSTABLE, "watchdog: |U| = " + std::to_string(nrm) + " after step " +
                                          std::to_string(c->n) + (std::isfinite(nrm) ? " exceeds the limit "
                                          + std::to_string(c->wd_max_norm) : " (state not finite)"));
      }
    }
  }
  c->n += nsteps;
  return SFM_OK;
}

sfm_status sfm_record_receivers(sfm_ctx c, float* out_dev, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs");
  if (c->nrec > 0 && !out_dev) return c->fail(SFM_EINVAL, "out_dev is NULL");
  SFM_TRY_HIP(c, hipSetDevice(c->device));
  RecParams r{};
  r.nrec = c->nrec;
  r.k = c->topo.k;
  r.P16 = c->geo.P16;
  r.rec_sub = c->rec_sub_d;
  r.perm = c->rec_perm_d;
  r.rows = c->rec_rows_d;
  r.U = c->U_d;
  r.out = out_dev;
  r.ld = 1;
  r.col = 0;
  SFM_TRY_HIP(c, launch_record(r, as_stream(stream)));
  return SFM_OK;
}

sfm_status sfm_apply_operator(sfm_ctx c, const float* u_dev, float* a_dev, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs");
  if (!u_dev || !a_dev) return c->fail(SFM_EINVAL, "u_dev and a_dev are required");
  if (u_dev == a_dev) return c->fail(SFM_EINVAL, "u_dev and a_dev must not alias");
  SFM_TRY_HIP(c, hipSetDevice(c->device));
  hipStream_t st = as_stream(stream);
  // The caller's arrays are [S][k][p]; the kernels work on [S][k][P16] (zero padding).
  const Topology& t = c->topo;
  const int P16 = c->geo.P16;
  if (P16 == t.p) {
    SFM_TRY_HIP(c, apply_operator(c, u_dev, a_dev, st));
    return SFM_OK;
  }
  SFM_TRY_HIP(c, hipMemsetAsync(c->work_a_d, 0, (size_t)t.S * t.k * P16 * sizeof(float), st));
  SFM_TRY_HIP(c, hipMemsetAsync(c->work_b_d, 0, (size_t)t.S * t.k * P16 * sizeof(float), st));
  SFM_TRY_HIP(c, hipMemcpy2DAsync(c->work_a_d, P16 * sizeof(float), u_dev, t.p * sizeof(float),
                                  t.p * sizeof(float), (size_t)t.S * t.k, hipMemcpyDeviceToDevice, st));
  SFM_TRY_HIP(c, apply_operator(c, c->work_a_d, c->work_b_d, st));
  SFM_TRY_HIP(c, hipMemcpy2DAsync(a_dev, t.p * sizeof(float), c->work_b_d, P16 * sizeof(float),
                                  t.p * sizeof(float), (size_t)t.S * t.k, hipMemcpyDeviceToDevice, st));
  return SFM_OK;
}

sfm_status sfm_set_watchdog(sfm_ctx c, int32_t every, double max_norm) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (every < 0) return c->fail(SFM_EINVAL, "every must be >= 0");
  if (every > 0 && !(max_norm > 0.0)) return c->fail(SFM_EINVAL, "max_norm must be > 0");
  c->wd_every = every;
  c->wd_max_norm = max_norm;
  c->wd_checks = 0;
  return SFM_OK;
}

sfm_status sfm_get_state(sfm_ctx c, float* u_now, float* u_incr, int64_t* n) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  const Topology& t = c->topo;
  const int P16 = c->geo.P16;
  SFM_TRY_HIP(c, hipSetDevice(c->device));
  SFM_TRY_HIP(c, hipDeviceSynchronize());
  if (u_now)
    SFM_TRY_HIP(c, hipMemcpy2D(u_now, t.p * sizeof(float), c->U_d, P16 * sizeof(float), t.p * sizeof(float),
                               (size_t)t.S * t.k, hipMemcpyDeviceToHost));
  if (u_incr)
    SFM_TRY_HIP(c, hipMemcpy2D(u_incr, t.p * sizeof(float), c->D_d, P16 * sizeof(float), t.p * sizeof(float),
                               (size_t)t.S * t.k, hipMemcpyDeviceToHost));
  if (n) *n = c->n;
  return SFM_OK;
}

sfm_status sfm_set_state(sfm_ctx c, const float* u_now, const float* u_incr, int64_t n) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (n < 0) return c->fail(SFM_EINVAL, "n must be >= 0");
  const Topology& t = c->topo;
  const int P16 = c->geo.P16;
  const size_t bytes = (size_t)t.S * t.k * P16 * sizeof(float);
  SFM_TRY_HIP(c, hipSetDevice(c->device));
  SFM_TRY_HIP(c, hipDeviceSynchronize());
  SFM_TRY_HIP(c, hipMemset(c->U_d, 0, bytes));
  SFM_TRY_HIP(c, hipMemset(c->D_d, 0, bytes));
  if (u_now)
    SFM_TRY_HIP(c, hipMemcpy2D(c->U_d, P16 * sizeof(float), u_now, t.p * sizeof(float), t.p * sizeof(float),
                               (size_t)t.S * t.k, hipMemcpyHostToDevice));
  if (u_incr)
    SFM_TRY_HIP(c, hipMemcpy2D(c->D_d, P16 * sizeof(float), u_incr, t.p * sizeof(float), t.p * sizeof(float),
                               (size_t)t.S * t.k, hipMemcpyHostToDevice));
  SFM_TRY_HIP(c, sfm::clear_extra_levels(c, c->U_d, 1, nullptr));
  SFM_TRY_HIP(c, sfm::clear_extra_levels(c, c->D_d, 1, nullptr));
  SFM_TRY_HIP(c, hipDeviceSynchronize());
  c->n = n;
  return SFM_OK;
}

sfm_status sfm_set_levels(sfm_ctx c, const int32_t* k_per_sub) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs: call sfm_build_roms or sfm_load_roms first");
  const Topology& t = c->topo;
  std::vector<int32_t> ks;
  if (k_per_sub) {
    ks.assign(k_per_sub, k_per_sub + t.S);
    for (int s = 0; s < t.S; ++s)
      if (ks[s] < 2 || ks[s] > t.k)
        return c->fail(SFM_EINVAL, "subdomain " + std::to_string(s) + ": levels " + std::to_string(ks[s]) +
                                       " outside [2, " + std::to_string(t.k) + "]");
    if (std::all_of(ks.begin(), ks.end(), [&](int32_t v) { return v == t.k; })) ks.clear();
  }
  SFM_TRY_HIP(c, hipSetDevice(c->device));
  SFM_TRY_HIP(c, hipDeviceSynchronize());
  sfm::drop_shot_graph(c);
  c->dfree(c->k_of_d);
  c->k_of_d = nullptr;
  c->dfree(c->order_d);
  c->order_d = nullptr;
  c->k_of = ks;
  if (!ks.empty()) {
    std::vector<int32_t> order(t.S);
    for (int s = 0; s < t.S; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return ks[a] > ks[b]; });
    hipError_t e = hipSuccess;
    c->k_of_d = alloc_copy(c, ks, &e);
    if (c->k_of_d && e == hipSuccess) c->order_d = alloc_copy(c, order, &e);
    if (!c->k_of_d || !c->order_d) {
      c->dfree(c->k_of_d);
      c->k_of_d = nullptr;
      c->k_of.clear();
      return c->fail(SFM_ENOMEM, "level table: out of device memory");
    }
    SFM_TRY_HIP(c, e);
  }
  // the stepped system changed: states restart from the initial condition, the limit is unknown
  hipLaunchKernelGGL(reset_state_kernel, dim3(1024), dim3(256), 0, nullptr, c->U_d, c->D_d, c->U0_d, nullptr, 0.f,
                     (int64_t)t.S * t.k * c->geo.P16);
  SFM_TRY_HIP(c, hipGetLastError());
  SFM_TRY_HIP(c, sfm::clear_extra_levels(c, c->U_d, 1, nullptr));
  SFM_TRY_HIP(c, sfm::clear_extra_levels(c, c->D_d, 1, nullptr));
  SFM_TRY_HIP(c, sfm::clear_extra_levels(c, c->Us_d, kShotCols, nullptr));
  SFM_TRY_HIP(c, sfm::clear_extra_levels(c, c->Ds_d, kShotCols, nullptr));
  SFM_TRY_HIP(c, hipDeviceSynchronize());
  c->n = 0;
  c->dt_max = -1.0;
  return SFM_OK;
}

sfm_status sfm_get_levels(sfm_ctx c, int32_t* k_per_sub) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!k_per_sub) return c->fail(SFM_EINVAL, "k_per_sub is NULL");
  for (int s = 0; s < c->topo.S; ++s) k_per_sub[s] = c->k_of.empty() ? c->topo.k : c->k_of[s];
  return SFM_OK;
}

sfm_status sfm_reset_state(sfm_ctx c, double dt, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs");
  if (!(dt >= 0.0)) return c->fail(SFM_EINVAL, "dt must be >= 0");
  SFM_TRY_HIP(c, hipSetDevice(c->device));
  const int64_t n = (int64_t)c->topo.S * c->topo.k * c->geo.P16;
  hipLaunchKernelGGL(reset_state_kernel, dim3(1024), dim3(256), 0, as_stream(stream), c->U_d, c->D_d, c->U0_d,
                     c->V0_d, (float)dt, n);
  SFM_TRY_HIP(c, hipGetLastError());
  SFM_TRY_HIP(c, sfm::clear_extra_levels(c, c->U_d, 1, as_stream(stream)));
  SFM_TRY_HIP(c, sfm::clear_extra_levels(c, c->D_d, 1, as_stream(stream)));
  c->n = 0;
  return SFM_OK;
}

}  // extern "C"
