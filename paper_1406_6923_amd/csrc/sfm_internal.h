// Internal declarations of libsfm: context, device layouts and kernel launchers.
//
// Layout of the streamed coefficient blocks ("tiles")
// ---------------------------------------------------
// Every symmetric p x p block (Gamma_j or Gamma-hat_j) is zero-padded to
// P16 = 16 * nt rows and cut into 16 x 16 tiles.  Only tiles on or above the
// diagonal are stored, each in "wrapped diagonal" order: for a tile at block
// rows 16I.. and columns 16J.., lane i (0..15) holds W_t[i] = A(16I + i, 16J + (i + t) mod 16).
//   * off-diagonal tile (I < J): t = 0..15, 256 words, stored [v][lane][e] with t = e v + i,
//     e = 16 bytes / word size (4 FP32, 8 BF16, 2 FP64), so each load instruction of a
//     16-lane row reads one contiguous 256-byte segment;
//   * diagonal tile (I = J): t = 0..7 in the tile, 128 words in the same [v][lane][e]
//     order; its t = 8 half-diagonal (16 lanes,
//     each entry present twice) sits in the block's tail, [I][lane], after all tiles, padded
//     to whole 128-byte lines.  Every tile then starts on a 128-byte line of HBM: a stream
//     whose rows start 64 bytes into a line reads about 10% slower.
// The symmetric product y = A x then needs each stored word once: W_t[i] multiplies
// x_J[i + t] into y_I[i], and, rotated by t lanes, x_I[c - t] into y_J[c] (DPP row
// rotations inside a 16-lane row).
// Tiles are grouped into "jobs" of one or two tile strips: job g covers strip g and
// strip nt - 1 - g (diagonal tile first, then the tiles to its right), so every job of
// an even-nt block holds nt + 1 tiles.  A block is the concatenation of its jobs and a
// subdomain stream is [Gamma_1 .. Gamma_k, Gamma-hat_2 .. Gamma-hat_k], each block being
// [job 0 .. job npairs-1][tail].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "sfm.h"

// Launch checks of the debug build (SFM_DEBUG): before a kernel is launched, the host verifies
// that shapes, grids and buffer extents match what the kernel's indexing assumes, and aborts with
// the failed condition otherwise.  Compiled out of the release build.
#ifdef SFM_DEBUG
#include <cstdio>
#include <cstdlib>
#define SFM_DCHECK(cond)                                                                         \
  do {                                                                                           \
    if (!(cond)) {                                                                               \
      std::fprintf(stderr, "SFM_DEBUG: launch check failed: %s (%s:%d)\n", #cond, __FILE__, __LINE__); \
      std::abort();                                                                              \
    }                                                                                            \
  } while (0)
#else
#define SFM_DCHECK(cond) \
  do {                   \
  } while (0)
#endif

namespace sfm {

constexpr int kTile = 16;
constexpr int kDiagWords = 128;        // t = 0..7 of a diagonal tile
constexpr int kHalfDiagWords = 16;     // t = 8 of a diagonal tile, in the block tail
constexpr int kOffWords = 256;
constexpr int kLineBytes = 128;
constexpr int kStepThreads = 256;      // 16 rows of 16 lanes per subdomain work-group
constexpr int kMaxNt = 16;             // p <= 256
constexpr int kShotCols = 64;                  // shots per multi-shot state row (the MFMA N dimension)
constexpr size_t kDefaultLdsBytes = 65536;     // dynamic LDS available without a kernel attribute
constexpr size_t kMaxLdsBytes = 163840;        // LDS of one CU (gfx950), the work-group limit

// Bytes of one stored coefficient word.
inline int tile_elem_bytes(int precision) {
  return precision == SFM_PREC_BF16_FP32ACC ? 2 : precision == SFM_PREC_FP64 ? 8 : 4;
}

// Geometry of the tile stream of one block.
struct TileGeometry {
  int p = 0, P16 = 0, nt = 0, npairs = 0, nslots = 0;
  int64_t words_per_block = 0;           // in stored elements (4 bytes FP32, 2 bytes BF16)
  int32_t job_off[kMaxNt / 2 + 1] = {};   // word offset of job g inside a block
  int32_t tail_off = 0;                   // word offset of the half-diagonals [nt][16]

  void init(int p_, int elem_bytes);
  // (row, col) of every stored word of a block, in stream order (row, col may be >= p: padding).
  void word_map(std::vector<int32_t>& rows, std::vector<int32_t>& cols, int elem_bytes) const;
};

// Decomposition of the global box into a tensor product of boxes and their faces.
struct Topology {
  int ncell[3] = {}, nsub[3] = {};
  std::vector<int32_t> cut[3];           // per axis: box planes 0 = x_0 < ... < x_nsub = ncell
  int S = 0, m = 0, m1 = 0, m2 = 0, p = 0, k = 0;
  int64_t N_max = 0;                     // nodes of the largest subdomain
  std::vector<int32_t> nbr;              // [S][6], -1 = outer face

  // box_cells: per axis the cell counts of its boxes (nbox[d] of them), or null for equal boxes
  // of cfg.sub_cells cells.  Returns "" or an error message.
  std::string init(const sfm_config& cfg, const int32_t* nbox = nullptr, const int32_t* box_cells = nullptr);
  int index(int bx, int by, int bz) const { return (bz * nsub[1] + by) * nsub[0] + bx; }
  void box_of(int s, int b[3]) const;
  // Subdomain holding global node (i, j, l): strictly inside if strict, else lowest index.
  int owner(int i, int j, int l, bool strict) const;
  void origin(int s, int o[3]) const;
  void cells(int s, int c[3]) const;     // cells per edge of subdomain s
};

struct StepParams {
  const void* tiles;          // [S][2k-1][words_per_block]
  int64_t words_per_sub;
  int64_t words_per_block;
  int32_t job_off[kMaxNt / 2 + 1];
  int32_t tail_off;
  int S, k, P16, nt, npairs, nslots;
  float* U;                   // [S][k][P16] state U^n (updated in place for layers 2..k)
  float* D;                   // [S][k][P16] increment U^n - U^{n-1} (step mode)
  const float* Uin;           // operator mode input (may alias nothing else)
  float* Aout;                // operator mode output
  float* exch;                // [S][P16] boundary-layer fluxes phi_1 (step 2.1 exchange)
  const int32_t* src_off;     // [S+1] CSR of sources interior to each subdomain
  const int32_t* src_ids;
  const float* src_vec;       // [nsrc][k][P16]
  const float* wavelet;       // [nsteps][nsrc] (row `step`)
  int nsrc;
  int64_t step;
  float dt2;
  int mode;                   // 0 = leapfrog step, 1 = apply operator
  const int32_t* k_of;        // optional [S]: levels of each subdomain's ROM (<= k; null: all k)
  const int32_t* order;       // optional [S]: subdomain of each work-group (longest ROMs first)
  float* kx_out;              // optional [S][k][P16]: the interior flux differences phi_j - phi_{j-1}
  float* u_out;               // optional [S][k][P16]: a copy of the state U^n the step starts from
                              // (j >= 2) of this step, for the adjoint's recomputed segments
  float* hist;                // receiver-subdomain state history [Tw][n_rs][k][P16] (or null)
  const int32_t* hist_slot;   // [S] history slot of each subdomain, -1 if it holds no receiver
  int64_t hist_off;           // offset of this step's time slot in hist
};

struct FaceParams {
  int S, k, P16, p, m;
  const int32_t* nbr;         // [S][6]
  const float* C;             // [S][P16] combined face mass
  const float* exch;
  const int32_t* sw_off;      // [S+1] CSR of layer-1 source weights
  const int32_t* sw_q;
  const int32_t* sw_src;
  const float* sw_w;
  const float* wavelet;
  int nsrc;
  int64_t step;
  float dt2;
  float* U;
  float* D;
  float* Aout;
  int mode;
  float* hist;
  const int32_t* hist_slot;
  int64_t hist_off;
};

// Receivers are stored sorted by subdomain (CSR over the receiver subdomains); perm maps the
// sorted position back to the caller's receiver index.
struct RecParams {
  int nrec, k, P16;
  const int32_t* rec_sub;     // [nrec] subdomain of each sorted receiver
  const int32_t* perm;        // [nrec] caller index of each sorted receiver
  const float* rows;          // [nrec][k][P16] (sorted)
  const float* U;             // [S][k][P16]
  float* out;                 // out[perm[r] * ld + col]
  int64_t ld, col;
};

// traces[perm[r]][col0 + t] = rows[r] . hist[t][slot(r)] for t < w (one GEMM per window).
struct RecWindowParams {
  int n_rs, k, P16, w;
  const int32_t* rs_off;      // [n_rs + 1] CSR of sorted receivers per receiver subdomain
  const int32_t* perm;
  const float* rows;
  const float* hist;          // [Tw][n_rs][k][P16]
  float* traces;
  int64_t ld, col0;
};
constexpr int kHistWindow = 64;

hipError_t launch_step_main(const StepParams& prm, int precision, hipStream_t st);
hipError_t launch_step_face(const FaceParams& prm, hipStream_t st);
hipError_t launch_record(const RecParams& prm, hipStream_t st);
hipError_t launch_record_window(const RecWindowParams& prm, hipStream_t st, int max_per_slot);
hipError_t launch_pack(const double* blocks, int64_t nblocks_total, int blocks_per_sub_in,
                       int k, int p, const TileGeometry& geo, const int32_t* wrow,
                       const int32_t* wcol, void* tiles, int precision, int S, hipStream_t st);
hipError_t launch_pad_rows(const double* src, int64_t nrows, int p, int P16, float* dst,
                           hipStream_t st);
size_t step_lds_bytes(const StepParams& prm, int precision);
hipError_t launch_gather_rows(const double* src, const int32_t* idx, int n, int64_t width, double* dst,
                              hipStream_t st);
// out: device double [kNormScratch0 + 1024]; out[0] = ||x||^2, the rest is scratch.
constexpr int kNormScratch0 = 64;
hipError_t launch_norm2(const float* x, int64_t n, double* out, hipStream_t st);
hipError_t launch_scale(const float* x, int64_t n, const double* num, float* y, hipStream_t st);

sfm_status locate_points(sfm_ctx c, int32_t nsrc, const int32_t* src_ijk, int32_t nrec, const int32_t* rec_ijk,
                         std::vector<int32_t>& src_sub, std::vector<int32_t>& src_local,
                         std::vector<int32_t>& rec_sub, std::vector<int32_t>& rec_local);
sfm_status finalize_roms(sfm_ctx c, const std::vector<double>& H, const std::vector<int32_t>& src_sub,
                         const std::vector<double>& src_vec_host, const std::vector<int32_t>& rec_sub,
                         hipStream_t st);
void release_roms(sfm_ctx c);
void release_shots(sfm_ctx c);
void drop_shot_graph(sfm_ctx c);   // destroys the cached shot-window graph (synchronizes)
// Fold the recorded step events `ev` (4 per timed step) into ms3 = {main, face, record} and
// *steps, then return the events to the context's pool.  Synchronizes on the last event.
sfm_status drain_events(sfm_ctx c, std::vector<hipEvent_t>& ev, double* ms3, int64_t* steps);
// Zero the levels j >= k_of[s] of a [S][k][P16][cols] state (no-op without a level table).
hipError_t clear_extra_levels(sfm_ctx c, float* X, int cols, hipStream_t st);
sfm_status forward_step(sfm_ctx c, double dt, const float* wavelet_row, float* kx_out, float* u_out,
                        hipStream_t st);
StepParams step_params(sfm_ctx c);
// Batched FP64 kernels of the ROM build (dgemm.hip), column-major like BLAS:
//   C_b = alpha op(A_b) op(B_b) + beta C_b, op(X) = X^T when tX.  work (work_bytes) holds the partial
//   tiles of split reductions (a split is only used when they fit; kMaxGemmSplit splits at most).
constexpr int kMaxGemmSplit = 16;
constexpr size_t kGemmWorkBytes = (size_t)8 * 4096 * 96 * 96;   // 4096 partial tiles of 96 x 96
hipError_t dgemm_batched(bool tA, bool tB, int M, int N, int K, double alpha, const double* A, int64_t lda,
                         int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, double* C, int64_t ldc,
                         int64_t sC, int batch, hipStream_t st, double* work, size_t work_bytes);
//   X_b = L_b^{-1}, L lower triangular non-unit p x p (ld p); X's strict upper triangle is zeroed.
hipError_t trtri_lower_batched(const double* L, int64_t sL, double* X, int64_t sX, int p, int batch, hipStream_t st);
//   B_b <- alpha op(L_b)^{-1} B_b, L lower triangular non-unit, B p x p (ld p each).
hipError_t trsm_lower_batched(bool trans, double alpha, const double* L, int64_t sL, double* B, int64_t sB, int p,
                              int batch, hipStream_t st);

// a = a(u) of the coupled scheme without forcing, [S][k][P16] each (step kernels in operator mode).
hipError_t apply_operator(sfm_ctx c, const float* u, float* a, hipStream_t st);

}  // namespace sfm

// ----------------------------------------------------------------------------- context
struct sfm_ctx_s {
  sfm_config cfg{};
  sfm::Topology topo;
  sfm::TileGeometry geo;
  int device = 0;
  std::string err;

  // device buffers (owned)
  std::vector<void*> owned;
  int32_t* nbr_d = nullptr;
  void* tiles_d = nullptr;
  double* coef64_d = nullptr;       // [S][2][k][p][p]: Gamma_j at [.][0], Gamma-hat_j at [.][1]
  size_t tile_elem = 4;             // bytes per streamed coefficient word
  uint32_t* wmap_d = nullptr;       // [words_per_block]: (row << 16) | col of every stored word
  float* C_d = nullptr;             // [S][P16]
  float* U_d = nullptr;             // [S][k][P16]
  float* D_d = nullptr;
  float* exch_d = nullptr;          // [S][P16]
  float* U0_d = nullptr;            // projected initial conditions (or null)
  float* V0_d = nullptr;
  // sources
  int nsrc = 0;
  std::vector<int32_t> src_sub;
  float* src_vec_d = nullptr;       // [nsrc][k][P16]
  double* src_vec64_d = nullptr;    // [nsrc][k][p]
  int32_t* src_off_d = nullptr;
  int32_t* src_ids_d = nullptr;
  int32_t* sw_off_d = nullptr;
  int32_t* sw_q_d = nullptr;
  int32_t* sw_src_d = nullptr;
  float* sw_w_d = nullptr;
  // receivers
  int nrec = 0;
  int32_t* rec_sub_d = nullptr;     // sorted receivers: subdomain
  int32_t* rec_perm_d = nullptr;    // sorted receivers: caller index
  float* rec_rows_d = nullptr;      // [nrec][k][P16], sorted by subdomain
  int n_rs = 0;                     // subdomains that hold receivers
  int rs_max = 0;                   // most receivers in one subdomain
  int32_t* rs_off_d = nullptr;      // [n_rs + 1]
  int32_t* hist_slot_d = nullptr;   // [S]
  float* hist_d = nullptr;          // [kHistWindow][n_rs][k][P16]
  float* plain_blocks_d = nullptr;  // comparator only: full FP32 blocks [S][2k-1][p][p]
  double* rec_rows64_d = nullptr;   // [nrec][k][p]
  // many shots (sfm_shots_*): state [S][k][P16][64], exchange [S][P16][64]
  int nshot = 0;
  float* Us_d = nullptr;
  float* Ds_d = nullptr;
  float* exch_s_d = nullptr;
  int32_t* src_shot_d = nullptr;    // [nsrc] shot driven by each source, -1 if none
  float* rec_stage_d = nullptr;     // receiver partial samples of the current window [32][4][nrec][64]
  int64_t shots_n = 0;
  int64_t shots_timed = 0;
  double shots_ms[3] = {0, 0, 0};   // main, face, record
  int shots_variant = 0;            // main-kernel variant in use
  int shots_tuned = 0;              // the variant the autotuner chose
  double shots_tune_ms[4] = {0, 0, 0, 0};
  // hipGraph of one receiver window of shot steps (replayed by sfm_shots_step)
  bool shots_graph = true;
  int64_t* shot_base_d = nullptr;   // device step counter read by the replayed kernels
  hipStream_t cap_stream = nullptr; // capture stream (the caller's may be the null stream)
  hipGraphExec_t shot_exec = nullptr;
  std::vector<uint64_t> shot_exec_key;
  int64_t shots_replays = 0;
  // scratch
  double* red_d = nullptr;          // reduction scratch
  float* work_a_d = nullptr;        // [S][k][P16] operator scratch
  float* work_b_d = nullptr;

  int32_t* k_of_d = nullptr;        // [S] per-subdomain levels (null: every subdomain uses k)
  int32_t* order_d = nullptr;       // [S] subdomains by decreasing levels (launch order of the shot
                                    // kernel: the longest first, so the grid's tail is short)
  std::vector<int32_t> k_of;        // host copy

  bool has_roms = false;
  int64_t n = 0;
  double dt_max = -1.0;
  double rho_est = 0.0;             // last sfm_cfl_dt: power-iteration estimate
  double rho_bound = 0.0;           // last sfm_cfl_dt: certified bound
  int32_t wd_every = 0;             // sfm_step watchdog: check every wd_every steps (0 = off)
  double wd_max_norm = 0.0;
  int64_t wd_checks = 0;
  double build_seconds = 0.0;
  // per-kernel timing of sfm_step and sfm_shots_step (events recorded on the caller's stream)
  bool timing = false;
  int32_t timing_every = 1;         // time one step in timing_every (counted from the enable call)
  int64_t timing_seen = 0;          // steps run since timing was enabled
  std::vector<hipEvent_t> ev;       // 4 events per timed step: main start, face start, record start, end
  std::vector<hipEvent_t> shot_ev;  // the same for the shot steps
  std::vector<hipEvent_t> ev_pool;  // created once, reused after every drain
  int64_t timed_steps = 0;
  double timed_ms[3] = {0, 0, 0};

  // Should the step about to run be timed?  Advances the step count.
  bool time_this_step() {
    if (!timing) return false;
    return timing_seen++ % timing_every == 0;
  }
  // Four events for one timed step, appended to `to` (from the pool when it has them).
  hipError_t take_events(std::vector<hipEvent_t>& to) {
    for (int q = 0; q < 4; ++q) {
      hipEvent_t e = nullptr;
      if (!ev_pool.empty()) {
        e = ev_pool.back();
        ev_pool.pop_back();
      } else {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
      }
      to.push_back(e);
    }
    return hipSuccess;
  }

  sfm_status fail(sfm_status code, const std::string& msg) {
    err = msg;
    return code;
  }
  void* dalloc(size_t bytes, hipError_t* e);
  void dfree_all();
  void dfree(void* p);
};
