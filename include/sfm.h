/*
 * sfm.h - C ABI of libsfm.so: S-fraction multiscale finite-volume wave propagation
 * (Druskin, Mamonov, Zaslavsky, arXiv 1406.6923) on one AMD MI355X (gfx950).
 *
 * The library implements the paper's Algorithm 1 for the 3-D constant-density
 * acoustic equation u_tt = c^2 Lap(u) on a box of ncell[0] x ncell[1] x ncell[2]
 * cells split into equal box subdomains:
 *
 *   Stage 1 (sfm_build_roms): per subdomain, the fine-grid operator A^alpha, the
 *     6m boundary functions F^alpha (m per face), block Lanczos on (A_+, F)
 *     (polynomial Krylov space, shift sigma = infinity), the S-fraction
 *     coefficients Gamma_j, Gamma-hat_j (eq. "GammaTrans") and the projections
 *     of sources and receivers (eq. "Uj").  Reductions are FP64 on the device.
 *   Stage 2 (sfm_step): explicit leapfrog of the coupled ROMs, eqs. "intrtstep"
 *     (interior layers) and "bdrytstep" (boundary layer, exchange of m numbers
 *     per shared face).  Coefficients stream from HBM in FP32, or BF16 with FP32
 *     accumulation.
 *
 * Conventions shared by every entry point
 *   - Grid nodes are x = h (i, j, l), 0 <= i <= ncell[0] etc.; nodal arrays are
 *     C-ordered [l][j][i] (x fastest); l = 0 is the surface.
 *   - Subdomain alpha = (bz * nsub_y + by) * nsub_x + bx.  Its boundary layer
 *     U_1 has p = 6m entries: face-major (x-, x+, y-, y+, z-, z+), then patch.
 *     ROM state arrays are [S][k][p] (layer j = 1..k, then entry).
 *   - Symmetric coefficient blocks are exchanged as full [p][p] row-major FP64.
 *   - Device pointers are borrowed: the caller keeps them alive and unaliased
 *     until the stream has passed the call.  Host arrays are read during the
 *     call and may be freed afterwards.
 *   - Every call returns an sfm_status.  No exception crosses the ABI.  On an
 *     error the context keeps its previous state and sfm_last_error(ctx)
 *     describes the failure.  Calls that take a stream are asynchronous on it
 *     unless marked "synchronizes".
 *   - A context is bound to the device current at sfm_create and is not
 *     thread-safe; distinct contexts are independent.
 */
#ifndef SFM_H
#define SFM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfm_ctx_s* sfm_ctx;

typedef enum {
  SFM_OK = 0,
  SFM_EINVAL = -1,      /* invalid argument or configuration */
  SFM_EHIP = -2,        /* HIP runtime or library failure (no device, launch error) */
  SFM_ENOMEM = -3,      /* device allocation failed */
  SFM_EBREAKDOWN = -4,  /* block Lanczos breakdown or non-SPD S-fraction level */
  SFM_ESTATE = -5,      /* call out of order (e.g. step before ROMs exist) */
  SFM_EUNSTABLE = -6,   /* time step above the stability limit */
  SFM_ENOCONV = -7      /* an iterative inner solve did not reach its tolerance */
} sfm_status;

typedef enum {
  SFM_PREC_FP32 = 0,         /* coefficient blocks stored FP32 */
  SFM_PREC_BF16_FP32ACC = 1, /* coefficient blocks stored BF16, FP32 accumulation */
  SFM_PREC_FP64 = 2          /* coefficient blocks stored FP64, FP64 products and sums (the
                                state arrays stay FP32): for ROMs whose S-fraction blocks are
                                too ill-conditioned for FP32 storage, e.g. finite-shift ROMs */
} sfm_precision;

typedef struct {
  int32_t ncell[3];      /* cells along x, y, z (nodes = ncell + 1) */
  int32_t sub_cells[3];  /* cells per subdomain edge; ncell[d] % sub_cells[d] == 0, sub_cells >= 2 */
  double h;              /* grid step (metres), > 0 */
  int32_t m;             /* boundary functions per face: m1 x m2 patches, m1 >= m2, m1 - m2 minimal */
  int32_t k;             /* S-fraction levels (blocks of the ROM), 2 <= k, 6mk <= subdomain nodes */
  int32_t precision;     /* sfm_precision */
  int32_t build_batch;   /* subdomains per ROM-build batch (device memory), 0 = automatic */
} sfm_config;

typedef struct {
  int32_t n_subdomains;      /* S */
  int32_t p;                 /* 6m */
  int32_t k;
  int32_t nsrc, nrec;        /* after sfm_build_roms / sfm_load_roms */
  int32_t has_roms;
  int64_t steps_done;        /* n of the current state U^n */
  int64_t coef_bytes;        /* device bytes of the streamed coefficient tiles */
  int64_t coef_bytes_algorithmic;  /* (2k-1) p (p+1)/2 words per subdomain in the stored precision */
  int64_t state_bytes;       /* one [S][k][p] FP32 state array */
  double build_seconds;      /* wall time of the last sfm_build_roms (device work included) */
  int64_t timed_steps;       /* steps launched by sfm_step while timing was enabled */
  double timed_main_ms;      /* summed device time of the step's main kernel over those steps */
  double timed_face_ms;      /* summed device time of the boundary-layer kernel */
  double timed_record_ms;    /* summed device time of the receiver kernel */
  double rho_estimate;       /* last sfm_cfl_dt: power-iteration estimate of rho (a lower bound), 0 if none */
  double rho_bound;          /* last sfm_cfl_dt: certified upper bound on rho, dt_max = 2 / sqrt(rho_bound) */
  int64_t watchdog_checks;   /* state checks made by the sfm_step watchdog since sfm_set_watchdog */
} sfm_info;

/* Validate cfg and allocate a context on the current device.
 * Errors: SFM_EINVAL (bad configuration, checked before any HIP call),
 *         SFM_EHIP (no usable device).  *out is NULL on failure. */
sfm_status sfm_create(const sfm_config* cfg, sfm_ctx* out);

/* As sfm_create with boxes of uneven size (the decomposition of the Introduction needs no equal
 * subdomains): the grid is the tensor product of nbox[0] x nbox[1] x nbox[2] boxes, and along
 * axis d box b has box_cells[nbox[0] + .. + nbox[d-1] + b] cells (each >= 2, adding up to
 * ncell[d]); cfg->sub_cells is ignored.  Neighbours across a face share the whole face, so its
 * m patches match on both sides; p = 6m on every subdomain, and 6mk must not exceed the nodes of
 * the smallest box.  The ROM build groups subdomains of one shape into its batches.
 *   nbox       host, int32 [3]
 *   box_cells  host, int32 [nbox[0] + nbox[1] + nbox[2]]; both NULL selects equal boxes.
 * Errors as sfm_create. */
sfm_status sfm_create_boxes(const sfm_config* cfg, const int32_t* nbox, const int32_t* box_cells, sfm_ctx* out);

/* Release every device buffer owned by ctx (NULL is ignored). */
void sfm_destroy(sfm_ctx ctx);

/* Per-context message of the last failing call ("" if none); valid until the next call on ctx.
 * With ctx == NULL, the message of the last failed sfm_create on this thread. */
const char* sfm_last_error(sfm_ctx ctx);

/* Sizes and counters of ctx.  Never fails for a valid ctx. */
sfm_status sfm_query(sfm_ctx ctx, sfm_info* out);

/* Algorithm 1, Stage 1 (steps 1.1-1.4), entirely on the device: per subdomain the
 * fine-grid operator from the nodal sound speed, the patch basis F, block Lanczos
 * with full two-pass FP64 re-orthogonalisation, the FP64 S-fraction transform,
 * the projections of point sources (s = G Z^T M^{-1/2} e_s) and receivers
 * (r = e_r^T M^{-1/2} Z G^{-1}), and (step 1.4) of optional initial conditions
 * (U(0) = G Z^T M^{1/2} u0, U_t(0) = G Z^T M^{1/2} v0, eq. "Uj").  Sets the state
 * to U^0 = U(0), U^0 - U^{-1} = 0 (see sfm_reset_state for a nonzero v0).
 *   vel_dev   device, float [nz+1][ny+1][nx+1] sound speed at the nodes (> 0)
 *   src_ijk   host, int32 [nsrc][3] source nodes, each strictly inside one subdomain
 *   rec_ijk   host, int32 [nrec][3] receiver nodes; a node on a subdomain boundary
 *             is reconstructed from the lowest-index subdomain that holds it
 *   u0_dev, v0_dev  device, float nodal fields like vel_dev, or NULL for zero
 *   stream    hipStream_t (NULL = default stream)
 * Synchronizes (the build reports breakdowns).  Errors: SFM_EINVAL,
 * SFM_EBREAKDOWN (rank-deficient Lanczos block or non-SPD Gamma_j, j < k),
 * SFM_ENOMEM, SFM_EHIP. */
sfm_status sfm_build_roms(sfm_ctx ctx, const float* vel_dev, int32_t nsrc, const int32_t* src_ijk,
                          int32_t nrec, const int32_t* rec_ijk, const float* u0_dev,
                          const float* v0_dev, void* stream);

/* Stage 1 with the rational projection subspace of a finite shift sigma > 0 (Stage 1
 * section: the Krylov space of the resolvent at one real shift, taken n times, with F
 * added as the coupling requires; the paper's K_n(0) with the shift moved off the null
 * space of a floating subdomain).  Per subdomain:
 *   1. V = orthonormal basis of span{F, (A_+ + sigma)^{-1} F, ..., (A_+ + sigma)^{-(k-1)} F}
 *      from block Lanczos on ((A_+ + sigma I)^{-1}, F) with the same FP64 two-pass
 *      re-orthogonalisation as sfm_build_roms; every shifted solve is a Jacobi-
 *      preconditioned conjugate-gradient iteration, one per column, stopped when
 *      |b - (A_+ + sigma) x| <= cg_rtol |b| (2-norms);
 *   2. the reduced pair (V^T A_+ V, V^T F) is tridiagonalised by block Lanczos
 *      (Algorithm 1, step 1.2); then steps 1.3 and 1.4 as in sfm_build_roms.
 * The result is the ROM whose transfer function interpolates the fine one at s^2 = sigma
 * (to the accuracy of the inner solves).  Arguments as sfm_build_roms, plus
 *   sigma        shift, positive and finite, in the units of A_+ (1/s^2)
 *   cg_rtol      relative residual of every inner solve, 0 < cg_rtol < 1
 *   cg_max_iter  iteration limit of every inner solve (>= 1)
 *   cg_iters     host, may be NULL: the largest iteration count of any inner solve
 * The context must store coefficients in FP64 (SFM_PREC_FP64): every subdomain is floating
 * (Neumann on its box faces), the rational space holds its constant mode, and the last
 * level Gamma_k is singular along it; rounding the blocks to FP32 or BF16 makes it
 * indefinite and the leapfrog diverges.
 * Synchronizes.  Errors: as sfm_build_roms, SFM_EINVAL for a context whose precision is not
 * SFM_PREC_FP64, and SFM_ENOCONV when an inner solve stops at cg_max_iter above cg_rtol (the
 * context then holds no ROMs). */
sfm_status sfm_build_roms_shifted(sfm_ctx ctx, double sigma, double cg_rtol, int32_t cg_max_iter,
                                  const float* vel_dev, int32_t nsrc, const int32_t* src_ijk, int32_t nrec,
                                  const int32_t* rec_ijk, const float* u0_dev, const float* v0_dev,
                                  int32_t* cg_iters, void* stream);

/* Restart from the projected initial conditions with step dt: U^0 = U(0) and
 * U^{-1} = U(0) - dt U_t(0) (first-order start, as the fine-grid leapfrog), n = 0.
 * Zero if the ROMs were built without initial conditions or loaded.  Errors: SFM_ESTATE. */
sfm_status sfm_reset_state(sfm_ctx ctx, double dt, void* stream);

/* Parity hook: install ROMs computed elsewhere instead of building them.
 *   gamma, gamma_hat  host, double [S][k][p][p]; gamma_hat[.][0] must be diagonal
 *   src_vec           host, double [nsrc][k][p] (source projections; may be NULL if nsrc == 0)
 *   rec_rows          host, double [nrec][k][p] (receiver rows; may be NULL if nrec == 0)
 * Face masses C_f = (sum over sides of Gamma-hat_1^{-1})^{-1} (eq. "bdrytstep") are
 * derived from the diagonal of gamma_hat[.][0].  Synchronizes; resets the state. */
sfm_status sfm_load_roms(sfm_ctx ctx, const double* gamma, const double* gamma_hat,
                         int32_t nsrc, const int32_t* src_ijk, const double* src_vec,
                         int32_t nrec, const int32_t* rec_ijk, const double* rec_rows);

/* Copy the FP64 S-fraction coefficients to host arrays double [S][k][p][p] (either may
 * be NULL).  Synchronizes. */
sfm_status sfm_export_roms(sfm_ctx ctx, double* gamma, double* gamma_hat);

/* Copy the FP64 source projections double [nsrc][k][p] and receiver rows
 * double [nrec][k][p] to the host (either may be NULL).  Synchronizes. */
sfm_status sfm_export_projections(sfm_ctx ctx, double* src_vec, double* rec_rows);

/* Stability limit of leapfrog for the coupled ROM (the time stepping of the Stage 2 section):
 * dt_max = 2 / sqrt(rho), rho the largest eigenvalue of M^{-1} K, the step operator with the
 * coefficients as they are stored (FP32, BF16 or FP64).  *dt_max never exceeds that limit:
 *   1. `iters` (>= 10) power iterations of the step operator from a fixed seeded start give an
 *      estimate rho_est <= rho;
 *   2. for mu on a ladder above rho_est (then bisected), every subdomain is tested for
 *      mu M^alpha - K^alpha > 0 by an FP64 block Cholesky factorisation of its block-tridiagonal
 *      S-fraction form on the stored coefficients (pivots must exceed 1e-9 mu); the first mu that
 *      passes everywhere bounds max_alpha lambda_max(K^alpha, M^alpha) >= rho (the coupled
 *      Rayleigh quotient is a mediant of the subdomains'), and dt_max = 2 / sqrt(mu).
 * rho_est and mu are reported in sfm_info.  Leaves the state unchanged.  Synchronizes.
 * Errors: SFM_ESTATE (no ROMs), SFM_EINVAL, SFM_ENOMEM (certificate scratch: 7 p^2 doubles for
 * each of min(S, 2048) subdomains processed together, plus 8 S bytes), SFM_EUNSTABLE (a stored
 * Gamma-hat_j is not positive definite, or nothing up to 1e6 rho_est passes: no time step is
 * stable). */
sfm_status sfm_cfl_dt(sfm_ctx ctx, int32_t iters, double* dt_max, void* stream);

/* Advance the coupled ROMs nsteps leapfrog steps of size dt (Algorithm 1, Stage 2):
 *   U^{n+1} = 2 U^n - U^{n-1} + dt^2 a(U^n, t_n),
 * a from eqs. "intrtstep" and "bdrytstep" with point forcing f_s(t_n).
 *   wavelet_dev  device, float [nsteps][nsrc] source samples f_s(t_n) (NULL iff nsrc == 0)
 *   traces_dev   device, float [nrec][ld]; if not NULL, receiver sample of U^{n+1} for the
 *                i-th step of this call goes to traces_dev[r * ld + i]  (ld >= nsteps)
 * If dt exceeds the last sfm_cfl_dt result (when one was computed) the call fails with
 * SFM_EUNSTABLE before launching anything; so does a failed watchdog check (sfm_set_watchdog).
 * Errors: SFM_ESTATE, SFM_EINVAL, SFM_EUNSTABLE. */
sfm_status sfm_step(sfm_ctx ctx, int32_t nsteps, double dt, const float* wavelet_dev,
                    float* traces_dev, int64_t ld, void* stream);

/* sfm_cfl_dt for callers that cannot allocate device memory (code that must not call hipMalloc,
 * tight serving loops, harnesses that forbid allocation): the same computation and result, with
 * the stability certificate's scratch in a static device array of 64 MiB instead of a per-call
 * allocation (the power iterations use buffers the context allocated at sfm_create).  Calls no
 * hipMalloc or hipFree.  Each device holds its own copy of the array, from the first call on that
 * device until the process ends; every call on a device shares it and leaves its contents behind
 * (nothing in it needs to start at zero), so calls that overlap on one device, from any context or
 * thread, race.  The subdomains processed together are limited to those whose 7 (6m)^2 FP64 work
 * matrices fit in 62 MiB (125 at 6m = 96, 17 at 6m = 256), which only lengthens the certificate:
 * every subdomain's arithmetic is the same in any batch, so the result equals sfm_cfl_dt's.
 * Errors: as sfm_cfl_dt except SFM_ENOMEM; SFM_EINVAL for more than 262,144 subdomains. */
sfm_status sfm_cfl_dt_noalloc(sfm_ctx ctx, int32_t iters, double* dt_max, void* stream);

/* The batched FP64 matrix product the ROM build runs on the FP64 matrix cores (block Lanczos
 * projections and re-orthogonalisation, Cholesky QR, S-fraction products of Stage 1), column-major
 * like BLAS:  C_b = alpha op(A_b) op(B_b) + beta C_b for b < batch, op(X) = X^T when trans_x != 0,
 * op(A) M x K, op(B) K x N, C M x N; X_b starts at X + b stride_x.  All pointers are device memory;
 * C must not overlap A or B.  work (device, work_bytes, may be NULL) holds partial tiles when a long
 * reduction (K in the thousands against a small C) is split over work-groups; the splits are summed
 * in a fixed order, so results are reproducible.  Asynchronous on stream.
 * Errors: SFM_EINVAL (sizes, leading dimensions, missing pointers), SFM_EHIP (launch). */
sfm_status sfm_dgemm_batched(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K, double alpha,
                             const double* A, int64_t lda, int64_t stride_a, const double* B, int64_t ldb,
                             int64_t stride_b, double beta, double* C, int64_t ldc, int64_t stride_c, int32_t batch,
                             double* work, int64_t work_bytes, void* stream);

/* Sustained rate of the FP64 matrix cores that sfm_dgemm_batched runs on, for reading its roofline:
 * `blocks` work-groups of four waves each run `iters` rounds of eight independent 16 x 16 x 4
 * FP64 matrix products on register operands, timed with events on stream.  out: device,
 * double [blocks * 256], written (one value per lane, to keep the products live).
 * *tflops = 2 * 16 * 16 * 4 * 8 * 4 * blocks * iters / seconds / 1e12.  Synchronizes.
 * Errors: SFM_EINVAL, SFM_EHIP. */
sfm_status sfm_probe_fp64_matrix_rate(int32_t blocks, int32_t iters, double* out, double* tflops, void* stream);

/* Run-time stability watchdog of sfm_step.  With every > 0, sfm_step computes ||U^n||_2 (FP64
 * sum over the whole state) after every `every`-th step of a call and after its last step,
 * synchronizes the stream, and stops with SFM_EUNSTABLE when the norm is not finite or exceeds
 * max_norm (> 0; INFINITY checks finiteness only).  The steps done before the failing check stay
 * applied (sfm_info.steps_done counts them).  every = 0 turns the watchdog off (the default).
 * Errors: SFM_EINVAL. */
sfm_status sfm_set_watchdog(sfm_ctx ctx, int32_t every, double max_norm);

/* Receiver samples of the current state: out_dev[r] = r_r . U^{alpha(r), n} (device,
 * float [nrec]).  Errors: SFM_ESTATE. */
sfm_status sfm_record_receivers(sfm_ctx ctx, float* out_dev, void* stream);

/* Apply the coupled step operator without forcing: a_dev = a(u_dev) as in sfm_step
 * (device, float [S][k][p] each; shared boundary entries of u must agree on both sides).
 * Errors: SFM_ESTATE. */
sfm_status sfm_apply_operator(sfm_ctx ctx, const float* u_dev, float* a_dev, void* stream);

/* Per-kernel device timing inside sfm_step and sfm_shots_step.  enable = 0 turns it off;
 * enable = n >= 1 times one step in n (the 1st, (n+1)th, ... step run after this call, counted
 * over both calls): four hipEvents are recorded on the caller's stream around that step's main,
 * face and receiver kernels, and the elapsed times are summed into the timed_* fields of
 * sfm_info (sfm_query synchronizes on the events and reads them; sfm_shots_timing does so for
 * the shot steps).  Every event record between two kernels costs device time of its own, so
 * n > 1 keeps the step rate of the untimed steps.  Enabling resets the sums; the events come
 * from a pool the context keeps until sfm_destroy.  Errors: SFM_EINVAL (enable < 0). */
sfm_status sfm_set_timing(sfm_ctx ctx, int32_t enable);

/* Checkpoint: copy U^n and the increment U^n - U^{n-1} (host, float [S][k][p] each; either
 * may be NULL) and n.  The increment is the stored leapfrog variable, so set_state of
 * what get_state returned resumes bit-identically.  Synchronizes. */
sfm_status sfm_get_state(sfm_ctx ctx, float* u_now, float* u_incr, int64_t* n);

/* Restore a checkpoint written by sfm_get_state (NULL arrays mean zero; levels a subdomain's
 * ROM does not use, see sfm_set_levels, are set to zero).  Synchronizes. */
sfm_status sfm_set_state(sfm_ctx ctx, const float* u_now, const float* u_incr, int64_t n);

/* Per-subdomain ROM size (Algorithm 1, Stage 1 run with its own k on each subdomain).  Block
 * Lanczos and the S-fraction recursions run forward in j, so the first k_s levels of a k-level
 * ROM (Gamma_j, Gamma-hat_j, source projections and receiver rows for j <= k_s) are exactly the
 * k_s-level ROM of the same subdomain: after a build or load with the largest k, this selects
 * k_s levels for subdomain s in every later sfm_step, sfm_apply_operator, sfm_cfl_dt,
 * sfm_shots_step and sfm_adjoint_gradient (levels j > k_s of the states are held at zero, their
 * gradients are zero).
 *   k_per_sub  host, int32 [S], 2 <= k_s <= k; NULL restores k levels everywhere.
 * Restarts both states from the initial condition (n = 0) and forgets the last sfm_cfl_dt
 * result (call it again: the limit grows as levels are dropped).  A new build or load clears
 * the table.  Synchronizes.  Errors: SFM_ESTATE (no ROMs), SFM_EINVAL (k_s out of range; the
 * previous table stays). */
sfm_status sfm_set_levels(sfm_ctx ctx, const int32_t* k_per_sub);

/* As sfm_build_roms (sigma = inf) with a ROM size of its own per subdomain: block Lanczos and the
 * S-fraction recursion run k_per_sub[s] steps on subdomain s (host int32 [S], 2 <= k_s <= k), its
 * later levels are stored as zero, and the level table is installed as by sfm_set_levels.  The
 * build batches subdomains of one box shape and one k_s together, so the cost follows the sizes
 * actually used.  Errors as sfm_build_roms and sfm_set_levels. */
sfm_status sfm_build_roms_levels(sfm_ctx ctx, const int32_t* k_per_sub, const float* vel_dev, int32_t nsrc,
                                 const int32_t* src_ijk, int32_t nrec, const int32_t* rec_ijk, const float* u0_dev,
                                 const float* v0_dev, void* stream);

/* The levels in use per subdomain, host int32 [S] (k everywhere without a table). */
sfm_status sfm_get_levels(sfm_ctx ctx, int32_t* k_per_sub);

/* ------------------------------------------------------------------------------------------
 * Comparators on the same GPU (baselines, not the method's hot path)
 * ------------------------------------------------------------------------------------------ */

/* Leapfrog on the reference fine grid itself (the scheme the ROMs reduce; Introduction, eq.
 * "wave"): M (u^{n+1} - 2u^n + u^{n-1}) / dt^2 = -K u^n + sum_s e_s f_s(t_n) with the node-based
 * 7-point operator and mirrored (Neumann) outer boundary, zero initial state, FP32.
 *   ncell      host, int32[3] cells (nodes = ncell + 1)
 *   vel_dev    device, float nodal sound speed [nz+1][ny+1][nx+1]
 *   wavelet_dev device, float [nsteps][nsrc]
 *   traces_dev device, float [nrec][ld] (may be NULL): u^{n+1} at the receivers after step n
 *   seconds    host, wall time of the step loop (may be NULL)
 * Allocates its own work arrays (3 nodal FP32 fields) for the duration of the call and
 * synchronizes.  Errors: SFM_EINVAL, SFM_EHIP (message in sfm_fdtd_last_error()). */
sfm_status sfm_fdtd_run(const int32_t* ncell, double h, const float* vel_dev, double dt, int32_t nsteps,
                        int32_t nsrc, const int32_t* src_ijk, const float* wavelet_dev, int32_t nrec,
                        const int32_t* rec_ijk, float* traces_dev, int64_t ld, double* seconds, void* stream);

/* Message of the last failing sfm_fdtd_run on this thread. */
const char* sfm_fdtd_last_error(void);

/* The same coupled leapfrog as sfm_step (eqs. "intrtstep", "bdrytstep"), done plainly: one kernel
 * launch per subdomain per step, full row-major FP32 p x p blocks (allocated on first use,
 * (2k-1) p^2 words per subdomain), one thread per row, no receivers.  Advances the context state. */
sfm_status sfm_step_plain(sfm_ctx ctx, int32_t nsteps, double dt, const float* wavelet_dev, void* stream);

/* ---- misfit gradients (discrete adjoint of the leapfrog step) ----
 * For traces t^n = R X^{n+1} of nsteps leapfrog steps from rest (as sfm_step after
 * sfm_reset_state without initial conditions) and a misfit J with trace gradient
 * r^n = dJ/dt^n, returns dJ/dGamma_j and dJ/dGamma-hat_j of every subdomain (the symmetric
 * parts; Gamma-hat_1, the face masses, and the source / receiver projections held fixed, so
 * grad_gamma_hat[.][0] = 0).  The adjoint runs backward with A^T = -K M^{-1} (the step with its
 * two block products swapped) and the residuals injected through the receiver rows; forward
 * states come from checkpoints every checkpoint_every = L steps and a recomputation of each
 * segment but the last, which the first forward pass stores: L >= nsteps runs the forward once.
 *   wavelet_dev      device, float [nsteps][nsrc] (as sfm_step)
 *   grad_traces_dev  device, float [nrec][ld]: r^n in column n (caller's receiver order)
 *   grad_gamma, grad_gamma_hat  host, double [S][k][p][p]
 * Device memory: checkpoints 2 (ceil(nsteps / L) - 1) states, a segment of 2 L + 1 states, 128
 * window states, 64 receiver-injection slices of n_rs k P16 floats, S (2k-1) p^2 doubles and
 * 2 S k p^2 doubles of output staging (state = S k P16 floats).  Requires SFM_PREC_FP32 and
 * receivers.  Synchronizes; the single-shot state is left at rest (n = 0).
 * Errors: SFM_ESTATE, SFM_EINVAL, SFM_EUNSTABLE, SFM_ENOMEM. */
sfm_status sfm_adjoint_gradient(sfm_ctx ctx, int32_t nsteps, double dt, const float* wavelet_dev,
                                const float* grad_traces_dev, int64_t ld, int32_t checkpoint_every,
                                double* grad_gamma, double* grad_gamma_hat, void* stream);

/* ---- many shots through the same ROMs (Stage 2 with a 64-column right-hand side) ----
 * The S-fraction blocks do not depend on the source, so up to 64 shots share one pass over
 * the coefficient stream per step: the block products of eq. "intrtstep" become (6m x 6m) x
 * (6m x 64) products on the matrix cores: FP32 MFMA with SFM_PREC_FP32, FP64 MFMA with
 * SFM_PREC_FP64 (for ROMs whose deep S-fraction levels do not survive FP32 rounding; the shot
 * states stay FP32).  Shot n is driven by source shot_src[n] of the last sfm_build_roms /
 * sfm_load_roms (its own wavelet column) and recorded at every receiver.  Requires FP32 or FP64
 * coefficient storage and 6m <= 112.  The single-shot state (sfm_step) is independent. */

/* Allocate and zero the shot state (U^0 = U^{-1} = 0) for nshot shots (1..64), then time every
 * compiled variant of the shot kernel on it (no sources, dt = 0: the state stays zero) and keep
 * the fastest (see sfm_shots_tuning).
 *   shot_src  host, int32 [nshot]: source index driving each shot (-1: no source), or NULL
 *             for shot n <- source n (then nshot <= nsrc).  A source drives at most one shot.
 * Device memory: U and D of S k P16 x 64 floats each, the boundary exchange, and a receiver
 * staging window of 32 steps x 4 partial sums x nrec x 64 floats.
 * Synchronizes.  Errors: SFM_ESTATE (no ROMs), SFM_EINVAL, SFM_ENOMEM. */
sfm_status sfm_shots_init(sfm_ctx ctx, int32_t nshot, const int32_t* shot_src, void* stream);

/* nsteps leapfrog steps of every shot (as sfm_step, per shot).
 *   wavelet_dev  device, float [nsteps][nshot]: amplitude of each shot's source at t_n
 *   traces_dev   device, float [nshot][nrec][ld] or NULL: receiver samples, column n = step n
 * Errors: SFM_ESTATE (no shot state), SFM_EINVAL, SFM_EUNSTABLE (dt above sfm_cfl_dt's limit). */
sfm_status sfm_shots_step(sfm_ctx ctx, int32_t nsteps, double dt, const float* wavelet_dev, float* traces_dev,
                          int64_t ld, void* stream);

/* hipGraph replay of the shot step loop.  With enable = 1 (the default) sfm_shots_step captures
 * one window of 32 steps (main, boundary and receiver kernels of each step, the window's trace
 * flush and a step-counter increment) into a graph once per (wavelet_dev, traces_dev, ld, dt,
 * level table, ROMs) and replays it floor(nsteps / 32) times (calls of fewer than 64 steps, and
 * calls with per-kernel timing on, launch every kernel); the kernels of a replay add a device
 * step counter to their relative step, and the remaining steps are launched directly.  Results
 * are bit-identical to enable = 0.  enable < 0 only queries.  *replays (may be NULL): windows
 * replayed so far.  Capture runs on a stream of the context's own (default priority); replays
 * go to the caller's stream. */
sfm_status sfm_shots_graph(sfm_ctx ctx, int32_t enable, int64_t* replays);

/* Copy the shot state U^n and D = U^n - U^{n-1} to / from host arrays float [S][k][p][nshot].
 * Synchronize.  Errors: SFM_ESTATE, SFM_EINVAL. */
sfm_status sfm_shots_get_state(sfm_ctx ctx, float* u_host, float* d_host);
sfm_status sfm_shots_set_state(sfm_ctx ctx, const float* u_host, const float* d_host);

/* Autotuner result of the last sfm_shots_init: *chosen_waves = the register budget (minimum
 * waves per SIMD) of the chosen variant; ms (host, double [2 cap]) = {waves, ms per step} of
 * each variant (up to cap; ms < 0 for a variant whose work-group limit, prefetch capacity or LDS
 * is below this 6m, which is not run); *count = number of variants.  The variants, in this
 * order: one work-group of 64 shots per subdomain at two register budgets, two work-groups of 32
 * shots per subdomain, and the first with two block buffers in LDS (the next block expanded while
 * the current one multiplies).  Errors: SFM_ESTATE. */
sfm_status sfm_shots_tuning(sfm_ctx ctx, int32_t* chosen_waves, double* ms, int32_t cap, int32_t* count);

/* Use shot-kernel variant `variant` (the order of sfm_shots_tuning; every variant computes the
 * same step) instead of the autotuner's choice, or go back to that choice with variant = -1; for
 * checking each variant against the others and for timing.  Lasts until the next sfm_shots_init.
 * Errors: SFM_ESTATE (no sfm_shots_init), SFM_EINVAL (out of range, or the variant's work-group
 * limit or prefetch capacity is below this 6m). */
sfm_status sfm_shots_select(sfm_ctx ctx, int32_t variant);

/* Device times of the shot kernels summed over the shot steps timed while sfm_set_timing was
 * on (one in n, as set there): *timed_steps, ms3 = {main, face, record}; then resets the
 * counters.  Synchronizes on the last recorded event.  Errors: SFM_EHIP. */
sfm_status sfm_shots_timing(sfm_ctx ctx, int64_t* timed_steps, double* ms3);

/* ------------------------------------------------------------------------------------------
 * Learned ROM surrogate network (a model of the many ROM builds FWI needs; Introduction)
 * ------------------------------------------------------------------------------------------
 * A 3D CNN: four 3x3x3 convolutions of stride 2 and zero padding 1 (n -> (n - 1) / 2 + 1 nodes
 * per axis), each with bias and ReLU, `channels` channels, then a dense head to n_out outputs.
 * Every product runs on the bf16 matrix cores with FP32 accumulation (operands rounded to
 * bfloat16, nearest-even); activations, gradients, master weights and Adam moments are FP32.
 * Layouts: inputs float [batch][n_in][n_in][n_in]; activations channels-last; the flat FP32
 * parameter vector is W1 b1 W2 b2 W3 b3 W4 b4 Wd bd with conv weights [co][t][ci] (tap
 * t = 9 dz + 3 dy + dx) and the dense weights [n_out][features] over the last activation in
 * [z][y][x][channel] order.  A net is bound to the current device; calls on one net do not
 * overlap.  Errors: SFM_EINVAL (bad sizes), SFM_ENOMEM, SFM_EHIP; message in sfm_cnn_last_error. */
typedef struct sfm_cnn_s* sfm_cnn;

/* Allocate a net for batches up to max_batch; weights He-initialised from seed (biases 0). */
sfm_status sfm_cnn_create(int32_t n_in, int32_t channels, int32_t n_out, int32_t max_batch, uint64_t seed,
                          sfm_cnn* out);
void sfm_cnn_destroy(sfm_cnn net);
/* Last error message of net (net == NULL: of the last failed sfm_cnn_create on this thread). */
const char* sfm_cnn_last_error(sfm_cnn net);
/* *n_params = parameter count, *features = inputs of the dense head, nodes5 (host int32 [5]) =
 * nodes per axis of the input and of each activation, dims4 (host int32 [4]) = {n_in, channels,
 * n_out, max_batch}; any may be NULL. */
sfm_status sfm_cnn_info(sfm_cnn net, int64_t* n_params, int32_t* features, int32_t* nodes5, int32_t* dims4);
/* Copy the flat parameters to get_host and/or from set_host (host float [n_params]; either may be
 * NULL; setting clears the Adam moments).  Synchronizes. */
sfm_status sfm_cnn_params(sfm_cnn net, float* get_host, const float* set_host);
/* y_dev (device float [batch][n_out], may be NULL) = net(x_dev) (device float
 * [batch][n_in^3]); x_dev must stay valid until a following sfm_cnn_backward. */
sfm_status sfm_cnn_forward(sfm_cnn net, const float* x_dev, int32_t batch, float* y_dev, void* stream);
/* Parameter gradients of sum(dy * y) for the last forward pass into grad_dev (device float
 * [n_params], flat layout); dy_dev device float [batch][n_out].  Errors: SFM_ESTATE (no forward). */
sfm_status sfm_cnn_backward(sfm_cnn net, const float* dy_dev, float* grad_dev, void* stream);
/* Input gradient: dx_dev (device float [batch][n_in^3]) = gradient of sum(dy * y) with respect to
 * the inputs of the last forward pass, y as sfm_cnn_forward returns it (with the output scale of
 * sfm_cnn_fit_scale when one is set); dy_dev device float [batch][n_out].  The same bf16 products
 * as sfm_cnn_backward, the first convolution's data gradient included; no parameter gradients.
 * Errors: SFM_ESTATE (no forward), SFM_EINVAL (NULL pointers). */
sfm_status sfm_cnn_input_grad(sfm_cnn net, const float* dy_dev, float* dx_dev, void* stream);
/* Output scale: per output, the mean and standard deviation (1 for a constant output) of
 * target_dev (device float [n_samples][n_out]); afterwards the net is trained on (target - mean)
 * / sd and sfm_cnn_forward returns mean + sd * (net output).  mean_host / sd_host (host float
 * [n_out], may be NULL) receive the scale. */
sfm_status sfm_cnn_fit_scale(sfm_cnn net, const float* target_dev, int64_t n_samples, float* mean_host,
                             float* sd_host, void* stream);
/* Train on n_samples pairs (x_dev [n_samples][n_in^3], target_dev [n_samples][n_out], device):
 * `epochs` passes in a seeded shuffled order, batches of `batch` (a final partial batch is
 * dropped), loss = mean squared error, Adam (beta 0.9 / 0.999, eps 1e-8, learning rate lr).
 * loss_per_epoch (host double [epochs], may be NULL): mean batch loss of each epoch.  Synchronizes
 * once per batch. */
sfm_status sfm_cnn_train(sfm_cnn net, const float* x_dev, const float* target_dev, int64_t n_samples,
                         int32_t batch, int32_t epochs, float lr, uint64_t seed, double* loss_per_epoch,
                         void* stream);

/* ------------------------------------------------------------------------------------------
 * Learned ROMs with block Lanczos as judge and fallback
 * ------------------------------------------------------------------------------------------
 * The network sees a subdomain's log(c / 3000 m/s) on its (n+1)^3 nodes ([z][y][x]; equal cubic
 * subdomains only) and predicts the upper triangles (row-major, i <= j) of Gamma_1..Gamma_k then
 * Gamma-hat_1..Gamma-hat_k: n_out = 2 k p(p+1)/2. */

/* Network inputs of every subdomain: x_dev device float [S][(n+1)^3] from vel_dev (as in
 * sfm_build_roms).  Errors: SFM_EINVAL (uneven or non-cubic boxes).  Synchronizes. */
sfm_status sfm_rom_inputs(sfm_ctx ctx, const float* vel_dev, float* x_dev, void* stream);

/* Training targets from the current ROMs: t_dev device float [S][n_out].  Synchronizes. */
sfm_status sfm_rom_targets(sfm_ctx ctx, float* t_dev, void* stream);

/* err_host[s] (host double [S]) = max over the 8 Laplace frequencies s_f = 2 pi f_peak {1/4, 1/2,
 * 3/4, 1, 3/2, 2, 5/2, 3} of ||M_a(s_f) - M(s_f)||_F / ||M(s_f)||_F, where M is the matrix
 * S-fraction NtD map (Stage 2 section) of the current ROM of subdomain s and M_a that of the
 * blocks coef_dev (device double [S][2][k][p][p], Gamma then Gamma-hat), evaluated in FP64 on
 * the device (Gauss-Jordan inverses with partial pivoting; a singular block gives +inf).
 * Requires 6m <= 64.  Synchronizes. */
sfm_status sfm_ntd_error(sfm_ctx ctx, const double* coef_dev, double f_peak, double* err_host, void* stream);

/* The network's blocks for every subdomain: coef_dev (device double [S][2][k][p][p], Gamma then
 * Gamma-hat, symmetric) from the predicted upper triangles of each subdomain's sound speed in
 * vel_dev (as sfm_build_roms), with Gamma-hat_1 (the face masses) copied from the current ROMs.
 * Errors: SFM_ESTATE (no ROMs), SFM_EINVAL (sizes as sfm_build_roms_surrogate, NULL pointers),
 * SFM_ENOMEM, SFM_EHIP.  Synchronizes. */
sfm_status sfm_surrogate_predict(sfm_ctx ctx, sfm_cnn net, const float* vel_dev, double* coef_dev, void* stream);

/* Learned ROM build: block Lanczos ROMs of every subdomain (as sfm_build_roms without initial
 * conditions; they judge and back up the network), the network's predictions of every
 * subdomain's blocks (Gamma-hat_1, the face masses, always taken from Lanczos), the NtD judge
 * above, and the prediction kept where its error is <= tol and the subdomain holds no source or
 * receiver.  accepted (host int32 [S]), ntd_err (host double [S]) and seconds (host double [4]:
 * Lanczos, network, judge, repack) may be NULL.  Afterwards the context steps the mixed ROMs
 * (call sfm_cfl_dt again).  Errors as sfm_build_roms, SFM_EINVAL for a network whose input or
 * output size does not match (n+1 nodes, 2 k p(p+1)/2 outputs) or 6m > 64.  Synchronizes. */
sfm_status sfm_build_roms_surrogate(sfm_ctx ctx, sfm_cnn net, double tol, double f_peak, const float* vel_dev,
                                    int32_t nsrc, const int32_t* src_ijk, int32_t nrec, const int32_t* rec_ijk,
                                    int32_t* accepted, double* ntd_err, double* seconds, void* stream);

/* Velocity gradient through the surrogate (the FWI use of the Introduction): for a misfit J that
 * depends on the blocks, with block gradients grad_gamma / grad_gamma_hat (host double
 * [S][k][p][p], as sfm_adjoint_gradient returns them), grad_vel_dev (device float, nodes as
 * vel_dev) = dJ/dc where the blocks are taken as the network's prediction from c: the chain
 * through the prediction's upper triangles (an off-diagonal output sets two entries and collects
 * both gradients; Gamma-hat_1 comes from Lanczos and collects none), the network (input gradient
 * as sfm_cnn_input_grad), the input log(c / 3000 m/s) (factor 1 / c), and every subdomain box
 * that holds the node.  Equal cubic subdomains; the network's sizes as in
 * sfm_build_roms_surrogate.  Runs the network forward again on every subdomain in batches of its
 * max_batch.  Errors: SFM_EINVAL (sizes, NULL pointers), SFM_ENOMEM, SFM_EHIP.  Synchronizes. */
sfm_status sfm_surrogate_velocity_gradient(sfm_ctx ctx, sfm_cnn net, const float* vel_dev, const double* grad_gamma,
                                           const double* grad_gamma_hat, float* grad_vel_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SFM_H */
