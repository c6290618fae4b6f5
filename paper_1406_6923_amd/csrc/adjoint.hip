// Discrete adjoint of the leapfrog step (Stage 2) and misfit gradients with respect to the
// S-fraction blocks, for full-waveform-inversion style use (Introduction, motivation).
//
// Forward (as sfm_step): X^{n+1} = 2 X^n - X^{n-1} + dt^2 (A X^n + b f^n), A = -M^{-1} K, with
// M^{-1} = Gamma-hat_j on interior layers and C_f on the shared boundary entries, K = sum over
// subdomains of D^T Gamma D ((D U)_j = U_{j+1} - U_j, U_{k+1} = 0); trace n = R X^{n+1}.
// For the misfit J with trace gradient r^n = dJ/dt^n the adjoint runs backward,
//   psi^m = R^T r^{m-1} + 2 psi^{m+1} - psi^{m+2} + dt^2 A^T psi^{m+1},  A^T = -K M^{-1},
// in increment form F^m = F^{m+1} + dt^2 A^T psi^{m+1} + R^T r^{m-1}, psi^m = psi^{m+1} + F^m, and
//   dJ/dGamma_j     = -dt^2 sum_m sym((D z^{m+1})_j (D X^m)_j^T),   z = M^{-1} psi,
//   dJ/dGamma-hat_j =  dt^2 sum_m sym(psi_j^{m+1} (-K X^m)_j^T),    j >= 2.
// Gamma-hat_1 (face masses) and the source / receiver projections are held fixed.
//
// A^T is the step kernel with its two phases swapped: adj_main_kernel first forms z_j =
// Gamma-hat_j psi_j (blocks k.. of the tile stream) and z_1 = C psi_1, then the fluxes
// phi_j = Gamma_j (z_{j+1} - z_j) and the interior update; adj_face_kernel sums phi_1 over both
// sides of a shared entry (no C: it was applied to z).  The forward states come from checkpoints
// every L steps and a recomputation of each segment (U^m and (-K X^m) stored per step; the last
// segment is stored by the first forward pass, so L >= nsteps runs the forward once).  The
// receiver injections R^T r of 64 adjoint steps come from one tiled product per window, and the
// gradient pairs of up to 64 adjoint steps are accumulated by one product per block into FP64,
// symmetric part only.
#include <algorithm>
#include <string>
#include <vector>

#include "tile_ops.h"

namespace sfm {
namespace {

constexpr int kGradWindow = 64;   // adjoint steps per gradient accumulation
constexpr int kInjWindow = 64;    // adjoint steps per receiver-injection product

struct AdjParams {
  StepParams geo;              // tile stream and block geometry
  float* Psi;                  // [S][k][P16]  psi^{m+1} -> psi^m
  float* F;                    // [S][k][P16]  psi^m - psi^{m+1}
  const float* C;              // [S][P16] combined face masses
  float* exch;                 // [S][P16] phi_1 of the adjoint fluxes
  const float* gslot;          // [n_rs][k][P16] R^T r of this step on each receiver subdomain (or null)
  const int32_t* slot_of;      // [S] receiver-subdomain slot or -1
  float* win_dz;               // window slot [S][k][P16]: (D z^{m+1})_j (or null)
  float* win_psi;              // window slot [S][k][P16]: psi_j^{m+1}, j >= 2 (or null)
  int p, m;                    // 6m, patches per face
  float dt2;
};

__global__ __launch_bounds__(kStepThreads) void adj_main_kernel(AdjParams prm) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* smem = reinterpret_cast<float*>(smem_raw);
  const StepParams& gp = prm.geo;
  const int s = gp.order ? gp.order[blockIdx.x] : (int)blockIdx.x, tid = threadIdx.x;
  const int k = gp.k, P = gp.P16;
  float* xs = smem;                       // [k][P] block inputs
  float* zs = xs + k * P;                 // [k][P] z = M^{-1} psi, later the fluxes phi
  float* part = zs + k * P;               // [k][nslots][16]
  const size_t sbase = (size_t)s * k * P;
  const float* tiles = reinterpret_cast<const float*>(gp.tiles) + (size_t)s * gp.words_per_sub;
  const int slot = prm.slot_of ? prm.slot_of[s] : -1;
  const int ks = gp.k_of ? gp.k_of[s] : k;      // this ROM's levels; the others stay zero

  // z_j = Gamma-hat_j psi_j, j = 2..ks (blocks k .. k + ks - 2 of the stream)
  for (int e = tid; e < (ks - 1) * P; e += kStepThreads) {
    const float v = prm.Psi[sbase + P + e];
    xs[e] = v;
    if (prm.win_psi) prm.win_psi[sbase + P + e] = v;
  }
  __syncthreads();
  run_phase<float>(tiles + (size_t)k * gp.words_per_block, ks - 1, gp, xs, P, part, tid);
  __syncthreads();
  for (int e = tid; e < (ks - 1) * P; e += kStepThreads) {
    const int b = e / P, i = e - b * P;
    zs[P + e] = reduce_entry(part, b, i, gp.nt, gp.nslots);
  }
  for (int e = tid; e < P; e += kStepThreads) zs[e] = prm.C[(size_t)s * P + e] * prm.Psi[sbase + e];   // z_1
  __syncthreads();
  // (D z)_j = z_{j+1} - z_j
  for (int e = tid; e < ks * P; e += kStepThreads) {
    const int j = e / P;
    const float v = (j + 1 < ks ? zs[e + P] : 0.f) - zs[e];
    xs[e] = v;
    if (prm.win_dz) prm.win_dz[sbase + e] = v;
  }
  __syncthreads();
  run_phase<float>(tiles, ks, gp, xs, P, part, tid);                     // phi_j = Gamma_j (D z)_j
  __syncthreads();
  for (int e = tid; e < ks * P; e += kStepThreads) {
    const int b = e / P, i = e - b * P;
    zs[e] = reduce_entry(part, b, i, gp.nt, gp.nslots);
  }
  __syncthreads();
  for (int e = tid; e < P; e += kStepThreads) prm.exch[(size_t)s * P + e] = zs[e];
  // interior layers: (A^T psi)_j = phi_j - phi_{j-1}
  for (int e = tid; e < (ks - 1) * P; e += kStepThreads) {
    const size_t idx = sbase + P + e;
    float f = fmaf(prm.dt2, zs[e + P] - zs[e], prm.F[idx]);
    if (slot >= 0 && prm.gslot) f += prm.gslot[((size_t)slot * k) * P + P + e];
    prm.F[idx] = f;
    prm.Psi[idx] = prm.Psi[idx] + f;
  }
}

// Shared boundary entries: (A^T psi)_f = phi_1^alpha + phi_1^beta, plus R^T r from both sides.
__global__ void adj_face_kernel(AdjParams prm, const int32_t* __restrict__ nbr) {
  const StepParams& gp = prm.geo;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)gp.S * prm.p) return;
  const int P = gp.P16, k = gp.k;
  const int s = (int)(idx / prm.p);
  const int q = (int)(idx - (int64_t)s * prm.p);
  const int f = q / prm.m, pat = q - f * prm.m;
  const int nb = nbr[s * 6 + f];
  const int qn = (f ^ 1) * prm.m + pat;
  float a = prm.exch[(size_t)s * P + q];
  if (nb >= 0) a += prm.exch[(size_t)nb * P + qn];
  float g = 0.f;
  if (prm.gslot) {
    const int sl = prm.slot_of[s];
    if (sl >= 0) g += prm.gslot[((size_t)sl * k) * P + q];
    if (nb >= 0) {
      const int sn = prm.slot_of[nb];
      if (sn >= 0) g += prm.gslot[((size_t)sn * k) * P + qn];
    }
  }
  const size_t u = (size_t)s * k * P + q;
  const float fv = fmaf(prm.dt2, a, prm.F[u]) + g;
  prm.F[u] = fv;
  prm.Psi[u] = prm.Psi[u] + fv;
}

constexpr int kIE = 64;   // injection entries per tile
constexpr int kIT = 64;   // adjoint steps per tile (= kInjWindow)
constexpr int kIR = 32;   // receivers per reduction chunk

// inj[t][slot][e] = sum over the slot's receivers r of res[perm[r]][col0 - t] rows[r][e], t < w:
// R^T r for w consecutive adjoint steps, so each receiver row is read once per window.
// blockIdx.y = receiver-subdomain slot, blockIdx.x = tile of 64 entries e; 4 x 4 outputs a thread.
__global__ __launch_bounds__(256) void adj_inject_window_kernel(const float* __restrict__ rows,
                                                                const int32_t* __restrict__ rs_off,
                                                                const int32_t* __restrict__ perm,
                                                                const float* __restrict__ res, int64_t ld,
                                                                int64_t col0, int w, int K, int n_rs,
                                                                float* __restrict__ inj) {
  __shared__ __align__(16) float Rs[kIR][kIE + 4];
  __shared__ __align__(16) float Qs[kIR][kIT + 4];
  const int slot = blockIdx.y, e0 = blockIdx.x * kIE, tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;        // entries e0 + 4tx.., steps 4ty..
  const int r0 = rs_off[slot], r1 = rs_off[slot + 1];
  float acc[4][4] = {};
  for (int rb = r0; rb < r1; rb += kIR) {
    for (int q = tid; q < kIR * kIE; q += 256) {
      const int rr = q / kIE, ee = q - rr * kIE;
      const int r = rb + rr, e = e0 + ee;
      Rs[rr][ee] = (r < r1 && e < K) ? rows[(size_t)r * K + e] : 0.f;
      Qs[rr][ee] = (r < r1 && ee < w) ? res[(size_t)perm[r] * ld + col0 - ee] : 0.f;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < kIR; ++rr) {
      const float4 a = *reinterpret_cast<const float4*>(&Qs[rr][ty * 4]);
      const float4 b = *reinterpret_cast<const float4*>(&Rs[rr][tx * 4]);
      const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int t = ty * 4 + i;
    if (t >= w) continue;
    float* out = inj + ((size_t)t * n_rs + slot) * K;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = e0 + tx * 4 + j;
      if (e < K) out[e] = acc[i][j];
    }
  }
}

struct GradParams {
  const float* win_dz;         // [T][S][k][P16]
  const float* win_psi;        // [T][S][k][P16]
  const float* useg;           // [L + 1][S][k][P16] forward states of the segment
  const float* kxseg;          // [L][S][k][P16] forward (-K X) of the segment
  const int32_t* k_of;         // [S] levels of each subdomain's ROM (null: all k)
  int first;                   // segment slot of window entry 0 (entry t is slot first - t)
  int w;                       // filled window entries
  int S, k, P, p;
  size_t state;                // S k P16
  double dt2;
  double* G;                   // [S][2k-1][p][p] accumulators
};

// One work-group per (subdomain, block): G[s][b] += factor sum_t (x_t y_t^T + y_t x_t^T), the
// symmetric part (twice it) of the pair products, on the tiles of 4 x 4 entries on or above the
// diagonal; below the diagonal only the diagonal tiles write (their mirror values).  The window
// of x and y sits in LDS ([w][P] each); a thread keeps one 4 x 4 tile in registers.
__global__ __launch_bounds__(256) void grad_accum_kernel(GradParams prm) {
  extern __shared__ __align__(16) unsigned char gsm_raw[];
  const int s = blockIdx.x, b = blockIdx.y;
  const int k = prm.k, P = prm.P, p = prm.p;
  float* xs = reinterpret_cast<float*>(gsm_raw);   // [w][P]
  float* ys = xs + (size_t)prm.w * P;              // [w][P]
  const bool hat = b >= k;
  const int j = hat ? b - k + 1 : b;           // layer index (0-based)
  if (j >= (prm.k_of ? prm.k_of[s] : k)) return;   // a level this ROM does not have: gradient zero
  for (int e = threadIdx.x; e < prm.w * P; e += 256) {
    const int t = e / P, i = e - t * P;
    const size_t lay = ((size_t)s * k + j) * P + i;
    const size_t slot = (size_t)(prm.first - t);
    if (hat) {
      xs[e] = prm.win_psi[(size_t)t * prm.state + lay];
      ys[e] = prm.kxseg[slot * prm.state + lay];
    } else {
      xs[e] = prm.win_dz[(size_t)t * prm.state + lay];
      const float* u = prm.useg + slot * prm.state;
      ys[e] = (j + 1 < k ? u[lay + P] : 0.f) - u[lay];
    }
  }
  __syncthreads();
  const double factor = hat ? prm.dt2 : -prm.dt2;
  double* G = prm.G + ((size_t)s * (2 * k - 1) + b) * p * p;
  const int nt = (p + 3) / 4;                  // 4 nt <= P: the tile reads stay inside a row
  for (int u = threadIdx.x; u < nt * (nt + 1) / 2; u += 256) {
    int bi = 0, rem = u;
    while (rem >= nt - bi) {
      rem -= nt - bi;
      ++bi;
    }
    const int r0 = 4 * bi, c0 = 4 * (bi + rem);
    float acc[4][4] = {};
    for (int t = 0; t < prm.w; ++t) {
      const float4 xr = *reinterpret_cast<const float4*>(xs + (size_t)t * P + r0);
      const float4 yr = *reinterpret_cast<const float4*>(ys + (size_t)t * P + r0);
      const float4 xc = *reinterpret_cast<const float4*>(xs + (size_t)t * P + c0);
      const float4 yc = *reinterpret_cast<const float4*>(ys + (size_t)t * P + c0);
      const float xrv[4] = {xr.x, xr.y, xr.z, xr.w}, yrv[4] = {yr.x, yr.y, yr.z, yr.w};
      const float xcv[4] = {xc.x, xc.y, xc.z, xc.w}, ycv[4] = {yc.x, yc.y, yc.z, yc.w};
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = fmaf(xrv[a], ycv[c], fmaf(yrv[a], xcv[c], acc[a][c]));
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int r = r0 + a, col = c0 + c;
        if (r < p && col < p) G[r * p + col] += factor * (double)acc[a][c];
      }
  }
}

size_t grad_lds_bytes(int w, int P) { return (size_t)2 * w * P * sizeof(float); }

// Caller layout [S][k][p][p]: dJ/dGamma_j and dJ/dGamma-hat_j (zero for j = 1), each half of the
// accumulated symmetric sum, which sits on or above the diagonal.
__global__ void grad_out_kernel(const double* __restrict__ G, int S, int k, int p, double* __restrict__ og,
                                double* __restrict__ oh) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t pp = (size_t)p * p;
  if (idx >= (size_t)S * k * pp) return;
  const size_t sj = idx / pp;
  const int e = (int)(idx - sj * pp);
  const int s = (int)(sj / k), j = (int)(sj - (size_t)s * k);
  const int r = e / p, q = e - r * p;
  const size_t up = (size_t)min(r, q) * p + max(r, q);
  const double* Gs = G + (size_t)s * (2 * k - 1) * pp;
  og[idx] = 0.5 * Gs[(size_t)j * pp + up];
  oh[idx] = j >= 1 ? 0.5 * Gs[(size_t)(k + j - 1) * pp + up] : 0.0;
}

struct Buffers {
  sfm_ctx c;
  hipError_t e = hipSuccess;
  std::vector<void*> ptrs;
  explicit Buffers(sfm_ctx ctx) : c(ctx) {}
  ~Buffers() {
    for (void* ptr : ptrs) c->dfree(ptr);
  }
  template <typename T>
  T* get(size_t count) {
    void* ptr = c->dalloc(count * sizeof(T), &e);
    if (ptr) ptrs.push_back(ptr);
    return static_cast<T*>(ptr);
  }
};

}  // namespace
}  // namespace sfm

using namespace sfm;

#define AD_TRY_HIP(call)                                                                      \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return c->fail(SFM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

extern "C" sfm_status sfm_adjoint_gradient(sfm_ctx c, int32_t nsteps, double dt, const float* wavelet_dev,
                                           const float* grad_traces_dev, int64_t ld, int32_t checkpoint_every,
                                           double* grad_gamma, double* grad_gamma_hat, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs: call sfm_build_roms or sfm_load_roms first");
  if (c->cfg.precision != SFM_PREC_FP32) return c->fail(SFM_EINVAL, "the adjoint needs FP32 coefficient storage");
  if (nsteps < 1) return c->fail(SFM_EINVAL, "nsteps must be >= 1");
  if (!(dt > 0.0) || !std::isfinite(dt)) return c->fail(SFM_EINVAL, "dt must be positive and finite");
  if (c->dt_max > 0.0 && dt > c->dt_max) return c->fail(SFM_EUNSTABLE, "dt above the stability limit");
  if (c->nsrc > 0 && !wavelet_dev) return c->fail(SFM_EINVAL, "wavelet_dev is required with sources");
  if (c->nrec == 0 || !grad_traces_dev) return c->fail(SFM_EINVAL, "the misfit needs receivers and grad_traces_dev");
  if (ld < nsteps) return c->fail(SFM_EINVAL, "ld must be >= nsteps");
  if (checkpoint_every < 1) return c->fail(SFM_EINVAL, "checkpoint_every must be >= 1");
  if (!grad_gamma || !grad_gamma_hat) return c->fail(SFM_EINVAL, "gradient arrays are NULL");
  AD_TRY_HIP(hipSetDevice(c->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const Topology& t = c->topo;
  const TileGeometry& geo = c->geo;
  const int S = t.S, k = t.k, p = t.p, P = geo.P16, N = nsteps;
  const int L = std::min(checkpoint_every, N);
  const size_t state = (size_t)S * k * P;
  const int nck = (N + L - 1) / L;
  const int nlast = (nck - 1) * L;              // first step of the last segment
  const int nblk = 2 * k - 1;
  const int K = k * P;
  Buffers B(c);
  float* ckU = B.get<float>(state * std::max(nck - 1, 1));
  float* ckD = B.get<float>(state * std::max(nck - 1, 1));
  float* useg = B.get<float>(state * (L + 1));
  float* kxseg = B.get<float>(state * L);
  float* wdz = B.get<float>(state * kGradWindow);
  float* wpsi = B.get<float>(state * kGradWindow);
  float* psi = B.get<float>(state);
  float* F = B.get<float>(state);
  float* injw = B.get<float>((size_t)kInjWindow * c->n_rs * K);
  double* G = B.get<double>((size_t)S * nblk * p * p);
  if (B.e != hipSuccess) return c->fail(SFM_ENOMEM, "adjoint buffers: out of device memory (lower checkpoint_every?)");
  AD_TRY_HIP(hipMemsetAsync(G, 0, (size_t)S * nblk * p * p * sizeof(double), st));
  AD_TRY_HIP(hipMemsetAsync(psi, 0, state * sizeof(float), st));
  AD_TRY_HIP(hipMemsetAsync(F, 0, state * sizeof(float), st));
  AD_TRY_HIP(hipMemsetAsync(kxseg, 0, state * L * sizeof(float), st));   // layer 0 rows stay zero
  // forward from rest with checkpoints of (U, D) before steps 0, L, .., nlast - L; the states of
  // the last segment are stored as they come
  AD_TRY_HIP(hipMemsetAsync(c->U_d, 0, state * sizeof(float), st));
  AD_TRY_HIP(hipMemsetAsync(c->D_d, 0, state * sizeof(float), st));
  const int nsrc = c->nsrc;
  for (int n = 0; n < N; ++n) {
    const bool last = n >= nlast;
    if (!last && n % L == 0) {
      AD_TRY_HIP(hipMemcpyAsync(ckU + state * (n / L), c->U_d, state * sizeof(float), hipMemcpyDeviceToDevice, st));
      AD_TRY_HIP(hipMemcpyAsync(ckD + state * (n / L), c->D_d, state * sizeof(float), hipMemcpyDeviceToDevice, st));
    }
    const sfm_status rc = forward_step(c, dt, wavelet_dev ? wavelet_dev + (size_t)n * nsrc : nullptr,
                                       last ? kxseg + state * (n - nlast) : nullptr,
                                       last ? useg + state * (n - nlast) : nullptr, st);
    if (rc != SFM_OK) return rc;
  }
  AdjParams ap{};
  ap.geo = step_params(c);
  ap.Psi = psi;
  ap.F = F;
  ap.C = c->C_d;
  ap.exch = c->exch_d;
  ap.slot_of = c->hist_slot_d;
  ap.p = p;
  ap.m = t.m;
  ap.dt2 = (float)(dt * dt);
  const size_t lds = step_lds_bytes(ap.geo, SFM_PREC_FP32);
  if (lds > kDefaultLdsBytes)
    AD_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&adj_main_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const size_t glds = grad_lds_bytes(kGradWindow, P);
  if (glds > kDefaultLdsBytes)
    AD_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&grad_accum_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)glds));
  const dim3 igrid((K + kIE - 1) / kIE, c->n_rs);
  const unsigned fgrid = (unsigned)(((int64_t)S * p + 255) / 256);
  GradParams gp{};
  gp.win_dz = wdz;
  gp.win_psi = wpsi;
  gp.useg = useg;
  gp.kxseg = kxseg;
  gp.k_of = c->k_of_d;
  gp.S = S;
  gp.k = k;
  gp.P = P;
  gp.p = p;
  gp.state = state;
  gp.dt2 = dt * dt;
  gp.G = G;
  // injections R^T r^{m-1} for the adjoint steps win_hi down to win_lo (m descends by one)
  int win_hi = 0, win_lo = N + 1;
  // one adjoint step psi^{m+1} -> psi^m; window slot wslot (or -1: no gradient pair)
  auto adjoint_step = [&](int m, int wslot) -> sfm_status {
    if (c->n_rs > 0 && m < win_lo) {
      win_hi = m;
      win_lo = std::max(1, m - kInjWindow + 1);
      hipLaunchKernelGGL(adj_inject_window_kernel, igrid, dim3(256), 0, st, c->rec_rows_d, c->rs_off_d,
                         c->rec_perm_d, grad_traces_dev, ld, (int64_t)(win_hi - 1), win_hi - win_lo + 1, K,
                         c->n_rs, injw);
      AD_TRY_HIP(hipGetLastError());
    }
    ap.gslot = c->n_rs > 0 ? injw + (size_t)(win_hi - m) * c->n_rs * K : nullptr;
    ap.win_dz = wslot >= 0 ? wdz + state * wslot : nullptr;
    ap.win_psi = wslot >= 0 ? wpsi + state * wslot : nullptr;
    hipLaunchKernelGGL(adj_main_kernel, dim3(S), dim3(kStepThreads), lds, st, ap);
    AD_TRY_HIP(hipGetLastError());
    hipLaunchKernelGGL(adj_face_kernel, dim3(fgrid), dim3(256), 0, st, ap, c->nbr_d);
    AD_TRY_HIP(hipGetLastError());
    return SFM_OK;
  };
  // m = N: psi^{N+1} = 0 pairs with nothing
  sfm_status rc = adjoint_step(N, -1);
  if (rc != SFM_OK) return rc;
  for (int seg = nck - 1; seg >= 0; --seg) {
    const int n0 = seg * L, n1 = std::min(N, n0 + L);
    if (seg < nck - 1) {                        // recompute the segment from its checkpoint
      AD_TRY_HIP(hipMemcpyAsync(c->U_d, ckU + state * seg, state * sizeof(float), hipMemcpyDeviceToDevice, st));
      AD_TRY_HIP(hipMemcpyAsync(c->D_d, ckD + state * seg, state * sizeof(float), hipMemcpyDeviceToDevice, st));
      for (int n = n0; n < n1; ++n) {
        rc = forward_step(c, dt, wavelet_dev ? wavelet_dev + (size_t)n * nsrc : nullptr, kxseg + state * (n - n0),
                          useg + state * (n - n0), st);
        if (rc != SFM_OK) return rc;
      }
    }
    // adjoint steps m = n1 - 1 .. max(n0, 1), each pairing psi^{m+1} with X^m
    int w = 0, first = 0;
    for (int m = n1 - 1; m >= std::max(n0, 1); --m) {
      if (w == 0) first = m - n0;
      rc = adjoint_step(m, w);
      if (rc != SFM_OK) return rc;
      ++w;
      if (w == kGradWindow || m == std::max(n0, 1)) {
        gp.first = first;
        gp.w = w;
        hipLaunchKernelGGL(grad_accum_kernel, dim3(S, nblk), dim3(256), grad_lds_bytes(w, P), st, gp);
        AD_TRY_HIP(hipGetLastError());
        w = 0;
      }
    }
  }
  // gradients to the caller: symmetric parts, Gamma-hat_1 held fixed
  const size_t nout = (size_t)S * k * p * p;
  double* og = B.get<double>(nout);
  double* oh = B.get<double>(nout);
  if (B.e != hipSuccess) return c->fail(SFM_ENOMEM, "adjoint output: out of device memory");
  hipLaunchKernelGGL(grad_out_kernel, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, st, G, S, k, p, og, oh);
  AD_TRY_HIP(hipGetLastError());
  AD_TRY_HIP(hipMemcpyAsync(grad_gamma, og, nout * sizeof(double), hipMemcpyDeviceToHost, st));
  AD_TRY_HIP(hipMemcpyAsync(grad_gamma_hat, oh, nout * sizeof(double), hipMemcpyDeviceToHost, st));
  AD_TRY_HIP(hipStreamSynchronize(st));
  // the single-shot state is left at rest
  AD_TRY_HIP(hipMemsetAsync(c->U_d, 0, state * sizeof(float), st));
  AD_TRY_HIP(hipMemsetAsync(c->D_d, 0, state * sizeof(float), st));
  AD_TRY_HIP(hipStreamSynchronize(st));
  c->n = 0;
  return SFM_OK;
}
