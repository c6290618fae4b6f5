// Certified upper bound on the spectral radius of the coupled ROM's step operator (the leapfrog
// stability limit dt_max = 2 / sqrt(rho) of the time stepping at the end of the Stage 2 section).
//
// The coupled scheme is  M X_tt = -K X  with M and K sums over subdomains of P^T M^a P and
// P^T K^a P, where per subdomain (eq. "intrtstep", eq. "bdrytstep")
//     M^a = blockdiag(diag(1/H), Gamma-hat_2^{-1}, ..., Gamma-hat_k^{-1}),   H = diag(Gamma-hat_1),
//     K^a = D^T Gamma D  (block tridiagonal: K_jj = Gamma_j + Gamma_{j-1}, K_{j,j+1} = -Gamma_j).
// The Rayleigh quotient of (K, M) is a mediant of the subdomains' quotients, so
//     rho = lambda_max(K, M) <= max_a lambda_max(K^a, M^a).
// lambda_max(K^a, M^a) < mu  iff  mu I - B^T K^a B is positive definite, B B^T = (M^a)^{-1}
// (B = blockdiag(sqrt(H), L_2, ..., L_k), L_j the Cholesky factor of Gamma-hat_j), and a block
// Cholesky factorisation of that block-tridiagonal matrix decides it:
//     S_1 = mu I - B_1 Gamma_1 B_1,
//     S_{j+1} = mu I - L_{j+1}^T (Gamma_{j+1} + Gamma_j) L_{j+1} - W_j^T W_j,
//     W_j = R_j^{-1} E_j^T,  R_j R_j^T = S_j,  E_j = -L_{j+1}^T Gamma_j B_j,
// positive definite iff every S_j is.  The test runs in FP64 on the coefficients exactly as the
// step kernels stream them (rounded to FP32 or BF16, or FP64), with the face masses widened by
// 4 units of FP32 rounding (the stored combined masses are FP32), and counts a pivot as positive
// only above 1e-9 mu.  One work-group per subdomain; its p x p work matrices live in a scratch
// slice of global memory.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "sfm_internal.h"

namespace sfm {
namespace {

constexpr int kCflThreads = 256;
constexpr int kCflMats = 5;        // Lc, Ln, Sm, Tm, Wm

__device__ __forceinline__ double stored(double v, int precision) {
  if (precision == SFM_PREC_FP64) return v;
  const float f = (float)v;
  if (precision == SFM_PREC_FP32) return (double)f;
  return (double)__bfloat162float(__float2bfloat16(f));
}

// In-place lower Cholesky of the p x p row-major matrix A (lower triangle read and written).
// Returns false (uniformly over the work-group) when a pivot is not above thr.
__device__ bool wg_cholesky(double* A, int p, double thr) {
  const int tid = threadIdx.x;
  for (int c = 0; c < p; ++c) {
    __syncthreads();
    const double d = A[(size_t)c * p + c];
    if (!(d > thr)) return false;
    const double l = sqrt(d);
    const double il = 1.0 / l;
    for (int i = c + 1 + tid; i < p; i += kCflThreads) A[(size_t)i * p + c] *= il;
    __syncthreads();
    if (tid == 0) A[(size_t)c * p + c] = l;
    const int n = p - c - 1;
    for (int e = tid; e < n * n; e += kCflThreads) {
      const int i = c + 1 + e / n, j = c + 1 + e % n;
      if (j <= i) A[(size_t)i * p + j] -= A[(size_t)i * p + c] * A[(size_t)j * p + c];
    }
  }
  __syncthreads();
  return true;
}

struct CflParams {
  const double* coef;       // [S][2][k][p][p]
  const int32_t* k_of;      // [S] or null
  int nsub, k, p, precision;
  double mu;
  double* scratch;          // [gridDim.x][kCflMats][p][p]
  int32_t* verdict;         // [nsub]: 1 = mu above every eigenvalue, 0 = not, -1 = Gamma-hat_j not
                            // positive definite as stored (every entry is written)
};

__global__ __launch_bounds__(kCflThreads) void inertia_kernel(CflParams prm) {
  const int p = prm.p, k = prm.k, tid = threadIdx.x;
  const size_t pp = (size_t)p * p;
  double* Lc = prm.scratch + (size_t)blockIdx.x * kCflMats * pp;
  double* Ln = Lc + pp;
  double* Sm = Ln + pp;
  double* Tm = Sm + pp;
  double* Wm = Tm + pp;
  const double mu = prm.mu;
  const double thr = 1e-9 * mu;
  const double widen = 1.0 + 4.0 * 5.9604644775390625e-08;   // 1 + 4 * 2^-24
  for (int q = blockIdx.x; q < prm.nsub; q += gridDim.x) {
    const int s = q;
    const int ks = prm.k_of ? prm.k_of[s] : k;
    const double* gam = prm.coef + (size_t)s * 2 * k * pp;     // Gamma_j at gam + j pp
    const double* hat = gam + (size_t)k * pp;                 // Gamma-hat_j at hat + j pp
    // level 1: B_1 = diag(sqrt(H)), kept in the diagonal of Lc
    for (int i = tid; i < p; i += kCflThreads) Lc[(size_t)i * p + i] = sqrt(hat[(size_t)i * p + i] * widen);
    __syncthreads();
    for (size_t e = tid; e < pp; e += kCflThreads) {
      const int i = (int)(e / p), c = (int)(e % p);
      Sm[e] = (i == c ? mu : 0.0) - Lc[(size_t)i * p + i] * stored(gam[e], prm.precision) * Lc[(size_t)c * p + c];
    }
    int verdict = 1;
    for (int j = 0; j + 1 < ks; ++j) {      // 0-based level j: S_j -> S_{j+1}
      if (!wg_cholesky(Sm, p, thr)) { verdict = 0; break; }
      // Ln = chol(Gamma-hat_{j+1}) as stored
      for (size_t e = tid; e < pp; e += kCflThreads) Ln[e] = stored(hat[(size_t)(j + 1) * pp + e], prm.precision);
      if (!wg_cholesky(Ln, p, 0.0)) { verdict = -1; break; }
      // Tm = Gamma_j B_j   (B_j diagonal for j = 0, lower triangular after)
      const double* Gj = gam + (size_t)j * pp;
      for (size_t e = tid; e < pp; e += kCflThreads) {
        const int i = (int)(e / p), c = (int)(e % p);
        double acc = 0.0;
        if (j == 0) {
          acc = stored(Gj[e], prm.precision) * Lc[(size_t)c * p + c];
        } else {
          for (int r = c; r < p; ++r) acc += stored(Gj[(size_t)i * p + r], prm.precision) * Lc[(size_t)r * p + c];
        }
        Tm[e] = acc;
      }
      __syncthreads();
      // Wm = E_j^T = -Tm^T Ln
      for (size_t e = tid; e < pp; e += kCflThreads) {
        const int i = (int)(e / p), c = (int)(e % p);
        double acc = 0.0;
        for (int r = c; r < p; ++r) acc += Tm[(size_t)r * p + i] * Ln[(size_t)r * p + c];
        Wm[e] = -acc;
      }
      __syncthreads();
      // Wm <- R_j^{-1} Wm (forward substitution, one column per thread)
      for (int c = tid; c < p; c += kCflThreads) {
        for (int r = 0; r < p; ++r) {
          double v = Wm[(size_t)r * p + c];
          for (int i = 0; i < r; ++i) v -= Sm[(size_t)r * p + i] * Wm[(size_t)i * p + c];
          Wm[(size_t)r * p + c] = v / Sm[(size_t)r * p + r];
        }
      }
      __syncthreads();
      // Tm = (Gamma_{j+1} + Gamma_j) Ln
      const double* Gn = gam + (size_t)(j + 1) * pp;
      for (size_t e = tid; e < pp; e += kCflThreads) {
        const int i = (int)(e / p), c = (int)(e % p);
        double acc = 0.0;
        for (int r = c; r < p; ++r)
          acc += (stored(Gn[(size_t)i * p + r], prm.precision) + stored(Gj[(size_t)i * p + r], prm.precision)) *
                 Ln[(size_t)r * p + c];
        Tm[e] = acc;
      }
      __syncthreads();
      // S_{j+1} = mu I - Ln^T Tm - Wm^T Wm
      for (size_t e = tid; e < pp; e += kCflThreads) {
        const int i = (int)(e / p), c = (int)(e % p);
        double acc = 0.0;
        for (int r = i; r < p; ++r) acc += Ln[(size_t)r * p + i] * Tm[(size_t)r * p + c];
        for (int r = 0; r < p; ++r) acc += Wm[(size_t)r * p + i] * Wm[(size_t)r * p + c];
        Sm[e] = (i == c ? mu : 0.0) - acc;
      }
      __syncthreads();
      double* t = Lc; Lc = Ln; Ln = t;
    }
    if (verdict == 1 && !wg_cholesky(Sm, p, thr)) verdict = 0;
    if (tid == 0) prm.verdict[q] = verdict;
    __syncthreads();
    // the next subdomain of this group starts from the original slots of the two rotating factors
    Lc = prm.scratch + (size_t)blockIdx.x * kCflMats * pp;
    Ln = Lc + pp;
  }
}

// Seeded start vector of the power iteration, [S][k][P16]: entry (s, j, q) is a counter-based
// uniform draw in [-0.5, 0.5) (splitmix64 of its index); padding is zero; a shared boundary entry
// takes the draw of the lower-index side, so both copies agree.
__global__ void start_vector_kernel(float* v, const int32_t* nbr, int S, int k, int p, int P16, int m) {
  const int64_t n = (int64_t)S * k * P16;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(i % P16);
    const int64_t sj = i / P16;
    const int j = (int)(sj % k);
    int s = (int)(sj / k);
    int qq = q;
    if (q >= p) { v[i] = 0.f; continue; }
    if (j == 0) {
      const int f = q / m, pat = q % m;
      const int nb = nbr[(size_t)s * 6 + f];
      if (nb >= 0 && nb < s) { s = nb; qq = (f ^ 1) * m + pat; }
    }
    uint64_t z = ((uint64_t)s * k + j) * (uint64_t)P16 + (uint64_t)qq + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    v[i] = (float)((double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5);
  }
}

}  // namespace

size_t cfl_scratch_bytes_per_group(int p) { return (size_t)kCflMats * p * p * sizeof(double); }

// dt_max of the coupled step operator: power iterations from the seeded start, then the smallest
// mu of a geometric ladder above that estimate which passes the inertia test in every subdomain,
// refined by bisection between the last failing and the first passing rung.  scratch holds
// nwg * cfl_scratch_bytes_per_group(p) bytes of work matrices followed by S int32 verdicts.
sfm_status cfl_limit(sfm_ctx c, int32_t iters, double* scratch, int nwg, double* dt_max, hipStream_t st) {
  const Topology& t = c->topo;
  const int S = t.S, p = t.p, k = t.k, P16 = c->geo.P16;
  const int64_t n = (int64_t)S * k * P16;
  hipError_t e = hipSuccess;
  auto hip_fail = [&](const char* what) {
    return c->fail(SFM_EHIP, std::string(what) + " failed: " + hipGetErrorString(e));
  };
  hipLaunchKernelGGL(start_vector_kernel, dim3(1024), dim3(256), 0, st, c->work_a_d, c->nbr_d, S, k, p, P16, t.m);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail("start vector");
  // padding entries of the boundary layer are never written by the operator: clear them
  if ((e = hipMemsetAsync(c->work_b_d, 0, n * sizeof(float), st)) != hipSuccess) return hip_fail("hipMemsetAsync");
  if ((e = launch_norm2(c->work_a_d, n, c->red_d, st)) != hipSuccess) return hip_fail("norm");
  if ((e = launch_scale(c->work_a_d, n, c->red_d, c->work_a_d, st)) != hipSuccess) return hip_fail("scale");
  for (int it = 0; it < iters; ++it) {
    if ((e = apply_operator(c, c->work_a_d, c->work_b_d, st)) != hipSuccess) return hip_fail("step operator");
    if ((e = launch_norm2(c->work_b_d, n, c->red_d, st)) != hipSuccess) return hip_fail("norm");
    if (it + 1 < iters && (e = launch_scale(c->work_b_d, n, c->red_d, c->work_a_d, st)) != hipSuccess)
      return hip_fail("scale");
  }
  double nrm2 = 0.0;
  if ((e = hipMemcpyAsync(&nrm2, c->red_d, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hip_fail("hipMemcpyAsync");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail("hipStreamSynchronize");
  // a = -M^{-1} K v with |v| = 1, so |a| tends to rho from below.
  const double rho_lo = std::sqrt(nrm2);
  if (!(rho_lo > 0.0) || !std::isfinite(rho_lo)) return c->fail(SFM_EBREAKDOWN, "spectral radius estimate failed");

  CflParams prm{};
  prm.coef = c->coef64_d;
  prm.k_of = c->k_of_d;
  prm.nsub = S;
  prm.k = k;
  prm.p = p;
  prm.precision = c->cfg.precision;
  prm.scratch = scratch;
  prm.verdict = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(scratch) + nwg * cfl_scratch_bytes_per_group(p));
  std::vector<int32_t> verdict(S);
  SFM_DCHECK(nwg >= 1 && nwg <= S && p >= 1 && k >= 1 && c->coef64_d && scratch);
  auto passes = [&](double mu, bool* ok) -> sfm_status {
    prm.mu = mu;
    hipLaunchKernelGGL(inertia_kernel, dim3(nwg), dim3(kCflThreads), 0, st, prm);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail("stability certificate");
    if ((e = hipMemcpyAsync(verdict.data(), prm.verdict, S * sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail("hipMemcpyAsync");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail("hipStreamSynchronize");
    *ok = true;
    for (int s = 0; s < S; ++s) {
      if (verdict[s] < 0)
        return c->fail(SFM_EUNSTABLE, "subdomain " + std::to_string(s) +
                                          ": a Gamma-hat block is not positive definite in the stored precision");
      if (verdict[s] == 0) *ok = false;
    }
    return SFM_OK;
  };
  const double rungs[] = {1e-4, 1e-3, 1e-2, 3e-2, 1e-1, 3e-1, 1.0, 3.0, 10.0, 1e2, 1e3, 1e4, 1e6};
  double lo = rho_lo, hi = -1.0;
  for (double r : rungs) {
    bool ok = false;
    const double mu = rho_lo * (1.0 + r);
    const sfm_status rc = passes(mu, &ok);
    if (rc != SFM_OK) return rc;
    if (ok) { hi = mu; break; }
    lo = mu;
  }
  if (hi < 0.0) return c->fail(SFM_EUNSTABLE, "no stability bound up to 1e6 times the power-iteration estimate");
  for (int it = 0; it < 4 && hi > lo * (1.0 + 2e-5); ++it) {
    const double mid = std::sqrt(lo * hi);
    bool ok = false;
    const sfm_status rc = passes(mid, &ok);
    if (rc != SFM_OK) return rc;
    if (ok) hi = mid; else lo = mid;
  }
  c->rho_est = rho_lo;
  c->rho_bound = hi;
  c->dt_max = 2.0 / std::sqrt(hi);
  *dt_max = c->dt_max;
  return SFM_OK;
}

}  // namespace sfm

extern "C" sfm_status sfm_cfl_dt(sfm_ctx c, int32_t iters, double* dt_max, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs");
  if (iters < 10 || !dt_max) return c->fail(SFM_EINVAL, "iters must be >= 10 and dt_max non-NULL");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return c->fail(SFM_EHIP, std::string("hipSetDevice failed: ") + hipGetErrorString(e));
  const int nwg = std::min(c->topo.S, 2048);
  const size_t bytes = nwg * sfm::cfl_scratch_bytes_per_group(c->topo.p) + (size_t)c->topo.S * sizeof(int32_t);
  double* scratch = static_cast<double*>(c->dalloc(bytes, &e));
  if (!scratch) return c->fail(SFM_ENOMEM, "stability certificate: out of device memory");
  const sfm_status rc = sfm::cfl_limit(c, iters, scratch, nwg, dt_max, reinterpret_cast<hipStream_t>(stream));
  c->dfree(scratch);
  return rc;
}

// ----------------------------------------------------------------------------- no-allocation variant
// The certificate's scratch (work matrices and verdicts) in one file-scope device array.  In host
// code `scratch` names a host-side stand-in, not device memory: its device address is taken once
// per device with hipGetSymbolAddress, with that device current, and only that address is used.
namespace {
constexpr size_t kStaticVerdictBytes = size_t(1) << 20;          // S <= 262,144
constexpr size_t kStaticScratchBytes = size_t(64) << 20;         // 63 MiB of work matrices + verdicts
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

extern "C" sfm_status sfm_cfl_dt_noalloc(sfm_ctx c, int32_t iters, double* dt_max, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  const size_t per_group = sfm::cfl_scratch_bytes_per_group(c->topo.p);
  const size_t verdict_bytes = (size_t)c->topo.S * sizeof(int32_t);
  if (verdict_bytes > kStaticVerdictBytes)
    return c->fail(SFM_EINVAL, "sfm_cfl_dt_noalloc: " + std::to_string(c->topo.S) +
                                   " subdomains exceed the static scratch limit of " +
                                   std::to_string(kStaticVerdictBytes / sizeof(int32_t)));
  const size_t groups = (kStaticScratchBytes - kStaticVerdictBytes) / per_group;
  if (groups < 1)
    return c->fail(SFM_EINVAL, "sfm_cfl_dt_noalloc: 6m = " + std::to_string(c->topo.p) +
                                   " needs more than the static scratch of one work-group");
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs");
  if (iters < 10 || !dt_max) return c->fail(SFM_EINVAL, "iters must be >= 10 and dt_max non-NULL");
  if (c->device < 0 || c->device >= kMaxDevices) return c->fail(SFM_EINVAL, "device index out of range");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return c->fail(SFM_EHIP, std::string("hipSetDevice failed: ") + hipGetErrorString(e));
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[c->device]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return c->fail(SFM_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
      g_scratch_dev[c->device] = ptr;
    }
    base = g_scratch_dev[c->device];
  }
  const int nwg = (int)std::min<size_t>({(size_t)c->topo.S, size_t(2048), groups});
  return sfm::cfl_limit(c, iters, static_cast<double*>(base), nwg, dt_max, reinterpret_cast<hipStream_t>(stream));
}
