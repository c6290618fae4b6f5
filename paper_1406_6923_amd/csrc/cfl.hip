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
// only above 1e-9 mu.  A trial mu runs level by level over batches of subdomains: the p x p
// products on the FP64 matrix cores, the factorisations and the substitution one work-group per
// subdomain, in LDS where the p x p blocks fit.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "sfm_internal.h"

namespace sfm {
namespace {

constexpr int kCflMats = 7;        // per batch member: Gamma_j, Gamma_{j+1}, B_j, L_{j+1}, T, W, S

__device__ __forceinline__ double stored(double v, int precision) {
  if (precision == SFM_PREC_FP64) return v;
  const float f = (float)v;
  if (precision == SFM_PREC_FP32) return (double)f;
  return (double)__bfloat162float(__float2bfloat16(f));
}

// dst[b] = the stored (rounded) value of block `which` (0: Gamma, 1: Gamma-hat) at level j of
// subdomain subs[b], p x p (symmetric, so row- and column-major agree).
__global__ void gather_rounded_kernel(const double* __restrict__ coef, const int32_t* __restrict__ subs, int nb, int k,
                                      int p, int which, int j, int precision, double* __restrict__ dst) {
  const int64_t pp = (int64_t)p * p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < pp * nb; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / pp, q = e - b * pp;
    dst[e] = stored(coef[(((int64_t)subs[b] * 2 + which) * k + j) * pp + q], precision);
  }
}

// Level 1: B_1 = diag(sqrt(H (1 + 4 2^-24))), H = diag(Gamma-hat_1) (the stored FP32 face masses are
// within 4 units of rounding of H); Bc = B_1 as a full matrix and S = mu I - B_1 Gamma_1 B_1.
__global__ void level_one_kernel(const double* __restrict__ coef, const int32_t* __restrict__ subs, int nb, int k,
                                 int p, const double* __restrict__ G1, double mu, double* __restrict__ Bc,
                                 double* __restrict__ Sm) {
  const int64_t pp = (int64_t)p * p;
  const double widen = 1.0 + 4.0 * 5.9604644775390625e-08;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < pp * nb; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / pp, q = e - b * pp;
    const int r = (int)(q % p), c = (int)(q / p);
    const double* hat1 = coef + (((int64_t)subs[b] * 2 + 1) * k) * pp;
    const double br = sqrt(hat1[(int64_t)r * p + r] * widen), bcol = sqrt(hat1[(int64_t)c * p + c] * widen);
    Bc[e] = r == c ? br : 0.0;
    Sm[e] = (r == c ? mu : 0.0) - br * G1[e] * bcol;
  }
}

__global__ void add_kernel(double* __restrict__ x, const double* __restrict__ y, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) x[e] += y[e];
}

__global__ void set_mu_kernel(double* __restrict__ Sm, int p, int nb, double mu) {
  const int64_t pp = (int64_t)p * p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < pp * nb; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e % pp;
    Sm[e] = (q % p == q / p) ? mu : 0.0;
  }
}

__global__ void fill_kernel(int32_t* __restrict__ v, int n, int32_t value) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) v[e] = value;
}

// Lower Cholesky in place of the p x p column-major matrix a (leading dimension p) held by the
// work-group (a multiple of 16 threads); the strict upper triangle is zeroed.  Returns, uniformly
// over the work-group, whether every pivot exceeded thr; a pivot that does not is replaced by 1 so
// the factorisation still ends.  Every thread forms the pivot itself; the trailing update runs
// over 16-lane groups, one column per group and consecutive rows across its lanes.
__device__ bool chol_body(double* a, int p, double thr) {
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4, nty = blockDim.x >> 4;
  if (tid == 0) bad = 0;
  for (int c = 0; c < p; ++c) {
    __syncthreads();                     // column c is final
    double d = a[c + (int64_t)c * p];
    const bool ok = d > thr;
    if (!ok) d = 1.0;
    const double piv = sqrt(d);
    const double inv = 1.0 / piv;
    for (int i = c + 1 + tid; i < p; i += blockDim.x) a[i + (int64_t)c * p] *= inv;
    __syncthreads();                     // the scaled column is visible, every thread has read a_cc
    if (tid == 0) {
      a[c + (int64_t)c * p] = piv;
      if (!ok) bad = 1;
    }
    const int nr = p - c - 1;
    const double* col = a + (int64_t)c * p + c + 1;
    for (int jj = ty; jj < nr; jj += nty) {
      const double lj = col[jj];
      double* dst = a + (c + 1) + (int64_t)(c + 1 + jj) * p;
      for (int ii = jj + tx; ii < nr; ii += 16) dst[ii] -= col[ii] * lj;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < p * p; e += blockDim.x)
    if (e % p < e / p) a[e] = 0.0;
  __syncthreads();
  return bad == 0;
}

// w <- r^{-1} w for the lower triangular r (p x p, leading dimension p) and p columns of w
// (leading dimension ldw), one column per thread, forward substitution.  Each row's dot product
// runs in eight interleaved partial sums (added in a fixed order), so the loads of the next terms
// are in flight while the current ones accumulate.
__device__ void solve_body(const double* r, double* w, int p, int ldw) {
  for (int c = threadIdx.x; c < p; c += blockDim.x) {
    double* x = w + (int64_t)c * ldw;
    for (int row = 0; row < p; ++row) {
      double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int i = 0;
      for (; i + 8 <= row; i += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = fma(r[row + (int64_t)(i + u) * p], x[i + u], acc[u]);
      }
      for (int u = 0; i < row; ++i, ++u) acc[u] = fma(r[row + (int64_t)i * p], x[i], acc[u]);
      const double dot = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
      x[row] = (x[row] - dot) / r[row + (int64_t)row * p];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void copy_block(double* dst, int ldd, const double* src, int lds_, int p) {
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int r = e % p, c = e / p;
    dst[r + (int64_t)c * ldd] = src[r + (int64_t)c * lds_];
  }
  __syncthreads();
}

__device__ __forceinline__ void mark(int32_t* verdict, bool ok, int fail_value) {
  if (threadIdx.x == 0 && !ok && fail_value < verdict[blockIdx.x]) verdict[blockIdx.x] = fail_value;
}

// A_b <- chol(A_b) for every batch member; a failing pivot lowers verdict[b] to fail_value.  With
// kLds the matrix is factored in LDS (p^2 doubles of dynamic LDS), else in place in global memory;
// the arithmetic and its order are the same.
template <bool kLds>
__global__ __launch_bounds__(256) void chol_kernel(double* __restrict__ A, int p, double thr, int fail_value,
                                                   int32_t* __restrict__ verdict) {
  extern __shared__ __align__(16) double cfl_lds[];
  double* g = A + (int64_t)blockIdx.x * p * p;
  double* a = kLds ? cfl_lds : g;
  if (kLds) copy_block(a, p, g, p, p);
  const bool ok = chol_body(a, p, thr);
  if (kLds) copy_block(g, p, a, p, p);
  mark(verdict, ok, fail_value);
}

// R_b = chol(S_b) (a failing pivot sets verdict[b] to 0), then W_b <- R_b^{-1} W_b.  With kLds, S
// and W live in LDS (p^2 + p (p + 1) doubles; W's columns padded by one), else in global memory.
template <bool kLds>
__global__ __launch_bounds__(256) void factor_solve_kernel(double* __restrict__ Sm, double* __restrict__ Wm, int p,
                                                           double thr, int32_t* __restrict__ verdict) {
  extern __shared__ __align__(16) double cfl_lds[];
  double* sg = Sm + (int64_t)blockIdx.x * p * p;
  double* wg = Wm + (int64_t)blockIdx.x * p * p;
  double* a = kLds ? cfl_lds : sg;
  double* w = kLds ? cfl_lds + (int64_t)p * p : wg;
  const int ldw = kLds ? p + 1 : p;
  if (kLds) copy_block(a, p, sg, p, p);
  const bool ok = chol_body(a, p, thr);
  mark(verdict, ok, 0);
  if (kLds) copy_block(w, ldw, wg, p, p);
  solve_body(a, w, p, ldw);
  if (kLds) copy_block(wg, p, w, ldw, p);
}

size_t chol_lds_bytes(int p) { return (size_t)p * p * sizeof(double); }
size_t factor_solve_lds_bytes(int p) { return ((size_t)p * p + (size_t)p * (p + 1)) * sizeof(double); }

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

size_t cfl_scratch_bytes_per_member(int p) { return (size_t)kCflMats * p * p * sizeof(double); }
size_t cfl_index_bytes(int S) { return (size_t)2 * S * sizeof(int32_t); }

// dt_max of the coupled step operator: power iterations from the seeded start, then the smallest
// mu of a geometric ladder above that estimate which passes the inertia test in every subdomain,
// refined by bisection between the last failing and the first passing rung.
//
// scratch holds cfl_index_bytes(S) bytes (verdicts and the level-sorted subdomain order) followed by
// batch * cfl_scratch_bytes_per_member(p) bytes of work matrices.  The subdomains are processed in
// batches of at most `batch` with equal level counts, one level at a time for the whole batch: the
// p x p products are batched FP64 matrix-core GEMMs (reduction depth p, never split, so a member's
// arithmetic does not depend on the batch it is in), the factorisations and the substitution are
// one work-group per member, in LDS when the blocks fit the work-group's limit.
sfm_status cfl_limit(sfm_ctx c, int32_t iters, void* scratch, int batch, double* dt_max, hipStream_t st) {
  const Topology& t = c->topo;
  const int S = t.S, p = t.p, k = t.k, P16 = c->geo.P16;
  const int64_t n = (int64_t)S * k * P16;
  const int64_t pp = (int64_t)p * p;
  hipError_t e = hipSuccess;
  auto hip_fail = [&](const char* what) {
    return c->fail(SFM_EHIP, std::string(what) + " failed: " + hipGetErrorString(e));
  };
  SFM_DCHECK(batch >= 1 && p >= 1 && k >= 1 && c->coef64_d && scratch);
  // subdomains sorted by level count (stable), so every batch shares one count
  std::vector<int32_t> order(S), levels(S);
  for (int s = 0; s < S; ++s) {
    order[s] = s;
    levels[s] = c->k_of.empty() ? k : c->k_of[s];
  }
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return levels[a] < levels[b]; });
  int32_t* verdict_d = static_cast<int32_t*>(scratch);
  int32_t* order_d = verdict_d + S;
  double* mats = reinterpret_cast<double*>(static_cast<char*>(scratch) + ((cfl_index_bytes(S) + 255) / 256) * 256);
  double* Gc = mats;
  double* Gn = Gc + batch * pp;
  double* La = Gn + batch * pp;
  double* Lb = La + batch * pp;
  double* Tm = Lb + batch * pp;
  double* Wm = Tm + batch * pp;
  double* Sm = Wm + batch * pp;
  if ((e = hipMemcpyAsync(order_d, order.data(), S * sizeof(int32_t), hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail("hipMemcpyAsync");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail("hipStreamSynchronize");

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

  const int prec = c->cfg.precision;
  std::vector<int32_t> verdict(S);
  auto grid = [](int64_t elems) { return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((elems + 255) / 256, 8192))); };
  const int chol_threads = std::min(256, (p + 63) / 64 * 64 * 2);
  const size_t chol_lds = chol_lds_bytes(p), fs_lds = factor_solve_lds_bytes(p);
  const bool chol_in_lds = chol_lds <= kMaxLdsBytes, fs_in_lds = fs_lds <= kMaxLdsBytes;
  if (chol_in_lds && chol_lds > kDefaultLdsBytes &&
      (e = hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_kernel<true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)chol_lds)) != hipSuccess)
    return hip_fail("hipFuncSetAttribute");
  if (fs_in_lds && fs_lds > kDefaultLdsBytes &&
      (e = hipFuncSetAttribute(reinterpret_cast<const void*>(&factor_solve_kernel<true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)fs_lds)) != hipSuccess)
    return hip_fail("hipFuncSetAttribute");
  auto chol = [&](double* A, int nb, double thr, int fail_value, int32_t* ver) {
    if (chol_in_lds)
      hipLaunchKernelGGL(chol_kernel<true>, dim3(nb), dim3(chol_threads), chol_lds, st, A, p, thr, fail_value, ver);
    else
      hipLaunchKernelGGL(chol_kernel<false>, dim3(nb), dim3(chol_threads), 0, st, A, p, thr, fail_value, ver);
  };
  auto factor_solve = [&](int nb, double thr, int32_t* ver) {
    if (fs_in_lds)
      hipLaunchKernelGGL(factor_solve_kernel<true>, dim3(nb), dim3(chol_threads), fs_lds, st, Sm, Wm, p, thr, ver);
    else
      hipLaunchKernelGGL(factor_solve_kernel<false>, dim3(nb), dim3(chol_threads), 0, st, Sm, Wm, p, thr, ver);
  };
  // one batch of nb subdomains (order[pos0 .. pos0 + nb)) with ks levels each
  auto run_batch = [&](int pos0, int nb, int ks, double mu) -> hipError_t {
    const int32_t* subs = order_d + pos0;
    int32_t* ver = verdict_d + pos0;
    const int64_t elems = nb * pp;
    const double thr = 1e-9 * mu;
    double* Bc = La;    // B_j of the current level
    double* Ln = Lb;    // L_{j+1}
    hipError_t r;
    hipLaunchKernelGGL(gather_rounded_kernel, grid(elems), dim3(256), 0, st, c->coef64_d, subs, nb, k, p, 0, 0, prec, Gc);
    hipLaunchKernelGGL(level_one_kernel, grid(elems), dim3(256), 0, st, c->coef64_d, subs, nb, k, p, Gc, mu, Bc, Sm);
    if ((r = hipGetLastError()) != hipSuccess) return r;
    for (int j = 0; j + 1 < ks; ++j) {     // 0-based level j: S_j -> S_{j+1}
      hipLaunchKernelGGL(gather_rounded_kernel, grid(elems), dim3(256), 0, st, c->coef64_d, subs, nb, k, p, 1, j + 1,
                         prec, Ln);
      chol(Ln, nb, 0.0, -1, ver);
      if (j > 0)
        hipLaunchKernelGGL(gather_rounded_kernel, grid(elems), dim3(256), 0, st, c->coef64_d, subs, nb, k, p, 0, j,
                           prec, Gc);
      hipLaunchKernelGGL(gather_rounded_kernel, grid(elems), dim3(256), 0, st, c->coef64_d, subs, nb, k, p, 0, j + 1,
                         prec, Gn);
      if ((r = hipGetLastError()) != hipSuccess) return r;
      // T = Gamma_j B_j;  W = E_j^T = -T^T L_{j+1};  R_j = chol(S_j), W <- R_j^{-1} W
      if ((r = dgemm_batched(false, false, p, p, p, 1.0, Gc, p, pp, Bc, p, pp, 0.0, Tm, p, pp, nb, st, nullptr, 0)) !=
          hipSuccess)
        return r;
      if ((r = dgemm_batched(true, false, p, p, p, -1.0, Tm, p, pp, Ln, p, pp, 0.0, Wm, p, pp, nb, st, nullptr, 0)) !=
          hipSuccess)
        return r;
      factor_solve(nb, thr, ver);
      // T = (Gamma_{j+1} + Gamma_j) L_{j+1};  S_{j+1} = mu I - L_{j+1}^T T - W^T W
      hipLaunchKernelGGL(add_kernel, grid(elems), dim3(256), 0, st, Gn, Gc, elems);
      hipLaunchKernelGGL(set_mu_kernel, grid(elems), dim3(256), 0, st, Sm, p, nb, mu);
      if ((r = hipGetLastError()) != hipSuccess) return r;
      if ((r = dgemm_batched(false, false, p, p, p, 1.0, Gn, p, pp, Ln, p, pp, 0.0, Tm, p, pp, nb, st, nullptr, 0)) !=
          hipSuccess)
        return r;
      if ((r = dgemm_batched(true, false, p, p, p, -1.0, Ln, p, pp, Tm, p, pp, 1.0, Sm, p, pp, nb, st, nullptr, 0)) !=
          hipSuccess)
        return r;
      if ((r = dgemm_batched(true, false, p, p, p, -1.0, Wm, p, pp, Wm, p, pp, 1.0, Sm, p, pp, nb, st, nullptr, 0)) !=
          hipSuccess)
        return r;
      std::swap(Bc, Ln);
    }
    chol(Sm, nb, thr, 0, ver);
    return hipGetLastError();
  };
  auto passes = [&](double mu, bool* ok) -> sfm_status {
    hipLaunchKernelGGL(fill_kernel, grid(S), dim3(256), 0, st, verdict_d, S, 1);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail("stability certificate");
    for (int pos = 0; pos < S;) {
      const int ks = levels[order[pos]];
      int end = pos;
      while (end < S && levels[order[end]] == ks && end - pos < batch) ++end;
      if ((e = run_batch(pos, end - pos, ks, mu)) != hipSuccess) return hip_fail("stability certificate");
      pos = end;
    }
    if ((e = hipMemcpyAsync(verdict.data(), verdict_d, S * sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail("hipMemcpyAsync");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail("hipStreamSynchronize");
    *ok = true;
    for (int q = 0; q < S; ++q) {
      if (verdict[q] < 0)
        return c->fail(SFM_EUNSTABLE, "subdomain " + std::to_string(order[q]) +
                                          ": a Gamma-hat block is not positive definite in the stored precision");
      if (verdict[q] == 0) *ok = false;
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
  const int batch = std::min(c->topo.S, 2048);
  const size_t bytes = (sfm::cfl_index_bytes(c->topo.S) + 255) / 256 * 256 +
                       batch * sfm::cfl_scratch_bytes_per_member(c->topo.p);
  void* scratch = c->dalloc(bytes, &e);
  if (!scratch) return c->fail(SFM_ENOMEM, "stability certificate: out of device memory");
  const sfm_status rc = sfm::cfl_limit(c, iters, scratch, batch, dt_max, reinterpret_cast<hipStream_t>(stream));
  c->dfree(scratch);
  return rc;
}

// ----------------------------------------------------------------------------- no-allocation variant
// The certificate's scratch (work matrices and verdicts) in one file-scope device array.  In host
// code `scratch` names a host-side stand-in, not device memory: its device address is taken once
// per device with hipGetSymbolAddress, with that device current, and only that address is used.
namespace {
constexpr size_t kStaticIndexBytes = size_t(2) << 20;            // verdicts + order: S <= 262,144
constexpr size_t kStaticScratchBytes = size_t(64) << 20;         // 62 MiB of work matrices + the index
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

extern "C" sfm_status sfm_cfl_dt_noalloc(sfm_ctx c, int32_t iters, double* dt_max, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  const size_t per_member = sfm::cfl_scratch_bytes_per_member(c->topo.p);
  if (sfm::cfl_index_bytes(c->topo.S) > kStaticIndexBytes)
    return c->fail(SFM_EINVAL, "sfm_cfl_dt_noalloc: " + std::to_string(c->topo.S) +
                                   " subdomains exceed the static scratch limit of " +
                                   std::to_string(kStaticIndexBytes / (2 * sizeof(int32_t))));
  const size_t members = (kStaticScratchBytes - kStaticIndexBytes) / per_member;
  if (members < 1)
    return c->fail(SFM_EINVAL, "sfm_cfl_dt_noalloc: 6m = " + std::to_string(c->topo.p) +
                                   " needs more than the static scratch of one subdomain");
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
  // the index region is a multiple of 256 bytes, so the matrices start where cfl_limit puts them
  static_assert(kStaticIndexBytes % 256 == 0, "index region alignment");
  const int batch = (int)std::min<size_t>({(size_t)c->topo.S, size_t(2048), members});
  return sfm::cfl_limit(c, iters, base, batch, dt_max, reinterpret_cast<hipStream_t>(stream));
}
