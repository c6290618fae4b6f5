// Batched FP64 dense kernels of the Stage 1 build (Algorithm 1, steps 1.1-1.3): the block Lanczos
// projections and re-orthogonalisation (eq. "krylov0" spaces), the Gram matrices and inverse
// factors of Cholesky QR, and the p x p products and triangular solves of the S-fraction
// recursion (eq. "GammaTrans").  Operands are column-major like BLAS:
//     C_b = alpha op(A_b) op(B_b) + beta C_b,   op(X) = X or X^T,   b < batch.
//
// dgemm_kernel runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  A work-group of four waves
// owns a BM x BN tile of C (BM = 32 TM, BN = 32 TN; waves in a 2 x 2 grid, each TM x TN MFMA tiles
// of 16 x 16) and walks K in stages of 16: the next stage of op(A) and op(B) is loaded from HBM into
// registers (coalesced along whichever index is contiguous in memory) while the MFMAs of the
// current stage read LDS.  The product is formed transposed (MFMA rows = columns of C), so each
// result register of a lane group maps to 16 consecutive rows of C and the stores are 128-byte
// runs.  Long reductions (K of tens of thousands of grid nodes against a small C) are split over
// work-groups; the partial tiles are summed in a fixed order by dgemm_reduce_kernel, so results
// are bit-reproducible.
//
// Triangular kernels (one work-group per matrix, one thread per right-hand-side column, forward
// or backward substitution with compensated sums: a product's rounding error is recovered with
// fma and carried in a second accumulator, so the solve is as accurate as one in twice the
// working precision for the moderately conditioned factors the build produces).
#include <algorithm>

#include "sfm_internal.h"

namespace sfm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

#ifndef SFM_GEMM_BK
#define SFM_GEMM_BK 16
#endif
constexpr int kBK = SFM_GEMM_BK;   // K per LDS stage
constexpr int kGemmThreads = 256;  // four waves
constexpr int kPad = 2;            // LDS row padding (doubles)

struct GemmArgs {
  int M, N, K, batch, ksplit, kchunk;
  double alpha, beta;
  const double* A;
  int64_t lda, sA;
  const double* B;
  int64_t ldb, sB;
  double* C;
  int64_t ldc, sC;
  double* part;   // ksplit > 1: partial tiles [batch][ksplit][N][M] (column-major, ld M)
};

template <bool TA, bool TB, int TM, int TN>
__global__ __launch_bounds__(kGemmThreads) void dgemm_kernel(GemmArgs g) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  constexpr int LA = BM * kBK / kGemmThreads, LB = BN * kBK / kGemmThreads;   // loads per thread
  __shared__ double As[kBK][BM + kPad];   // op(A)(m, k) at As[k][m]
  __shared__ double Bs[kBK][BN + kPad];   // op(B)(k, n) at Bs[k][n]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int tiles_m = (g.M + BM - 1) / BM;
  const int m0 = (blockIdx.x % tiles_m) * BM, n0 = (blockIdx.x / tiles_m) * BN;
  const int split = blockIdx.y, b = blockIdx.z;
  const int kbeg = split * g.kchunk, kend = min(g.K, kbeg + g.kchunk);
  const double* A = g.A + (int64_t)b * g.sA;
  const double* B = g.B + (int64_t)b * g.sB;
  // element e of a stage: the index that is contiguous in memory runs fastest across threads
  auto load_a = [&](int k0, double (&r)[LA]) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int e = tid + q * kGemmThreads;
      const int m = TA ? e / kBK : e % BM, k = TA ? e % kBK : e / BM;
      const int gm = m0 + m, gk = k0 + k;
      r[q] = (gm < g.M && gk < kend) ? (TA ? A[gk + (int64_t)gm * g.lda] : A[gm + (int64_t)gk * g.lda]) : 0.0;
    }
  };
  auto load_b = [&](int k0, double (&r)[LB]) {
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + q * kGemmThreads;
      const int n = TB ? e % BN : e / kBK, k = TB ? e / BN : e % kBK;
      const int gn = n0 + n, gk = k0 + k;
      r[q] = (gn < g.N && gk < kend) ? (TB ? B[gn + (int64_t)gk * g.ldb] : B[gk + (int64_t)gn * g.ldb]) : 0.0;
    }
  };
  auto store_a = [&](const double (&r)[LA]) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int e = tid + q * kGemmThreads;
      const int m = TA ? e / kBK : e % BM, k = TA ? e % kBK : e / BM;
      As[k][m] = r[q];
    }
  };
  auto store_b = [&](const double (&r)[LB]) {
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + q * kGemmThreads;
      const int n = TB ? e % BN : e / kBK, k = TB ? e / BN : e % kBK;
      Bs[k][n] = r[q];
    }
  };
  // wave (wm, wn): rows m0 + wm 16 TM .., columns n0 + wn 16 TN ..
  const int wm = wave & 1, wn = wave >> 1;
  d4 acc[TN][TM];
#pragma unroll
  for (int j = 0; j < TN; ++j)
#pragma unroll
    for (int i = 0; i < TM; ++i) acc[j][i] = d4{0.0, 0.0, 0.0, 0.0};
  double ra[LA], rb[LB];
  if (kbeg < kend) {
    load_a(kbeg, ra);
    load_b(kbeg, rb);
  }
  for (int k0 = kbeg; k0 < kend; k0 += kBK) {
    __syncthreads();                 // the previous stage's MFMAs are done with LDS
    store_a(ra);
    store_b(rb);
    __syncthreads();
    if (k0 + kBK < kend) {           // next stage in flight during this stage's MFMAs
      load_a(k0 + kBK, ra);
      load_b(k0 + kBK, rb);
    }
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      double av[TM], bv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) av[i] = As[kk + lg][wm * 16 * TM + i * 16 + li];
#pragma unroll
      for (int j = 0; j < TN; ++j) bv[j] = Bs[kk + lg][wn * 16 * TN + j * 16 + li];
      // D(n, m) += sum_k op(B)(k, n) op(A)(m, k): the MFMA's rows are C's columns
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int i = 0; i < TM; ++i) acc[j][i] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[j], av[i], acc[j][i], 0, 0, 0);
    }
  }
  // acc[j][i] element v: column n = .. j 16 + lg + 4 v, row m = .. i 16 + li
#pragma unroll
  for (int j = 0; j < TN; ++j)
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * 16 * TM + i * 16 + li;
        const int n = n0 + wn * 16 * TN + j * 16 + lg + 4 * v;
        if (m < g.M && n < g.N) {
          if (g.ksplit > 1) {
            g.part[(((int64_t)b * g.ksplit + split) * g.N + n) * g.M + m] = acc[j][i][v];
          } else {
            double* c = g.C + (int64_t)b * g.sC + m + (int64_t)n * g.ldc;
            *c = g.beta == 0.0 ? g.alpha * acc[j][i][v] : fma(g.alpha, acc[j][i][v], g.beta * *c);
          }
        }
      }
}

// C = alpha sum_split part + beta C, the splits summed in order.
__global__ void dgemm_reduce_kernel(GemmArgs g) {
  const int64_t mn = (int64_t)g.M * g.N;
  const int64_t total = mn * g.batch;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / mn, r = e - b * mn;
    const int n = (int)(r / g.M), m = (int)(r - (int64_t)n * g.M);
    const double* p = g.part + b * g.ksplit * mn + r;
    double s = 0.0;
    for (int q = 0; q < g.ksplit; ++q) s += p[q * mn];
    double* c = g.C + b * g.sC + m + (int64_t)n * g.ldc;
    *c = g.beta == 0.0 ? g.alpha * s : fma(g.alpha, s, g.beta * *c);
  }
}

// Compensated accumulation: s + e carries sum a_i b_i with the product and sum errors of each term.
__device__ __forceinline__ void acc2(double& s, double& e, double a, double b) {
  const double p = a * b;
  const double pe = fma(a, b, -p);            // a b = p + pe exactly
  const double t = s + p;
  const double z = t - s;
  e += ((s - (t - z)) + (p - z)) + pe;        // s + p = t + (that) exactly
  s = t;
}

// X_b = L_b^{-1} (lower triangular, non-unit), p x p column-major (lda p), written to X; one thread
// per column of X (X has the identity's column), forward substitution.  With kLds, L and X are
// staged in LDS (X's columns padded to p + 1); the arithmetic and its order are the same.
template <bool kLds>
__global__ void trtri_lower_kernel(const double* __restrict__ L, int64_t sL, double* __restrict__ X, int64_t sX,
                                   int p) {
  extern __shared__ __align__(16) double tri_lds[];
  const double* Lg = L + (int64_t)blockIdx.x * sL;
  double* Xg = X + (int64_t)blockIdx.x * sX;
  const int ldx = kLds ? p + 1 : p;
  if (kLds) {
    for (int e = threadIdx.x; e < p * p; e += blockDim.x) tri_lds[e] = Lg[e];
    __syncthreads();
  }
  const double* Lb = kLds ? tri_lds : Lg;
  double* Xb = kLds ? tri_lds + p * p : Xg;
  for (int c = threadIdx.x; c < p; c += blockDim.x) {
    for (int r = 0; r < c; ++r) Xb[r + (int64_t)c * ldx] = 0.0;
    for (int r = c; r < p; ++r) {
      double s = r == c ? 1.0 : 0.0, e = 0.0;
      for (int i = c; i < r; ++i) acc2(s, e, -Lb[r + (int64_t)i * p], Xb[i + (int64_t)c * ldx]);
      Xb[r + (int64_t)c * ldx] = (s + e) / Lb[r + (int64_t)r * p];
    }
  }
  if (kLds) {
    __syncthreads();
    for (int e = threadIdx.x; e < p * p; e += blockDim.x) Xg[e] = Xb[e % p + (int64_t)(e / p) * ldx];
  }
}

// B_b <- alpha op(L_b)^{-1} B_b, L lower triangular non-unit (p x p, ld p), B p x p (ld p); one
// thread per column of B: forward substitution for op = N, backward for op = T.  With kLds, L and B
// are staged in LDS (B's columns padded to p + 1); the arithmetic and its order are the same.
template <bool kLds>
__global__ void trsm_lower_kernel(const double* __restrict__ L, int64_t sL, double* __restrict__ Bm, int64_t sB,
                                  int p, int trans, double alpha) {
  extern __shared__ __align__(16) double tri_lds[];
  const double* Lg = L + (int64_t)blockIdx.x * sL;
  double* Bg = Bm + (int64_t)blockIdx.x * sB;
  const int ldb = kLds ? p + 1 : p;
  if (kLds) {
    for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
      tri_lds[e] = Lg[e];
      tri_lds[p * p + e % p + (e / p) * ldb] = Bg[e];
    }
    __syncthreads();
  }
  const double* Lb = kLds ? tri_lds : Lg;
  double* Bb = kLds ? tri_lds + p * p : Bg;
  for (int c = threadIdx.x; c < p; c += blockDim.x) {
    double* x = Bb + (int64_t)c * ldb;
    if (!trans) {
      for (int r = 0; r < p; ++r) {
        double s = alpha * x[r], e = fma(alpha, x[r], -s);
        for (int i = 0; i < r; ++i) acc2(s, e, -Lb[r + (int64_t)i * p], x[i]);
        x[r] = (s + e) / Lb[r + (int64_t)r * p];
      }
    } else {   // L^T is upper: row r of L^T is column r of L
      for (int r = p - 1; r >= 0; --r) {
        double s = alpha * x[r], e = fma(alpha, x[r], -s);
        for (int i = r + 1; i < p; ++i) acc2(s, e, -Lb[i + (int64_t)r * p], x[i]);
        x[r] = (s + e) / Lb[r + (int64_t)r * p];
      }
    }
  }
  if (kLds) {
    __syncthreads();
    for (int e = threadIdx.x; e < p * p; e += blockDim.x) Bg[e] = Bb[e % p + (int64_t)(e / p) * ldb];
  }
}

// LDS of the staged triangular kernels: L and a padded p x p right-hand side.  Staging pays while
// several matrices still share a CU's LDS in flight with the global version's occupancy: measured
// faster at 6m = 72 (the many-shot build: 14.6 -> 13.7 s), slower at 6m = 96 (one work-group of
// 96 busy threads per CU; the 512^3 build 23.0 -> 24.6 s), so it is used up to 6m = 80.
size_t tri_lds_bytes(int p) { return ((size_t)p * p + (size_t)p * (p + 1)) * sizeof(double); }
constexpr int kTriLdsMaxP = 80;

template <bool TA, bool TB, int TM, int TN>
hipError_t launch_tile(GemmArgs& g, hipStream_t st) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  hipLaunchKernelGGL((dgemm_kernel<TA, TB, TM, TN>), dim3(tiles, g.ksplit, g.batch), dim3(kGemmThreads), 0, st, g);
  return hipGetLastError();
}

template <bool TA, bool TB>
hipError_t launch_trans(GemmArgs& g, int tm, int tn, hipStream_t st) {
  if (tm == 3 && tn == 3) return launch_tile<TA, TB, 3, 3>(g, st);
  if (tm == 3 && tn == 1) return launch_tile<TA, TB, 3, 1>(g, st);
  if (tm == 1 && tn == 3) return launch_tile<TA, TB, 1, 3>(g, st);
  return launch_tile<TA, TB, 1, 1>(g, st);
}

// Sustained FP64 matrix-core rate: every wave runs `iters` rounds of eight independent
// 16 x 16 x 4 MFMA accumulation chains on register operands (no memory traffic in the loop).
__global__ __launch_bounds__(256) void mfma_rate_kernel(double* out, int iters) {
  d4 acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  const double a = 1.0 + threadIdx.x * 1e-9, b = 1.0 - threadIdx.x * 1e-9;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

size_t dgemm_workspace_bytes(int M, int N, int K, int batch) {
  (void)K;
  return (size_t)8 * kMaxGemmSplit * M * N * batch;
}

hipError_t dgemm_batched(bool tA, bool tB, int M, int N, int K, double alpha, const double* A, int64_t lda,
                         int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, double* C, int64_t ldc,
                         int64_t sC, int batch, hipStream_t st, double* work, size_t work_bytes) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  GemmArgs g{};
  g.M = M; g.N = N; g.K = std::max(K, 0); g.batch = batch;
  g.alpha = alpha; g.beta = beta;
  g.A = A; g.lda = lda; g.sA = sA;
  g.B = B; g.ldb = ldb; g.sB = sB;
  g.C = C; g.ldc = ldc; g.sC = sC;
  // tiles of 96 (3 MFMA tiles per wave) along a dimension above 32, else 32; a short reduction
  // that also reads C back (beta != 0) is bound by the C traffic, and narrower column tiles
  // (twice the work-groups per CU) move it faster
  const int tm = M > 32 ? 3 : 1, tn = (N > 32 && (K > 256 || beta == 0.0)) ? 3 : 1;
  const int64_t tiles = (int64_t)((M + 32 * tm - 1) / (32 * tm)) * ((N + 32 * tn - 1) / (32 * tn)) * batch;
  // split long reductions until the grid holds about 2048 work-groups, each at least 1024 deep
  int ksplit = 1;
  while (ksplit < kMaxGemmSplit && tiles * ksplit < 2048 && (int64_t)g.K / (2 * ksplit) >= 1024) ksplit *= 2;
  if ((size_t)8 * ksplit * M * N * batch > work_bytes || !work) ksplit = 1;
  g.ksplit = ksplit;
  g.kchunk = ksplit == 1 ? std::max(g.K, 1) : (g.K + ksplit - 1) / ksplit;
  g.kchunk = (g.kchunk + kBK - 1) / kBK * kBK;
  g.part = work;
  SFM_DCHECK(lda >= (tA ? K : M) && ldb >= (tB ? N : K) && ldc >= M);
  hipError_t e;
  if (!tA && !tB) e = launch_trans<false, false>(g, tm, tn, st);
  else if (!tA && tB) e = launch_trans<false, true>(g, tm, tn, st);
  else if (tA && !tB) e = launch_trans<true, false>(g, tm, tn, st);
  else e = launch_trans<true, true>(g, tm, tn, st);
  if (e != hipSuccess || ksplit == 1) return e;
  const int64_t total = (int64_t)M * N * batch;
  hipLaunchKernelGGL(dgemm_reduce_kernel, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65536)), dim3(256), 0,
                     st, g);
  return hipGetLastError();
}

hipError_t trtri_lower_batched(const double* L, int64_t sL, double* X, int64_t sX, int p, int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  const dim3 threads(std::min(256, (p + 63) / 64 * 64));
  const size_t lds = tri_lds_bytes(p);
  if (p <= kTriLdsMaxP && lds <= kMaxLdsBytes) {
    if (lds > kDefaultLdsBytes) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&trtri_lower_kernel<true>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(trtri_lower_kernel<true>, dim3(batch), threads, lds, st, L, sL, X, sX, p);
  } else {
    hipLaunchKernelGGL(trtri_lower_kernel<false>, dim3(batch), threads, 0, st, L, sL, X, sX, p);
  }
  return hipGetLastError();
}

hipError_t trsm_lower_batched(bool trans, double alpha, const double* L, int64_t sL, double* B, int64_t sB, int p,
                              int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  const dim3 threads(std::min(256, (p + 63) / 64 * 64));
  const size_t lds = tri_lds_bytes(p);
  if (p <= kTriLdsMaxP && lds <= kMaxLdsBytes) {
    if (lds > kDefaultLdsBytes) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&trsm_lower_kernel<true>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(trsm_lower_kernel<true>, dim3(batch), threads, lds, st, L, sL, B, sB, p, trans ? 1 : 0, alpha);
  } else {
    hipLaunchKernelGGL(trsm_lower_kernel<false>, dim3(batch), threads, 0, st, L, sL, B, sB, p, trans ? 1 : 0, alpha);
  }
  return hipGetLastError();
}

}  // namespace sfm

extern "C" sfm_status sfm_dgemm_batched(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K,
                                        double alpha, const double* A, int64_t lda, int64_t stride_a,
                                        const double* B, int64_t ldb, int64_t stride_b, double beta, double* C,
                                        int64_t ldc, int64_t stride_c, int32_t batch, double* work,
                                        int64_t work_bytes, void* stream) {
  if (M < 0 || N < 0 || K < 0 || batch < 0 || lda < std::max(1, trans_a ? K : M) ||
      ldb < std::max(1, trans_b ? N : K) || ldc < std::max(1, M) || work_bytes < 0)
    return SFM_EINVAL;
  if ((int64_t)M * N * batch > 0 && (!C || (K > 0 && (!A || !B)))) return SFM_EINVAL;
  const hipError_t e = sfm::dgemm_batched(trans_a != 0, trans_b != 0, M, N, K, alpha, A, lda, stride_a, B, ldb,
                                          stride_b, beta, C, ldc, stride_c, batch,
                                          reinterpret_cast<hipStream_t>(stream), work, (size_t)work_bytes);
  return e == hipSuccess ? SFM_OK : SFM_EHIP;
}

extern "C" sfm_status sfm_probe_fp64_matrix_rate(int32_t blocks, int32_t iters, double* out, double* tflops,
                                                 void* stream) {
  if (blocks < 1 || iters < 1 || !out || !tflops) return SFM_EINVAL;
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return SFM_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SFM_EHIP;
  }
  float ms = 0.0f;
  hipError_t e = hipEventRecord(e0, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(sfm::mfma_rate_kernel, dim3(blocks), dim3(256), 0, st, out, iters);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess || !(ms > 0.0f)) return SFM_EHIP;
  // four waves per work-group, eight 16 x 16 x 4 products (2 * 1024 flops) per wave and round
  *tflops = (double)blocks * 4 * 8 * (double)iters * 2048.0 / (ms * 1e-3) / 1e12;
  return SFM_OK;
}
