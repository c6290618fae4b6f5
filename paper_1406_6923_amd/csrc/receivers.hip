// Receiver recording: u(x_r) = e_r^T M^{-1/2} Z G^{-1} U = sum_j r_j . U_j (inverse of eq. "Uj").
//
// Per step the leapfrog kernels copy the new state of every subdomain that holds receivers into
// a history ring of kHistWindow time slots; once per window a tiled FP32 product
//   traces[r][t] = rows[r] . hist[t][slot(r)]
// turns the ring into trace samples, so each receiver row (k p words) is read from HBM once per
// window instead of once per step.  record_kernel samples the current state directly.
#include <algorithm>

#include "sfm_internal.h"

namespace sfm {
namespace {

// One wave per (sorted) receiver.
__global__ __launch_bounds__(256) void record_kernel(RecParams prm) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + wave;
  if (r >= prm.nrec) return;
  const int n = prm.k * prm.P16;
  const float* row = prm.rows + (size_t)r * n;
  const float* u = prm.U + (size_t)prm.rec_sub[r] * n;
  float acc = 0.f;
  for (int e = lane; e < n; e += 64) acc = fmaf(row[e], u[e], acc);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) prm.out[(size_t)prm.perm[r] * prm.ld + prm.col] = acc;
}

constexpr int kTR = 64;   // receivers per tile
constexpr int kTT = 64;   // time samples per tile (= kHistWindow)
constexpr int kTK = 32;   // reduction chunk

// C[r][t] = sum_e R[r][e] H[t][e] for one receiver subdomain: blockIdx.y = subdomain slot,
// blockIdx.x = tile of 64 receivers; 256 threads, 4 x 4 outputs each.  The next 64 x 32 chunks of
// R and H are loaded into registers while the products of the current ones run from LDS.
__global__ __launch_bounds__(256) void record_window_kernel(RecWindowParams prm) {
  __shared__ float Rs[kTK][kTR + 4];
  __shared__ float Hs[kTK][kTT + 4];
  const int slot = blockIdx.y;
  const int r0 = prm.rs_off[slot] + blockIdx.x * kTR;
  const int r1 = prm.rs_off[slot + 1];
  if (r0 >= r1) return;
  const int K = prm.k * prm.P16;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const float* H = prm.hist + (size_t)slot * K;
  const size_t hstride = (size_t)prm.n_rs * K;
  constexpr int kPer = kTR * kTK / 256;   // words of each tile per thread
  static_assert(kTR == kTT && kTR * kTK % 256 == 0, "tile shape");
  float rv[kPer], hv[kPer];
  // 64 x 32 tiles of R and H, coalesced along e
  auto load = [&](int k0) {
#pragma unroll
    for (int v = 0; v < kPer; ++v) {
      const int q = tid + 256 * v;
      const int rr = q / kTK, kk = q % kTK;
      const int r = r0 + rr, e = k0 + kk;
      rv[v] = (r < r1 && e < K) ? prm.rows[(size_t)r * K + e] : 0.f;
      hv[v] = (rr < prm.w && e < K) ? H[(size_t)rr * hstride + e] : 0.f;
    }
  };
  float acc[4][4] = {};
  load(0);
  for (int k0 = 0; k0 < K; k0 += kTK) {
#pragma unroll
    for (int v = 0; v < kPer; ++v) {
      const int q = tid + 256 * v;
      const int rr = q / kTK, kk = q % kTK;
      Rs[kk][rr] = rv[v];
      Hs[kk][rr] = hv[v];
    }
    __syncthreads();
    if (k0 + kTK < K) load(k0 + kTK);
#pragma unroll 8
    for (int kk = 0; kk < kTK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = Rs[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Hs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + ty * 4 + i;
    if (r >= r1) continue;
    float* out = prm.traces + (size_t)prm.perm[r] * prm.ld + prm.col0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = tx * 4 + j;
      if (t < prm.w) out[t] = acc[i][j];
    }
  }
}

}  // namespace

hipError_t launch_record(const RecParams& prm, hipStream_t st) {
  if (prm.nrec == 0) return hipSuccess;
  hipLaunchKernelGGL(record_kernel, dim3((prm.nrec + 3) / 4), dim3(256), 0, st, prm);
  return hipGetLastError();
}

hipError_t launch_record_window(const RecWindowParams& prm, hipStream_t st, int max_per_slot) {
  if (prm.n_rs == 0 || prm.w <= 0) return hipSuccess;
  SFM_DCHECK(prm.w <= kHistWindow && max_per_slot >= 1 && prm.rs_off && prm.perm && prm.rows && prm.hist);
  SFM_DCHECK(prm.traces && prm.ld >= prm.col0 + prm.w);
  const dim3 grid((max_per_slot + kTR - 1) / kTR, prm.n_rs);
  hipLaunchKernelGGL(record_window_kernel, grid, dim3(256), 0, st, prm);
  return hipGetLastError();
}

}  // namespace sfm
