// Stage 2 kernels: one leapfrog step of the coupled subdomain ROMs (Algorithm 1, steps 2.1-2.3).
//
// step_main  (one work-group per subdomain, 16 rows of 16 lanes)
//   layer fluxes   phi_j = Gamma_j (U_{j+1} - U_j), j = 1..k, U_{k+1} = 0          (eq. "intrtstep")
//   exchange       phi_1 -> exch[s]  (the m-vectors of step 2.1)
//   interior       a_j = Gamma-hat_j (phi_j - phi_{j-1}) + f(t_n) s_j, j = 2..k  (step 2.2)
//   leapfrog       D_j += dt^2 a_j, U_j += D_j  (D = U^n - U^{n-1}, same recursion as
//                  U^{n+1} = 2U^n - U^{n-1} + dt^2 a with better rounding)
// step_face  (one lane per boundary-layer entry)
//   boundary       a_f = C_f (phi_1^alpha + phi_1^beta) + f(t_n) w_f                  (eq. "bdrytstep", 2.3)
//
// The coefficient blocks stream from HBM once per step in the tile layout described in
// sfm_internal.h; each 16-lane row holds one tile and forms both halves of the symmetric
// product with DPP row rotations, so no coefficient word is read twice and no LDS
// staging of coefficients is needed.  Partial sums go to distinct LDS slots and are
// reduced in a fixed order: results are bit-reproducible run to run.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <type_traits>

#include "sfm_internal.h"

#include "tile_ops.h"

namespace sfm {
namespace {

template <typename T>
__global__ __launch_bounds__(kStepThreads) void step_main_kernel(StepParams prm) {
  typedef typename Acc<T>::type R;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* smem = reinterpret_cast<R*>(smem_raw);
  const int s = prm.order ? prm.order[blockIdx.x] : (int)blockIdx.x;
  const int tid = threadIdx.x;
  const int k = prm.k, P = prm.P16;
  const int vstride = P;
  R* xs = smem;                           // [k][P]   block inputs
  R* ph = xs + k * vstride;               // [k][P]   layer fluxes phi_j
  R* part = ph + k * vstride;             // [k][nslots][16]
  const size_t sbase = (size_t)s * k * P;
  const float* Uin = prm.mode == 0 ? prm.U : prm.Uin;
  const T* tiles = reinterpret_cast<const T*>(prm.tiles) + (size_t)s * prm.words_per_sub;
  // levels of this subdomain's ROM (the leading ks of the stored k; the others stay zero)
  const int ks = prm.k_of ? prm.k_of[s] : k;

  // U_{j+1} - U_j with U_{ks+1} = 0
  for (int e = tid; e < ks * P; e += kStepThreads) {
    const int j = e / P;
    const float uf = Uin[sbase + e];
    const R u = uf;
    const R un = (j + 1 < ks) ? (R)Uin[sbase + e + P] : (R)0;
    xs[e] = un - u;
    if (prm.u_out) prm.u_out[sbase + e] = uf;
  }
  if (prm.u_out)
    for (int e = ks * P + tid; e < k * P; e += kStepThreads) prm.u_out[sbase + e] = Uin[sbase + e];
  __syncthreads();
  run_phase<T, R>(tiles, ks, prm, xs, vstride, part, tid);      // phi_j = Gamma_j dU_j
  __syncthreads();
  for (int e = tid; e < ks * P; e += kStepThreads) {
    const int b = e / P, i = e - b * P;
    ph[e] = reduce_entry(part, b, i, prm.nt, prm.nslots);
  }
  __syncthreads();
  for (int e = tid; e < P; e += kStepThreads) prm.exch[(size_t)s * P + e] = (float)ph[e];   // step 2.1
  for (int e = tid; e < (ks - 1) * P; e += kStepThreads) {
    xs[e] = ph[e + P] - ph[e];                                          // phi_j - phi_{j-1}
    if (prm.kx_out) prm.kx_out[sbase + P + e] = (float)xs[e];           // (-K U)_j, j >= 2
  }
  __syncthreads();
  run_phase<T, R>(tiles + (size_t)k * prm.words_per_block, ks - 1, prm, xs, vstride, part, tid);
  __syncthreads();
  const int slot = (prm.mode == 0 && prm.hist) ? prm.hist_slot[s] : -1;
  const int s0 = prm.src_off ? prm.src_off[s] : 0;
  const int s1 = prm.src_off ? prm.src_off[s + 1] : 0;
  if (prm.mode != 0)
    for (int e = (ks - 1) * P + tid; e < (k - 1) * P; e += kStepThreads) prm.Aout[sbase + P + e] = 0.f;
  for (int e = tid; e < (ks - 1) * P; e += kStepThreads) {
    const int b = e / P, i = e - b * P;
    R a = reduce_entry(part, b, i, prm.nt, prm.nslots);
    for (int q = s0; q < s1; ++q) {
      const int src = prm.src_ids[q];
      a = mad((R)prm.wavelet[prm.step * prm.nsrc + src], (R)prm.src_vec[((size_t)src * k + b + 1) * P + i], a);
    }
    const size_t idx = sbase + (size_t)(b + 1) * P + i;
    if (prm.mode == 0) {
      const float d = (float)mad((R)prm.dt2, a, (R)prm.D[idx]);
      const float un = prm.U[idx] + d;
      prm.D[idx] = d;
      prm.U[idx] = un;
      if (slot >= 0) prm.hist[prm.hist_off + ((size_t)slot * k + b + 1) * P + i] = un;
    } else {
      prm.Aout[idx] = (float)a;
    }
  }
}

__global__ void step_face_kernel(FaceParams prm) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)prm.S * prm.p) return;
  const int s = (int)(idx / prm.p);
  const int q = (int)(idx - (int64_t)s * prm.p);
  const int f = q / prm.m, pat = q - f * prm.m;
  const int nb = prm.nbr[s * 6 + f];
  float flux = prm.exch[(size_t)s * prm.P16 + q];
  if (nb >= 0) flux += prm.exch[(size_t)nb * prm.P16 + (f ^ 1) * prm.m + pat];
  float a = prm.C[(size_t)s * prm.P16 + q] * flux;
  if (prm.sw_off) {
    for (int e = prm.sw_off[s]; e < prm.sw_off[s + 1]; ++e) {
      if (prm.sw_q[e] == q) a = fmaf(prm.sw_w[e], prm.wavelet[prm.step * prm.nsrc + prm.sw_src[e]], a);
    }
  }
  const size_t u = (size_t)s * prm.k * prm.P16 + q;
  if (prm.mode == 0) {
    const float d = fmaf(prm.dt2, a, prm.D[u]);
    const float un = prm.U[u] + d;
    prm.D[u] = d;
    prm.U[u] = un;
    if (prm.hist) {
      const int slot = prm.hist_slot[s];
      if (slot >= 0) prm.hist[prm.hist_off + (size_t)slot * prm.k * prm.P16 + q] = un;
    }
  } else {
    prm.Aout[u] = a;
  }
}

// Pack full FP64 blocks into the tile stream: out[s][b][w] = blk(s, b)[wrow[w]][wcol[w]].
template <typename T>
__global__ void pack_kernel(const double* __restrict__ blocks, int k, int p, int64_t wpb,
                            const int32_t* __restrict__ wrow, const int32_t* __restrict__ wcol,
                            T* __restrict__ out, int S) {
  const int64_t nb_out = 2 * k - 1;
  const int64_t total = (int64_t)S * nb_out * wpb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = idx % wpb;
    const int64_t sb = idx / wpb;
    const int64_t s = sb / nb_out;
    const int b = (int)(sb - s * nb_out);
    // input blocks: [S][2][k][p][p] with Gamma at [.][0] and Gamma-hat at [.][1]
    const int which = b < k ? 0 : 1;
    const int j = b < k ? b : b - k + 1;
    const int r = wrow[w], c = wcol[w];
    double v = 0.0;
    if (r < p && c < p) v = blocks[((((size_t)s * 2 + which) * k + j) * p + r) * p + c];
    if constexpr (std::is_same<T, double>::value) {
      out[idx] = v;
    } else if constexpr (std::is_same<T, float>::value) {
      out[idx] = (float)v;
    } else {
      out[idx] = __bfloat16_as_ushort(__float2bfloat16((float)v));
    }
  }
}

// dst[i] = src[idx[i]] for rows of `width` doubles.
__global__ void gather_rows_kernel(const double* __restrict__ src, const int32_t* __restrict__ idx, int n,
                                   int64_t width, double* __restrict__ dst) {
  const int64_t total = (int64_t)n * width;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q / width;
    dst[q] = src[(int64_t)idx[i] * width + (q - i * width)];
  }
}

__global__ void pad_rows_kernel(const double* __restrict__ src, int64_t nrows, int p, int P16,
                                float* __restrict__ dst) {
  const int64_t total = nrows * P16;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / P16;
    const int c = (int)(idx - r * P16);
    dst[idx] = c < p ? (float)src[r * p + c] : 0.f;
  }
}

// Sum of squares of x (FP64 accumulation), single work-group (used by the CFL estimate).
// ||x||^2 in two passes: kNormBlocks partial sums (FP64) into part, then one work-group sums them
// in a fixed order (the result does not depend on scheduling).
constexpr int kNormBlocks = 1024;

__global__ __launch_bounds__(256) void norm2_partial_kernel(const float* __restrict__ x, int64_t n,
                                                            double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += (double)x[i] * (double)x[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void norm2_final_kernel(const double* __restrict__ part, int np, double* out) {
  __shared__ double red[1024];
  red[threadIdx.x] = (int)threadIdx.x < np ? part[threadIdx.x] : 0.0;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void scale_kernel(const float* __restrict__ x, int64_t n, const double* __restrict__ nrm2,
                             float* __restrict__ y) {
  const double inv = 1.0 / sqrt(*nrm2);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)(x[i] * inv);
}

}  // namespace

size_t step_lds_bytes(const StepParams& prm, int precision) {
  const size_t acc = precision == SFM_PREC_FP64 ? sizeof(double) : sizeof(float);
  return acc * ((size_t)2 * prm.k * prm.P16 + (size_t)prm.k * prm.nslots * kTile);
}

template <typename T>
static hipError_t launch_main_t(const StepParams& prm, size_t lds, hipStream_t st) {
  if (lds > kDefaultLdsBytes) {
    // beyond the default dynamic-LDS limit (the work-group limit is kMaxLdsBytes, checked at create)
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&step_main_kernel<T>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(step_main_kernel<T>, dim3(prm.S), dim3(kStepThreads), lds, st, prm);
  return hipGetLastError();
}

hipError_t launch_step_main(const StepParams& prm, int precision, hipStream_t st) {
  const size_t lds = step_lds_bytes(prm, precision);
  SFM_DCHECK(prm.S > 0 && prm.k >= 1 && prm.P16 == kTile * prm.nt && prm.nt >= 1 && prm.nt <= kMaxNt);
  SFM_DCHECK(prm.npairs == (prm.nt + 1) / 2 && prm.nslots == prm.nt + prm.nt * (prm.nt - 1) / 2);
  SFM_DCHECK(prm.words_per_sub == (2 * (int64_t)prm.k - 1) * prm.words_per_block);
  SFM_DCHECK(lds <= kMaxLdsBytes && prm.tiles && prm.exch);
  SFM_DCHECK(prm.mode == 1 ? (prm.Uin && prm.Aout) : (prm.U && prm.D));
  SFM_DCHECK(!prm.hist || (prm.hist_slot && prm.mode == 0));
  if (precision == SFM_PREC_FP32) return launch_main_t<float>(prm, lds, st);
  if (precision == SFM_PREC_FP64) return launch_main_t<double>(prm, lds, st);
  return launch_main_t<uint16_t>(prm, lds, st);
}

hipError_t launch_step_face(const FaceParams& prm, hipStream_t st) {
  const int64_t n = (int64_t)prm.S * prm.p;
  SFM_DCHECK(prm.p == 6 * prm.m && prm.p <= prm.P16 && prm.nbr && prm.C && prm.exch);
  SFM_DCHECK(n > 0 && (n + 255) / 256 <= 0x7fffffff);
  const int threads = 256;
  hipLaunchKernelGGL(step_face_kernel, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0, st, prm);
  return hipGetLastError();
}

hipError_t launch_pack(const double* blocks, int64_t /*nblocks_total*/, int /*blocks_per_sub_in*/, int k, int p,
                       const TileGeometry& geo, const int32_t* wrow, const int32_t* wcol, void* tiles,
                       int precision, int S, hipStream_t st) {
  const int threads = 256;
  const int64_t total = (int64_t)S * (2 * k - 1) * geo.words_per_block;
  SFM_DCHECK(geo.p == p && geo.P16 >= p && blocks && wrow && wcol && tiles && total > 0);
  const unsigned grid = (unsigned)std::min<int64_t>((total + threads - 1) / threads, 65536);
  if (precision == SFM_PREC_FP32) {
    hipLaunchKernelGGL(pack_kernel<float>, dim3(grid), dim3(threads), 0, st, blocks, k, p, geo.words_per_block,
                       wrow, wcol, reinterpret_cast<float*>(tiles), S);
  } else if (precision == SFM_PREC_FP64) {
    hipLaunchKernelGGL(pack_kernel<double>, dim3(grid), dim3(threads), 0, st, blocks, k, p, geo.words_per_block,
                       wrow, wcol, reinterpret_cast<double*>(tiles), S);
  } else {
    hipLaunchKernelGGL(pack_kernel<uint16_t>, dim3(grid), dim3(threads), 0, st, blocks, k, p,
                       geo.words_per_block, wrow, wcol, reinterpret_cast<uint16_t*>(tiles), S);
  }
  return hipGetLastError();
}

hipError_t launch_pad_rows(const double* src, int64_t nrows, int p, int P16, float* dst, hipStream_t st) {
  if (nrows == 0) return hipSuccess;
  const int threads = 256;
  const int64_t total = nrows * P16;
  const unsigned grid = (unsigned)std::min<int64_t>((total + threads - 1) / threads, 65536);
  hipLaunchKernelGGL(pad_rows_kernel, dim3(grid), dim3(threads), 0, st, src, nrows, p, P16, dst);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const double* src, const int32_t* idx, int n, int64_t width, double* dst,
                              hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int threads = 256;
  const unsigned grid = (unsigned)std::min<int64_t>((n * width + threads - 1) / threads, 65536);
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid), dim3(threads), 0, st, src, idx, n, width, dst);
  return hipGetLastError();
}

hipError_t launch_norm2(const float* x, int64_t n, double* out, hipStream_t st) {
  // out[0] receives the result; out[kNormScratch0 ..] holds the partial sums
  hipLaunchKernelGGL(norm2_partial_kernel, dim3(kNormBlocks), dim3(256), 0, st, x, n, out + kNormScratch0);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(norm2_final_kernel, dim3(1), dim3(1024), 0, st, out + kNormScratch0, kNormBlocks, out);
  return hipGetLastError();
}

hipError_t launch_scale(const float* x, int64_t n, const double* num, float* y, hipStream_t st) {
  const int threads = 256;
  const unsigned grid = (unsigned)std::min<int64_t>((n + threads - 1) / threads, 65536);
  hipLaunchKernelGGL(scale_kernel, dim3(grid), dim3(threads), 0, st, x, n, num, y);
  return hipGetLastError();
}

}  // namespace sfm
