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

namespace sfm {
namespace {

template <int R>
__device__ __forceinline__ float row_ror(float v) {
  // DPP row_ror:R -- lane i of each 16-lane row receives lane (i - R) mod 16.
  static_assert(R >= 1 && R <= 15, "rotation amount");
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x120 + R, 0xF, 0xF, true));
}

template <int R>
__device__ __forceinline__ double row_ror(double v) {
  static_assert(R >= 1 && R <= 15, "rotation amount");
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), 0x120 + R, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x120 + R, 0xF, 0xF, true);
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// ------------------------------------------------------------------ tile loads
template <typename T>
struct TileIO;

template <>
struct TileIO<float> {
  static constexpr int kDiag = kDiagWords;
  static constexpr int kOff = kOffWords;
  // p: the tile (t = 0..7); h: its half-diagonal t = 8 in the block tail
  __device__ __forceinline__ static void diag(const float* __restrict__ p, const float* __restrict__ h,
                                              int lane, float (&w)[9]) {
    const f32x4* q = reinterpret_cast<const f32x4*>(p);
    f32x4 a = __builtin_nontemporal_load(q + lane);
    f32x4 b = __builtin_nontemporal_load(q + 16 + lane);
    w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
    w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
    w[8] = __builtin_nontemporal_load(h + lane);
  }
  __device__ __forceinline__ static void off(const float* __restrict__ p, int lane, float (&w)[16]) {
    const f32x4* q = reinterpret_cast<const f32x4*>(p);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      f32x4 a = __builtin_nontemporal_load(q + v * 16 + lane);
      w[4 * v + 0] = a.x; w[4 * v + 1] = a.y; w[4 * v + 2] = a.z; w[4 * v + 3] = a.w;
    }
  }
};

template <>
struct TileIO<uint16_t> {
  static constexpr int kDiag = kDiagWords;
  static constexpr int kOff = kOffWords;
  __device__ __forceinline__ static void unpack8(u32x4 a, float* w) {
    w[0] = bf16_lo(a.x); w[1] = bf16_hi(a.x); w[2] = bf16_lo(a.y); w[3] = bf16_hi(a.y);
    w[4] = bf16_lo(a.z); w[5] = bf16_hi(a.z); w[6] = bf16_lo(a.w); w[7] = bf16_hi(a.w);
  }
  __device__ __forceinline__ static void diag(const uint16_t* __restrict__ p, const uint16_t* __restrict__ h,
                                              int lane, float (&w)[9]) {
    const u32x4* q = reinterpret_cast<const u32x4*>(p);
    u32x4 a = __builtin_nontemporal_load(q + lane);
    unpack8(a, w);
    uint32_t t8 = __builtin_nontemporal_load(h + lane);
    w[8] = __uint_as_float(t8 << 16);
  }
  __device__ __forceinline__ static void off(const uint16_t* __restrict__ p, int lane, float (&w)[16]) {
    const u32x4* q = reinterpret_cast<const u32x4*>(p);
    u32x4 a = __builtin_nontemporal_load(q + lane);
    u32x4 b = __builtin_nontemporal_load(q + 16 + lane);
    unpack8(a, w);
    unpack8(b, w + 8);
  }
};

template <>
struct TileIO<double> {
  typedef double f64x2 __attribute__((ext_vector_type(2)));
  static constexpr int kDiag = kDiagWords;
  static constexpr int kOff = kOffWords;
  __device__ __forceinline__ static void diag(const double* __restrict__ p, const double* __restrict__ h,
                                              int lane, double (&w)[9]) {
    const f64x2* q = reinterpret_cast<const f64x2*>(p);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      f64x2 a = __builtin_nontemporal_load(q + v * 16 + lane);
      w[2 * v] = a.x;
      w[2 * v + 1] = a.y;
    }
    w[8] = __builtin_nontemporal_load(h + lane);
  }
  __device__ __forceinline__ static void off(const double* __restrict__ p, int lane, double (&w)[16]) {
    const f64x2* q = reinterpret_cast<const f64x2*>(p);
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      f64x2 a = __builtin_nontemporal_load(q + v * 16 + lane);
      w[2 * v] = a.x;
      w[2 * v + 1] = a.y;
    }
  }
};

// Arithmetic type of the products and sums for a stored coefficient type.
template <typename T>
struct Acc {
  typedef float type;
};
template <>
struct Acc<double> {
  typedef double type;
};

__device__ __forceinline__ float mad(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double mad(double a, double b, double c) { return fma(a, b, c); }

// ------------------------------------------------------------------ tile products
// Diagonal tile: y_I[i] += sum_c A(i, c) x_I[c] using W_0..W_8 (symmetric inside the tile).
template <typename R>
__device__ __forceinline__ void diag_tile(const R (&w)[9], R xI, const R (&xr)[16], R& yI) {
  yI = mad(w[0], xI, yI);
  static_for<1, 8>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    yI = mad(w[t], row_ror<16 - t>(xI), yI);   // A(i, i+t) x[i+t]
    yI = mad(row_ror<t>(w[t]), xr[t], yI);     // A(i-t, i) x[i-t]
  });
  yI = mad(w[8], row_ror<8>(xI), yI);
}

// Off-diagonal tile (I < J): y_I += A x_J and y_J += A^T x_I.
template <typename R>
__device__ __forceinline__ void off_tile(const R (&w)[16], R xJ, const R (&xr)[16], R& yI, R& yJ) {
  yI = mad(w[0], xJ, yI);
  yJ = mad(w[0], xr[0], yJ);
  static_for<1, 16>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    yI = mad(w[t], row_ror<16 - t>(xJ), yI);   // A(i, i+t) x_J[i+t]
    yJ = mad(row_ror<t>(w[t]), xr[t], yJ);     // A(c-t, c) x_I[c-t]
  });
}

__device__ __forceinline__ int tri_index(int I, int J, int nt) {
  return I * (2 * nt - I - 1) / 2 + (J - I - 1);
}

// One job: strips g and nt-1-g of one block.  x: block input vector (LDS); part: the
// block's partial-sum slots (LDS): slot I = row sums of strip I, slot nt + tri(I,J) =
// transposed contribution of tile (I, J) to segment J.
template <typename T, typename R = typename Acc<T>::type>
__device__ __forceinline__ void run_job(const T* __restrict__ blk, int job_off, int tail_off, int g, int nt,
                                        const R* __restrict__ x, R* __restrict__ part, int lane) {
  const int I0 = g, I1 = nt - 1 - g;
  const int nstrip = (I0 == I1) ? 1 : 2;
  const T* ptr = blk + job_off;
  for (int st = 0; st < nstrip; ++st) {
    const int I = st ? I1 : I0;
    const R xI = x[kTile * I + lane];
    R xr[16];
    xr[0] = xI;
    static_for<1, 16>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      xr[t] = row_ror<t>(xI);
    });
    R yI = 0;
    {
      R w[9];
      TileIO<T>::diag(ptr, blk + tail_off + kHalfDiagWords * I, lane, w);
      ptr += TileIO<T>::kDiag;
      diag_tile(w, xI, xr, yI);
    }
    R wn[16];
    if (I + 1 < nt) TileIO<T>::off(ptr, lane, wn);
    for (int J = I + 1; J < nt; ++J) {
      R w[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) w[t] = wn[t];
      ptr += TileIO<T>::kOff;
      if (J + 1 < nt) TileIO<T>::off(ptr, lane, wn);   // prefetch the next tile
      const R xJ = x[kTile * J + lane];
      R yJ = 0;
      off_tile(w, xJ, xr, yI, yJ);
      part[(nt + tri_index(I, J, nt)) * kTile + lane] = yJ;
    }
    part[I * kTile + lane] = yI;
  }
}

// All jobs of nb consecutive blocks.  The four rows of a wave take the same job shape g
// on four different blocks so that their control flow is identical.
template <typename T, typename R = typename Acc<T>::type>
__device__ __forceinline__ void run_phase(const T* __restrict__ tiles, int nb, const StepParams& prm,
                                          const R* xs, int vstride, R* part, int tid) {
  const int lane = tid & 15;
  const int rw = (tid >> 4) & 3;
  const int wave = tid >> 6;
  const int per_g = (nb + 3) >> 2;
  const int ngroups = prm.npairs * per_g;
  for (int grp = wave; grp < ngroups; grp += kStepThreads / 64) {
    const int g = grp / per_g;
    const int b = (grp - g * per_g) * 4 + rw;
    if (b < nb) {
      run_job<T, R>(tiles + b * prm.words_per_block, prm.job_off[g], prm.tail_off, g, prm.nt, xs + b * vstride,
                 part + b * prm.nslots * kTile, lane);
    }
  }
}

template <typename R>
__device__ __forceinline__ R reduce_entry(const R* part, int b, int i, int nt, int nslots) {
  const int J = i >> 4, c = i & 15;
  const R* pb = part + b * nslots * kTile;
  R v = pb[J * kTile + c];
  for (int I = 0; I < J; ++I) v += pb[(nt + tri_index(I, J, nt)) * kTile + c];
  return v;
}

template <typename T>
__global__ __launch_bounds__(kStepThreads) void step_main_kernel(StepParams prm) {
  typedef typename Acc<T>::type R;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* smem = reinterpret_cast<R*>(smem_raw);
  const int s = blockIdx.x;
  const int tid = threadIdx.x;
  const int k = prm.k, P = prm.P16;
  const int vstride = P;
  R* xs = smem;                           // [k][P]   block inputs
  R* ph = xs + k * vstride;               // [k][P]   layer fluxes phi_j
  R* part = ph + k * vstride;             // [k][nslots][16]
  const size_t sbase = (size_t)s * k * P;
  const float* Uin = prm.mode == 0 ? prm.U : prm.Uin;
  const T* tiles = reinterpret_cast<const T*>(prm.tiles) + (size_t)s * prm.words_per_sub;

  // U_{j+1} - U_j with U_{k+1} = 0
  for (int e = tid; e < k * P; e += kStepThreads) {
    const int j = e / P;
    const R u = Uin[sbase + e];
    const R un = (j + 1 < k) ? (R)Uin[sbase + e + P] : (R)0;
    xs[e] = un - u;
  }
  __syncthreads();
  run_phase<T, R>(tiles, k, prm, xs, vstride, part, tid);       // phi_j = Gamma_j dU_j
  __syncthreads();
  for (int e = tid; e < k * P; e += kStepThreads) {
    const int b = e / P, i = e - b * P;
    ph[e] = reduce_entry(part, b, i, prm.nt, prm.nslots);
  }
  __syncthreads();
  for (int e = tid; e < P; e += kStepThreads) prm.exch[(size_t)s * P + e] = (float)ph[e];   // step 2.1
  for (int e = tid; e < (k - 1) * P; e += kStepThreads) xs[e] = ph[e + P] - ph[e];   // phi_j - phi_{j-1}
  __syncthreads();
  run_phase<T, R>(tiles + (size_t)k * prm.words_per_block, k - 1, prm, xs, vstride, part, tid);
  __syncthreads();
  const int slot = (prm.mode == 0 && prm.hist) ? prm.hist_slot[s] : -1;
  const int s0 = prm.src_off ? prm.src_off[s] : 0;
  const int s1 = prm.src_off ? prm.src_off[s + 1] : 0;
  for (int e = tid; e < (k - 1) * P; e += kStepThreads) {
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
__global__ __launch_bounds__(1024) void norm2_kernel(const float* __restrict__ x, int64_t n, double* out) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += (double)x[i] * (double)x[i];
  red[threadIdx.x] = acc;
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
  if (precision == SFM_PREC_FP32) return launch_main_t<float>(prm, lds, st);
  if (precision == SFM_PREC_FP64) return launch_main_t<double>(prm, lds, st);
  return launch_main_t<uint16_t>(prm, lds, st);
}

hipError_t launch_step_face(const FaceParams& prm, hipStream_t st) {
  const int64_t n = (int64_t)prm.S * prm.p;
  const int threads = 256;
  hipLaunchKernelGGL(step_face_kernel, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0, st, prm);
  return hipGetLastError();
}

hipError_t launch_pack(const double* blocks, int64_t /*nblocks_total*/, int /*blocks_per_sub_in*/, int k, int p,
                       const TileGeometry& geo, const int32_t* wrow, const int32_t* wcol, void* tiles,
                       int precision, int S, hipStream_t st) {
  const int threads = 256;
  const int64_t total = (int64_t)S * (2 * k - 1) * geo.words_per_block;
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
  hipLaunchKernelGGL(norm2_kernel, dim3(1), dim3(1024), 0, st, x, n, out);
  return hipGetLastError();
}

hipError_t launch_scale(const float* x, int64_t n, const double* num, float* y, hipStream_t st) {
  const int threads = 256;
  const unsigned grid = (unsigned)std::min<int64_t>((n + threads - 1) / threads, 65536);
  hipLaunchKernelGGL(scale_kernel, dim3(grid), dim3(threads), 0, st, x, n, num, y);
  return hipGetLastError();
}

}  // namespace sfm
