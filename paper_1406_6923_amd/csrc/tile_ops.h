// Device code shared by the kernels that stream the packed coefficient tiles (the leapfrog step
// and its adjoint): tile loads in the stored word order, the symmetric 16 x 16 tile products with
// DPP row rotations, and the job / phase loops over the blocks of one subdomain (layout in
// sfm_internal.h).  Included by each kernel source; everything is internal to its file.
#pragma once

#include <hip/hip_bf16.h>

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

}  // namespace
}  // namespace sfm
