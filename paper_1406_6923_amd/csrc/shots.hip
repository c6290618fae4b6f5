// Many shots through one set of subdomain ROMs: Algorithm 1, Stage 2 for up to 64 independent
// sources at once.  The coefficient blocks do not depend on the source, so one pass over the
// coefficient stream serves every shot and the block products become small dense GEMMs
//   phi_j = Gamma_j (U_{j+1} - U_j),   a_j = Gamma-hat_j (phi_j - phi_{j-1})    (eq. "intrtstep")
// with a p x 64 right-hand side (one column per shot) instead of a matrix-vector product.
// They run on the FP32 matrix cores (v_mfma_f32_16x16x4f32), or with FP64 coefficient storage on
// the FP64 ones (v_mfma_f64_16x16x4f64, the same lane layout with doubles): the deep levels of a
// large polynomial-Krylov S-fraction do not survive rounding to FP32 (the rounded operator's
// spectral radius grows by orders of magnitude), so such ROMs are stepped with FP64 blocks and
// FP64 products while the states stay FP32.
//
// State layout: U, D [S][k][P16][64] (shot fastest); exch [S][P16][64].
//
// shots_main_kernel: one work-group per subdomain, two waves per 16-row tile of the block (each
// wave 32 of the 64 shots; 2 P16/16 waves, which spreads the matrix-core work evenly over the
// four SIMDs of a CU for every even P16/16).  Per level j the block is read from the packed tile stream once (prefetched into
// registers while the previous block computes), expanded to a dense symmetric P16 x P16 copy in
// LDS through the stored word map, and multiplied by the level input held transposed in LDS
// ([shot][row], rows padded to PP = P16 + 4 floats).  phi_{j-1} stays in registers, so one sweep
// over the levels does both halves of the step without an HBM round trip for phi; U_j, U_{j+1},
// U_{j+2} and D_j are held in registers in a layout where every thread owns one shot of 8 rows
// (coalesced 256-byte rows), the loads of the next level issued before the matrix-core work.
// LDS is the dense block and one [64][PP] array (64 KB at 6m = 96): two work-groups per CU.  Within each
// 16-wide reduction chunk the MFMA number c takes k = kk + 4 g + c in lane group g, so a lane
// reads its four k values of A and of B with one 16-byte LDS load each.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "sfm_internal.h"

namespace sfm {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));

// Per coefficient type: the 16-byte load unit of the tile stream, 4-wide accumulator, MFMA.
template <typename T>
struct ShotMath;
template <>
struct ShotMath<float> {
  typedef f4 Load;               // 4 words per 16-byte load
  typedef f4 Acc;
  static constexpr int kWords = 4;
  static constexpr int kPrefetch = 2;   // 16-byte loads of the next block held per thread
  __device__ __forceinline__ static Acc mfma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of output element v held by lane group g (column: the lane within its group of 16)
  __device__ __forceinline__ static int out_row(int g, int v) { return 4 * g + v; }
};
template <>
struct ShotMath<double> {
  typedef d2 Load;               // 2 words per 16-byte load
  typedef d4 Acc;
  static constexpr int kWords = 2;
  static constexpr int kPrefetch = 4;
  __device__ __forceinline__ static Acc mfma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // the FP64 16x16x4 result interleaves the lane groups: element v of group g is row g + 4 v
  __device__ __forceinline__ static int out_row(int g, int v) { return g + 4 * v; }
};

// Xt[col][rbase + out_row(g, v)] = x[v]: one 16-byte store where the four rows are consecutive.
template <typename T>
__device__ __forceinline__ void store_rows(T* __restrict__ dst, int g, const typename ShotMath<T>::Acc& x) {
  if constexpr (std::is_same<T, float>::value) {
    *reinterpret_cast<f4*>(dst + 4 * g) = x;
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[ShotMath<T>::out_row(g, v)] = x[v];
  }
}

constexpr int kMaxShotP16 = 112;        // work-group size (2 P16 / 16 waves) and prefetch capacity
constexpr int kShotRowsPerThread = 8;   // P16 rows x 64 shots over 2 P16 / 16 waves
constexpr int kShotWindow = 32;         // receiver samples staged per shot before the flush

struct ShotParams {
  const void* tiles;           // packed tile stream [S][2k-1][words_per_block] (FP32 or FP64 words)
  int64_t words_per_sub, words_per_block;
  const uint32_t* wmap;        // [words_per_block]: (row << 16) | col of every stored word
  int S, k, P, PP;
  float* U;                    // [S][k][P][64]
  float* D;
  float* exch;                 // [S][P][64]
  const int32_t* k_of;         // [S] levels of each subdomain's ROM (null: all k)
  const int32_t* order;        // [S] subdomain of each launch slot (null: the identity)
  const int32_t* src_off;      // [S+1] interior sources of each subdomain
  const int32_t* src_ids;
  const int32_t* src_shot;     // [nsrc] shot driven by each source (-1: none)
  const float* src_vec;        // [nsrc][k][P]
  const float* wavelet;        // [nsteps][nshot] (row `step`, plus *step_base when set)
  const int64_t* step_base;    // device step counter of a replayed window (or null)
  int nshot;
  int64_t step;
  float dt2;
};

__device__ __forceinline__ size_t block_word(const ShotParams& prm, int s, int b) {
  return (size_t)s * prm.words_per_sub + (size_t)b * prm.words_per_block;
}

template <typename T, int kPF = ShotMath<T>::kPrefetch>
using ShotBuf = typename ShotMath<T>::Load[kPF];

template <typename T, int kPF>
__device__ __forceinline__ void prefetch_block(const T* __restrict__ blk, int nq, int tid, int nthr,
                                               ShotBuf<T, kPF>& buf) {
  typedef typename ShotMath<T>::Load L;
  const L* q = reinterpret_cast<const L*>(blk);
#pragma unroll
  for (int i = 0; i < kPF; ++i) {
    const int qi = tid + i * nthr;
    if (qi < nq) buf[i] = __builtin_nontemporal_load(q + qi);
  }
}

// Dense symmetric copy of the block in LDS: word (r, c) goes to G[r][c] and G[c][r].
template <typename T, int kPF>
__device__ __forceinline__ void expand_block(T* __restrict__ G, int PP, int P, const uint32_t* __restrict__ wmap,
                                             int nq, int tid, int nthr, const ShotBuf<T, kPF>& buf) {
  constexpr int kW = ShotMath<T>::kWords;
  typedef uint32_t MapLoad __attribute__((ext_vector_type(kW)));   // the map entries of one load
#pragma unroll
  for (int i = 0; i < kPF; ++i) {
    const int qi = tid + i * nthr;
    if (qi < nq) {
      const MapLoad ms = reinterpret_cast<const MapLoad*>(wmap)[qi];
#pragma unroll
      for (int e = 0; e < kW; ++e) {
        const uint32_t m = ms[e];
        const int r = (int)(m >> 16), c = (int)(m & 0xffff);
        if (r < P) {
          const T v = buf[i][e];
          G[r * PP + c] = v;
          G[c * PP + r] = v;
        }
      }
    }
  }
}

// acc[h] (16 x 16, shots 16 (sh + h)..) = G[16 I .. 16 I + 15][:] * X[:][16 (sh + h) ..] for the
// wave's two shot tiles, X held as Xt[shot][row].
template <typename T>
__device__ __forceinline__ void block_product(const T* __restrict__ G, const T* __restrict__ Xt, int PP, int P, int I,
                                              int sh, int g, int li, typename ShotMath<T>::Acc (&acc)[2]) {
  typedef typename ShotMath<T>::Acc A4;
  typedef T V4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int h = 0; h < 2; ++h) acc[h] = A4{0, 0, 0, 0};
  const T* arow = G + (16 * I + li) * PP + 4 * g;
  const T* brow = Xt + (16 * sh + li) * PP + 4 * g;
  for (int kk = 0; kk < P; kk += 16) {
    const V4 a = *reinterpret_cast<const V4*>(arow + kk);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const V4 b = *reinterpret_cast<const V4*>(brow + 16 * h * PP + kk);
      acc[h] = ShotMath<T>::mfma(a.x, b.x, acc[h]);
      acc[h] = ShotMath<T>::mfma(a.y, b.y, acc[h]);
      acc[h] = ShotMath<T>::mfma(a.z, b.z, acc[h]);
      acc[h] = ShotMath<T>::mfma(a.w, b.w, acc[h]);
    }
  }
}

// kMinWaves: waves per SIMD the register allocation must allow (2: one work-group per CU, no
// spills; 3: two work-groups per CU at 6m = 96, some registers spilled).  sfm_shots_init times
// every instantiation and keeps the fastest.
// kCols = 64: one work-group per subdomain, two waves per row tile (32 shots each).  kCols = 32:
// two work-groups per subdomain (shots 0..31 and 32..63), one wave per row tile; the half-size
// Xt lets two work-groups share a CU where the 64-shot one needs most of its LDS (FP64 blocks).
// Work-groups g and g + 8 of every 16 take the two halves of one subdomain: the same XCD (and L2)
// reads the subdomain's blocks for both.  kPF: 16-byte prefetch loads per thread.
// kDB: two dense block buffers in LDS; each block product runs while the next block of the stream
// (Gamma_1, Gamma_2, Gamma-hat_2, Gamma_3, Gamma-hat_3, ...) is expanded into the other buffer, so the
// expansion leaves the products' critical path (the same arithmetic, in the same order).
template <typename T, int kMinWaves, int kMaxNtWG = kMaxShotP16 / kTile, int kCols = 64,
          int kPF = ShotMath<T>::kPrefetch, bool kDB = false>
__global__ __launch_bounds__((kCols == 64 ? 128 : 64) * kMaxNtWG, kMinWaves) void shots_main_kernel(ShotParams prm) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  typedef typename ShotMath<T>::Acc A4;
  const int P = prm.P, PP = prm.PP, k = prm.k;
  T* G = reinterpret_cast<T*>(lds_raw);  // [P][PP]      dense block
  T* G2 = kDB ? G + P * PP : G;          // [P][PP]      second block buffer (kDB)
  T* Xt = G2 + P * PP;                   // [kCols][PP]  block input, then a_j, transposed
  const T* tiles = static_cast<const T*>(prm.tiles);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index: uniform
  const int nw = nthr >> 6;              // 2 P / 16 (kCols = 64) or P / 16 waves
  const int I = kCols == 64 ? w >> 1 : w;              // row tile
  const int sh = kCols == 64 ? 2 * (w & 1) : 0;        // first of the wave's two shot tiles (local)
  const int lane = tid & 63, g = lane >> 4, li = lane & 15;
  int s = blockIdx.x, c0 = 0;
  if (kCols == 32) {
    const int grp = blockIdx.x >> 4, r = blockIdx.x & 15;
    s = grp * 8 + (r & 7);
    c0 = (r >> 3) * 32;
    if (s >= prm.S) return;              // the whole work-group: the last group of 8 is partial
  }
  if (prm.order) s = prm.order[s];
  const int nq = (int)(prm.words_per_block / ShotMath<T>::kWords);
  const size_t sbase = (size_t)s * k * P * kShotCols;
  const int ns0 = prm.src_off ? prm.src_off[s] : 0;
  const int ns1 = prm.src_off ? prm.src_off[s + 1] : 0;
  const int ks = prm.k_of ? prm.k_of[s] : k;   // this ROM's levels (>= 2); the others stay zero
  // X layout: this thread owns column col of rows (w + i nw) * (64 / kCols) + lane / kCols (i < 8)
  // of every level; a wave's global accesses are whole 64-shot rows (kCols = 64) or two 32-shot
  // halves of consecutive rows, at a wave-uniform offset.
  constexpr int kRowMul = 64 / kCols;
  const int xl = lane % kCols;           // local column (shot c0 + xl)
  const int ro = lane / kCols;
  float* const Uw = prm.U + sbase + (size_t)(w * kRowMul + ro) * kShotCols + c0 + xl;
  float* const Dw = prm.D + sbase + (size_t)(w * kRowMul + ro) * kShotCols + c0 + xl;
  auto xrow = [&](int j, int i) { return ((j * P + i * nw * kRowMul) * kShotCols); };
  auto trow = [&](int i) { return (w + i * nw) * kRowMul + ro; };   // row of the thread's i-th value
  constexpr int R = kShotRowsPerThread;
  float Ua[R], Ub[R], Un[R], Dr[R];      // U_j, U_{j+1}, U_{j+2}, D_j
  A4 phip[2];                            // phi_{j-1} in the MFMA output layout
  A4 acc[2];
  ShotBuf<T, kPF> buf;
  prefetch_block<T, kPF>(tiles + block_word(prm, s, 0), nq, tid, nthr, buf);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    Ua[i] = Uw[xrow(0, i)];
    Ub[i] = Uw[xrow(1, i)];
  }
  const int rb = 16 * I;                 // first row of the wave's row tile
  if constexpr (!kDB) {
    for (int j = 0; j < ks; ++j) {
      __syncthreads();                                       // G, Xt free
      expand_block<T, kPF>(G, PP, P, prm.wmap, nq, tid, nthr, buf);  // G <- Gamma_j
#pragma unroll
      for (int i = 0; i < R; ++i) Xt[xl * PP + trow(i)] = (T)Ub[i] - (T)Ua[i];   // U_{j+1} - U_j
      __syncthreads();
      if (j >= 1) {
        prefetch_block<T, kPF>(tiles + block_word(prm, s, k + j - 1), nq, tid, nthr, buf);   // Gamma-hat_j
#pragma unroll
        for (int i = 0; i < R; ++i) Dr[i] = Dw[xrow(j, i)];
      } else {
        prefetch_block<T, kPF>(tiles + block_word(prm, s, 1), nq, tid, nthr, buf);           // Gamma_2
      }
#pragma unroll
      for (int i = 0; i < R; ++i) Un[i] = (j + 2 < ks) ? Uw[xrow(j + 2, i)] : 0.f;
      block_product<T>(G, Xt, PP, P, I, sh, g, li, acc);     // phi_j
      __syncthreads();                                       // every wave done with G, Xt
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int n = 16 * (sh + h) + li;   // local column
        if (j == 0) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            prm.exch[((size_t)s * P + rb + ShotMath<T>::out_row(g, v)) * kShotCols + c0 + n] = (float)acc[h][v];  // 2.1
        } else {
          store_rows<T>(Xt + n * PP + rb, g, acc[h] - phip[h]);   // phi_j - phi_{j-1}
        }
        phip[h] = acc[h];
      }
      if (j >= 1) {
        expand_block<T, kPF>(G, PP, P, prm.wmap, nq, tid, nthr, buf);  // G <- Gamma-hat_j
        __syncthreads();
        if (j + 1 < ks) prefetch_block<T, kPF>(tiles + block_word(prm, s, j + 1), nq, tid, nthr, buf);  // Gamma_{j+1}
        block_product<T>(G, Xt, PP, P, I, sh, g, li, acc);     // a_j
        // sources of this subdomain: a_j += f_n(t) s_j for the shot n each source drives
        for (int q = ns0; q < ns1; ++q) {
          const int src = prm.src_ids[q];
          const int n = prm.src_shot[src];
          const int nl = n - c0;               // local column of the shot (outside: another half)
          if (n < 0 || nl < 0 || nl >= kCols || (nl & 15) != li || (nl >> 4) < sh || (nl >> 4) > sh + 1) continue;
          const int64_t stp = prm.step + (prm.step_base ? *prm.step_base : 0);
          const float wv = prm.wavelet[stp * prm.nshot + n];
          const float* sv = prm.src_vec + ((size_t)src * k + j) * P + rb;
          const int h = (nl >> 4) - sh;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T x = (T)sv[ShotMath<T>::out_row(g, v)];
            if constexpr (std::is_same<T, float>::value) acc[h][v] = fmaf(wv, x, acc[h][v]);
            else acc[h][v] = fma((double)wv, x, acc[h][v]);
          }
        }
        __syncthreads();                                     // every wave done reading Xt
#pragma unroll
        for (int h = 0; h < 2; ++h) store_rows<T>(Xt + (16 * (sh + h) + li) * PP + rb, g, acc[h]);
        __syncthreads();
        // leapfrog in increment form: D_j += dt^2 a_j, U_j += D_j
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const float d = std::is_same<T, float>::value
                              ? fmaf(prm.dt2, (float)Xt[xl * PP + trow(i)], Dr[i])
                              : (float)fma((double)prm.dt2, (double)Xt[xl * PP + trow(i)], (double)Dr[i]);
          Dw[xrow(j, i)] = d;
          Uw[xrow(j, i)] = Ua[i] + d;
        }
      }
#pragma unroll
      for (int i = 0; i < R; ++i) {
        Ua[i] = Ub[i];
        Ub[i] = Un[i];
      }
    }

  } else {
    // the blocks in order of use: t = 0 the Gamma block of level 0 (block 0); for a level j >= 1,
    // t = 2j - 1 its Gamma block (block j) and t = 2j its Gamma-hat block (block k + j - 1)
    const int nt_s = 2 * ks - 1;
    auto block_of = [&](int t) { return t == 0 ? 0 : ((t & 1) ? (t + 1) / 2 : k + t / 2 - 1); };
    expand_block<T, kPF>(G, PP, P, prm.wmap, nq, tid, nthr, buf);               // stream block 0
    prefetch_block<T, kPF>(tiles + block_word(prm, s, block_of(1)), nq, tid, nthr, buf);
    int t = 0;
    for (int j = 0; j < ks; ++j) {
      T* Gc = (t & 1) ? G2 : G;
      T* Gn = (t & 1) ? G : G2;
      __syncthreads();                                     // Xt and Gn free, Gc expanded
#pragma unroll
      for (int i = 0; i < R; ++i) Xt[xl * PP + trow(i)] = (T)Ub[i] - (T)Ua[i];   // U_{j+1} - U_j
      __syncthreads();
      if (j >= 1) {
#pragma unroll
        for (int i = 0; i < R; ++i) Dr[i] = Dw[xrow(j, i)];
      }
#pragma unroll
      for (int i = 0; i < R; ++i) Un[i] = (j + 2 < ks) ? Uw[xrow(j + 2, i)] : 0.f;
      if (t + 1 < nt_s) {
        expand_block<T, kPF>(Gn, PP, P, prm.wmap, nq, tid, nthr, buf);          // next block, other buffer
        if (t + 2 < nt_s) prefetch_block<T, kPF>(tiles + block_word(prm, s, block_of(t + 2)), nq, tid, nthr, buf);
      }
      block_product<T>(Gc, Xt, PP, P, I, sh, g, li, acc);  // phi_j
      ++t;
      __syncthreads();                                     // every wave done with Xt; Gn expanded
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int n = 16 * (sh + h) + li;   // local column
        if (j == 0) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            prm.exch[((size_t)s * P + rb + ShotMath<T>::out_row(g, v)) * kShotCols + c0 + n] = (float)acc[h][v];  // 2.1
        } else {
          store_rows<T>(Xt + n * PP + rb, g, acc[h] - phip[h]);   // phi_j - phi_{j-1}
        }
        phip[h] = acc[h];
      }
      if (j >= 1) {
        Gc = (t & 1) ? G2 : G;
        Gn = (t & 1) ? G : G2;
        __syncthreads();                                   // phi_j - phi_{j-1} in Xt
        if (t + 1 < nt_s) {
          expand_block<T, kPF>(Gn, PP, P, prm.wmap, nq, tid, nthr, buf);
          if (t + 2 < nt_s) prefetch_block<T, kPF>(tiles + block_word(prm, s, block_of(t + 2)), nq, tid, nthr, buf);
        }
        block_product<T>(Gc, Xt, PP, P, I, sh, g, li, acc);   // a_j
        ++t;
        for (int q = ns0; q < ns1; ++q) {
          const int src = prm.src_ids[q];
          const int n = prm.src_shot[src];
          const int nl = n - c0;
          if (n < 0 || nl < 0 || nl >= kCols || (nl & 15) != li || (nl >> 4) < sh || (nl >> 4) > sh + 1) continue;
          const int64_t stp = prm.step + (prm.step_base ? *prm.step_base : 0);
          const float wv = prm.wavelet[stp * prm.nshot + n];
          const float* sv = prm.src_vec + ((size_t)src * k + j) * P + rb;
          const int h = (nl >> 4) - sh;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T x = (T)sv[ShotMath<T>::out_row(g, v)];
            if constexpr (std::is_same<T, float>::value) acc[h][v] = fmaf(wv, x, acc[h][v]);
            else acc[h][v] = fma((double)wv, x, acc[h][v]);
          }
        }
        __syncthreads();                                   // every wave done reading Xt
#pragma unroll
        for (int h = 0; h < 2; ++h) store_rows<T>(Xt + (16 * (sh + h) + li) * PP + rb, g, acc[h]);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const float d = std::is_same<T, float>::value
                              ? fmaf(prm.dt2, (float)Xt[xl * PP + trow(i)], Dr[i])
                              : (float)fma((double)prm.dt2, (double)Xt[xl * PP + trow(i)], (double)Dr[i]);
          Dw[xrow(j, i)] = d;
          Uw[xrow(j, i)] = Ua[i] + d;
        }
      }
#pragma unroll
      for (int i = 0; i < R; ++i) {
        Ua[i] = Ub[i];
        Ub[i] = Un[i];
      }
    }
  }
}

struct ShotFaceParams {
  int S, k, P, p, m;
  const int32_t* nbr;
  const float* C;
  const float* exch;
  const int32_t* sw_off;
  const int32_t* sw_q;
  const int32_t* sw_src;
  const float* sw_w;
  const int32_t* src_shot;
  const float* wavelet;
  const int64_t* step_base;    // as in ShotParams
  int nshot;
  int64_t step;
  float dt2;
  float* U;
  float* D;
};

// a_f = C_f (phi_1^alpha + phi_1^beta) + f_n(t) w_f per shot n (eq. "bdrytstep"); four shots per
// thread (16-byte accesses).
__global__ void shots_face_kernel(ShotFaceParams prm) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int kQ = kShotCols / 4;
  if (idx >= (int64_t)prm.S * prm.p * kQ) return;
  const int n0 = 4 * (int)(idx % kQ);
  const int64_t sq = idx / kQ;
  const int s = (int)(sq / prm.p);
  const int q = (int)(sq - (int64_t)s * prm.p);
  const int f = q / prm.m, pat = q - f * prm.m;
  const int nb = prm.nbr[s * 6 + f];
  f4 flux = *reinterpret_cast<const f4*>(prm.exch + ((size_t)s * prm.P + q) * kShotCols + n0);
  if (nb >= 0) flux += *reinterpret_cast<const f4*>(prm.exch + ((size_t)nb * prm.P + (f ^ 1) * prm.m + pat) * kShotCols + n0);
  f4 a = prm.C[(size_t)s * prm.P + q] * flux;
  if (prm.sw_off) {
    const int64_t stp = prm.step + (prm.step_base ? *prm.step_base : 0);
    for (int e = prm.sw_off[s]; e < prm.sw_off[s + 1]; ++e) {
      if (prm.sw_q[e] != q) continue;
      const int n = prm.src_shot[prm.sw_src[e]];
      if (n < n0 || n >= n0 + 4) continue;
      a[n - n0] = fmaf(prm.sw_w[e], prm.wavelet[stp * prm.nshot + n], a[n - n0]);
    }
  }
  const size_t u = ((size_t)s * prm.k * prm.P + q) * kShotCols + n0;
  f4 d = *reinterpret_cast<const f4*>(prm.D + u);
  const f4 uu = *reinterpret_cast<const f4*>(prm.U + u);
#pragma unroll
  for (int c = 0; c < 4; ++c) d[c] = fmaf(prm.dt2, a[c], d[c]);
  *reinterpret_cast<f4*>(prm.D + u) = d;
  *reinterpret_cast<f4*>(prm.U + u) = uu + d;
}

struct ShotRecParams {
  const float* rows;           // [nrec][k][P], sorted by subdomain
  const int32_t* rs_off;       // [n_rs + 1]
  const int32_t* rec_sub;      // sorted receivers: subdomain
  const int32_t* perm;         // sorted receivers: caller index
  const float* U;              // [S][k][P][64]
  const int32_t* k_of;         // [S] levels of each subdomain's ROM (null: all k)
  float* stage;                // [kShotWindow][nsplit][nrec][64] partial samples of the window (sorted order)
  int nsplit;                  // reduction segments of the receiver product (1 .. kRecSplit)
  float* out;                  // [nshot][nrec][ld]
  int k, P, nrec, nshot;
  int64_t ld;
  int slot;                    // time slot of this step in the window
  int64_t col0;                // flush: trace column of slot 0 (plus *step_base when set)
  const int64_t* step_base;
  int w;                       // flush: filled slots
};

constexpr int kRecSplit = 4;   // most reduction segments of the receiver product

// stage[slot][z][r][n] = rows[r][K_z] . U[s(r)][K_z][n], K_z the z-th of nsplit segments of the
// k P words of a row (multiples of 64; the segments past the subdomain's k_s P sum nothing):
// per receiver subdomain a (receivers x kP) (kP x 64) product on the matrix cores, 64 receivers x
// 64 shots per work-group (one wave per 16 receivers).  With ROM sizes that differ, the work-groups
// of the deepest ROMs set the kernel's length, so the reduction is split over kRecSplit
// work-groups (nsplit = 1 otherwise: the split only adds partial traffic).  The flush adds the
// segments in order.
// The reduction runs in chunks of 64 staged through LDS (rows as [r][e], U as [e][n]); the next
// chunk is loaded into registers (16-byte loads) while the current one is multiplied.  The 64
// shots of a receiver are one 256-byte row of the window.
__global__ __launch_bounds__(256) void shots_record_kernel(ShotRecParams prm) {
  constexpr int kR = 64, kK = 64, kKP = kK + 4, kNP = kShotCols + 4;
  __shared__ __align__(16) float Rs[kR][kKP];
  __shared__ __align__(16) float Us[kK][kNP];
  const int slot = blockIdx.y;
  const int r0 = prm.rs_off[slot] + blockIdx.x * kR;
  const int r1 = prm.rs_off[slot + 1];
  if (r0 >= r1) return;
  const int K = prm.k * prm.P;            // row length and level stride; a multiple of 16 (P = P16)
  const int sub = prm.rec_sub[r0];
  const int Kr = (prm.k_of ? prm.k_of[sub] : prm.k) * prm.P;   // levels past k_s are zero: skipped
  const int seg = ((K + prm.nsplit - 1) / prm.nsplit + kK - 1) / kK * kK;
  const int z = blockIdx.z;
  const int kb = z * seg, ke = min(kb + seg, Kr);               // this work-group's words of the rows
  const float* Ub = prm.U + (size_t)sub * K * kShotCols;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, g = lane >> 4, li = lane & 15;
  // loader layout: 4 passes of 16 rows x 16 quads
  const int lr = tid >> 4, lq = tid & 15;
  f4 rbuf[4], ubuf[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
      const int rr = lr + 16 * pass;
      const int r = r0 + rr, e = k0 + 4 * lq;
      rbuf[pass] = (r < r1 && e < ke) ? *reinterpret_cast<const f4*>(prm.rows + (size_t)r * K + e) : f4{0.f, 0.f, 0.f, 0.f};
      const int e2 = k0 + rr;
      ubuf[pass] = e2 < ke ? *reinterpret_cast<const f4*>(Ub + (size_t)e2 * kShotCols + 4 * lq) : f4{0.f, 0.f, 0.f, 0.f};
    }
  };
  f4 acc[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) acc[h] = f4{0.f, 0.f, 0.f, 0.f};
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += kK) {
    __syncthreads();
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
      *reinterpret_cast<f4*>(&Rs[lr + 16 * pass][4 * lq]) = rbuf[pass];
      *reinterpret_cast<f4*>(&Us[lr + 16 * pass][4 * lq]) = ubuf[pass];
    }
    __syncthreads();
    if (k0 + kK < ke) load(k0 + kK);
#pragma unroll
    for (int kk = 0; kk < kK; kk += 16) {
      const f4 a = *reinterpret_cast<const f4*>(&Rs[16 * wv + li][kk + 4 * g]);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int n = 16 * h + li;
        const float* ub = &Us[kk + 4 * g][n];
        acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, ub[0], acc[h], 0, 0, 0);
        acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, ub[kNP], acc[h], 0, 0, 0);
        acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, ub[2 * kNP], acc[h], 0, 0, 0);
        acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, ub[3 * kNP], acc[h], 0, 0, 0);
      }
    }
  }
  // acc[h][v]: receiver r0 + 16 wv + 4 g + v, shot 16 h + li
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = r0 + 16 * wv + 4 * g + v;
    if (r >= r1) continue;
    float* row = prm.stage + (((size_t)prm.slot * prm.nsplit + z) * prm.nrec + r) * kShotCols;
#pragma unroll
    for (int h = 0; h < 4; ++h) row[16 * h + li] = acc[h][v];
  }
}

// out[n][perm[r]][col0 + t] = sum over z of stage[t][z][r][n] for t < w: one work-group per receiver, transposed
// through LDS so that both the window rows (64 shots) and the trace runs (w samples) are contiguous.
__global__ __launch_bounds__(256) void shots_flush_kernel(ShotRecParams prm) {
  __shared__ float tile[kShotWindow][kShotCols + 1];
  const int r = blockIdx.x;
  for (int e = threadIdx.x; e < prm.w * kShotCols; e += 256) {
    const int t = e / kShotCols, n = e - t * kShotCols;
    float v = 0.f;
    for (int z = 0; z < prm.nsplit; ++z) v += prm.stage[(((size_t)t * prm.nsplit + z) * prm.nrec + r) * kShotCols + n];
    tile[t][n] = v;
  }
  __syncthreads();
  const size_t orow = (size_t)prm.perm[r];
  const int64_t col0 = prm.col0 + (prm.step_base ? *prm.step_base : 0);
  for (int e = threadIdx.x; e < prm.w * prm.nshot; e += 256) {
    const int n = e / prm.w, t = e - n * prm.w;
    prm.out[((size_t)n * prm.nrec + orow) * prm.ld + col0 + t] = tile[t][n];
  }
}

// The replayed window's last node: advance the step counter (one thread, a vector store).
__global__ void step_base_kernel(int64_t* base, int64_t add, int set) {
  if (blockIdx.x == 0 && threadIdx.x == 0) base[0] = set ? add : base[0] + add;
}

typedef void (*ShotKernel)(ShotParams);
// FP32: 4 waves per SIMD, one 12-wave work-group per CU at 6m = 96 with no spills; 6: two
// work-groups per CU with some registers spilled.  FP64 (twice the accumulator and prefetch
// registers): for 6m <= 80 a work-group of at most 10 waves allows 3 waves per SIMD (170
// registers, no spills); the 4-wave variant serves every 6m <= 112.
// Third variant of each: 32 shots per work-group (two per subdomain), with twice the prefetch
// loads per thread since the work-group is half the size.
// Fourth variant of each: the first with two block buffers (kDB), where its LDS fits.
constexpr int kNumShotVariants = 4;
constexpr ShotKernel kShotVariants[2][kNumShotVariants] = {
    {shots_main_kernel<float, 4>, shots_main_kernel<float, 6>, shots_main_kernel<float, 3, 7, 32, 4>,
     shots_main_kernel<float, 4, 7, 64, 2, true>},
    {shots_main_kernel<double, 3, 5>, shots_main_kernel<double, 4>, shots_main_kernel<double, 3, 5, 32, 6>,
     shots_main_kernel<double, 3, 5, 64, 4, true>}};
constexpr int kShotVariantWaves[2][kNumShotVariants] = {{4, 6, 3, 4}, {3, 4, 3, 3}};
constexpr int kShotVariantMaxNt[2][kNumShotVariants] = {{7, 7, 7, 7}, {5, 7, 5, 5}};   // largest P16 / 16
constexpr int kShotVariantCols[kNumShotVariants] = {64, 64, 32, 64};
constexpr int kShotVariantPrefetch[2][kNumShotVariants] = {{2, 2, 4, 2}, {4, 4, 6, 4}};
constexpr bool kShotVariantDB[kNumShotVariants] = {false, false, false, true};

size_t shots_lds_bytes(int P, size_t elem, int cols = kShotCols, bool db = false) {
  const int PP = P + 4;
  return elem * ((size_t)(db ? 2 : 1) * P * PP + (size_t)cols * PP);
}

int shot_kind(sfm_ctx c) { return c->cfg.precision == SFM_PREC_FP64 ? 1 : 0; }

}  // namespace

void drop_shot_graph(sfm_ctx c) {
  if (c->shot_exec) {
    (void)hipDeviceSynchronize();
    (void)hipGraphExecDestroy(c->shot_exec);
  }
  c->shot_exec = nullptr;
  c->shot_exec_key.clear();
}

void release_shots(sfm_ctx c) {
  drop_shot_graph(c);
  void* bufs[] = {c->Us_d, c->Ds_d, c->exch_s_d, c->src_shot_d, c->rec_stage_d, c->shot_base_d};
  for (void* b : bufs) c->dfree(b);
  c->Us_d = c->Ds_d = c->exch_s_d = c->rec_stage_d = nullptr;
  c->src_shot_d = nullptr;
  c->shot_base_d = nullptr;
  c->nshot = 0;
  c->shots_n = 0;
}

}  // namespace sfm

using namespace sfm;

namespace {
sfm_status autotune_shots(sfm_ctx c, hipStream_t st);
}

#define SH_TRY_HIP(call)                                                                      \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return c->fail(SFM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

extern "C" {

sfm_status sfm_shots_init(sfm_ctx c, int32_t nshot, const int32_t* shot_src, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs: call sfm_build_roms or sfm_load_roms first");
  if (c->cfg.precision != SFM_PREC_FP32 && c->cfg.precision != SFM_PREC_FP64)
    return c->fail(SFM_EINVAL, "shots need FP32 or FP64 coefficient storage");
  if (c->geo.P16 > kMaxShotP16)
    return c->fail(SFM_EINVAL, "shots support 6m <= " + std::to_string(kMaxShotP16) + " (LDS of one CU)");
  const int64_t cap = shot_kind(c) ? (int64_t)ShotMath<double>::kPrefetch * ShotMath<double>::kWords
                                    : (int64_t)ShotMath<float>::kPrefetch * ShotMath<float>::kWords;
  if (c->geo.words_per_block > cap * 128 * c->geo.nt)
    return c->fail(SFM_EINVAL, "coefficient block larger than the shot kernel's prefetch");
  if (shots_lds_bytes(c->geo.P16, shot_kind(c) ? sizeof(double) : sizeof(float)) > (size_t)kMaxLdsBytes)
    return c->fail(SFM_EINVAL, "shot kernel LDS above the 160 KB of a CU for this 6m");
  if (nshot < 1 || nshot > kShotCols) return c->fail(SFM_EINVAL, "nshot must lie in 1..64");
  std::vector<int32_t> src_shot(std::max(c->nsrc, 1), -1);
  for (int n = 0; n < nshot; ++n) {
    const int src = shot_src ? shot_src[n] : n;
    if (src < -1 || src >= c->nsrc)
      return c->fail(SFM_EINVAL, "shot " + std::to_string(n) + " names source " + std::to_string(src) + " of " +
                                     std::to_string(c->nsrc));
    if (src < 0) continue;
    if (src_shot[src] >= 0) return c->fail(SFM_EINVAL, "source " + std::to_string(src) + " drives two shots");
    src_shot[src] = n;
  }
  SH_TRY_HIP(hipSetDevice(c->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  release_shots(c);
  const Topology& t = c->topo;
  const size_t nstate = (size_t)t.S * t.k * c->geo.P16 * kShotCols;
  hipError_t e = hipSuccess;
  c->Us_d = static_cast<float*>(c->dalloc(nstate * sizeof(float), &e));
  c->Ds_d = static_cast<float*>(c->dalloc(nstate * sizeof(float), &e));
  c->exch_s_d = static_cast<float*>(c->dalloc((size_t)t.S * c->geo.P16 * kShotCols * sizeof(float), &e));
  c->src_shot_d = static_cast<int32_t*>(c->dalloc(src_shot.size() * sizeof(int32_t), &e));
  c->shot_base_d = static_cast<int64_t*>(c->dalloc(sizeof(int64_t), &e));
  if (c->nrec > 0)
    c->rec_stage_d =
        static_cast<float*>(c->dalloc((size_t)kShotWindow * kRecSplit * c->nrec * kShotCols * sizeof(float), &e));
  // every pointer is checked: a later allocation that succeeds overwrites the status of a failed one
  if (!c->Us_d || !c->Ds_d || !c->exch_s_d || !c->src_shot_d || !c->shot_base_d ||
      (c->nrec > 0 && !c->rec_stage_d)) {
    release_shots(c);
    return c->fail(SFM_ENOMEM, "shot state: out of device memory");
  }
  SH_TRY_HIP(hipMemcpy(c->src_shot_d, src_shot.data(), src_shot.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  SH_TRY_HIP(hipMemsetAsync(c->Us_d, 0, nstate * sizeof(float), st));
  SH_TRY_HIP(hipMemsetAsync(c->Ds_d, 0, nstate * sizeof(float), st));
  SH_TRY_HIP(hipMemsetAsync(c->exch_s_d, 0, (size_t)t.S * c->geo.P16 * kShotCols * sizeof(float), st));
  SH_TRY_HIP(hipStreamSynchronize(st));
  c->nshot = nshot;
  c->shots_n = 0;
  const sfm_status rc = autotune_shots(c, st);
  if (rc != SFM_OK) release_shots(c);
  return rc;
}

}  // extern "C"

namespace {

ShotParams main_params(sfm_ctx c, const float* wavelet_dev, double dt) {
  const Topology& t = c->topo;
  const TileGeometry& g = c->geo;
  ShotParams prm{};
  prm.tiles = c->tiles_d;
  prm.words_per_block = g.words_per_block;
  prm.words_per_sub = (int64_t)(2 * t.k - 1) * g.words_per_block;
  prm.wmap = c->wmap_d;
  prm.S = t.S;
  prm.k = t.k;
  prm.k_of = c->k_of_d;
  prm.order = c->order_d;
  prm.P = g.P16;
  prm.PP = g.P16 + 4;
  prm.U = c->Us_d;
  prm.D = c->Ds_d;
  prm.exch = c->exch_s_d;
  prm.src_off = c->nsrc ? c->src_off_d : nullptr;
  prm.src_ids = c->src_ids_d;
  prm.src_shot = c->src_shot_d;
  prm.src_vec = c->src_vec_d;
  prm.wavelet = wavelet_dev;
  prm.nshot = c->nshot;
  prm.dt2 = (float)(dt * dt);
  return prm;
}

hipError_t launch_shots_main(int kind, int variant, const ShotParams& prm, int nt, hipStream_t st,
                             bool set_attr = true) {
  const int cols = kShotVariantCols[variant];
  const size_t lds = shots_lds_bytes(prm.P, kind ? sizeof(double) : sizeof(float), cols, kShotVariantDB[variant]);
  const ShotKernel kern = kShotVariants[kind][variant];
  if (lds > kDefaultLdsBytes && set_attr) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const unsigned grid = cols == 64 ? (unsigned)prm.S : (unsigned)((prm.S + 7) / 8 * 16);
  hipLaunchKernelGGL(kern, dim3(grid), dim3((cols == 64 ? 128 : 64) * nt), lds, st, prm);
  return hipGetLastError();
}

// The variant's prefetch holds a whole coefficient block for this 6m and fits its work-group limit.
bool shot_variant_fits(sfm_ctx c, int v) {
  const int kind = shot_kind(c);
  const int64_t words = kind ? ShotMath<double>::kWords : ShotMath<float>::kWords;
  const int64_t threads = (kShotVariantCols[v] == 64 ? 128 : 64) * (int64_t)c->geo.nt;
  return c->geo.nt <= kShotVariantMaxNt[kind][v] &&
         c->geo.words_per_block <= (int64_t)kShotVariantPrefetch[kind][v] * words * threads &&
         shots_lds_bytes(c->geo.P16, kind ? sizeof(double) : sizeof(float), kShotVariantCols[v],
                         kShotVariantDB[v]) <= (size_t)kMaxLdsBytes;
}

// Times every kernel variant on the (zero) shot state with no sources and dt = 0, which leaves
// the state unchanged, and keeps the fastest.
sfm_status autotune_shots(sfm_ctx c, hipStream_t st) {
  ShotParams prm = main_params(c, nullptr, 0.0);
  prm.src_off = nullptr;
  hipEvent_t a, b;
  SH_TRY_HIP(hipEventCreate(&a));
  SH_TRY_HIP(hipEventCreate(&b));
  int best = -1;
  for (int v = 0; v < kNumShotVariants; ++v) {
    c->shots_tune_ms[v] = -1.0;
    if (!shot_variant_fits(c, v)) continue;   // work-group limit or prefetch capacity below this 6m
    for (int r = 0; r < 2; ++r) SH_TRY_HIP(launch_shots_main(shot_kind(c), v, prm, c->geo.nt, st));
    SH_TRY_HIP(hipEventRecord(a, st));
    constexpr int kReps = 5;
    for (int r = 0; r < kReps; ++r) SH_TRY_HIP(launch_shots_main(shot_kind(c), v, prm, c->geo.nt, st));
    SH_TRY_HIP(hipEventRecord(b, st));
    SH_TRY_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    SH_TRY_HIP(hipEventElapsedTime(&ms, a, b));
    c->shots_tune_ms[v] = ms / kReps;
    if (best < 0 || c->shots_tune_ms[v] < c->shots_tune_ms[best]) best = v;
  }
  SH_TRY_HIP(hipEventDestroy(a));
  SH_TRY_HIP(hipEventDestroy(b));
  c->shots_variant = best;
  c->shots_tuned = best;
  return SFM_OK;
}

}  // namespace

extern "C" {

sfm_status sfm_shots_step(sfm_ctx c, int32_t nsteps, double dt, const float* wavelet_dev, float* traces_dev,
                          int64_t ld, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (c->nshot == 0) return c->fail(SFM_ESTATE, "call sfm_shots_init first");
  if (nsteps < 0) return c->fail(SFM_EINVAL, "nsteps must be >= 0");
  if (!(dt > 0.0)) return c->fail(SFM_EINVAL, "dt must be positive");
  if (c->dt_max > 0.0 && dt > c->dt_max)
    return c->fail(SFM_EUNSTABLE, "dt above the stability limit from sfm_cfl_dt");
  if (c->nsrc > 0 && !wavelet_dev) return c->fail(SFM_EINVAL, "wavelet_dev is NULL but sources exist");
  if (traces_dev && c->nrec > 0 && ld < nsteps) return c->fail(SFM_EINVAL, "ld must be >= nsteps");
  SH_TRY_HIP(hipSetDevice(c->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const Topology& t = c->topo;
  const TileGeometry& g = c->geo;
  ShotParams prm = main_params(c, wavelet_dev, dt);
  ShotFaceParams fp{};
  fp.S = t.S;
  fp.k = t.k;
  fp.P = g.P16;
  fp.p = t.p;
  fp.m = t.m;
  fp.nbr = c->nbr_d;
  fp.C = c->C_d;
  fp.exch = c->exch_s_d;
  fp.sw_off = c->nsrc ? c->sw_off_d : nullptr;
  fp.sw_q = c->sw_q_d;
  fp.sw_src = c->sw_src_d;
  fp.sw_w = c->sw_w_d;
  fp.src_shot = c->src_shot_d;
  fp.wavelet = wavelet_dev;
  fp.nshot = c->nshot;
  fp.dt2 = prm.dt2;
  fp.U = c->Us_d;
  fp.D = c->Ds_d;
  ShotRecParams rp{};
  rp.rows = c->rec_rows_d;
  rp.rs_off = c->rs_off_d;
  rp.rec_sub = c->rec_sub_d;
  rp.perm = c->rec_perm_d;
  rp.U = c->Us_d;
  rp.k_of = c->k_of_d;
  rp.stage = c->rec_stage_d;
  rp.out = traces_dev;
  rp.k = t.k;
  rp.P = g.P16;
  rp.nrec = c->nrec;
  rp.nshot = c->nshot;
  rp.ld = ld;
  const int64_t nface = (int64_t)t.S * t.p * (kShotCols / 4);
  const bool record = traces_dev && c->nrec > 0;
  bool mixed = false;                    // ROM sizes that differ: split the receiver product
  for (size_t q = 1; q < c->k_of.size(); ++q) mixed = mixed || c->k_of[q] != c->k_of[0];
  rp.nsplit = mixed ? kRecSplit : 1;
  const dim3 rgrid((c->rs_max + 63) / 64, c->n_rs, rp.nsplit);
  // one step at relative index n (absolute with base == null); closes the window with a flush
  auto launch_step = [&](int n, int64_t col0, bool close, const int64_t* base, hipStream_t s,
                         bool set_attr) -> hipError_t {
    prm.step = n;
    prm.step_base = base;
    fp.step = n;
    fp.step_base = base;
    hipError_t e = launch_shots_main(shot_kind(c), c->shots_variant, prm, g.nt, s, set_attr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(shots_face_kernel, dim3((unsigned)((nface + 255) / 256)), dim3(256), 0, s, fp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (record) {
      rp.slot = n % kShotWindow;
      hipLaunchKernelGGL(shots_record_kernel, rgrid, dim3(256), 0, s, rp);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if (close) {
        rp.w = rp.slot + 1;
        rp.col0 = col0;
        rp.step_base = base;
        hipLaunchKernelGGL(shots_flush_kernel, dim3(c->nrec), dim3(256), 0, s, rp);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
    }
    return hipSuccess;
  };
  const bool timing = c->timing;
  const int nwin = nsteps / kShotWindow;
  int n_done = 0;
  if (c->shots_graph && !timing && nwin >= 2) {
    // Capture one window of kShotWindow steps (relative steps 0..W-1, flush at the end, counter
    // += W) and replay it nwin times; the kernels add the device counter to their step.
    const uint64_t dtb = (uint64_t)__builtin_bit_cast(uint32_t, prm.dt2);
    const std::vector<uint64_t> key = {(uint64_t)(uintptr_t)wavelet_dev, (uint64_t)(uintptr_t)traces_dev,
                                       (uint64_t)ld, dtb, (uint64_t)c->shots_variant,
                                       (uint64_t)(uintptr_t)c->k_of_d, (uint64_t)(uintptr_t)c->Us_d,
                                       (uint64_t)(uintptr_t)c->tiles_d};
    if (c->shot_exec && key != c->shot_exec_key) drop_shot_graph(c);
    if (!c->shot_exec) {
      if (!c->cap_stream) SH_TRY_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
      SH_TRY_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipSuccess;
      for (int q = 0; q < kShotWindow && e == hipSuccess; ++q)
        e = launch_step(q, 0, q == kShotWindow - 1, c->shot_base_d, c->cap_stream, false);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(step_base_kernel, dim3(1), dim3(64), 0, c->cap_stream, c->shot_base_d,
                           (int64_t)kShotWindow, 0);
        e = hipGetLastError();
      }
      hipGraph_t graph = nullptr;
      const hipError_t ee = hipStreamEndCapture(c->cap_stream, &graph);
      if (e == hipSuccess) e = ee;
      if (e == hipSuccess) e = hipGraphInstantiate(&c->shot_exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        c->shot_exec = nullptr;
        return c->fail(SFM_EHIP, std::string("shot-window graph capture: ") + hipGetErrorString(e));
      }
      c->shot_exec_key = key;
    }
    hipLaunchKernelGGL(step_base_kernel, dim3(1), dim3(64), 0, st, c->shot_base_d, (int64_t)0, 1);
    SH_TRY_HIP(hipGetLastError());
    for (int r = 0; r < nwin; ++r) SH_TRY_HIP(hipGraphLaunch(c->shot_exec, st));
    c->shots_replays += nwin;
    // the rest of the steps eagerly, relative to the counter (now nwin W)
    for (int n = 0; n < nsteps - nwin * kShotWindow; ++n)
      SH_TRY_HIP(launch_step(n, 0, n + 1 == nsteps - nwin * kShotWindow, c->shot_base_d, st, true));
    n_done = nsteps;
  }
  for (int n = n_done; n < nsteps; ++n) {
    hipEvent_t* ev = nullptr;
    if (c->time_this_step()) {
      SH_TRY_HIP(c->take_events(c->shot_ev));
      ev = &c->shot_ev[c->shot_ev.size() - 4];
      SH_TRY_HIP(hipEventRecord(ev[0], st));
    }
    prm.step = n;
    prm.step_base = nullptr;
    SH_TRY_HIP(launch_shots_main(shot_kind(c), c->shots_variant, prm, g.nt, st));
    if (ev) SH_TRY_HIP(hipEventRecord(ev[1], st));
    fp.step = n;
    fp.step_base = nullptr;
    hipLaunchKernelGGL(shots_face_kernel, dim3((unsigned)((nface + 255) / 256)), dim3(256), 0, st, fp);
    SH_TRY_HIP(hipGetLastError());
    if (ev) SH_TRY_HIP(hipEventRecord(ev[2], st));
    if (record) {
      rp.slot = n % kShotWindow;
      hipLaunchKernelGGL(shots_record_kernel, rgrid, dim3(256), 0, st, rp);
      SH_TRY_HIP(hipGetLastError());
      if (rp.slot == kShotWindow - 1 || n + 1 == nsteps) {
        rp.w = rp.slot + 1;
        rp.col0 = n - rp.slot;
        rp.step_base = nullptr;
        hipLaunchKernelGGL(shots_flush_kernel, dim3(c->nrec), dim3(256), 0, st, rp);
        SH_TRY_HIP(hipGetLastError());
      }
    }
    if (ev) SH_TRY_HIP(hipEventRecord(ev[3], st));
  }
  c->shots_n += nsteps;
  return SFM_OK;
}

sfm_status sfm_shots_graph(sfm_ctx c, int32_t enable, int64_t* replays) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (enable >= 0) {
    c->shots_graph = enable != 0;
    if (!c->shots_graph) drop_shot_graph(c);
  }
  if (replays) *replays = c->shots_replays;
  return SFM_OK;
}

sfm_status sfm_shots_get_state(sfm_ctx c, float* u_host, float* d_host) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (c->nshot == 0) return c->fail(SFM_ESTATE, "call sfm_shots_init first");
  SH_TRY_HIP(hipSetDevice(c->device));
  SH_TRY_HIP(hipDeviceSynchronize());
  const Topology& t = c->topo;
  const int P = c->geo.P16;
  std::vector<float> buf((size_t)t.S * t.k * P * kShotCols);
  float* outs[2] = {u_host, d_host};
  float* srcs[2] = {c->Us_d, c->Ds_d};
  for (int a = 0; a < 2; ++a) {
    if (!outs[a]) continue;
    SH_TRY_HIP(hipMemcpy(buf.data(), srcs[a], buf.size() * sizeof(float), hipMemcpyDeviceToHost));
    // [S][k][P16][64] -> [S][k][p][nshot]
    for (size_t sj = 0; sj < (size_t)t.S * t.k; ++sj)
      for (int q = 0; q < t.p; ++q)
        std::memcpy(outs[a] + (sj * t.p + q) * c->nshot, buf.data() + (sj * P + q) * kShotCols,
                    c->nshot * sizeof(float));
  }
  return SFM_OK;
}

sfm_status sfm_shots_set_state(sfm_ctx c, const float* u_host, const float* d_host) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (c->nshot == 0) return c->fail(SFM_ESTATE, "call sfm_shots_init first");
  if (!u_host || !d_host) return c->fail(SFM_EINVAL, "state arrays are NULL");
  SH_TRY_HIP(hipSetDevice(c->device));
  SH_TRY_HIP(hipDeviceSynchronize());
  const Topology& t = c->topo;
  const int P = c->geo.P16;
  std::vector<float> buf((size_t)t.S * t.k * P * kShotCols);
  const float* ins[2] = {u_host, d_host};
  float* dsts[2] = {c->Us_d, c->Ds_d};
  for (int a = 0; a < 2; ++a) {
    std::fill(buf.begin(), buf.end(), 0.f);
    for (size_t sj = 0; sj < (size_t)t.S * t.k; ++sj)
      for (int q = 0; q < t.p; ++q)
        std::memcpy(buf.data() + (sj * P + q) * kShotCols, ins[a] + (sj * t.p + q) * c->nshot,
                    c->nshot * sizeof(float));
    SH_TRY_HIP(hipMemcpy(dsts[a], buf.data(), buf.size() * sizeof(float), hipMemcpyHostToDevice));
    SH_TRY_HIP(clear_extra_levels(c, dsts[a], kShotCols, nullptr));
  }
  SH_TRY_HIP(hipDeviceSynchronize());
  return SFM_OK;
}

sfm_status sfm_shots_tuning(sfm_ctx c, int32_t* chosen_waves, double* ms, int32_t cap, int32_t* count) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (c->nshot == 0) return c->fail(SFM_ESTATE, "call sfm_shots_init first");
  if (chosen_waves) *chosen_waves = kShotVariantWaves[shot_kind(c)][c->shots_tuned];
  if (count) *count = kNumShotVariants;
  for (int v = 0; v < std::min<int>(cap, kNumShotVariants); ++v) {
    if (ms) ms[2 * v] = kShotVariantWaves[shot_kind(c)][v];
    if (ms) ms[2 * v + 1] = c->shots_tune_ms[v];
  }
  return SFM_OK;
}

sfm_status sfm_shots_select(sfm_ctx c, int32_t variant) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (c->nshot == 0) return c->fail(SFM_ESTATE, "call sfm_shots_init first");
  if (variant == -1) {
    c->shots_variant = c->shots_tuned;
    return SFM_OK;
  }
  if (variant < 0 || variant >= kNumShotVariants)
    return c->fail(SFM_EINVAL, "variant must be -1 or in [0, " + std::to_string(kNumShotVariants) + ")");
  if (!shot_variant_fits(c, variant))
    return c->fail(SFM_EINVAL, "variant " + std::to_string(variant) + " does not fit 6m = " + std::to_string(c->topo.p));
  c->shots_variant = variant;
  return SFM_OK;
}

sfm_status sfm_shots_timing(sfm_ctx c, int64_t* timed_steps, double* ms3) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  SH_TRY_HIP(hipSetDevice(c->device));
  const sfm_status rc = drain_events(c, c->shot_ev, c->shots_ms, &c->shots_timed);
  if (rc != SFM_OK) return rc;
  if (timed_steps) *timed_steps = c->shots_timed;
  if (ms3)
    for (int q = 0; q < 3; ++q) ms3[q] = c->shots_ms[q];
  c->shots_timed = 0;
  for (double& x : c->shots_ms) x = 0.0;
  return SFM_OK;
}

}  // extern "C"
