// Many shots through one set of subdomain ROMs: Algorithm 1, Stage 2 for up to 64 independent
// sources at once.  The coefficient blocks do not depend on the source, so one pass over the
// coefficient stream serves every shot and the block products become small dense GEMMs
//   phi_j = Gamma_j (U_{j+1} - U_j),   a_j = Gamma-hat_j (phi_j - phi_{j-1})    (eq. "intrtstep")
// with a p x 64 right-hand side (one column per shot) instead of a matrix-vector product.
// They run on the FP32 matrix cores (v_mfma_f32_16x16x4f32).
//
// State layout: U, D [S][k][P16][64] (shot fastest); exch [S][P16][64].
//
// shots_main_kernel: one work-group per subdomain, one wave per 16-row tile of the block (P16/16
// waves).  Per level j the block is read from the packed tile stream once (prefetched into
// registers while the previous block computes), expanded to a dense symmetric P16 x P16 copy in
// LDS through the stored word map, and multiplied by the level input held transposed in LDS
// ([shot][row], rows padded to PP = P16 + 4 floats).  phi_{j-1} stays in LDS, so one sweep over
// the levels does both halves of the step without an HBM round trip for phi.  Within each
// 16-wide reduction chunk the MFMA number c takes k = kk + 4 g + c in lane group g, so a lane
// reads its four k values of A and of B with one 16-byte LDS load each.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "sfm_internal.h"

namespace sfm {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kMaxShotP16 = 112;        // LDS: dense block + three [64][P16 + 4] arrays <= 160 KB
constexpr int kPrefetchQuads = 5;       // 16-byte words of the next block held per thread

struct ShotParams {
  const float* tiles;          // packed FP32 tile stream [S][2k-1][words_per_block]
  int64_t words_per_sub, words_per_block;
  const uint32_t* wmap;        // [words_per_block]: (row << 16) | col of every stored word
  int S, k, P, PP;
  float* U;                    // [S][k][P][64]
  float* D;
  float* exch;                 // [S][P][64]
  const int32_t* src_off;      // [S+1] interior sources of each subdomain
  const int32_t* src_ids;
  const int32_t* src_shot;     // [nsrc] shot driven by each source (-1: none)
  const float* src_vec;        // [nsrc][k][P]
  const float* wavelet;        // [nsteps][nshot] (row `step`)
  int nshot;
  int64_t step;
  float dt2;
};

__device__ __forceinline__ size_t block_word(const ShotParams& prm, int s, int b) {
  return (size_t)s * prm.words_per_sub + (size_t)b * prm.words_per_block;
}

__device__ __forceinline__ void prefetch_block(const float* __restrict__ blk, int nq, int tid, int nthr,
                                               f4 (&buf)[kPrefetchQuads]) {
  const f4* q = reinterpret_cast<const f4*>(blk);
#pragma unroll
  for (int i = 0; i < kPrefetchQuads; ++i) {
    const int qi = tid + i * nthr;
    if (qi < nq) buf[i] = __builtin_nontemporal_load(q + qi);
  }
}

// Dense symmetric copy of the block in LDS: word (r, c) goes to G[r][c] and G[c][r].
__device__ __forceinline__ void expand_block(float* __restrict__ G, int PP, int P, const uint32_t* __restrict__ wmap,
                                             int nq, int tid, int nthr, const f4 (&buf)[kPrefetchQuads]) {
  const uint4* wm = reinterpret_cast<const uint4*>(wmap);
#pragma unroll
  for (int i = 0; i < kPrefetchQuads; ++i) {
    const int qi = tid + i * nthr;
    if (qi < nq) {
      const uint4 m = wm[qi];
      const uint32_t ms[4] = {m.x, m.y, m.z, m.w};
      const float vs[4] = {buf[i].x, buf[i].y, buf[i].z, buf[i].w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = (int)(ms[e] >> 16), c = (int)(ms[e] & 0xffff);
        if (r < P) {
          G[r * PP + c] = vs[e];
          G[c * PP + r] = vs[e];
        }
      }
    }
  }
}

// acc[s4] (16 x 16, shots 16 s4..) = G[16 I .. 16 I + 15][:] * X[:][16 s4 ..] with X held as Xt[shot][row].
__device__ __forceinline__ void block_product(const float* __restrict__ G, const float* __restrict__ Xt, int PP,
                                              int P, int I, int g, int li, f4 (&acc)[4]) {
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) acc[s4] = f4{0.f, 0.f, 0.f, 0.f};
  const float* arow = G + (16 * I + li) * PP + 4 * g;
  const float* brow = Xt + li * PP + 4 * g;
  for (int kk = 0; kk < P; kk += 16) {
    const f4 a = *reinterpret_cast<const f4*>(arow + kk);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const f4 b = *reinterpret_cast<const f4*>(brow + 16 * s4 * PP + kk);
      acc[s4] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc[s4], 0, 0, 0);
      acc[s4] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc[s4], 0, 0, 0);
      acc[s4] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc[s4], 0, 0, 0);
      acc[s4] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc[s4], 0, 0, 0);
    }
  }
}

__global__ __launch_bounds__(64 * (kMaxShotP16 / kTile)) void shots_main_kernel(ShotParams prm) {
  extern __shared__ __align__(16) float lds[];
  const int P = prm.P, PP = prm.PP, k = prm.k;
  float* G = lds;                        // [P][PP]   dense block
  float* Xt = G + P * PP;                // [64][PP]  block input, transposed
  float* Ut = Xt + kShotCols * PP;       // [64][PP]  U_{j+1} of the previous level = U_j
  float* Ft = Ut + kShotCols * PP;       // [64][PP]  phi_{j-1}
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int I = tid >> 6, lane = tid & 63, g = lane >> 4, li = lane & 15;
  const int s = blockIdx.x;
  const int nq = (int)(prm.words_per_block / 4);
  const size_t sbase = (size_t)s * k * P * kShotCols;
  const int ns0 = prm.src_off ? prm.src_off[s] : 0;
  const int ns1 = prm.src_off ? prm.src_off[s + 1] : 0;

  for (int e = tid; e < P * kShotCols; e += nthr) {
    const int r = e / kShotCols, n = e - r * kShotCols;
    Ut[n * PP + r] = prm.U[sbase + e];
  }
  f4 buf[kPrefetchQuads];
  prefetch_block(prm.tiles + block_word(prm, s, 0), nq, tid, nthr, buf);
  f4 acc[4];
  for (int j = 0; j < k; ++j) {
    __syncthreads();                                       // G, Xt free
    expand_block(G, PP, P, prm.wmap, nq, tid, nthr, buf);  // G <- Gamma_j
    // X = U_{j+1} - U_j (U_{k+1} = 0); Ut <- U_{j+1}
    for (int e = tid; e < P * kShotCols; e += nthr) {
      const int r = e / kShotCols, n = e - r * kShotCols;
      const float un = (j + 1 < k) ? prm.U[sbase + (size_t)(j + 1) * P * kShotCols + e] : 0.f;
      Xt[n * PP + r] = un - Ut[n * PP + r];
      Ut[n * PP + r] = un;
    }
    __syncthreads();
    if (j >= 1) prefetch_block(prm.tiles + block_word(prm, s, k + j - 1), nq, tid, nthr, buf);   // Gamma-hat_j
    else if (k > 1) prefetch_block(prm.tiles + block_word(prm, s, 1), nq, tid, nthr, buf);       // Gamma_2
    block_product(G, Xt, PP, P, I, g, li, acc);            // phi_j
    __syncthreads();                                       // every wave done with G, Xt
    const int row0 = 16 * I + 4 * g;
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int n = 16 * s4 + li;
      float* fp = Ft + n * PP + row0;
      if (j == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) prm.exch[((size_t)s * P + row0 + v) * kShotCols + n] = acc[s4][v];   // step 2.1
      } else {
        const f4 prev = *reinterpret_cast<const f4*>(fp);
        *reinterpret_cast<f4*>(Xt + n * PP + row0) = acc[s4] - prev;   // phi_j - phi_{j-1}
      }
      *reinterpret_cast<f4*>(fp) = acc[s4];
    }
    if (j == 0) continue;                                  // the boundary layer is the face kernel's
    expand_block(G, PP, P, prm.wmap, nq, tid, nthr, buf);  // G <- Gamma-hat_j
    __syncthreads();
    if (j + 1 < k) prefetch_block(prm.tiles + block_word(prm, s, j + 1), nq, tid, nthr, buf);   // Gamma_{j+1}
    block_product(G, Xt, PP, P, I, g, li, acc);            // a_j
    // sources of this subdomain: a_j += f_n(t) s_j for the shot n each source drives
    for (int q = ns0; q < ns1; ++q) {
      const int src = prm.src_ids[q];
      const int n = prm.src_shot[src];
      if (n < 0 || (n & 15) != li) continue;
      const float w = prm.wavelet[prm.step * prm.nshot + n];
      const float* sv = prm.src_vec + ((size_t)src * k + j) * P + row0;
      const int s4 = n >> 4;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[s4][v] = fmaf(w, sv[v], acc[s4][v]);
    }
    // leapfrog in increment form: D_j += dt^2 a_j, U_j += D_j
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int n = 16 * s4 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const size_t idx = sbase + ((size_t)j * P + row0 + v) * kShotCols + n;
        const float d = fmaf(prm.dt2, acc[s4][v], prm.D[idx]);
        prm.D[idx] = d;
        prm.U[idx] = prm.U[idx] + d;
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
  int nshot;
  int64_t step;
  float dt2;
  float* U;
  float* D;
};

// a_f = C_f (phi_1^alpha + phi_1^beta) + f_n(t) w_f per shot n (eq. "bdrytstep").
__global__ void shots_face_kernel(ShotFaceParams prm) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)prm.S * prm.p * kShotCols) return;
  const int n = (int)(idx % kShotCols);
  const int64_t sq = idx / kShotCols;
  const int s = (int)(sq / prm.p);
  const int q = (int)(sq - (int64_t)s * prm.p);
  const int f = q / prm.m, pat = q - f * prm.m;
  const int nb = prm.nbr[s * 6 + f];
  float flux = prm.exch[((size_t)s * prm.P + q) * kShotCols + n];
  if (nb >= 0) flux += prm.exch[((size_t)nb * prm.P + (f ^ 1) * prm.m + pat) * kShotCols + n];
  float a = prm.C[(size_t)s * prm.P + q] * flux;
  if (prm.sw_off) {
    for (int e = prm.sw_off[s]; e < prm.sw_off[s + 1]; ++e)
      if (prm.sw_q[e] == q && prm.src_shot[prm.sw_src[e]] == n)
        a = fmaf(prm.sw_w[e], prm.wavelet[prm.step * prm.nshot + n], a);
  }
  const size_t u = ((size_t)s * prm.k * prm.P + q) * kShotCols + n;
  const float d = fmaf(prm.dt2, a, prm.D[u]);
  prm.D[u] = d;
  prm.U[u] = prm.U[u] + d;
}

struct ShotRecParams {
  const float* rows;           // [nrec][k][P], sorted by subdomain
  const int32_t* rs_off;       // [n_rs + 1]
  const int32_t* rec_sub;      // sorted receivers: subdomain
  const int32_t* perm;         // sorted receivers: caller index
  const float* U;              // [S][k][P][64]
  float* out;                  // [nshot][nrec][ld]
  int k, P, nrec, nshot;
  int64_t ld, col;
};

// out[n][r][col] = rows[r] . U[s(r)][:][:][n]: per receiver subdomain a (receivers x kP) (kP x 64)
// product, 64 x 64 outputs per work-group staged through LDS in chunks of 32.
__global__ __launch_bounds__(256) void shots_record_kernel(ShotRecParams prm) {
  constexpr int kR = 64, kK = 32;
  __shared__ float Rs[kK][kR + 4];
  __shared__ float Us[kK][kShotCols + 4];
  const int slot = blockIdx.y;
  const int r0 = prm.rs_off[slot] + blockIdx.x * kR;
  const int r1 = prm.rs_off[slot + 1];
  if (r0 >= r1) return;
  const int K = prm.k * prm.P;
  const float* Ub = prm.U + (size_t)prm.rec_sub[r0] * K * kShotCols;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += kK) {
    for (int q = tid; q < kR * kK; q += 256) {
      const int rr = q / kK, kk = q - rr * kK;
      const int r = r0 + rr, e = k0 + kk;
      Rs[kk][rr] = (r < r1 && e < K) ? prm.rows[(size_t)r * K + e] : 0.f;
      const int kk2 = q / kShotCols, n = q - kk2 * kShotCols;
      const int e2 = k0 + kk2;
      Us[kk2][n] = e2 < K ? Ub[(size_t)e2 * kShotCols + n] : 0.f;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = Rs[kk][ty * 4 + i];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) b[jj] = Us[kk][tx * 4 + jj];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) acc[i][jj] = fmaf(a[i], b[jj], acc[i][jj]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + ty * 4 + i;
    if (r >= r1) continue;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int n = tx * 4 + jj;
      if (n < prm.nshot) prm.out[((size_t)n * prm.nrec + prm.perm[r]) * prm.ld + prm.col] = acc[i][jj];
    }
  }
}

size_t shots_lds_bytes(int P) {
  const int PP = P + 4;
  return sizeof(float) * ((size_t)P * PP + (size_t)3 * kShotCols * PP);
}

}  // namespace

void release_shots(sfm_ctx c) {
  void* bufs[] = {c->Us_d, c->Ds_d, c->exch_s_d, c->src_shot_d};
  for (void* b : bufs) c->dfree(b);
  c->Us_d = c->Ds_d = c->exch_s_d = nullptr;
  c->src_shot_d = nullptr;
  c->nshot = 0;
  c->shots_n = 0;
}

}  // namespace sfm

using namespace sfm;

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
  if (c->cfg.precision != SFM_PREC_FP32) return c->fail(SFM_EINVAL, "shots need FP32 coefficient storage");
  if (c->geo.P16 > kMaxShotP16)
    return c->fail(SFM_EINVAL, "shots support 6m <= " + std::to_string(kMaxShotP16) + " (LDS of one CU)");
  if (c->geo.words_per_block > (int64_t)kPrefetchQuads * 4 * 64 * c->geo.nt)
    return c->fail(SFM_EINVAL, "coefficient block larger than the shot kernel's prefetch");
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
  if (e != hipSuccess) {
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
  return SFM_OK;
}

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
  ShotParams prm{};
  prm.tiles = static_cast<const float*>(c->tiles_d);
  prm.words_per_block = g.words_per_block;
  prm.words_per_sub = (int64_t)(2 * t.k - 1) * g.words_per_block;
  prm.wmap = c->wmap_d;
  prm.S = t.S;
  prm.k = t.k;
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
  rp.out = traces_dev;
  rp.k = t.k;
  rp.P = g.P16;
  rp.nrec = c->nrec;
  rp.nshot = c->nshot;
  rp.ld = ld;
  const size_t lds = shots_lds_bytes(g.P16);
  if (lds > kDefaultLdsBytes)
    SH_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&shots_main_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const int64_t nface = (int64_t)t.S * t.p * kShotCols;
  const bool record = traces_dev && c->nrec > 0;
  const dim3 rgrid((c->rs_max + 63) / 64, c->n_rs);
  hipEvent_t ev[4] = {};
  const bool timing = c->timing;
  for (int n = 0; n < nsteps; ++n) {
    prm.step = n;
    fp.step = n;
    if (timing) {
      for (auto& x : ev) SH_TRY_HIP(hipEventCreate(&x));
      SH_TRY_HIP(hipEventRecord(ev[0], st));
    }
    hipLaunchKernelGGL(shots_main_kernel, dim3(t.S), dim3(64 * g.nt), lds, st, prm);
    SH_TRY_HIP(hipGetLastError());
    if (timing) SH_TRY_HIP(hipEventRecord(ev[1], st));
    hipLaunchKernelGGL(shots_face_kernel, dim3((unsigned)((nface + 255) / 256)), dim3(256), 0, st, fp);
    SH_TRY_HIP(hipGetLastError());
    if (timing) SH_TRY_HIP(hipEventRecord(ev[2], st));
    if (record) {
      rp.col = n;
      hipLaunchKernelGGL(shots_record_kernel, rgrid, dim3(256), 0, st, rp);
      SH_TRY_HIP(hipGetLastError());
    }
    if (timing) {
      SH_TRY_HIP(hipEventRecord(ev[3], st));
      SH_TRY_HIP(hipEventSynchronize(ev[3]));
      float ms[3];
      for (int q = 0; q < 3; ++q) SH_TRY_HIP(hipEventElapsedTime(&ms[q], ev[q], ev[q + 1]));
      for (int q = 0; q < 3; ++q) c->shots_ms[q] += ms[q];
      c->shots_timed++;
      for (auto& x : ev) SH_TRY_HIP(hipEventDestroy(x));
    }
  }
  c->shots_n += nsteps;
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
  }
  return SFM_OK;
}

sfm_status sfm_shots_timing(sfm_ctx c, int64_t* timed_steps, double* ms3) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (timed_steps) *timed_steps = c->shots_timed;
  if (ms3)
    for (int q = 0; q < 3; ++q) ms3[q] = c->shots_ms[q];
  c->shots_timed = 0;
  for (double& x : c->shots_ms) x = 0.0;
  return SFM_OK;
}

}  // extern "C"
