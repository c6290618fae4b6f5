// Learned ROMs: the surrogate network predicts every subdomain's S-fraction blocks from its sound
// speed; block Lanczos (Algorithm 1, Stage 1) is the judge and the fallback.  A prediction is kept
// where the relative Frobenius error of its NtD map (the matrix S-fraction of the Stage 2
// section, evaluated at 8 real Laplace frequencies 2 pi f_p {1/4, 1/2, 3/4, 1, 3/2, 2, 5/2, 3})
// against the Lanczos ROM's is at most tol; subdomains that hold sources or receivers keep the
// Lanczos ROM (their projections belong to its coordinates), and so does every Gamma-hat_1 (the
// face masses, exact and cheap).
//
// Network input: log(c / 3000 m/s) on the subdomain's (n+1)^3 nodes, [z][y][x].  Network output:
// the upper triangles (row-major, i <= j) of Gamma_1..Gamma_k, then Gamma-hat_1..Gamma-hat_k.
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "sfm_internal.h"

namespace sfm {
namespace {

constexpr int kNtdFreq = 8;
constexpr int kJudgeThreads = 256;
constexpr int kMaxJudgeP = 64;

__global__ void box_inputs_kernel(const float* __restrict__ vel, int ncx, int ncy, const int32_t* __restrict__ org,
                                  int nn, int S, float* __restrict__ x) {
  const int64_t per = (int64_t)nn * nn * nn, total = (int64_t)S * per;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(e / per);
    int64_t r = e - (int64_t)s * per;
    const int i = (int)(r % nn);
    r /= nn;
    const int j = (int)(r % nn), l = (int)(r / nn);
    const float c = vel[((int64_t)(org[3 * s + 2] + l) * (ncy + 1) + org[3 * s + 1] + j) * (ncx + 1) + org[3 * s] + i];
    x[e] = logf(c / 3000.f);
  }
}

// t[s][b][e] = block b of subdomain s at upper-triangle entry e = (ti[e], tj[e]).
__global__ void rom_targets_kernel(const double* __restrict__ coef, int S, int k, int p, const int32_t* __restrict__ ti,
                                   const int32_t* __restrict__ tj, float* __restrict__ t) {
  const int64_t ntri = (int64_t)p * (p + 1) / 2, per = 2LL * k * ntri, total = (int64_t)S * per;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = idx / per, r = idx - s * per;
    const int64_t b = r / ntri, e = r - b * ntri;
    t[idx] = (float)coef[(s * 2 * k + b) * p * p + (int64_t)ti[e] * p + tj[e]];
  }
}

// Symmetric FP64 blocks from the predicted triangles; Gamma-hat_1 (block k) copied from ref.
__global__ void unpack_pred_kernel(const float* __restrict__ y, const double* __restrict__ ref, int S, int k, int p,
                                   double* __restrict__ out) {
  const int64_t pp = (int64_t)p * p, per = 2LL * k * pp, total = (int64_t)S * per;
  const int64_t ntri = (int64_t)p * (p + 1) / 2;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = idx / per, r = idx - s * per;
    const int b = (int)(r / pp);
    const int64_t q = r - (int64_t)b * pp;
    int i = (int)(q / p), j = (int)(q - (int64_t)i * p);
    if (b == k) {
      out[idx] = ref[idx];
      continue;
    }
    if (i > j) {
      const int tmp = i;
      i = j;
      j = tmp;
    }
    const int64_t e = (int64_t)i * p - (int64_t)i * (i - 1) / 2 + (j - i);   // row-major upper triangle
    out[idx] = (double)y[(s * 2 * k + b) * ntri + e];
  }
}

// out = a^{-1} (p x p, row-major, LDS) by Gauss-Jordan elimination with partial pivoting in the
// [p][2p] workspace w; *bad is set for a zero pivot.
__device__ void gj_inverse(const double* a, double* out, double* w, double* fac, int p, int* piv_s, int* bad) {
  const int tid = threadIdx.x, nthr = blockDim.x, p2 = 2 * p;
  for (int e = tid; e < p * p2; e += nthr) {
    const int r = e / p2, c = e - r * p2;
    w[e] = c < p ? a[r * p + c] : (c - p == r ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int col = 0; col < p; ++col) {
    if (tid < 64) {
      double best = -1.0;
      int bi = col;
      for (int r = col + tid; r < p; r += 64) {
        const double v = fabs(w[r * p2 + col]);
        if (v > best) {
          best = v;
          bi = r;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > best || (ov == best && oi < bi)) {
          best = ov;
          bi = oi;
        }
      }
      if (tid == 0) *piv_s = bi;
    }
    __syncthreads();
    const int piv = *piv_s;
    if (piv != col)
      for (int c = tid; c < p2; c += nthr) {
        const double t = w[col * p2 + c];
        w[col * p2 + c] = w[piv * p2 + c];
        w[piv * p2 + c] = t;
      }
    __syncthreads();
    const double pv = w[col * p2 + col];
    if (pv == 0.0 && tid == 0) *bad = 1;
    for (int r = tid; r < p; r += nthr) fac[r] = w[r * p2 + col];
    __syncthreads();
    const double inv_pv = 1.0 / pv;
    for (int c = tid; c < p2; c += nthr) w[col * p2 + c] *= inv_pv;
    __syncthreads();
    for (int e = tid; e < p * p2; e += nthr) {
      const int r = e / p2, c = e - r * p2;
      if (r != col) w[e] -= fac[r] * w[col * p2 + c];
    }
    __syncthreads();
  }
  for (int e = tid; e < p * p; e += nthr) {
    const int r = e / p, c = e - r * p;
    out[e] = w[r * p2 + p + c];
  }
  __syncthreads();
}

// M(s) = X_1^{-1} of the matrix S-fraction: X_k = Gamma-hat_k^{-1} s^2 + Gamma_k,
// X_j = Gamma-hat_j^{-1} s^2 + (Gamma_j^{-1} + X_{j+1}^{-1})^{-1}; result in X.
__device__ void sfraction_ntd(const double* gam, const double* hat, int k, int p, double s2, double* X, double* T1,
                              double* T2, double* w, double* fac, int* piv_s, int* bad) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int64_t pp = (int64_t)p * p;
  for (int e = tid; e < p * p; e += nthr) T1[e] = hat[(k - 1) * pp + e];
  __syncthreads();
  gj_inverse(T1, T2, w, fac, p, piv_s, bad);
  for (int e = tid; e < p * p; e += nthr) X[e] = T2[e] * s2 + gam[(k - 1) * pp + e];
  __syncthreads();
  for (int j = k - 2; j >= 0; --j) {
    gj_inverse(X, T1, w, fac, p, piv_s, bad);                 // X^{-1}
    for (int e = tid; e < p * p; e += nthr) X[e] = gam[j * pp + e];
    __syncthreads();
    gj_inverse(X, T2, w, fac, p, piv_s, bad);                 // Gamma_j^{-1}
    for (int e = tid; e < p * p; e += nthr) X[e] = T1[e] + T2[e];
    __syncthreads();
    gj_inverse(X, T1, w, fac, p, piv_s, bad);                 // (Gamma_j^{-1} + X^{-1})^{-1}
    for (int e = tid; e < p * p; e += nthr) X[e] = hat[j * pp + e];
    __syncthreads();
    gj_inverse(X, T2, w, fac, p, piv_s, bad);                 // Gamma-hat_j^{-1}
    for (int e = tid; e < p * p; e += nthr) X[e] = T2[e] * s2 + T1[e];
    __syncthreads();
  }
  gj_inverse(X, T1, w, fac, p, piv_s, bad);
  for (int e = tid; e < p * p; e += nthr) X[e] = T1[e];
  __syncthreads();
}

// err[s][f] = ||M_a - M_b||_F / ||M_b||_F at Laplace frequency svals[f]; blocks [S][2][k][p][p].
__global__ __launch_bounds__(kJudgeThreads) void ntd_judge_kernel(const double* __restrict__ A, const double* __restrict__ Bm,
                                                                  int k, int p, const double* __restrict__ svals,
                                                                  double* __restrict__ err) {
  extern __shared__ __align__(16) unsigned char raw[];
  double* X = reinterpret_cast<double*>(raw);
  const int64_t pp = (int64_t)p * p;
  double* Mb = X + pp;
  double* T1 = Mb + pp;
  double* T2 = T1 + pp;
  double* w = T2 + pp;
  double* fac = w + 2 * pp;
  __shared__ int piv_s, bad;
  __shared__ double red[kJudgeThreads][2];
  const int s = blockIdx.x, f = blockIdx.y, tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  const double s2 = svals[f] * svals[f];
  const double* b0 = Bm + (int64_t)s * 2 * k * pp;
  const double* a0 = A + (int64_t)s * 2 * k * pp;
  sfraction_ntd(b0, b0 + k * pp, k, p, s2, X, T1, T2, w, fac, &piv_s, &bad);
  for (int e = tid; e < p * p; e += blockDim.x) Mb[e] = X[e];
  __syncthreads();
  sfraction_ntd(a0, a0 + k * pp, k, p, s2, X, T1, T2, w, fac, &piv_s, &bad);
  double num = 0.0, den = 0.0;
  for (int e = tid; e < p * p; e += blockDim.x) {
    const double d = X[e] - Mb[e];
    num += d * d;
    den += Mb[e] * Mb[e];
  }
  red[tid][0] = num;
  red[tid][1] = den;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (tid < h) {
      red[tid][0] += red[tid + h][0];
      red[tid][1] += red[tid + h][1];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double e = sqrt(red[0][0] / red[0][1]);
    err[(int64_t)s * gridDim.y + f] = (bad || !(e == e)) ? INFINITY : e;
  }
}

size_t judge_lds(int p) { return sizeof(double) * (6 * (size_t)p * p + p); }

struct Buf {
  sfm_ctx c;
  hipError_t e = hipSuccess;
  std::vector<void*> ptrs;
  explicit Buf(sfm_ctx ctx) : c(ctx) {}
  ~Buf() {
    for (void* q : ptrs) c->dfree(q);
  }
  template <typename T>
  T* get(size_t n) {
    void* q = c->dalloc(n * sizeof(T), &e);
    if (q) ptrs.push_back(q);
    return static_cast<T*>(q);
  }
};

// Gradient with respect to the network outputs of subdomains s0 .. s0 + nb - 1 from the block
// gradients gg / gh ([S][k][p][p], Gamma_j / Gamma-hat_j): an upper-triangle output sets both
// (i, l) and (l, i) of its block, so it collects both entries' gradients; Gamma-hat_1 (taken from
// Lanczos, not from the network) collects none.
__global__ void output_grad_kernel(const double* __restrict__ gg, const double* __restrict__ gh, int s0, int nb, int k,
                                   int p, const int32_t* __restrict__ ti, const int32_t* __restrict__ tj,
                                   float* __restrict__ dy) {
  const int64_t ntri = (int64_t)p * (p + 1) / 2, per = 2LL * k * ntri, total = (int64_t)nb * per;
  const int64_t pp = (int64_t)p * p;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx / per, r = idx - b * per;
    const int64_t blk = r / ntri, e = r - blk * ntri;
    const bool hat = blk >= k;
    const int j = (int)(hat ? blk - k : blk);
    const int i = ti[e], l = tj[e];
    double v = 0.0;
    if (!(hat && j == 0)) {
      const double* G = (hat ? gh : gg) + ((s0 + b) * k + j) * pp;
      v = i == l ? G[(int64_t)i * p + i] : G[(int64_t)i * p + l] + G[(int64_t)l * p + i];
    }
    dy[idx] = (float)v;
  }
}

// dJ/dc at every node: the input gradients of all subdomain boxes that hold the node (up to 8 on
// shared corners), times d log(c / 3000) / dc = 1 / c.  Equal cubic boxes of n cells; box b along
// an axis holds nodes b n .. (b + 1) n.
__global__ void velocity_gather_kernel(const float* __restrict__ dx, const float* __restrict__ vel, int ncx, int ncy,
                                       int ncz, int n, float* __restrict__ out) {
  const int nbx = ncx / n, nby = ncy / n, nbz = ncz / n, nn = n + 1;
  const int64_t nx = ncx + 1, ny = ncy + 1, total = nx * ny * (ncz + 1), per = (int64_t)nn * nn * nn;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int ix = (int)(e % nx), iy = (int)((e / nx) % ny), iz = (int)(e / (nx * ny));
    int bx[2], by[2], bz[2], cx = 0, cy = 0, cz = 0;
    if (ix / n < nbx) bx[cx++] = ix / n;
    if (ix % n == 0 && ix > 0) bx[cx++] = ix / n - 1;
    if (iy / n < nby) by[cy++] = iy / n;
    if (iy % n == 0 && iy > 0) by[cy++] = iy / n - 1;
    if (iz / n < nbz) bz[cz++] = iz / n;
    if (iz % n == 0 && iz > 0) bz[cz++] = iz / n - 1;
    float acc = 0.f;
    for (int a = 0; a < cz; ++a)
      for (int b = 0; b < cy; ++b)
        for (int c = 0; c < cx; ++c) {
          const int64_t s = ((int64_t)bz[a] * nby + by[b]) * nbx + bx[c];
          const int lz = iz - bz[a] * n, ly = iy - by[b] * n, lx = ix - bx[c] * n;
          acc += dx[s * per + ((int64_t)lz * nn + ly) * nn + lx];
        }
    out[e] = acc / vel[e];
  }
}

bool uniform_boxes(const Topology& t, int* cells) {
  int w[3];
  t.cells(0, w);
  if (w[0] != w[1] || w[1] != w[2]) return false;
  for (int s = 1; s < t.S; ++s) {
    int v[3];
    t.cells(s, v);
    if (v[0] != w[0] || v[1] != w[1] || v[2] != w[2]) return false;
  }
  *cells = w[0];
  return true;
}

}  // namespace
}  // namespace sfm

using namespace sfm;

#define SG_TRY(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return c->fail(SFM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

extern "C" {

sfm_status sfm_rom_inputs(sfm_ctx c, const float* vel_dev, float* x_dev, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!vel_dev || !x_dev) return c->fail(SFM_EINVAL, "vel_dev and x_dev are required");
  int cells = 0;
  if (!uniform_boxes(c->topo, &cells)) return c->fail(SFM_EINVAL, "network inputs need equal cubic subdomains");
  SG_TRY(hipSetDevice(c->device));
  const Topology& t = c->topo;
  std::vector<int32_t> org((size_t)t.S * 3);
  for (int s = 0; s < t.S; ++s) t.origin(s, &org[(size_t)s * 3]);
  Buf b(c);
  int32_t* org_d = b.get<int32_t>(org.size());
  if (b.e != hipSuccess) return c->fail(SFM_ENOMEM, "out of device memory");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  SG_TRY(hipMemcpyAsync(org_d, org.data(), org.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  const int nn = cells + 1;
  hipLaunchKernelGGL(box_inputs_kernel, dim3(4096), dim3(256), 0, st, vel_dev, t.ncell[0], t.ncell[1], org_d, nn, t.S,
                     x_dev);
  SG_TRY(hipGetLastError());
  SG_TRY(hipStreamSynchronize(st));
  return SFM_OK;
}

sfm_status sfm_rom_targets(sfm_ctx c, float* t_dev, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs");
  if (!t_dev) return c->fail(SFM_EINVAL, "t_dev is NULL");
  SG_TRY(hipSetDevice(c->device));
  const Topology& t = c->topo;
  const int p = t.p;
  std::vector<int32_t> ti, tj;
  for (int i = 0; i < p; ++i)
    for (int j = i; j < p; ++j) {
      ti.push_back(i);
      tj.push_back(j);
    }
  Buf b(c);
  int32_t* ti_d = b.get<int32_t>(ti.size());
  int32_t* tj_d = b.get<int32_t>(tj.size());
  if (b.e != hipSuccess) return c->fail(SFM_ENOMEM, "out of device memory");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  SG_TRY(hipMemcpyAsync(ti_d, ti.data(), ti.size() * 4, hipMemcpyHostToDevice, st));
  SG_TRY(hipMemcpyAsync(tj_d, tj.data(), tj.size() * 4, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(rom_targets_kernel, dim3(4096), dim3(256), 0, st, c->coef64_d, t.S, t.k, p, ti_d, tj_d, t_dev);
  SG_TRY(hipGetLastError());
  SG_TRY(hipStreamSynchronize(st));
  return SFM_OK;
}

sfm_status sfm_ntd_error(sfm_ctx c, const double* coef_dev, double f_peak, double* err_host, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs");
  if (!coef_dev || !err_host || !(f_peak > 0.0)) return c->fail(SFM_EINVAL, "coef_dev, err_host and f_peak > 0 required");
  const Topology& t = c->topo;
  if (t.p > kMaxJudgeP) return c->fail(SFM_EINVAL, "the NtD judge supports 6m <= 64");
  SG_TRY(hipSetDevice(c->device));
  double sv[kNtdFreq];
  const double mult[kNtdFreq] = {0.25, 0.5, 0.75, 1.0, 1.5, 2.0, 2.5, 3.0};
  for (int f = 0; f < kNtdFreq; ++f) sv[f] = 2.0 * M_PI * f_peak * mult[f];
  Buf b(c);
  double* sv_d = b.get<double>(kNtdFreq);
  double* err_d = b.get<double>((size_t)t.S * kNtdFreq);
  if (b.e != hipSuccess) return c->fail(SFM_ENOMEM, "out of device memory");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  SG_TRY(hipMemcpyAsync(sv_d, sv, sizeof(sv), hipMemcpyHostToDevice, st));
  const size_t lds = judge_lds(t.p);
  if (lds > kDefaultLdsBytes)
    SG_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&ntd_judge_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
  hipLaunchKernelGGL(ntd_judge_kernel, dim3(t.S, kNtdFreq), dim3(kJudgeThreads), lds, st, coef_dev, c->coef64_d, t.k,
                     t.p, sv_d, err_d);
  SG_TRY(hipGetLastError());
  std::vector<double> e((size_t)t.S * kNtdFreq);
  SG_TRY(hipMemcpyAsync(e.data(), err_d, e.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  SG_TRY(hipStreamSynchronize(st));
  for (int s = 0; s < t.S; ++s) {
    double m = 0.0;
    for (int f = 0; f < kNtdFreq; ++f) m = std::max(m, e[(size_t)s * kNtdFreq + f]);
    err_host[s] = m;
  }
  return SFM_OK;
}

sfm_status sfm_surrogate_predict(sfm_ctx c, sfm_cnn net, const float* vel_dev, double* coef_dev, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!net) return c->fail(SFM_EINVAL, "net is NULL");
  if (!vel_dev || !coef_dev) return c->fail(SFM_EINVAL, "vel_dev and coef_dev are required");
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs: Gamma-hat_1 comes from the current ROMs");
  const Topology& t = c->topo;
  int cells = 0;
  if (!uniform_boxes(t, &cells)) return c->fail(SFM_EINVAL, "the surrogate needs equal cubic subdomains");
  int32_t dims[4] = {};
  sfm_cnn_info(net, nullptr, nullptr, nullptr, dims);
  const int64_t ntri = (int64_t)t.p * (t.p + 1) / 2, n_out = 2LL * t.k * ntri;
  if (dims[0] != cells + 1) return c->fail(SFM_EINVAL, "network input size differs from the subdomain nodes");
  if (dims[2] != n_out) return c->fail(SFM_EINVAL, "network output size differs from 2k p(p+1)/2");
  SG_TRY(hipSetDevice(c->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t nin3 = (int64_t)(cells + 1) * (cells + 1) * (cells + 1);
  Buf b(c);
  float* x = b.get<float>((size_t)t.S * nin3);
  float* y = b.get<float>((size_t)t.S * n_out);
  if (b.e != hipSuccess) return c->fail(SFM_ENOMEM, "surrogate buffers: out of device memory");
  sfm_status rc = sfm_rom_inputs(c, vel_dev, x, stream);
  if (rc != SFM_OK) return rc;
  const int32_t maxb = dims[3];
  for (int s0 = 0; s0 < t.S; s0 += maxb) {
    const int nb = std::min<int>(maxb, t.S - s0);
    rc = sfm_cnn_forward(net, x + (int64_t)s0 * nin3, nb, y + (int64_t)s0 * n_out, stream);
    if (rc != SFM_OK) return c->fail(rc, std::string("surrogate forward: ") + sfm_cnn_last_error(net));
  }
  hipLaunchKernelGGL(unpack_pred_kernel, dim3(4096), dim3(256), 0, st, y, c->coef64_d, t.S, t.k, t.p, coef_dev);
  SG_TRY(hipGetLastError());
  SG_TRY(hipStreamSynchronize(st));
  return SFM_OK;
}

sfm_status sfm_build_roms_surrogate(sfm_ctx c, sfm_cnn net, double tol, double f_peak, const float* vel_dev,
                                    int32_t nsrc, const int32_t* src_ijk, int32_t nrec, const int32_t* rec_ijk,
                                    int32_t* accepted, double* ntd_err, double* seconds, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!net) return c->fail(SFM_EINVAL, "net is NULL");
  if (!(tol >= 0.0) || !(f_peak > 0.0)) return c->fail(SFM_EINVAL, "need tol >= 0 and f_peak > 0");
  const Topology& t = c->topo;
  int cells = 0;
  if (!uniform_boxes(t, &cells)) return c->fail(SFM_EINVAL, "the surrogate needs equal cubic subdomains");
  int64_t n_params = 0;
  int32_t dims[4] = {};
  sfm_cnn_info(net, &n_params, nullptr, nullptr, dims);
  const int64_t ntri = (int64_t)t.p * (t.p + 1) / 2, n_out = 2LL * t.k * ntri;
  if (dims[0] != cells + 1) return c->fail(SFM_EINVAL, "network input size differs from the subdomain nodes");
  if (dims[2] != n_out) return c->fail(SFM_EINVAL, "network output size differs from 2k p(p+1)/2");
  if (t.p > kMaxJudgeP) return c->fail(SFM_EINVAL, "the NtD judge supports 6m <= 64");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto secs = [](auto a, auto b) { return std::chrono::duration<double>(b - a).count(); };
  // judge and fallback: the Lanczos ROMs of every subdomain
  auto t0 = now();
  sfm_status rc = sfm_build_roms(c, vel_dev, nsrc, src_ijk, nrec, rec_ijk, nullptr, nullptr, stream);
  if (rc != SFM_OK) return rc;
  SG_TRY(hipStreamSynchronize(st));
  auto t1 = now();
  // predictions
  const int64_t pp = (int64_t)t.p * t.p;
  Buf b(c);
  double* pred = b.get<double>((size_t)t.S * 2 * t.k * pp);
  if (b.e != hipSuccess) return c->fail(SFM_ENOMEM, "surrogate buffers: out of device memory");
  rc = sfm_surrogate_predict(c, net, vel_dev, pred, stream);
  if (rc != SFM_OK) return rc;
  auto t2 = now();
  std::vector<double> err((size_t)t.S);
  rc = sfm_ntd_error(c, pred, f_peak, err.data(), stream);
  if (rc != SFM_OK) return rc;
  auto t3 = now();
  // keep the accepted predictions, repack the coefficient stream
  std::vector<uint8_t> pinned((size_t)t.S, 0);
  for (int32_t s : c->src_sub) pinned[(size_t)s] = 1;
  {
    std::vector<int32_t> rs(c->nrec);
    if (c->nrec) SG_TRY(hipMemcpy(rs.data(), c->rec_sub_d, rs.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int32_t s : rs) pinned[(size_t)s] = 1;
  }
  int n_acc = 0;
  for (int s = 0; s < t.S; ++s) {
    const bool ok = !pinned[(size_t)s] && err[(size_t)s] <= tol;
    if (accepted) accepted[s] = ok ? 1 : 0;
    if (ntd_err) ntd_err[s] = err[(size_t)s];
    if (ok) {
      SG_TRY(hipMemcpyAsync(c->coef64_d + (int64_t)s * 2 * t.k * pp, pred + (int64_t)s * 2 * t.k * pp,
                            (size_t)2 * t.k * pp * sizeof(double), hipMemcpyDeviceToDevice, st));
      ++n_acc;
    }
  }
  if (n_acc) {
    std::vector<int32_t> wrow, wcol;
    c->geo.word_map(wrow, wcol, (int)c->tile_elem);
    int32_t* wr = b.get<int32_t>(wrow.size());
    int32_t* wc = b.get<int32_t>(wcol.size());
    if (b.e != hipSuccess) return c->fail(SFM_ENOMEM, "out of device memory");
    SG_TRY(hipMemcpyAsync(wr, wrow.data(), wrow.size() * 4, hipMemcpyHostToDevice, st));
    SG_TRY(hipMemcpyAsync(wc, wcol.data(), wcol.size() * 4, hipMemcpyHostToDevice, st));
    SG_TRY(launch_pack(c->coef64_d, 0, 0, t.k, t.p, c->geo, wr, wc, c->tiles_d, c->cfg.precision, t.S, st));
    c->dt_max = -1.0;
  }
  SG_TRY(hipStreamSynchronize(st));
  auto t4 = now();
  if (seconds) {
    seconds[0] = secs(t0, t1);   // Lanczos ROMs (judge and fallback)
    seconds[1] = secs(t1, t2);   // network inputs, inference, unpacking
    seconds[2] = secs(t2, t3);   // NtD judge
    seconds[3] = secs(t3, t4);   // accept and repack
  }
  return SFM_OK;
}

sfm_status sfm_surrogate_velocity_gradient(sfm_ctx c, sfm_cnn net, const float* vel_dev, const double* grad_gamma,
                                           const double* grad_gamma_hat, float* grad_vel_dev, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!net) return c->fail(SFM_EINVAL, "net is NULL");
  if (!vel_dev || !grad_gamma || !grad_gamma_hat || !grad_vel_dev)
    return c->fail(SFM_EINVAL, "vel_dev, grad_gamma, grad_gamma_hat and grad_vel_dev are required");
  const Topology& t = c->topo;
  int cells = 0;
  if (!uniform_boxes(t, &cells)) return c->fail(SFM_EINVAL, "the surrogate needs equal cubic subdomains");
  int32_t dims[4] = {};
  sfm_cnn_info(net, nullptr, nullptr, nullptr, dims);
  const int p = t.p, k = t.k;
  const int64_t ntri = (int64_t)p * (p + 1) / 2, n_out = 2LL * k * ntri;
  if (dims[0] != cells + 1) return c->fail(SFM_EINVAL, "network input size differs from the subdomain nodes");
  if (dims[2] != n_out) return c->fail(SFM_EINVAL, "network output size differs from 2k p(p+1)/2");
  SG_TRY(hipSetDevice(c->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t nin3 = (int64_t)(cells + 1) * (cells + 1) * (cells + 1);
  const size_t ng = (size_t)t.S * k * p * p;
  const int32_t maxb = dims[3];
  std::vector<int32_t> ti, tj;
  for (int i = 0; i < p; ++i)
    for (int j = i; j < p; ++j) {
      ti.push_back(i);
      tj.push_back(j);
    }
  Buf b(c);
  double* gg = b.get<double>(ng);
  double* gh = b.get<double>(ng);
  float* x = b.get<float>((size_t)t.S * nin3);
  float* dx = b.get<float>((size_t)t.S * nin3);
  float* dy = b.get<float>((size_t)maxb * n_out);
  int32_t* ti_d = b.get<int32_t>(ti.size());
  int32_t* tj_d = b.get<int32_t>(tj.size());
  if (b.e != hipSuccess) return c->fail(SFM_ENOMEM, "velocity gradient buffers: out of device memory");
  SG_TRY(hipMemcpyAsync(gg, grad_gamma, ng * sizeof(double), hipMemcpyHostToDevice, st));
  SG_TRY(hipMemcpyAsync(gh, grad_gamma_hat, ng * sizeof(double), hipMemcpyHostToDevice, st));
  SG_TRY(hipMemcpyAsync(ti_d, ti.data(), ti.size() * 4, hipMemcpyHostToDevice, st));
  SG_TRY(hipMemcpyAsync(tj_d, tj.data(), tj.size() * 4, hipMemcpyHostToDevice, st));
  sfm_status rc = sfm_rom_inputs(c, vel_dev, x, stream);
  if (rc != SFM_OK) return rc;
  for (int s0 = 0; s0 < t.S; s0 += maxb) {
    const int nb = std::min<int>(maxb, t.S - s0);
    rc = sfm_cnn_forward(net, x + (int64_t)s0 * nin3, nb, nullptr, stream);
    if (rc != SFM_OK) return c->fail(rc, std::string("surrogate forward: ") + sfm_cnn_last_error(net));
    hipLaunchKernelGGL(output_grad_kernel, dim3(2048), dim3(256), 0, st, gg, gh, s0, nb, k, p, ti_d, tj_d, dy);
    SG_TRY(hipGetLastError());
    rc = sfm_cnn_input_grad(net, dy, dx + (int64_t)s0 * nin3, stream);
    if (rc != SFM_OK) return c->fail(rc, std::string("surrogate input gradient: ") + sfm_cnn_last_error(net));
  }
  hipLaunchKernelGGL(velocity_gather_kernel, dim3(4096), dim3(256), 0, st, dx, vel_dev, t.ncell[0], t.ncell[1],
                     t.ncell[2], cells, grad_vel_dev);
  SG_TRY(hipGetLastError());
  SG_TRY(hipStreamSynchronize(st));
  return SFM_OK;
}

}  // extern "C"
