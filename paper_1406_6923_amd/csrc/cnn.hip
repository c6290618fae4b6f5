// Learned ROM surrogate network: a 3D CNN (four 3x3x3 stride-2 convolution blocks with ReLU,
// then a dense head) that maps a subdomain's sound speed to its S-fraction coefficients, so that
// many ROM builds (the many forward solves FWI needs, Introduction) can be predicted instead of
// computed, with block Lanczos as judge and fallback.
//
// Every product runs on the bf16 matrix cores with FP32 accumulation
// (v_mfma_f32_16x16x16_bf16): forward convolutions, both halves of the backward pass and the
// dense layer are one implicit GEMM kernel whose operands are gathered through a problem-specific
// index map (no im2col buffers), rounded to bfloat16 (nearest, ties to even) on the way into LDS.
// Activations, gradients, master weights and the Adam moments stay FP32.
//
// Layouts (shared with the host side and the flat parameter vector):
//   activations channels-last [batch][z][y][x][channel] (the input has one channel);
//   conv weights W[co][t][ci], t = 9 dz + 3 dy + dx, then bias[co]; dense Wd[j][i], then bd[j];
//   flat parameters W1 b1 W2 b2 W3 b3 W4 b4 Wd bd; gradients use the same layout.
// A stride-2, pad-1, size-3 convolution maps n nodes per axis to (n - 1) / 2 + 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "sfm.h"

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kConv = 4;
constexpr int kBM = 64, kBN = 64, kBK = 16, kThreads = 256;
constexpr int64_t kSplitTarget = 2048;   // work-groups a split-K product aims for

// K per work-group slice of a product whose M x N tiles alone do not fill the device: enough
// slices for about kSplitTarget work-groups, at least 256 per slice (a multiple of the K step).
int64_t split_k(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
  if (tiles >= kSplitTarget) return K;
  const int64_t want = (K * tiles + kSplitTarget - 1) / kSplitTarget;
  return std::min<int64_t>(K, std::max<int64_t>(256, (want + 15) / 16 * 16));
}

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);     // round to nearest, ties to even (finite inputs)
  return (uint16_t)(u >> 16);
}

// C[m][n] = sum_k A(m, k) B(k, n) over the K slice of blockIdx.z; P supplies M, N, K, a(), b() and
// store(m, n, value, slice).  A work-group computes a 64 x 64 tile, each of its four waves a
// 32 x 32 quarter as 2 x 2 MFMA tiles.  Lane l of an MFMA holds A[l % 16][4 (l / 16) + 0..3] and
// B[4 (l / 16) + 0..3][l % 16]; its result element v is C[4 (l / 16) + v][l % 16].
template <class P>
__global__ __launch_bounds__(kThreads) void gemm_bf16_kernel(P pb, int64_t kslice) {
  __shared__ __align__(16) uint16_t As[kBM][kBK + 4];
  __shared__ __align__(16) uint16_t Bt[kBN][kBK + 4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t m0 = (int64_t)blockIdx.x * kBM, n0 = (int64_t)blockIdx.y * kBN;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int64_t kb = (int64_t)blockIdx.z * kslice, ke = std::min<int64_t>(pb.K, kb + kslice);
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  for (int64_t k0 = kb; k0 < ke; k0 += kBK) {
    for (int e = tid; e < kBM * kBK; e += kThreads) {
      const int r = e / kBK, kk = e % kBK;
      const int64_t m = m0 + r, k = k0 + kk;
      As[r][kk] = to_bf16((m < pb.M && k < ke) ? pb.a(m, k) : 0.f);
    }
    for (int e = tid; e < kBN * kBK; e += kThreads) {
      const int c = e / kBK, kk = e % kBK;
      const int64_t n = n0 + c, k = k0 + kk;
      Bt[c][kk] = to_bf16((n < pb.N && k < ke) ? pb.b(k, n) : 0.f);
    }
    __syncthreads();
    s4 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const s4*>(&As[wm + 16 * i + li][4 * g]);
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const s4*>(&Bt[wn + 16 * j + li][4 * g]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + wm + 16 * i + 4 * g + v, n = n0 + wn + 16 * j + li;
        if (m < pb.M && n < pb.N) pb.store(m, n, acc[i][j][v], (int)blockIdx.z);
      }
}

struct Grid3 {
  int n;   // nodes per axis
  __device__ __forceinline__ void split(int64_t r, int& b, int& z, int& y, int& x) const {
    x = (int)(r % n);
    r /= n;
    y = (int)(r % n);
    r /= n;
    z = (int)(r % n);
    b = (int)(r / n);
  }
};

// Forward convolution + bias + ReLU: rows = output positions, columns = output channels,
// k = t ci_count + ci.
struct ConvFwd {
  int64_t M, N, K;
  const float* x;
  const float* W;
  const float* bias;
  float* out;
  Grid3 gi, go;
  int ci;
  __device__ float a(int64_t r, int64_t k) const {
    const int t = (int)(k / ci), c = (int)(k - (int64_t)t * ci);
    int b, zo, yo, xo;
    go.split(r, b, zo, yo, xo);
    const int z = 2 * zo - 1 + t / 9, y = 2 * yo - 1 + (t / 3) % 3, xx = 2 * xo - 1 + t % 3;
    const int n = gi.n;
    if (z < 0 || z >= n || y < 0 || y >= n || xx < 0 || xx >= n) return 0.f;
    return x[((((int64_t)b * n + z) * n + y) * n + xx) * ci + c];
  }
  __device__ float b(int64_t k, int64_t c) const { return W[c * K + k]; }
  __device__ void store(int64_t r, int64_t c, float v, int) const { out[r * N + c] = fmaxf(v + bias[c], 0.f); }
};

// Gradient of the layer input: rows = input positions, columns = input channels, k = t co + o;
// dpre = dact where the layer's output was positive (ReLU), else 0.
struct ConvBwdData {
  int64_t M, N, K;
  const float* dact;
  const float* act;
  const float* W;
  float* dx;
  Grid3 gi, go;
  int co;
  __device__ float a(int64_t r, int64_t k) const {
    const int t = (int)(k / co), o = (int)(k - (int64_t)t * co);
    int b, z, y, x;
    gi.split(r, b, z, y, x);
    const int sz = z + 1 - t / 9, sy = y + 1 - (t / 3) % 3, sx = x + 1 - t % 3;
    if ((sz | sy | sx) & 1) return 0.f;
    const int zo = sz >> 1, yo = sy >> 1, xo = sx >> 1;
    const int m = go.n;
    if (sz < 0 || sy < 0 || sx < 0 || zo >= m || yo >= m || xo >= m) return 0.f;
    const int64_t idx = ((((int64_t)b * m + zo) * m + yo) * m + xo) * co + o;
    return act[idx] > 0.f ? dact[idx] : 0.f;
  }
  __device__ float b(int64_t k, int64_t c) const {
    const int t = (int)(k / co), o = (int)(k - (int64_t)t * co);
    return W[((int64_t)o * 27 + t) * N + c];
  }
  __device__ void store(int64_t r, int64_t c, float v, int) const { dx[r * N + c] = v; }
};

// Gradient of the weights, split over K (output positions): partial[slice][o][t ci + c].
struct ConvBwdW {
  int64_t M, N, K;
  const float* dact;
  const float* act;
  const float* x;
  float* part;
  Grid3 gi, go;
  int ci;
  __device__ float a(int64_t o, int64_t k) const {
    const int64_t idx = k * M + o;
    return act[idx] > 0.f ? dact[idx] : 0.f;
  }
  __device__ float b(int64_t k, int64_t c) const {
    const int t = (int)(c / ci), cc = (int)(c - (int64_t)t * ci);
    int b, zo, yo, xo;
    go.split(k, b, zo, yo, xo);
    const int z = 2 * zo - 1 + t / 9, y = 2 * yo - 1 + (t / 3) % 3, xx = 2 * xo - 1 + t % 3;
    const int n = gi.n;
    if (z < 0 || z >= n || y < 0 || y >= n || xx < 0 || xx >= n) return 0.f;
    return x[((((int64_t)b * n + z) * n + y) * n + xx) * ci + cc];
  }
  __device__ void store(int64_t o, int64_t c, float v, int s) const { part[((int64_t)s * M + o) * N + c] = v; }
};

// Dense layer: y[b][j] = feat[b] . Wd[j] + bd[j].
struct DenseFwd {
  int64_t M, N, K;
  const float* feat;
  const float* Wd;
  const float* bd;
  float* y;
  __device__ float a(int64_t b, int64_t i) const { return feat[b * K + i]; }
  __device__ float b(int64_t i, int64_t j) const { return Wd[j * K + i]; }
  __device__ void store(int64_t b, int64_t j, float v, int) const { y[b * N + j] = v + bd[j]; }
};

// dfeat[b][i] = sum_j dy[b][j] Wd[j][i], split over j: partial[slice][b][i].
struct DenseBwdData {
  int64_t M, N, K;
  const float* dy;
  const float* Wd;
  float* part;
  __device__ float a(int64_t b, int64_t j) const { return dy[b * K + j]; }
  __device__ float b(int64_t j, int64_t i) const { return Wd[j * N + i]; }
  __device__ void store(int64_t b, int64_t i, float v, int s) const { part[((int64_t)s * M + b) * N + i] = v; }
};

// dWd[j][i] = sum_b dy[b][j] feat[b][i].
struct DenseBwdW {
  int64_t M, N, K;
  const float* dy;
  const float* feat;
  float* dW;
  __device__ float a(int64_t j, int64_t b) const { return dy[b * M + j]; }
  __device__ float b(int64_t b, int64_t i) const { return feat[b * N + i]; }
  __device__ void store(int64_t j, int64_t i, float v, int) const { dW[j * N + i] = v; }
};

// out[i] = sum over slices of part[s][i]
__global__ void sum_slices_kernel(const float* __restrict__ part, int slices, int64_t n, float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float acc = 0.f;
    for (int s = 0; s < slices; ++s) acc += part[(int64_t)s * n + i];
    out[i] = acc;
  }
}

// Column sums of [rows][cols] (dpre = d where act > 0 when act is given): one partial per block,
// part[block][col]; the host-side launch sums the partials with sum_slices_kernel.
__global__ void column_sum_kernel(const float* __restrict__ d, const float* __restrict__ act, int64_t rows, int cols,
                                  float* __restrict__ part) {
  const int c = threadIdx.x % cols;
  const int lanes = blockDim.x / cols;
  const int sub = threadIdx.x / cols;
  if (sub >= lanes) return;
  __shared__ float red[256];
  float acc = 0.f;
  for (int64_t r = (int64_t)blockIdx.x * lanes + sub; r < rows; r += (int64_t)gridDim.x * lanes) {
    const int64_t idx = r * cols + c;
    acc += (!act || act[idx] > 0.f) ? d[idx] : 0.f;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (sub == 0) {
    float s = 0.f;
    for (int q = 0; q < lanes; ++q) s += red[q * cols + c];
    part[(int64_t)blockIdx.x * cols + c] = s;
  }
}

// Column sums of a short, wide [rows][cols] array (rows <= a batch): one thread per column.
__global__ void column_sum_wide_kernel(const float* __restrict__ d, int64_t rows, int64_t cols, float* __restrict__ out) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += (int64_t)gridDim.x * blockDim.x) {
    float acc = 0.f;
    for (int64_t r = 0; r < rows; ++r) acc += d[r * cols + c];
    out[c] = acc;
  }
}

// dy = 2 (y - t) / count; part[block] = sum of (y - t)^2 over the block's entries (FP64).
__global__ void mse_kernel(const float* __restrict__ y, const float* __restrict__ t, int64_t n, float* __restrict__ dy,
                           double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  const float scale = 2.f / (float)n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float r = y[i] - t[i];
    dy[i] = scale * r;
    acc += (double)r * (double)r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam (bias-corrected moments): c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Per-output mean and standard deviation over n samples of [n][cols] (FP64 sums); a constant
// output gets std 1.
__global__ void fit_scale_kernel(const float* __restrict__ t, int64_t n, int64_t cols, float* __restrict__ mean,
                                 float* __restrict__ sd) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += (int64_t)gridDim.x * blockDim.x) {
    double s1 = 0.0;
    for (int64_t r = 0; r < n; ++r) s1 += t[r * cols + c];
    const double mu = s1 / (double)n;
    double s2 = 0.0;
    for (int64_t r = 0; r < n; ++r) {
      const double d = t[r * cols + c] - mu;
      s2 += d * d;
    }
    const double sdv = sqrt(s2 / (double)n);
    mean[c] = (float)mu;
    sd[c] = sdv > 1e-30 * (fabs(mu) + 1e-300) && sdv > 0.0 ? (float)sdv : 1.f;
  }
}

// x[r][c] = (x[r][c] - mean[c]) / sd[c]  (dir = +1), or mean[c] + sd[c] x[r][c]  (dir = -1)
__global__ void apply_scale_kernel(float* __restrict__ x, int64_t rows, int64_t cols, const float* __restrict__ mean,
                                   const float* __restrict__ sd, int dir) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e % cols;
    x[e] = dir > 0 ? (x[e] - mean[c]) / sd[c] : fmaf(sd[c], x[e], mean[c]);
  }
}

// out[r][c] = sd[c] dy[r][c]: a gradient with respect to the scaled output, carried to the net's own
__global__ void scale_grad_kernel(const float* __restrict__ dy, int64_t rows, int64_t cols, const float* __restrict__ sd,
                                  float* __restrict__ out) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = sd[e % cols] * dy[e];
}

// rows of x gathered by index: dst[r] = src[idx[r]] (rows of `len` floats)
__global__ void gather_rows_kernel(const float* __restrict__ src, const int32_t* __restrict__ idx, int rows, int64_t len,
                                   float* __restrict__ dst) {
  const int64_t total = (int64_t)rows * len;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / len, c = e - r * len;
    dst[e] = src[(int64_t)idx[r] * len + c];
  }
}

template <class P>
hipError_t launch_gemm(const P& pb, int64_t kslice, hipStream_t st) {
  const int64_t slices = (pb.K + kslice - 1) / kslice;
  dim3 grid((unsigned)((pb.M + kBM - 1) / kBM), (unsigned)((pb.N + kBN - 1) / kBN), (unsigned)std::max<int64_t>(1, slices));
  hipLaunchKernelGGL(gemm_bf16_kernel<P>, grid, dim3(kThreads), 0, st, pb, kslice);
  return hipGetLastError();
}

unsigned blocks_for(int64_t n) { return (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256)); }

}  // namespace

struct sfm_cnn_s {
  int n_in = 0, ch = 0, n_out = 0, max_batch = 0;
  int nodes[kConv + 1] = {};            // nodes per axis of the input and of each activation
  int64_t off_W[kConv] = {}, off_b[kConv] = {}, off_Wd = 0, off_bd = 0, n_params = 0, feat = 0;
  int device = 0;
  std::string err;
  std::vector<void*> owned;
  float* params = nullptr;              // FP32 master weights (flat)
  float* grads = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* xin = nullptr;                 // [max_batch][n_in^3] gathered inputs
  float* tgt = nullptr;                 // [max_batch][n_out] gathered targets
  float* act[kConv + 1] = {};           // act[0] = input (aliased), act[l] = layer-l output
  float* dact[kConv + 1] = {};
  float* y = nullptr;
  float* dy = nullptr;
  float* out_mean = nullptr;            // output scale: the net predicts (target - mean) / sd
  float* out_sd = nullptr;
  bool scaled = false;
  float* part = nullptr;                // split-K / column-sum partials
  int64_t part_len = 0;
  double* loss_part = nullptr;
  int32_t* idx_d = nullptr;
  int64_t adam_t = 0;
  int last_batch = 0;

  sfm_status fail(sfm_status s, const std::string& m) {
    err = m;
    return s;
  }
  // *e is written only on failure: the first failure of a run of allocations is kept
  void* alloc(size_t bytes, hipError_t* e) {
    void* p = nullptr;
    const hipError_t r = hipMalloc(&p, std::max<size_t>(bytes, 16));
    if (r != hipSuccess) {
      *e = r;
      return nullptr;
    }
    owned.push_back(p);
    return p;
  }
};

#define CNN_TRY(call)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return net->fail(SFM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

thread_local std::string g_cnn_create_error;

// Largest partial buffer any product of a batch of B needs.
int64_t partial_len(const sfm_cnn_s& c, int B) {
  int64_t need = 0;
  for (int l = 0; l < kConv; ++l) {
    const int ci = l == 0 ? 1 : c.ch;
    const int64_t K = (int64_t)B * c.nodes[l + 1] * c.nodes[l + 1] * c.nodes[l + 1];
    const int64_t ks = split_k(c.ch, 27LL * ci, K);
    need = std::max<int64_t>(need, (K + ks - 1) / ks * c.ch * 27 * ci);
    need = std::max<int64_t>(need, (int64_t)4096 * c.ch);               // column sums
  }
  const int64_t kd = split_k(B, c.feat, c.n_out);
  need = std::max<int64_t>(need, ((int64_t)c.n_out + kd - 1) / kd * B * c.feat);
  return need;
}

sfm_status forward_pass(sfm_cnn net, const float* x, int B, hipStream_t st) {
  net->act[0] = const_cast<float*>(x);
  for (int l = 0; l < kConv; ++l) {
    const int ci = l == 0 ? 1 : net->ch, n = net->nodes[l], m = net->nodes[l + 1];
    ConvFwd pb{};
    pb.M = (int64_t)B * m * m * m;
    pb.N = net->ch;
    pb.K = 27LL * ci;
    pb.x = net->act[l];
    pb.W = net->params + net->off_W[l];
    pb.bias = net->params + net->off_b[l];
    pb.out = net->act[l + 1];
    pb.gi = Grid3{n};
    pb.go = Grid3{m};
    pb.ci = ci;
    CNN_TRY(launch_gemm(pb, pb.K, st));
  }
  DenseFwd d{};
  d.M = B;
  d.N = net->n_out;
  d.K = net->feat;
  d.feat = net->act[kConv];
  d.Wd = net->params + net->off_Wd;
  d.bd = net->params + net->off_bd;
  d.y = net->y;
  CNN_TRY(launch_gemm(d, d.K, st));
  net->last_batch = B;
  return SFM_OK;
}

sfm_status column_sums(sfm_cnn net, const float* d, const float* act, int64_t rows, int cols, float* out, hipStream_t st) {
  if (cols > 256) {                      // the dense bias: rows = batch
    hipLaunchKernelGGL(column_sum_wide_kernel, dim3(blocks_for(cols)), dim3(256), 0, st, d, rows, (int64_t)cols, out);
    CNN_TRY(hipGetLastError());
    return SFM_OK;
  }
  const int lanes = 256 / cols;
  const unsigned blocks = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (rows + lanes - 1) / lanes));
  hipLaunchKernelGGL(column_sum_kernel, dim3(blocks), dim3(lanes * cols), 0, st, d, act, rows, cols, net->part);
  CNN_TRY(hipGetLastError());
  hipLaunchKernelGGL(sum_slices_kernel, dim3(blocks_for(cols)), dim3(256), 0, st, net->part, (int)blocks,
                     (int64_t)cols, out);
  CNN_TRY(hipGetLastError());
  return SFM_OK;
}

// Gradients of sum(dy * y) into g (flat layout), for the last forward pass.
// Gradients of sum(dy * y) for the last forward pass (y the net's own, unscaled output): the
// parameters into g (flat layout; skipped when g is null) and the input into dx ([B][n_in^3];
// skipped when dx is null).
sfm_status backward_pass(sfm_cnn net, const float* dy, int B, float* g, float* dx, hipStream_t st) {
  const int64_t F = net->feat;
  {  // dense layer
    if (g) {
      DenseBwdW w{};
      w.M = net->n_out;
      w.N = F;
      w.K = B;
      w.dy = dy;
      w.feat = net->act[kConv];
      w.dW = g + net->off_Wd;
      CNN_TRY(launch_gemm(w, w.K, st));
      sfm_status rc = column_sums(net, dy, nullptr, B, net->n_out, g + net->off_bd, st);
      if (rc != SFM_OK) return rc;
    }
    DenseBwdData d{};
    d.M = B;
    d.N = F;
    d.K = net->n_out;
    d.dy = dy;
    d.Wd = net->params + net->off_Wd;
    d.part = net->part;
    const int64_t kd = split_k(d.M, d.N, d.K);
    const int slices = (int)((d.K + kd - 1) / kd);
    if ((int64_t)slices * d.M * d.N > net->part_len) return net->fail(SFM_EINVAL, "partial-sum buffer too small");
    CNN_TRY(launch_gemm(d, kd, st));
    hipLaunchKernelGGL(sum_slices_kernel, dim3(blocks_for((int64_t)B * F)), dim3(256), 0, st, net->part, slices,
                       (int64_t)B * F, net->dact[kConv]);
    CNN_TRY(hipGetLastError());
  }
  for (int l = kConv - 1; l >= 0; --l) {
    const int ci = l == 0 ? 1 : net->ch, n = net->nodes[l], m = net->nodes[l + 1];
    const int64_t rows = (int64_t)B * m * m * m;
    if (g) {
      ConvBwdW w{};
      w.M = net->ch;
      w.N = 27LL * ci;
      w.K = rows;
      w.dact = net->dact[l + 1];
      w.act = net->act[l + 1];
      w.x = net->act[l];
      w.part = net->part;
      w.gi = Grid3{n};
      w.go = Grid3{m};
      w.ci = ci;
      const int64_t kw = split_k(w.M, w.N, w.K);
      const int slices = (int)((rows + kw - 1) / kw);
      if ((int64_t)slices * w.M * w.N > net->part_len) return net->fail(SFM_EINVAL, "partial-sum buffer too small");
      CNN_TRY(launch_gemm(w, kw, st));
      hipLaunchKernelGGL(sum_slices_kernel, dim3(blocks_for(w.M * w.N)), dim3(256), 0, st, net->part, slices,
                         w.M * w.N, g + net->off_W[l]);
      CNN_TRY(hipGetLastError());
      sfm_status rc = column_sums(net, net->dact[l + 1], net->act[l + 1], rows, net->ch, g + net->off_b[l], st);
      if (rc != SFM_OK) return rc;
    }
    if (l > 0 || dx) {            // gradient of this layer's input (the net's input for l = 0)
      ConvBwdData d{};
      d.M = (int64_t)B * n * n * n;
      d.N = ci;
      d.K = 27LL * net->ch;
      d.dact = net->dact[l + 1];
      d.act = net->act[l + 1];
      d.W = net->params + net->off_W[l];
      d.dx = l > 0 ? net->dact[l] : dx;
      d.gi = Grid3{n};
      d.go = Grid3{m};
      d.co = net->ch;
      CNN_TRY(launch_gemm(d, d.K, st));
    }
  }
  return SFM_OK;
}

}  // namespace

extern "C" {

sfm_status sfm_cnn_create(int32_t n_in, int32_t channels, int32_t n_out, int32_t max_batch, uint64_t seed,
                          sfm_cnn* out) {
  if (!out) return SFM_EINVAL;
  *out = nullptr;
  if (n_in < 3 || channels < 1 || channels > 256 || n_out < 1 || max_batch < 1) {
    g_cnn_create_error = "need n_in >= 3, 1 <= channels <= 256, n_out >= 1, max_batch >= 1";
    return SFM_EINVAL;
  }
  auto* net = new (std::nothrow) sfm_cnn_s();
  if (!net) return SFM_ENOMEM;
  net->n_in = n_in;
  net->ch = channels;
  net->n_out = n_out;
  net->max_batch = max_batch;
  net->nodes[0] = n_in;
  for (int l = 0; l < kConv; ++l) net->nodes[l + 1] = (net->nodes[l] - 1) / 2 + 1;
  int64_t o = 0;
  for (int l = 0; l < kConv; ++l) {
    const int ci = l == 0 ? 1 : channels;
    net->off_W[l] = o;
    o += (int64_t)channels * 27 * ci;
    net->off_b[l] = o;
    o += channels;
  }
  const int64_t nl = net->nodes[kConv];
  net->feat = nl * nl * nl * channels;
  net->off_Wd = o;
  o += net->feat * n_out;
  net->off_bd = o;
  o += n_out;
  net->n_params = o;
  (void)hipGetDevice(&net->device);
  hipError_t e = hipSuccess;
  auto F = [&](int64_t count) { return static_cast<float*>(net->alloc((size_t)count * sizeof(float), &e)); };
  net->params = F(o);
  net->grads = F(o);
  net->m1 = F(o);
  net->m2 = F(o);
  const int64_t nin3 = (int64_t)n_in * n_in * n_in;
  net->xin = F((int64_t)max_batch * nin3);
  net->tgt = F((int64_t)max_batch * n_out);
  for (int l = 1; l <= kConv; ++l) {
    const int64_t nn = net->nodes[l];
    net->act[l] = F((int64_t)max_batch * nn * nn * nn * channels);
    net->dact[l] = F((int64_t)max_batch * nn * nn * nn * channels);
  }
  net->y = F((int64_t)max_batch * n_out);
  net->dy = F((int64_t)max_batch * n_out);
  net->out_mean = F(n_out);
  net->out_sd = F(n_out);
  net->part_len = 0;
  for (int b = 1; b <= max_batch; ++b) net->part_len = std::max<int64_t>(net->part_len, partial_len(*net, b));
  net->part = F(net->part_len);
  net->loss_part = static_cast<double*>(net->alloc(4096 * sizeof(double), &e));
  net->idx_d = static_cast<int32_t*>(net->alloc((size_t)max_batch * sizeof(int32_t), &e));
  if (e != hipSuccess) {
    g_cnn_create_error = std::string("device allocation failed: ") + hipGetErrorString(e);
    sfm_cnn_destroy(net);
    return SFM_ENOMEM;
  }
  // He initialisation of the convolutions, 1/sqrt(fan_in) of the dense head, zero biases
  std::vector<float> h((size_t)o, 0.f);
  std::mt19937_64 rng(seed);
  for (int l = 0; l < kConv; ++l) {
    const int ci = l == 0 ? 1 : channels;
    std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (27.f * ci)));
    for (int64_t i = 0; i < (int64_t)channels * 27 * ci; ++i) h[net->off_W[l] + i] = nd(rng);
  }
  std::normal_distribution<float> nd(0.f, 1.f / std::sqrt((float)net->feat));
  for (int64_t i = 0; i < net->feat * n_out; ++i) h[net->off_Wd + i] = nd(rng);
  if ((e = hipMemcpy(net->params, h.data(), (size_t)o * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(net->m1, 0, (size_t)o * sizeof(float))) != hipSuccess ||
      (e = hipMemset(net->m2, 0, (size_t)o * sizeof(float))) != hipSuccess) {
    g_cnn_create_error = std::string("initialisation failed: ") + hipGetErrorString(e);
    sfm_cnn_destroy(net);
    return SFM_EHIP;
  }
  *out = net;
  return SFM_OK;
}

void sfm_cnn_destroy(sfm_cnn net) {
  if (!net) return;
  (void)hipDeviceSynchronize();
  for (void* p : net->owned) (void)hipFree(p);
  delete net;
}

const char* sfm_cnn_last_error(sfm_cnn net) { return net ? net->err.c_str() : g_cnn_create_error.c_str(); }

sfm_status sfm_cnn_info(sfm_cnn net, int64_t* n_params, int32_t* feat, int32_t* nodes5, int32_t* dims4) {
  if (!net) return SFM_EINVAL;
  if (n_params) *n_params = net->n_params;
  if (feat) *feat = (int32_t)net->feat;
  if (nodes5)
    for (int l = 0; l <= kConv; ++l) nodes5[l] = net->nodes[l];
  if (dims4) {
    dims4[0] = net->n_in;
    dims4[1] = net->ch;
    dims4[2] = net->n_out;
    dims4[3] = net->max_batch;
  }
  return SFM_OK;
}

sfm_status sfm_cnn_params(sfm_cnn net, float* get_host, const float* set_host) {
  if (!net) return SFM_EINVAL;
  net->err.clear();
  CNN_TRY(hipDeviceSynchronize());
  if (set_host) {
    CNN_TRY(hipMemcpy(net->params, set_host, (size_t)net->n_params * sizeof(float), hipMemcpyHostToDevice));
    CNN_TRY(hipMemset(net->m1, 0, (size_t)net->n_params * sizeof(float)));
    CNN_TRY(hipMemset(net->m2, 0, (size_t)net->n_params * sizeof(float)));
    net->adam_t = 0;
  }
  if (get_host)
    CNN_TRY(hipMemcpy(get_host, net->params, (size_t)net->n_params * sizeof(float), hipMemcpyDeviceToHost));
  return SFM_OK;
}

sfm_status sfm_cnn_forward(sfm_cnn net, const float* x_dev, int32_t batch, float* y_dev, void* stream) {
  if (!net) return SFM_EINVAL;
  net->err.clear();
  if (batch < 1 || batch > net->max_batch) return net->fail(SFM_EINVAL, "batch must lie in 1..max_batch");
  if (!x_dev) return net->fail(SFM_EINVAL, "x_dev is NULL");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const sfm_status rc = forward_pass(net, x_dev, batch, st);
  if (rc != SFM_OK) return rc;
  if (y_dev) {
    CNN_TRY(hipMemcpyAsync(y_dev, net->y, (size_t)batch * net->n_out * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (net->scaled) {
      hipLaunchKernelGGL(apply_scale_kernel, dim3(blocks_for((int64_t)batch * net->n_out)), dim3(256), 0, st, y_dev,
                         (int64_t)batch, (int64_t)net->n_out, net->out_mean, net->out_sd, -1);
      CNN_TRY(hipGetLastError());
    }
  }
  return SFM_OK;
}

sfm_status sfm_cnn_fit_scale(sfm_cnn net, const float* target_dev, int64_t n_samples, float* mean_host,
                             float* sd_host, void* stream) {
  if (!net) return SFM_EINVAL;
  net->err.clear();
  if (!target_dev || n_samples < 1) return net->fail(SFM_EINVAL, "need target_dev and n_samples >= 1");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(fit_scale_kernel, dim3(blocks_for(net->n_out)), dim3(256), 0, st, target_dev, n_samples,
                     (int64_t)net->n_out, net->out_mean, net->out_sd);
  CNN_TRY(hipGetLastError());
  net->scaled = true;
  if (mean_host || sd_host) {
    CNN_TRY(hipStreamSynchronize(st));
    if (mean_host) CNN_TRY(hipMemcpy(mean_host, net->out_mean, (size_t)net->n_out * sizeof(float), hipMemcpyDeviceToHost));
    if (sd_host) CNN_TRY(hipMemcpy(sd_host, net->out_sd, (size_t)net->n_out * sizeof(float), hipMemcpyDeviceToHost));
  }
  return SFM_OK;
}

sfm_status sfm_cnn_backward(sfm_cnn net, const float* dy_dev, float* grad_dev, void* stream) {
  if (!net) return SFM_EINVAL;
  net->err.clear();
  if (net->last_batch < 1) return net->fail(SFM_ESTATE, "call sfm_cnn_forward first");
  if (!dy_dev || !grad_dev) return net->fail(SFM_EINVAL, "dy_dev and grad_dev are required");
  return backward_pass(net, dy_dev, net->last_batch, grad_dev, nullptr, reinterpret_cast<hipStream_t>(stream));
}

sfm_status sfm_cnn_input_grad(sfm_cnn net, const float* dy_dev, float* dx_dev, void* stream) {
  if (!net) return SFM_EINVAL;
  net->err.clear();
  if (net->last_batch < 1) return net->fail(SFM_ESTATE, "call sfm_cnn_forward first");
  if (!dy_dev || !dx_dev) return net->fail(SFM_EINVAL, "dy_dev and dx_dev are required");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const float* dy = dy_dev;
  if (net->scaled) {             // y = mean + sd * (net output)
    const int64_t ny = (int64_t)net->last_batch * net->n_out;
    hipLaunchKernelGGL(scale_grad_kernel, dim3(blocks_for(ny)), dim3(256), 0, st, dy_dev, (int64_t)net->last_batch,
                       (int64_t)net->n_out, net->out_sd, net->dy);
    CNN_TRY(hipGetLastError());
    dy = net->dy;
  }
  return backward_pass(net, dy, net->last_batch, nullptr, dx_dev, st);
}

sfm_status sfm_cnn_train(sfm_cnn net, const float* x_dev, const float* target_dev, int64_t n_samples,
                         int32_t batch, int32_t epochs, float lr, uint64_t seed, double* loss_per_epoch, void* stream) {
  if (!net) return SFM_EINVAL;
  net->err.clear();
  if (!x_dev || !target_dev) return net->fail(SFM_EINVAL, "x_dev and target_dev are required");
  if (batch < 1 || batch > net->max_batch || n_samples < batch || epochs < 0)
    return net->fail(SFM_EINVAL, "need 1 <= batch <= max_batch, batch <= n_samples, epochs >= 0");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t nin3 = (int64_t)net->n_in * net->n_in * net->n_in;
  std::vector<int32_t> order((size_t)n_samples);
  for (int64_t i = 0; i < n_samples; ++i) order[(size_t)i] = (int32_t)i;
  std::mt19937_64 rng(seed);
  std::vector<double> lp(4096);
  for (int ep = 0; ep < epochs; ++ep) {
    std::shuffle(order.begin(), order.end(), rng);
    double loss_sum = 0.0;
    int64_t nb = 0;
    for (int64_t b0 = 0; b0 + batch <= n_samples; b0 += batch, ++nb) {
      CNN_TRY(hipMemcpyAsync(net->idx_d, order.data() + b0, (size_t)batch * sizeof(int32_t), hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for((int64_t)batch * nin3)), dim3(256), 0, st, x_dev,
                         net->idx_d, batch, nin3, net->xin);
      CNN_TRY(hipGetLastError());
      hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for((int64_t)batch * net->n_out)), dim3(256), 0, st,
                         target_dev, net->idx_d, batch, (int64_t)net->n_out, net->tgt);
      CNN_TRY(hipGetLastError());
      if (net->scaled) {
        hipLaunchKernelGGL(apply_scale_kernel, dim3(blocks_for((int64_t)batch * net->n_out)), dim3(256), 0, st,
                           net->tgt, (int64_t)batch, (int64_t)net->n_out, net->out_mean, net->out_sd, 1);
        CNN_TRY(hipGetLastError());
      }
      sfm_status rc = forward_pass(net, net->xin, batch, st);
      if (rc != SFM_OK) return rc;
      const int64_t ny = (int64_t)batch * net->n_out;
      const unsigned lb = blocks_for(ny);
      hipLaunchKernelGGL(mse_kernel, dim3(lb), dim3(256), 0, st, net->y, net->tgt, ny, net->dy, net->loss_part);
      CNN_TRY(hipGetLastError());
      rc = backward_pass(net, net->dy, batch, net->grads, nullptr, st);
      if (rc != SFM_OK) return rc;
      ++net->adam_t;
      const float c1 = 1.f - std::pow(0.9f, (float)net->adam_t), c2 = 1.f - std::pow(0.999f, (float)net->adam_t);
      hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(net->n_params)), dim3(256), 0, st, net->params, net->grads,
                         net->m1, net->m2, net->n_params, lr, 0.9f, 0.999f, 1e-8f, c1, c2);
      CNN_TRY(hipGetLastError());
      CNN_TRY(hipMemcpyAsync(lp.data(), net->loss_part, lb * sizeof(double), hipMemcpyDeviceToHost, st));
      CNN_TRY(hipStreamSynchronize(st));
      double s = 0.0;
      for (unsigned i = 0; i < lb; ++i) s += lp[i];
      loss_sum += s / (double)ny;
    }
    if (loss_per_epoch) loss_per_epoch[ep] = loss_sum / (double)std::max<int64_t>(1, nb);
  }
  return SFM_OK;
}

}  // extern "C"
