// Comparators on the same GPU (not part of the method's hot path):
//
//  * fine-grid FDTD: the reference fine grid the ROMs are built from (Introduction, eq. "wave";
//    the "traditional FDTD" of the Abstract), leapfrog M (u^{n+1} - 2u^n + u^{n-1}) / dt^2 = -K u^n + f,
//    which for the node-based 7-point operator is u^{n+1} = 2u^n - u^{n-1} + dt^2 c^2 Lap_h u^n with
//    mirrored ghost nodes on the outer boundary, plus dt^2 f c^2 / (w h^3) at a source node.
//  * plain per-subdomain ROM stepping: the same coupled leapfrog as sfm_step, but one launch per
//    subdomain per step reading full row-major p x p FP32 blocks with one thread per row (no
//    batching, no symmetric packing, no coalescing) -- the straightforward port of the scheme.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "sfm_internal.h"
#include "xcd.h"

namespace sfm {
namespace {

__global__ void fdtd_coef_kernel(const float* __restrict__ vel, int64_t n, float s, float* __restrict__ coef) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float c = vel[i];
    coef[i] = s * c * c;   // dt^2 c^2 / h^2
  }
}

// u_nm1 <- 2 u - u_nm1 + coef * Lap_h(u) (mirror closure); one thread per node, x fastest.
__global__ __launch_bounds__(256) void fdtd_step_kernel(const float* __restrict__ u, float* __restrict__ unm1,
                                                        const float* __restrict__ coef, int nx, int ny, int nz) {
  const int64_t sxy = (int64_t)nx * ny;
  const int64_t n = sxy * nz;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int i = (int)(idx % nx);
  const int64_t r = idx / nx;
  const int j = (int)(r % ny);
  const int l = (int)(r / ny);
  const float uc = u[idx];
  const float xm = u[i > 0 ? idx - 1 : idx + 1];
  const float xp = u[i < nx - 1 ? idx + 1 : idx - 1];
  const float ym = u[j > 0 ? idx - nx : idx + nx];
  const float yp = u[j < ny - 1 ? idx + nx : idx - nx];
  const float zm = u[l > 0 ? idx - sxy : idx + sxy];
  const float zp = u[l < nz - 1 ? idx + sxy : idx - sxy];
  const float lap = (xm + xp) + (ym + yp) + (zm + zp) - 6.f * uc;
  unm1[idx] = fmaf(coef[idx], lap, 2.f * uc - unm1[idx]);
}

// The same update, marching along z: a work-group owns a 64 x 4 tile of (x, y) columns and a
// chunk of kFdtdChunk planes; each thread keeps its column's u at planes l-1, l, l+1 in registers
// (each plane's operands loaded one plane ahead) and takes its x / y neighbours from plane l staged
// in LDS with a one-node ring of the neighbouring tiles' nodes; mirror ghosts on the outer faces are
// taken in the stencil itself.  Per node and step it reads u, u^{n-1} and the coefficient once
// (plus the ring and two planes per chunk) and writes u^{n+1}: 16 bytes.
constexpr int kFdtdTx = 64, kFdtdTy = 4, kFdtdChunk = 32;

__global__ __launch_bounds__(kFdtdTx * kFdtdTy) void fdtd_march_kernel(const float* __restrict__ u,
                                                                    float* __restrict__ unm1,
                                                                    const float* __restrict__ coef, int nx, int ny,
                                                                    int nz) {
  __shared__ float pl[2][kFdtdTy + 2][kFdtdTx + 2];
  const int tx = threadIdx.x % kFdtdTx, ty = threadIdx.x / kFdtdTx;
  // tiles in XCD-contiguous order, so the ring nodes a tile reads from its neighbours come
  // through the same L2
  int bx, by, bz;
  {
    const int64_t X = gridDim.x, Y = gridDim.y;
    const int64_t lb = xcd_contiguous_id(blockIdx.x + X * (blockIdx.y + Y * (int64_t)blockIdx.z), X * Y * gridDim.z);
    bx = (int)(lb % X);
    by = (int)((lb / X) % Y);
    bz = (int)(lb / (X * Y));
  }
  const int x0 = bx * kFdtdTx, y0 = by * kFdtdTy;
  const int x = x0 + tx, y = y0 + ty;
  const int l0 = bz * kFdtdChunk;
  const int l1 = min(nz, l0 + kFdtdChunk);
  const int64_t sxy = (int64_t)nx * ny;
  const bool act = x < nx && y < ny;
  const int64_t col = act ? (int64_t)y * nx + x : 0;
  // the ring: rows y0 - 1 and y0 + 4 (64 nodes each), columns x0 - 1 and x0 + 64 (4 nodes each),
  // where they exist in the grid
  const int t = threadIdx.x;
  int rx = -1, ry = -1, slot_r = 0, slot_c = 0;
  if (t < 2 * kFdtdTx) {
    const int side = t / kFdtdTx;
    slot_r = side ? kFdtdTy + 1 : 0;
    slot_c = t % kFdtdTx + 1;
    rx = x0 + t % kFdtdTx;
    ry = side ? y0 + kFdtdTy : y0 - 1;
  } else if (t < 2 * kFdtdTx + 2 * kFdtdTy) {
    const int q = t - 2 * kFdtdTx;
    const int side = q / kFdtdTy;
    slot_r = q % kFdtdTy + 1;
    slot_c = side ? kFdtdTx + 1 : 0;
    rx = side ? x0 + kFdtdTx : x0 - 1;
    ry = y0 + q % kFdtdTy;
  }
  const bool ring = rx >= 0 && rx < nx && ry >= 0 && ry < ny;
  const int64_t rcol = ring ? (int64_t)ry * nx + rx : 0;
  // plane above l with the mirror ghost at the last plane
  auto above = [&](int l) { return l + 1 < nz ? l + 1 : (nz > 1 ? l - 1 : l); };
  float um = 0.f, uc = 0.f, up = 0.f, vn = 0.f, cn = 0.f, rg = 0.f;
  if (act) {
    uc = u[l0 * sxy + col];
    um = u[(l0 > 0 ? l0 - 1 : above(l0)) * sxy + col];
    up = u[above(l0) * sxy + col];
    vn = unm1[l0 * sxy + col];
    cn = coef[l0 * sxy + col];
  }
  if (ring) rg = u[l0 * sxy + rcol];
  int b = 0;
  for (int l = l0; l < l1; ++l) {
    pl[b][ty + 1][tx + 1] = uc;
    if (ring) pl[b][slot_r][slot_c] = rg;
    const float vc = vn, cc = cn, uz = up;
    if (l + 1 < l1) {       // operands of the next plane
      if (act) {
        vn = unm1[(l + 1) * sxy + col];
        cn = coef[(l + 1) * sxy + col];
        up = u[above(l + 1) * sxy + col];
      }
      if (ring) rg = u[(l + 1) * sxy + rcol];
    }
    __syncthreads();
    if (act) {
      const float xm = pl[b][ty + 1][x > 0 ? tx : tx + 2];
      const float xp = pl[b][ty + 1][x < nx - 1 ? tx + 2 : tx];
      const float ym = pl[b][y > 0 ? ty : ty + 2][tx + 1];
      const float yp = pl[b][y < ny - 1 ? ty + 2 : ty][tx + 1];
      const float lap = (xm + xp) + (ym + yp) + (um + uz) - 6.f * uc;
      unm1[l * sxy + col] = fmaf(cc, lap, 2.f * uc - vc);
    }
    um = uc;
    uc = uz;
    b ^= 1;
  }
}

// Point sources (added after the stencil update of the same step) and receiver samples.
__global__ void fdtd_source_kernel(float* __restrict__ unext, const int64_t* __restrict__ node,
                                   const float* __restrict__ scale, const float* __restrict__ wavelet, int nsrc) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nsrc) unext[node[q]] += scale[q] * wavelet[q];
}

__global__ void fdtd_record_kernel(const float* __restrict__ u, const int64_t* __restrict__ node, int nrec,
                                   float* __restrict__ traces, int64_t ld, int64_t col) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nrec) traces[(int64_t)q * ld + col] = u[node[q]];
}

// One subdomain, one work-group of p threads: the coupled-ROM step with dense row-major blocks.
__global__ void plain_subdomain_kernel(const float* __restrict__ blocks, int k, int p, int P16, int s,
                                       float* __restrict__ U, float* __restrict__ D, float* __restrict__ exch,
                                       const int32_t* __restrict__ src_off, const int32_t* __restrict__ src_ids,
                                       const float* __restrict__ src_vec, const float* __restrict__ wavelet,
                                       int nsrc, int64_t step, float dt2) {
  extern __shared__ float sh[];
  float* x = sh;             // [k][p]
  float* ph = sh + k * p;    // [k][p]
  const int i = threadIdx.x;
  const float* Bs = blocks + (size_t)s * (2 * k - 1) * p * p;
  float* Us = U + (size_t)s * k * P16;
  float* Ds = D + (size_t)s * k * P16;
  for (int j = 0; j < k; ++j) x[j * p + i] = (j + 1 < k ? Us[(j + 1) * P16 + i] : 0.f) - Us[j * P16 + i];
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    const float* G = Bs + (size_t)j * p * p + (size_t)i * p;
    float acc = 0.f;
    for (int c = 0; c < p; ++c) acc = fmaf(G[c], x[j * p + c], acc);
    ph[j * p + i] = acc;
  }
  __syncthreads();
  exch[(size_t)s * P16 + i] = ph[i];
  for (int j = 1; j < k; ++j) x[j * p + i] = ph[j * p + i] - ph[(j - 1) * p + i];
  __syncthreads();
  const int s0 = src_off ? src_off[s] : 0, s1 = src_off ? src_off[s + 1] : 0;
  for (int j = 1; j < k; ++j) {
    const float* G = Bs + (size_t)(k + j - 1) * p * p + (size_t)i * p;
    float a = 0.f;
    for (int c = 0; c < p; ++c) a = fmaf(G[c], x[j * p + c], a);
    for (int q = s0; q < s1; ++q) {
      const int src = src_ids[q];
      a = fmaf(wavelet[step * nsrc + src], src_vec[((size_t)src * k + j) * P16 + i], a);
    }
    const float d = fmaf(dt2, a, Ds[j * P16 + i]);
    Ds[j * P16 + i] = d;
    Us[j * P16 + i] += d;
  }
}

// Full row-major FP32 blocks [S][2k-1][p][p] (Gamma_1..k, Gamma-hat_2..k) from the FP64 store.
__global__ void full_blocks_kernel(const double* __restrict__ coef64, int k, int p, int S, float* __restrict__ out) {
  const int64_t nb = 2 * k - 1;
  const int64_t pp = (int64_t)p * p;
  const int64_t total = (int64_t)S * nb * pp;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = q % pp;
    const int64_t sb = q / pp;
    const int64_t s = sb / nb;
    const int b = (int)(sb - s * nb);
    const int which = b < k ? 0 : 1;
    const int j = b < k ? b : b - k + 1;
    out[q] = (float)coef64[(((size_t)s * 2 + which) * k + j) * pp + e];
  }
}

}  // namespace
}  // namespace sfm

using namespace sfm;

#define C_TRY(call)                                                                         \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      err = std::string(#call) + ": " + hipGetErrorString(e_);                              \
      goto fail;                                                                            \
    }                                                                                       \
  } while (0)

namespace {
thread_local std::string g_fdtd_error;
}

extern "C" const char* sfm_fdtd_last_error(void) { return g_fdtd_error.c_str(); }

extern "C" sfm_status sfm_fdtd_run(const int32_t* ncell, double h, const float* vel_dev, double dt, int32_t nsteps,
                                   int32_t nsrc, const int32_t* src_ijk, const float* wavelet_dev, int32_t nrec,
                                   const int32_t* rec_ijk, float* traces_dev, int64_t ld, double* seconds,
                                   void* stream) {
  std::string err;
  g_fdtd_error.clear();
  if (!ncell || !vel_dev || !(h > 0) || !(dt > 0) || nsteps < 0 || nsrc < 0 || nrec < 0 ||
      (nsrc > 0 && (!src_ijk || !wavelet_dev)) || (nrec > 0 && (!rec_ijk || (traces_dev && ld < nsteps)))) {
    g_fdtd_error = "invalid argument";
    return SFM_EINVAL;
  }
  const int nx = ncell[0] + 1, ny = ncell[1] + 1, nz = ncell[2] + 1;
  if (ncell[0] < 1 || ncell[1] < 1 || ncell[2] < 1) {
    g_fdtd_error = "ncell must be positive";
    return SFM_EINVAL;
  }
  const int64_t n = (int64_t)nx * ny * nz;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<int64_t> sn(nsrc), rn(nrec);
  std::vector<float> sscale(nsrc);
  std::vector<float> vel_h(nsrc);
  float *u = nullptr, *v = nullptr, *coef = nullptr, *scale_d = nullptr;
  int64_t *sn_d = nullptr, *rn_d = nullptr;
  std::chrono::steady_clock::time_point t0;
  for (int q = 0; q < nsrc; ++q) {
    const int32_t* g = src_ijk + 3 * q;
    if (g[0] < 0 || g[0] >= nx || g[1] < 0 || g[1] >= ny || g[2] < 0 || g[2] >= nz) {
      g_fdtd_error = "source outside the grid";
      return SFM_EINVAL;
    }
    sn[q] = ((int64_t)g[2] * ny + g[1]) * nx + g[0];
  }
  for (int q = 0; q < nrec; ++q) {
    const int32_t* g = rec_ijk + 3 * q;
    if (g[0] < 0 || g[0] >= nx || g[1] < 0 || g[1] >= ny || g[2] < 0 || g[2] >= nz) {
      g_fdtd_error = "receiver outside the grid";
      return SFM_EINVAL;
    }
    rn[q] = ((int64_t)g[2] * ny + g[1]) * nx + g[0];
  }
  C_TRY(hipMalloc(&u, n * 4));
  C_TRY(hipMalloc(&v, n * 4));
  C_TRY(hipMalloc(&coef, n * 4));
  C_TRY(hipMalloc(&sn_d, std::max<size_t>(1, nsrc) * 8));
  C_TRY(hipMalloc(&rn_d, std::max<size_t>(1, nrec) * 8));
  C_TRY(hipMalloc(&scale_d, std::max<size_t>(1, nsrc) * 4));
  C_TRY(hipMemsetAsync(u, 0, n * 4, st));
  C_TRY(hipMemsetAsync(v, 0, n * 4, st));
  hipLaunchKernelGGL(fdtd_coef_kernel, dim3(4096), dim3(256), 0, st, vel_dev, n, (float)(dt * dt / (h * h)), coef);
  C_TRY(hipGetLastError());
  // source scale dt^2 c^2 / (w h^3) with the node's dual-volume weight w
  for (int q = 0; q < nsrc; ++q) C_TRY(hipMemcpy(&vel_h[q], vel_dev + sn[q], 4, hipMemcpyDeviceToHost));
  for (int q = 0; q < nsrc; ++q) {
    const int32_t* g = src_ijk + 3 * q;
    double w = 1.0;
    for (int d = 0; d < 3; ++d) {
      const int nn = d == 0 ? nx : d == 1 ? ny : nz;
      if (g[d] == 0 || g[d] == nn - 1) w *= 0.5;
    }
    sscale[q] = (float)(dt * dt * (double)vel_h[q] * vel_h[q] / (w * h * h * h));
  }
  if (nsrc) C_TRY(hipMemcpy(sn_d, sn.data(), nsrc * 8, hipMemcpyHostToDevice));
  if (nsrc) C_TRY(hipMemcpy(scale_d, sscale.data(), nsrc * 4, hipMemcpyHostToDevice));
  if (nrec) C_TRY(hipMemcpy(rn_d, rn.data(), nrec * 8, hipMemcpyHostToDevice));
  C_TRY(hipStreamSynchronize(st));
  SFM_DCHECK(nx >= 2 && ny >= 2 && nz >= 1 && (int64_t)nx * ny * nz == n);
  t0 = std::chrono::steady_clock::now();
  for (int32_t s = 0; s < nsteps; ++s) {
    hipLaunchKernelGGL(fdtd_march_kernel,
                       dim3((unsigned)((nx + kFdtdTx - 1) / kFdtdTx), (unsigned)((ny + kFdtdTy - 1) / kFdtdTy),
                            (unsigned)((nz + kFdtdChunk - 1) / kFdtdChunk)),
                       dim3(kFdtdTx * kFdtdTy), 0, st, u, v, coef, nx, ny, nz);
    if (nsrc)
      hipLaunchKernelGGL(fdtd_source_kernel, dim3((nsrc + 63) / 64), dim3(64), 0, st, v, sn_d, scale_d,
                         wavelet_dev + (int64_t)s * nsrc, nsrc);
    std::swap(u, v);   // u = u^{n+1}, v = u^n
    if (nrec && traces_dev)
      hipLaunchKernelGGL(fdtd_record_kernel, dim3((nrec + 255) / 256), dim3(256), 0, st, u, rn_d, nrec, traces_dev, ld,
                         (int64_t)s);
  }
  C_TRY(hipGetLastError());
  C_TRY(hipStreamSynchronize(st));
  if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  (void)hipFree(u); (void)hipFree(v); (void)hipFree(coef); (void)hipFree(sn_d); (void)hipFree(rn_d); (void)hipFree(scale_d);
  return SFM_OK;
fail:
  g_fdtd_error = err;
  (void)hipFree(u); (void)hipFree(v); (void)hipFree(coef); (void)hipFree(sn_d); (void)hipFree(rn_d); (void)hipFree(scale_d);
  return SFM_EHIP;
}

extern "C" sfm_status sfm_step_plain(sfm_ctx c, int32_t nsteps, double dt, const float* wavelet_dev, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!c->has_roms) return c->fail(SFM_ESTATE, "no ROMs");
  if (nsteps < 0 || !(dt > 0)) return c->fail(SFM_EINVAL, "bad nsteps or dt");
  if (c->nsrc > 0 && nsteps > 0 && !wavelet_dev) return c->fail(SFM_EINVAL, "wavelet_dev is required with sources");
  const Topology& t = c->topo;
  const int S = t.S, k = t.k, p = t.p, P16 = c->geo.P16;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return c->fail(SFM_EHIP, hipGetErrorString(e));
  if (!c->plain_blocks_d) {
    c->plain_blocks_d = static_cast<float*>(c->dalloc((size_t)S * (2 * k - 1) * p * p * sizeof(float), &e));
    if (!c->plain_blocks_d) return c->fail(SFM_ENOMEM, "plain blocks: out of device memory");
    hipLaunchKernelGGL(full_blocks_kernel, dim3(65536), dim3(256), 0, st, c->coef64_d, k, p, S, c->plain_blocks_d);
    if ((e = hipGetLastError()) != hipSuccess) return c->fail(SFM_EHIP, hipGetErrorString(e));
  }
  FaceParams f{};
  f.S = S; f.k = k; f.P16 = P16; f.p = p; f.m = t.m; f.nbr = c->nbr_d; f.C = c->C_d; f.exch = c->exch_d;
  f.U = c->U_d; f.D = c->D_d; f.mode = 0; f.dt2 = (float)(dt * dt); f.nsrc = c->nsrc; f.wavelet = wavelet_dev;
  if (c->nsrc > 0) { f.sw_off = c->sw_off_d; f.sw_q = c->sw_q_d; f.sw_src = c->sw_src_d; f.sw_w = c->sw_w_d; }
  const size_t lds = (size_t)2 * k * p * sizeof(float);
  for (int32_t i = 0; i < nsteps; ++i) {
    for (int s = 0; s < S; ++s) {
      hipLaunchKernelGGL(plain_subdomain_kernel, dim3(1), dim3(p), lds, st, c->plain_blocks_d, k, p, P16, s, c->U_d,
                         c->D_d, c->exch_d, c->nsrc ? c->src_off_d : nullptr, c->src_ids_d, c->src_vec_d,
                         wavelet_dev, c->nsrc, (int64_t)i, f.dt2);
    }
    f.step = i;
    if ((e = launch_step_face(f, st)) != hipSuccess) return c->fail(SFM_EHIP, hipGetErrorString(e));
  }
  if ((e = hipGetLastError()) != hipSuccess) return c->fail(SFM_EHIP, hipGetErrorString(e));
  c->n += nsteps;
  return SFM_OK;
}
