// Stage 1 of Algorithm 1 on the device: one ROM per subdomain, built in batches.
//
//  a1  operator and basis: A_+ = M^{-1/2} K M^{-1/2} of the subdomain box (node-based
//      7-point stencil with mirror closure on the box faces, shared interface nodes with
//      halved dual volumes) and F = M^{-1/2} E (m piecewise-constant patches per face;
//      each boundary node owned by one face, interface faces first).  Because the patch
//      functions do not overlap, F^T F = diag(H) and Q_1 = F diag(H)^{-1/2}, B_1 = diag(H^{1/2}).
//  a2  block Lanczos on (A_+, F) (polynomial Krylov space, the combined steps 1.1 + 1.2 of
//      Algorithm 1): W = A_+ Q_j, the three-term recurrence (W -= Q_j A_j + Q_{j-1} B_j^T),
//      one pass of classical Gram-Schmidt against all blocks so far (full
//      reorthogonalisation: after the recurrence only rounding drift is left, so this pass
//      is the second pass of a CGS2 for the two latest blocks; A_j gets its correction), then
//      two passes of Cholesky QR, W = Q_{j+1} B_{j+1} with B upper triangular, all in FP64.
//  a3  S-fraction (eq. "GammaTrans"), FP64, with G_1 = B_1^T and
//        Gamma-hat_j = G_j G_j^T,  Gamma_j = G_j^{-T} A_j G_j^{-1} - Gamma_{j-1},
//        G_{j+1} = -Gamma_j^{-1} G_j^{-T} B_{j+1}^T,  G_{j+1}^{-1} = -B_{j+1}^{-T} G_j^T Gamma_j
//      (the last identity keeps every inverse triangular or SPD: no pivoting).
//  a4  projections (eq. "Uj"): s = G Z^T M^{-1/2} e_s, r = e_r^T M^{-1/2} Z G^{-1}, and
//      U(0) = G Z^T M^{1/2} u0.
// The reductions run in FP64 on the device; the dense products (Z^T W, Z C, W^T W, the products
// with the inverse Cholesky factors and the p x p products of the S-fraction) run on the batched
// FP64 matrix-core kernel of dgemm.hip, the triangular inverses and solves on its compensated
// substitution kernels.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "sfm_internal.h"
#include "xcd.h"

namespace sfm {
namespace {

// Relative Gram pivot below which a Lanczos block counts as rank deficient: the independent
// part of a column is below ~3e-7 of its norm, where Cholesky QR can no longer orthogonalise it.
constexpr double kGramRelTol = 1e-13;
// Gamma_j (j < k) and Gamma-hat_j = G_j G_j^T (j >= 2) must be positive definite: a Cholesky pivot
// at or below 1e-13 of its diagonal entry is rounding-level in FP64, so such a level is reported as
// a breakdown rather than left to the sign of a rounding error.  Gamma-hat_j squares the
// conditioning of G_j, so a near-singular level falls to ~1e-16 whatever the rounding order.  The
// S-fraction levels of the workloads here keep every pivot above 1.6e-11 of its diagonal (the
// k = 32 polynomial ROMs of the many-shot workload; 2e-10 and up for finite shifts).
constexpr double kGammaRelTol = 1e-13;

struct BoxGeo {
  int sub[3];        // cells per edge
  int n[3];          // nodes per edge
  int m, m1, m2, p;
  double h;
};

__device__ __forceinline__ void local_ijk(const BoxGeo& g, int64_t node, int& i, int& j, int& l) {
  i = (int)(node % g.n[0]);
  const int64_t r = node / g.n[0];
  j = (int)(r % g.n[1]);
  l = (int)(r / g.n[1]);
}

__device__ __forceinline__ double half_if(bool on) { return on ? 0.5 : 1.0; }

// Owner face of a boundary node (-1 for interior nodes): among the faces whose plane holds
// the node, the first interface face in the order x-, x+, y-, y+, z-, z+, else the first outer one.
__device__ __forceinline__ int owner_face(const BoxGeo& g, int i, int j, int l, int nbmask) {
  const bool on[6] = {i == 0, i == g.sub[0], j == 0, j == g.sub[1], l == 0, l == g.sub[2]};
  for (int f = 0; f < 6; ++f)
    if (on[f] && ((nbmask >> f) & 1)) return f;
  for (int f = 0; f < 6; ++f)
    if (on[f]) return f;
  return -1;
}

// Patch index of a node on face f: strips min(floor(a m1 / n1), m1-1) x min(floor(b m2 / n2), m2-1)
// over the tangential axes in increasing order.
__device__ __forceinline__ int patch_of(const BoxGeo& g, int f, const int c[3]) {
  const int d = f >> 1;
  const int t1 = d == 0 ? 1 : 0;
  const int t2 = d == 2 ? 1 : 2;
  const int q1 = min(c[t1] * g.m1 / g.sub[t1], g.m1 - 1);
  const int q2 = min(c[t2] * g.m2 / g.sub[t2], g.m2 - 1);
  return q1 * g.m2 + q2;
}

// Dual face area of a boundary node inside its owner face: h^2 halved per tangential box plane.
__device__ __forceinline__ double patch_weight(const BoxGeo& g, int f, const int c[3]) {
  const int d = f >> 1;
  double w = g.h * g.h;
  for (int t = 0; t < 3; ++t)
    if (t != d) w *= half_if(c[t] == 0 || c[t] == g.sub[t]);
  return w;
}

// S = M^{-1/2} = c / sqrt(w h^3) at every node of every subdomain of the batch.
__global__ void node_scale_kernel(BoxGeo g, const float* __restrict__ vel, int ncx, int ncy, const int32_t* __restrict__ org,
                                  int64_t N, int nb, double* __restrict__ S, int* __restrict__ bad) {
  const int64_t total = (int64_t)nb * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx / N);
    const int64_t n = idx - (int64_t)b * N;
    int i, j, l;
    local_ijk(g, n, i, j, l);
    const int gi = org[3 * b] + i, gj = org[3 * b + 1] + j, gl = org[3 * b + 2] + l;
    const double c = vel[((int64_t)gl * (ncy + 1) + gj) * (ncx + 1) + gi];
    if (!(c > 0.0) || !isfinite(c)) *bad = 1;
    const double w = half_if(i == 0 || i == g.sub[0]) * half_if(j == 0 || j == g.sub[1]) *
                     half_if(l == 0 || l == g.sub[2]);
    S[idx] = c / sqrt(w * g.h * g.h * g.h);
  }
}

// H[b][col] = sum over the patch's owned nodes of (E S)^2 = (F^T F)_{col,col}.
__global__ void face_mass_kernel(BoxGeo g, const double* __restrict__ S, const int32_t* __restrict__ nbmask, int64_t N,
                                 int nb, double* __restrict__ H) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nb * g.p) return;
  const int b = idx / g.p, col = idx - b * g.p;
  const int f = col / g.m, q = col - f * g.m;
  const int d = f >> 1;
  const int t1 = d == 0 ? 1 : 0;
  const int t2 = d == 2 ? 1 : 2;
  double acc = 0.0;
  for (int a = 0; a <= g.sub[t1]; ++a) {
    if (min(a * g.m1 / g.sub[t1], g.m1 - 1) != q / g.m2) continue;
    for (int bb = 0; bb <= g.sub[t2]; ++bb) {
      if (min(bb * g.m2 / g.sub[t2], g.m2 - 1) != q % g.m2) continue;
      int c[3];
      c[d] = (f & 1) ? g.sub[d] : 0;
      c[t1] = a;
      c[t2] = bb;
      if (owner_face(g, c[0], c[1], c[2], nbmask[b]) != f) continue;
      const int64_t n = ((int64_t)c[2] * g.n[1] + c[1]) * g.n[0] + c[0];
      const double e = patch_weight(g, f, c) * S[(int64_t)b * N + n];
      acc += e * e;
    }
  }
  H[idx] = acc;
}

// Q_1 = F diag(H)^{-1/2} into columns 0..p-1 of Z (node-major, ld = kp).
__global__ void init_q1_kernel(BoxGeo g, const double* __restrict__ S, const int32_t* __restrict__ nbmask,
                               const double* __restrict__ H, int64_t N, int kp, int nb, double* __restrict__ Z) {
  const int64_t total = (int64_t)nb * N * g.p;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(idx % g.p);
    const int64_t bn = idx / g.p;
    const int b = (int)(bn / N);
    const int64_t n = bn - (int64_t)b * N;
    int c[3];
    local_ijk(g, n, c[0], c[1], c[2]);
    double v = 0.0;
    const int f = owner_face(g, c[0], c[1], c[2], nbmask[b]);
    if (f >= 0 && col == f * g.m + patch_of(g, f, c))
      v = patch_weight(g, f, c) * S[(int64_t)b * N + n] / sqrt(H[(int64_t)b * g.p + col]);
    Z[((int64_t)b * N + n) * kp + col] = v;
  }
}

// W = (A_+ + shift I) X = S K S X + shift X for the p columns of X (ld ldx) into W (ld ldw).
// K is the geometric stiffness: coefficient h per edge, halved for every box plane holding the edge.
// One thread per (subdomain, node column (i, j), column of X) marches along z with the scale and
// value of the planes l - 1, l, l + 1 in registers, so a z-neighbour (a whole plane of rows away)
// is loaded once; the x- and y-neighbours lie in the plane the neighbouring threads load (on the
// same XCD, through xcd_contiguous_id).  Every term is formed as y_n - S_nb X_nb with
// y_n = S_n X_n, in the order x-, x+, y-, y+, z-, z+.
__global__ void stencil_kernel(BoxGeo g, const double* __restrict__ S, int64_t N, int nb, const double* __restrict__ X,
                               int ldx, int64_t sx, double* __restrict__ W, int ldw, int64_t sw, double shift) {
  const int nx = g.n[0], nz = g.n[2];
  const int64_t plane = (int64_t)nx * g.n[1];
  const int64_t total = (int64_t)nb * plane * g.p;
  const int64_t lb = xcd_contiguous_id(blockIdx.x, gridDim.x);
  for (int64_t idx = lb * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(idx % g.p);
    const int64_t bq = idx / g.p;
    const int b = (int)(bq / plane);
    const int64_t q = bq - (int64_t)b * plane;
    const int i = (int)(q % nx), j = (int)(q / nx);
    const double* Sb = S + (int64_t)b * N;
    const double* Xb = X + (int64_t)b * sx + col;
    double* Wb = W + (int64_t)b * sw + col;
    const double wi = half_if(i == 0 || i == g.sub[0]);
    const double wj = half_if(j == 0 || j == g.sub[1]);
    const double cz = g.h * wi * wj;     // z-edges lie in the planes normal to x and y that hold them
    int64_t n = q;
    double sm = 0.0, xm = 0.0;                               // plane l - 1
    double sn = Sb[n], xn = Xb[n * ldx];                     // plane l
    double sp = Sb[n + plane], xp = Xb[(n + plane) * ldx];   // plane l + 1 (nz >= 2)
    for (int l = 0; l < nz; ++l) {
      const double wl = half_if(l == 0 || l == g.sub[2]);
      const double cx = g.h * wj * wl, cy = g.h * wi * wl;
      const double yn = sn * xn;
      double acc = 0.0;
      if (i > 0) acc += cx * (yn - Sb[n - 1] * Xb[(n - 1) * ldx]);
      if (i < g.sub[0]) acc += cx * (yn - Sb[n + 1] * Xb[(n + 1) * ldx]);
      if (j > 0) acc += cy * (yn - Sb[n - nx] * Xb[(n - nx) * ldx]);
      if (j < g.sub[1]) acc += cy * (yn - Sb[n + nx] * Xb[(n + nx) * ldx]);
      if (l > 0) acc += cz * (yn - sm * xm);
      if (l < g.sub[2]) acc += cz * (yn - sp * xp);
      Wb[n * ldw] = sn * acc + shift * xn;
      sm = sn;
      xm = xn;
      sn = sp;
      xn = xp;
      n += plane;
      if (l + 2 < nz) {
        sp = Sb[n + plane];
        xp = Xb[(n + plane) * ldx];
      }
    }
  }
}

// Jacobi preconditioner of A_+ + sigma I: dinv = 1 / (S_n^2 sum of the node's edge coefficients + sigma).
__global__ void shifted_diag_kernel(BoxGeo g, const double* __restrict__ S, int64_t N, int nb, double sigma,
                                    double* __restrict__ dinv) {
  const int64_t total = (int64_t)nb * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = idx % N;
    int i, j, l;
    local_ijk(g, n, i, j, l);
    const double wi = half_if(i == 0 || i == g.sub[0]);
    const double wj = half_if(j == 0 || j == g.sub[1]);
    const double wl = half_if(l == 0 || l == g.sub[2]);
    const int nx = (i > 0) + (i < g.sub[0]), ny = (j > 0) + (j < g.sub[1]), nz = (l > 0) + (l < g.sub[2]);
    const double ksum = g.h * (nx * wj * wl + ny * wi * wl + nz * wi * wj);
    const double sn = S[idx];
    dinv[idx] = 1.0 / (sn * sn * ksum + sigma);
  }
}

// ---------------------------------------------------------------- batched Jacobi PCG
// Solves (A_+ + sigma I) X = B for the p columns of every subdomain of a batch, one CG
// recurrence per column.  Vectors R, P, Q are node-major [b][N][p]; X and B may be column
// blocks of a wider node-major array (ld, stride).  Column sums over the N nodes are taken in
// two stages: a chunk kernel writes partial sums part[.][b][chunk][col] (block (chunk, b);
// thread t handles column t % p of every (256 / p)-th row of the chunk), then a per-column
// kernel adds the chunks in order, so every sum is reproducible.  A column stops (alpha = 0)
// once |r| <= rtol |b|; it is never updated again.
struct CgVec {
  int64_t N;
  int p, nchunk, nb;
};

__device__ __forceinline__ void chunk_range(const CgVec& v, int chunk, int64_t& n0, int64_t& n1) {
  const int64_t rows = (v.N + v.nchunk - 1) / v.nchunk;
  n0 = (int64_t)chunk * rows;
  n1 = min(v.N, n0 + rows);
}

// Sums s[0..NS) of each column over the rows of this block into part[q][b][chunk][col].
template <int NS>
__device__ __forceinline__ void chunk_col_sums(const CgVec& v, const double (&sv)[NS], double* __restrict__ part) {
  __shared__ double red[NS][256];
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NS; ++q) red[q][t] = sv[q];
  __syncthreads();
  const int rpp = 256 / v.p;
  if (t < v.p) {
    const int64_t slot = ((int64_t)blockIdx.y * v.nchunk + blockIdx.x) * v.p + t;
    const int64_t plane = (int64_t)v.nb * v.nchunk * v.p;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      double acc = 0.0;
      for (int r = 0; r < rpp; ++r) acc += red[q][r * v.p + t];
      part[q * plane + slot] = acc;
    }
  }
}

// x = 0, r = b, p = D^{-1} r; partial sums of r.z and r.r.
__global__ __launch_bounds__(256) void cg_init_kernel(CgVec v, const double* __restrict__ B, int ldb, int64_t sb,
                                                      const double* __restrict__ dinv, double* __restrict__ X, int ldx,
                                                      int64_t sx, double* __restrict__ R, double* __restrict__ P,
                                                      double* __restrict__ part) {
  const int b = blockIdx.y, t = threadIdx.x;
  const int rpp = 256 / v.p, col = t % v.p, r0 = t / v.p;
  int64_t n0, n1;
  chunk_range(v, blockIdx.x, n0, n1);
  double sv[2] = {0.0, 0.0};
  if (r0 < rpp) {
    for (int64_t n = n0 + r0; n < n1; n += rpp) {
      const double bv = B[(int64_t)b * sb + n * ldb + col];
      const double z = dinv[(int64_t)b * v.N + n] * bv;
      const int64_t e = ((int64_t)b * v.N + n) * v.p + col;
      X[(int64_t)b * sx + n * ldx + col] = 0.0;
      R[e] = bv;
      P[e] = z;
      sv[0] += bv * z;
      sv[1] += bv * bv;
    }
  }
  chunk_col_sums<2>(v, sv, part);
}

// partial sums of p.q
__global__ __launch_bounds__(256) void cg_dot_kernel(CgVec v, const double* __restrict__ P, const double* __restrict__ Q,
                                                     double* __restrict__ part) {
  const int b = blockIdx.y, t = threadIdx.x;
  const int rpp = 256 / v.p, col = t % v.p, r0 = t / v.p;
  int64_t n0, n1;
  chunk_range(v, blockIdx.x, n0, n1);
  double sv[1] = {0.0};
  if (r0 < rpp) {
    for (int64_t n = n0 + r0; n < n1; n += rpp) {
      const int64_t e = ((int64_t)b * v.N + n) * v.p + col;
      sv[0] += P[e] * Q[e];
    }
  }
  chunk_col_sums<1>(v, sv, part);
}

// x += alpha p, r -= alpha q; partial sums of r.z (z = D^{-1} r) and r.r.
__global__ __launch_bounds__(256) void cg_update_kernel(CgVec v, const double* __restrict__ alpha,
                                                        const double* __restrict__ dinv, const double* __restrict__ P,
                                                        const double* __restrict__ Q, double* __restrict__ X, int ldx,
                                                        int64_t sx, double* __restrict__ R, double* __restrict__ part) {
  const int b = blockIdx.y, t = threadIdx.x;
  const int rpp = 256 / v.p, col = t % v.p, r0 = t / v.p;
  int64_t n0, n1;
  chunk_range(v, blockIdx.x, n0, n1);
  double sv[2] = {0.0, 0.0};
  if (r0 < rpp) {
    const double a = alpha[(int64_t)b * v.p + col];
    for (int64_t n = n0 + r0; n < n1; n += rpp) {
      const int64_t e = ((int64_t)b * v.N + n) * v.p + col;
      double* x = X + (int64_t)b * sx + n * ldx + col;
      *x = fma(a, P[e], *x);
      const double r = fma(-a, Q[e], R[e]);
      R[e] = r;
      sv[0] += r * dinv[(int64_t)b * v.N + n] * r;
      sv[1] += r * r;
    }
  }
  chunk_col_sums<2>(v, sv, part);
}

// Per-column scalars sc = [rz][bb][alpha][beta] ([4][nb * p]) and active flags.
__device__ __forceinline__ double sum_chunks(const CgVec& v, const double* part, int q, int b, int col) {
  const int64_t plane = (int64_t)v.nb * v.nchunk * v.p;
  const double* pp = part + q * plane + (int64_t)b * v.nchunk * v.p + col;
  double acc = 0.0;
  for (int ch = 0; ch < v.nchunk; ++ch) acc += pp[(int64_t)ch * v.p];
  return acc;
}

__global__ void cg_start_kernel(CgVec v, const double* __restrict__ part, double* __restrict__ sc, int* __restrict__ active) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = v.nb * v.p;
  if (idx >= n) return;
  const int b = idx / v.p, col = idx - b * v.p;
  const double rz = sum_chunks(v, part, 0, b, col);
  const double bb = sum_chunks(v, part, 1, b, col);
  sc[idx] = rz;
  sc[n + idx] = bb;
  sc[2 * n + idx] = 0.0;
  sc[3 * n + idx] = 0.0;
  active[idx] = bb > 0.0 ? 1 : 0;
}

__global__ void cg_alpha_kernel(CgVec v, const double* __restrict__ part, double* __restrict__ sc,
                                const int* __restrict__ active) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = v.nb * v.p;
  if (idx >= n) return;
  const int b = idx / v.p, col = idx - b * v.p;
  const double pq = sum_chunks(v, part, 0, b, col);
  sc[2 * n + idx] = (active[idx] && pq > 0.0) ? sc[idx] / pq : 0.0;
}

__global__ void cg_beta_kernel(CgVec v, const double* __restrict__ part, double* __restrict__ sc, int* __restrict__ active,
                               double rtol2) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = v.nb * v.p;
  if (idx >= n) return;
  const int b = idx / v.p, col = idx - b * v.p;
  double beta = 0.0;
  if (active[idx]) {
    const double rzn = sum_chunks(v, part, 0, b, col);
    const double rr = sum_chunks(v, part, 1, b, col);
    const double rz = sc[idx];
    beta = rz > 0.0 ? rzn / rz : 0.0;
    sc[idx] = rzn;
    if (rr <= rtol2 * sc[n + idx]) active[idx] = 0;
  }
  sc[3 * n + idx] = beta;
}

// p = D^{-1} r + beta p
__global__ void cg_dir_kernel(CgVec v, const double* __restrict__ dinv, const double* __restrict__ R,
                              const double* __restrict__ beta, double* __restrict__ P) {
  const int64_t total = (int64_t)v.nb * v.N * v.p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(e % v.p);
    const int64_t bn = e / v.p;
    const int b = (int)(bn / v.N);
    P[e] = fma(dinv[bn], R[e], beta[(int64_t)b * v.p + col] * P[e]);
  }
}

// count[0] = number of active columns (one work-group)
__global__ __launch_bounds__(256) void count_active_kernel(const int* __restrict__ active, int n, int* __restrict__ count) {
  __shared__ int red[256];
  int acc = 0;
  for (int i = threadIdx.x; i < n; i += 256) acc += active[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) count[0] = red[0];
}

// First block of the reduced-space Lanczos basis: columns 0..p-1 of the identity (rows kp, ld kp).
__global__ void eye_block_kernel(int kp, int p, int nb, double* __restrict__ Z, int64_t sz) {
  const int64_t total = (int64_t)nb * kp * p;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(idx % p);
    const int64_t bn = idx / p;
    const int b = (int)(bn / kp);
    const int n = (int)(bn - (int64_t)b * kp);
    Z[(int64_t)b * sz + (int64_t)n * kp + col] = n == col ? 1.0 : 0.0;
  }
}

// Cholesky A = L L^T in place (column-major p x p, lower), one work-group per matrix.
// A pivot d_c marks a breakdown of matrix b when d_c <= max(thr[b], rel * A_cc) with A_cc the
// diagonal before factorisation.  For a Gram matrix W^T W the relative test catches a column
// whose component independent of the previous ones has fallen to rounding level (forming the
// Gram squares the condition number, so such a pivot is noise of size eps * A_cc, not ~0).
__global__ __launch_bounds__(256) void cholesky_kernel(double* __restrict__ A, int p, int64_t stride,
                                                       const double* __restrict__ thr, double rel,
                                                       int* __restrict__ flag) {
  double* a = A + (int64_t)blockIdx.x * stride;
  __shared__ int bad;
  __shared__ double diag0[kTile * kMaxNt];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4, nty = blockDim.x >> 4;   // 16-lane column groups
  const double tb = thr ? thr[blockIdx.x] : 0.0;
  if (tid == 0) bad = 0;
  for (int c = tid; c < p; c += blockDim.x) diag0[c] = a[c + (int64_t)c * p];
  for (int c = 0; c < p; ++c) {
    __syncthreads();                     // column c is final
    double d = a[c + (int64_t)c * p];    // every thread forms the pivot
    const bool ok = d > fmax(tb, rel * diag0[c]);
    if (!ok) d = 1.0;
    const double piv = sqrt(d);
    const double inv = 1.0 / piv;
    for (int i = c + 1 + tid; i < p; i += blockDim.x) a[i + (int64_t)c * p] *= inv;
    __syncthreads();                     // the scaled column is visible, every thread has read a_cc
    if (tid == 0) {
      a[c + (int64_t)c * p] = piv;
      if (!ok) bad = 1;
    }
    const int nr = p - c - 1;
    const double* col = a + (int64_t)c * p + c + 1;
    for (int jj = ty; jj < nr; jj += nty) {
      const double lj = col[jj];
      double* dst = a + (c + 1) + (int64_t)(c + 1 + jj) * p;
      for (int ii = jj + tx; ii < nr; ii += 16) dst[ii] -= col[ii] * lj;
    }
  }
  __syncthreads();
  for (int e = tid; e < p * p; e += blockDim.x) {
    const int i = e % p, j = e / p;
    if (i < j) a[e] = 0.0;
  }
  if (tid == 0 && bad) flag[blockIdx.x] = 1;
}

// Strict upper triangle of column-major p x p blocks set to zero.
__global__ void zero_upper_kernel(double* __restrict__ A, int p, int64_t stride, int nb) {
  const int64_t total = (int64_t)nb * p * p;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx / ((int64_t)p * p));
    const int e = (int)(idx - (int64_t)b * p * p);
    if (e % p < e / p) A[b * stride + e] = 0.0;
  }
}

// out_j = sym(C1 block j + C2 block j) (projection coefficients of W on Q_j) -> A_j.
__global__ void accum_a_kernel(const double* __restrict__ C1, const double* __restrict__ C2, int p, int64_t sc,
                               int off, double* __restrict__ A, int64_t sa, int nb) {
  const int64_t total = (int64_t)nb * p * p;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx / ((int64_t)p * p));
    const int e = (int)(idx - (int64_t)b * p * p);
    const int r = e % p, c = e / p;
    const double* c1 = C1 + b * sc + (int64_t)off * p;
    const double* c2 = C2 ? C2 + b * sc + (int64_t)off * p : nullptr;
    double v = c1[r + c * p] + c1[c + r * p];
    if (c2) v += c2[r + c * p] + c2[c + r * p];
    A[b * sa + e] = 0.5 * v;
  }
}

__global__ void symmetrize_kernel(double* __restrict__ A, int p, int64_t stride, int nb) {
  const int64_t total = (int64_t)nb * p * p;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx / ((int64_t)p * p));
    const int e = (int)(idx - (int64_t)b * p * p);
    const int r = e % p, c = e / p;
    if (r < c) {
      double* a = A + b * stride;
      const double v = 0.5 * (a[r + c * p] + a[c + r * p]);
      a[r + c * p] = v;
      a[c + r * p] = v;
    }
  }
}

// diag(v) or diag(1/v) (column-major p x p) from H: G_1 = B_1^T = diag(H^{1/2}), G_1^{-1}, and B_1^T.
__global__ void diag_kernel(const double* __restrict__ H, int p, int nb, double* __restrict__ D, int64_t sd, int mode) {
  const int64_t total = (int64_t)nb * p * p;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx / ((int64_t)p * p));
    const int e = (int)(idx - (int64_t)b * p * p);
    const int r = e % p, c = e / p;
    double v = 0.0;
    if (r == c) {
      const double s = sqrt(H[(int64_t)b * p + r]);
      v = mode == 0 ? s : 1.0 / s;
    }
    D[b * sd + e] = v;
  }
}

__global__ void copy_blocks_kernel(const double* __restrict__ src, int64_t ss, double* __restrict__ dst, int64_t sd,
                                   int64_t n, int nb, double scale) {
  const int64_t total = (int64_t)nb * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx / n);
    const int64_t e = idx - (int64_t)b * n;
    dst[b * sd + e] = scale * src[b * ss + e];
  }
}

// dst[ids[b] * sd + e] = src[b * ss + e], e < n: batch results to their subdomains' slots.
__global__ void scatter_blocks_kernel(const double* __restrict__ src, int64_t ss, double* __restrict__ dst, int64_t sd,
                                      int64_t n, int nb, const int32_t* __restrict__ ids) {
  const int64_t total = (int64_t)nb * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx / n);
    const int64_t e = idx - (int64_t)b * n;
    dst[(int64_t)ids[b] * sd + e] = src[b * ss + e];
  }
}

// Source vectors s_j = G_j z_j and receiver rows r_j = z_j^T G_j^{-1} with z = M^{-1/2} Z^T e_node.
__global__ void project_points_kernel(const double* __restrict__ Z, const double* __restrict__ S, int64_t N, int k, int kb,
                                      int p, const double* __restrict__ G, const double* __restrict__ Gi, int64_t sg,
                                      const int32_t* __restrict__ pb, const int32_t* __restrict__ pnode,
                                      const int32_t* __restrict__ pid, int npts, int mode, double* __restrict__ out) {
  const int64_t total = (int64_t)npts * k * p;
  const int kp = k * p;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(idx % p);
    const int64_t pj = idx / p;
    const int j = (int)(pj % k);
    const int pt = (int)(pj / k);
    if (j >= kb) {                      // a level past this batch's ROM size
      out[((int64_t)pid[pt] * k + j) * p + e] = 0.0;
      continue;
    }
    const int b = pb[pt];
    const int64_t n = pnode[pt];
    const double sn = S[(int64_t)b * N + n];
    const double* z = Z + ((int64_t)b * N + n) * kp + (int64_t)j * p;
    const double* M = (mode == 0 ? G : Gi) + b * sg + (int64_t)j * p * p;
    double acc = 0.0;
    if (mode == 0) {
      for (int c = 0; c < p; ++c) acc += M[e + (int64_t)c * p] * z[c];       // (G_j z_j)[e]
    } else {
      for (int r = 0; r < p; ++r) acc += z[r] * M[r + (int64_t)e * p];       // (z_j^T G_j^{-1})[e]
    }
    out[((int64_t)pid[pt] * k + j) * p + e] = sn * acc;
  }
}

// y[b][col] = sum_n Z[b][n][col] u(n) / S_n for col < kp (Z^T M^{1/2} u).
__global__ void project_field_kernel(BoxGeo g, const double* __restrict__ Z, const double* __restrict__ S, int64_t N,
                                     int kp, int nb, const float* __restrict__ u, int ncx, int ncy,
                                     const int32_t* __restrict__ org, double* __restrict__ y) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nb * kp) return;
  const int b = idx / kp, col = idx - b * kp;
  double acc = 0.0;
  for (int64_t n = 0; n < N; ++n) {
    int i, j, l;
    local_ijk(g, n, i, j, l);
    const int gi = org[3 * b] + i, gj = org[3 * b + 1] + j, gl = org[3 * b + 2] + l;
    const double un = u[((int64_t)gl * (ncy + 1) + gj) * (ncx + 1) + gi];
    acc += Z[((int64_t)b * N + n) * kp + col] * un / S[(int64_t)b * N + n];
  }
  y[idx] = acc;
}

// U_j = G_j y_j into the FP32 state layout [S][k][P16].
__global__ void apply_g_kernel(const double* __restrict__ y, const double* __restrict__ G, int64_t sg, int k, int kb,
                               int p, int P16, int nb, const int32_t* __restrict__ ids, float* __restrict__ U) {
  const int64_t total = (int64_t)nb * k * p;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(idx % p);
    const int64_t bj = idx / p;
    const int j = (int)(bj % k);
    const int b = (int)(bj / k);
    double acc = 0.0;
    if (j < kb) {                       // levels past this batch's ROM size stay zero
      const double* M = G + b * sg + (int64_t)j * p * p;
      const double* yj = y + (int64_t)b * k * p + (int64_t)j * p;
      for (int c = 0; c < p; ++c) acc += M[e + (int64_t)c * p] * yj[c];
    }
    U[(((int64_t)ids[b]) * k + j) * P16 + e] = (float)acc;
  }
}

// Boundary-layer entries shared with a lower-index neighbour take that neighbour's value.
__global__ void unify_ports_kernel(const int32_t* __restrict__ nbr, int S, int k, int p, int m, int P16,
                                   float* __restrict__ U) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)S * p) return;
  const int s = (int)(idx / p), q = (int)(idx - (int64_t)s * p);
  const int f = q / m, pat = q - f * m;
  const int nb = nbr[s * 6 + f];
  if (nb >= 0 && nb < s) U[(int64_t)s * k * P16 + q] = U[(int64_t)nb * k * P16 + (f ^ 1) * m + pat];
}

// A_b = [B_j | C2_j] (p x 2p, column-major, ld p): B_j from its stored transpose (column-major
// B_j^T at Bt), then the recurrence's projection C2_j, so that W -= Q_{j-1} B_j^T + Q_j A_j is one
// product with the adjacent basis blocks [Q_{j-1} Q_j].
__global__ void recurrence_coef_kernel(const double* __restrict__ Bt, int64_t sBt, const double* __restrict__ C2,
                                       int64_t sC2, int p, int nb, double* __restrict__ Af) {
  const int64_t per = 2 * (int64_t)p * p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < per * nb; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / per, q = e - b * per;
    const int c = (int)(q / p), r = (int)(q - (int64_t)c * p);
    Af[e] = c < p ? Bt[b * sBt + c + (int64_t)r * p] : C2[b * sC2 + r + (int64_t)(c - p) * p];
  }
}

unsigned grid_for(int64_t n, int threads = 256) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + threads - 1) / threads, 1 << 20));
}

}  // namespace

}  // namespace sfm

using namespace sfm;

#define B_TRY_HIP(call)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return c->fail(SFM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define B_LAUNCH(kernel, n, ...)                                                              \
  do {                                                                                        \
    hipLaunchKernelGGL(kernel, dim3(grid_for(n)), dim3(256), 0, st, __VA_ARGS__);             \
    B_TRY_HIP(hipGetLastError());                                                             \
  } while (0)

namespace {

// Device scratch of one build, released on every return path.
struct Scratch {
  sfm_ctx c;
  hipError_t e = hipSuccess;
  std::vector<void*> ptrs;
  explicit Scratch(sfm_ctx ctx) : c(ctx) {}
  ~Scratch() {
    for (void* ptr : ptrs) c->dfree(ptr);
  }
  template <typename T = double>
  T* get(size_t count) {
    void* ptr = c->dalloc(count * sizeof(T), &e);
    if (ptr) ptrs.push_back(ptr);
    return static_cast<T*>(ptr);
  }
};

// Shift and inner-solver settings of one build; sigma = +inf selects the polynomial space.
struct ShiftSpec {
  double sigma;
  double rtol;
  int max_iter;
};

constexpr int kCgCheck = 10;   // CG iterations between convergence checks on the host

// levels: optional [S] ROM size per subdomain (block Lanczos and the S-fraction run levels[s]
// steps there; the blocks and projections of later levels are zero).  sigma = inf only.
sfm_status build_roms(sfm_ctx c, const ShiftSpec& shift, const float* vel_dev, int32_t nsrc, const int32_t* src_ijk,
                      int32_t nrec, const int32_t* rec_ijk, const float* u0_dev, const float* v0_dev,
                      int32_t* cg_iters_out, void* stream, const int32_t* levels = nullptr) {
  c->err.clear();
  if (!vel_dev) return c->fail(SFM_EINVAL, "vel_dev is NULL");
  const bool finite = std::isfinite(shift.sigma);
  const auto t_start = std::chrono::steady_clock::now();
  B_TRY_HIP(hipSetDevice(c->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const Topology& t = c->topo;
  const int S = t.S, k = t.k, p = t.p, kp = k * p, P16 = c->geo.P16;
  const int64_t Nmax = t.N_max;
  const int64_t pp = (int64_t)p * p;
  const int64_t kpkp = (int64_t)kp * kp;
  std::vector<int32_t> src_sub, src_local, rec_sub, rec_local;
  sfm_status rc = locate_points(c, nsrc, src_ijk, nrec, rec_ijk, src_sub, src_local, rec_sub, rec_local);
  if (rc != SFM_OK) return rc;

  release_roms(c);
  hipError_t e = hipSuccess;
  c->coef64_d = static_cast<double*>(c->dalloc((size_t)S * 2 * k * pp * sizeof(double), &e));
  if (!c->coef64_d) return c->fail(SFM_ENOMEM, "FP64 coefficients: out of device memory");
  if (levels) B_TRY_HIP(hipMemsetAsync(c->coef64_d, 0, (size_t)S * 2 * k * pp * sizeof(double), st));
  if (nsrc > 0) c->src_vec64_d = static_cast<double*>(c->dalloc((size_t)nsrc * kp * sizeof(double), &e));
  if (nrec > 0) c->rec_rows64_d = static_cast<double*>(c->dalloc((size_t)nrec * kp * sizeof(double), &e));
  const bool ic = u0_dev || v0_dev;
  if (ic) {
    c->U0_d = static_cast<float*>(c->dalloc((size_t)S * k * P16 * sizeof(float), &e));
    c->V0_d = static_cast<float*>(c->dalloc((size_t)S * k * P16 * sizeof(float), &e));
    if (e == hipSuccess) e = hipMemsetAsync(c->U0_d, 0, (size_t)S * k * P16 * sizeof(float), st);
    if (e == hipSuccess) e = hipMemsetAsync(c->V0_d, 0, (size_t)S * k * P16 * sizeof(float), st);
  }
  if (e != hipSuccess) return c->fail(SFM_ENOMEM, "projection buffers: out of device memory");

  // batch size from the free device memory
  int64_t per_sub = (int64_t)sizeof(double) *
                    (Nmax * kp + Nmax * p + Nmax + 2 * (int64_t)kp * p + 7 * (int64_t)k * pp + 6 * pp + kp + 8);
  if (finite) per_sub += (int64_t)sizeof(double) * (3 * Nmax * p + Nmax + 2 * kpkp + 16 * (int64_t)p) +
                         (int64_t)sizeof(double) * 2 * 1024 * p;
  int nbmax = c->cfg.build_batch;
  if (nbmax <= 0) {
    size_t fr = 0, tot = 0;
    B_TRY_HIP(hipMemGetInfo(&fr, &tot));
    nbmax = (int)std::max<int64_t>(1, std::min<int64_t>(256, (int64_t)(0.6 * (double)fr) / per_sub));
  }
  nbmax = std::min(nbmax, S);
  // CG chunks: enough work-groups per column sum to fill the device, at most 1024
  auto chunks_for = [&](int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, std::min<int64_t>(n, (2048 + nbmax - 1) / nbmax)));
  };
  const int nchunk_max = chunks_for(Nmax);
  Scratch sc(c);
  double* Z = sc.get((size_t)nbmax * Nmax * kp);
  double* Wl = sc.get((size_t)nbmax * Nmax * p);
  double* Sd = sc.get((size_t)nbmax * Nmax);
  double* C1 = sc.get((size_t)nbmax * kp * p);
  double* C2 = sc.get((size_t)nbmax * kp * p);
  double* A = sc.get((size_t)nbmax * k * pp);
  double* Bt = sc.get((size_t)nbmax * k * pp);
  double* G = sc.get((size_t)nbmax * k * pp);
  double* Gi = sc.get((size_t)nbmax * k * pp);
  double* Gam = sc.get((size_t)nbmax * k * pp);
  double* Gh = sc.get((size_t)nbmax * k * pp);
  double* L1 = sc.get((size_t)nbmax * pp);
  double* L2 = sc.get((size_t)nbmax * pp);
  double* T1 = sc.get((size_t)nbmax * pp);
  double* Hb = sc.get((size_t)nbmax * p);
  double* thr = sc.get((size_t)nbmax);
  double* ybuf = sc.get((size_t)nbmax * kp);
  int32_t* flags = sc.get<int32_t>((size_t)nbmax + 1);
  int32_t* meta = sc.get<int32_t>((size_t)nbmax * 5);
  int32_t* pts = sc.get<int32_t>((size_t)(std::max(nsrc, nrec) + 1) * 3);
  double* gw = sc.get(kGemmWorkBytes / sizeof(double));      // split-reduction partial tiles
  double* Af = sc.get((size_t)nbmax * 2 * pp);                // [B_j | C2_j] of the fused recurrence update
  // finite shift: PCG vectors, reduced operator and reduced-space basis
  double *Dinv = nullptr, *Rv = nullptr, *Pv = nullptr, *Qv = nullptr, *part = nullptr, *cgs = nullptr;
  double *At = nullptr, *Zh = nullptr;
  int32_t *active = nullptr, *count = nullptr;
  if (finite) {
    Dinv = sc.get((size_t)nbmax * Nmax);
    Rv = sc.get((size_t)nbmax * Nmax * p);
    Pv = sc.get((size_t)nbmax * Nmax * p);
    Qv = sc.get((size_t)nbmax * Nmax * p);
    part = sc.get((size_t)2 * nbmax * nchunk_max * p);
    cgs = sc.get((size_t)4 * nbmax * p);
    At = sc.get((size_t)nbmax * kpkp);
    Zh = sc.get((size_t)nbmax * kpkp);
    active = sc.get<int32_t>((size_t)nbmax * p);
    count = sc.get<int32_t>(1);
  }
  if (sc.e != hipSuccess) return c->fail(SFM_ENOMEM, "ROM build scratch: out of device memory (lower build_batch)");
  std::vector<double> Hall((size_t)S * p);
  const double one = 1.0, zero = 0.0, mone = -1.0;
  const bool NN = false, TT = true;   // operand not transposed / transposed

  const char* vb = std::getenv("SFM_VERBOSE");
  const bool verbose = vb && vb[0] && vb[0] != '0';
  int cg_iters_max = 0;
  sfm_status status = SFM_OK;
  // Batches: up to nbmax subdomains of one box shape (all of them for equal boxes), in
  // subdomain order within a shape.  ids[b] is the subdomain of batch member b.
  std::vector<int32_t> order(S);
  for (int s = 0; s < S; ++s) order[s] = s;
  auto shape_key = [&](int s) {
    int w[3];
    t.cells(s, w);
    const int64_t kb = levels ? levels[s] : k;   // one ROM size per batch too
    return ((kb * (t.ncell[2] + 1) + w[2]) * (t.ncell[1] + 1) + w[1]) * (t.ncell[0] + 1) + w[0];
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return shape_key(a) < shape_key(b); });
  std::vector<int32_t> batch_of(S), pos_of(S);
  int nbatch_done = 0;
  for (size_t i0 = 0; i0 < order.size() && status == SFM_OK;) {
    size_t i1 = i0 + 1;
    while (i1 < order.size() && (int)(i1 - i0) < nbmax && shape_key(order[i1]) == shape_key(order[i0])) ++i1;
    const int nb = (int)(i1 - i0);
    const std::vector<int32_t> ids(order.begin() + i0, order.begin() + i1);
    i0 = i1;
    for (int b = 0; b < nb; ++b) {
      batch_of[ids[b]] = nbatch_done;
      pos_of[ids[b]] = b;
    }
    const int bidx = nbatch_done++;
    const int kb = levels ? levels[ids[0]] : k;    // Lanczos steps and S-fraction levels of this batch
    int w[3];
    t.cells(ids[0], w);
    const BoxGeo g{{w[0], w[1], w[2]}, {w[0] + 1, w[1] + 1, w[2] + 1}, t.m, t.m1, t.m2, p, c->cfg.h};
    const int64_t N = (int64_t)(w[0] + 1) * (w[1] + 1) * (w[2] + 1);
    const int64_t sZ = N * kp;
    const int nchunk = chunks_for(N);
    // batch metadata: origins, neighbour masks, subdomain ids
    std::vector<int32_t> org(3 * nb), mask(nb);
    for (int b = 0; b < nb; ++b) {
      int o[3];
      t.origin(ids[b], o);
      org[3 * b] = o[0]; org[3 * b + 1] = o[1]; org[3 * b + 2] = o[2];
      int mk = 0;
      for (int f = 0; f < 6; ++f)
        if (t.nbr[(size_t)ids[b] * 6 + f] >= 0) mk |= 1 << f;
      mask[b] = mk;
    }
    int32_t* org_d = meta;
    int32_t* mask_d = meta + 3 * nbmax;
    int32_t* ids_d = meta + 4 * nbmax;
    B_TRY_HIP(hipMemcpyAsync(org_d, org.data(), org.size() * 4, hipMemcpyHostToDevice, st));
    B_TRY_HIP(hipMemcpyAsync(mask_d, mask.data(), mask.size() * 4, hipMemcpyHostToDevice, st));
    B_TRY_HIP(hipMemcpyAsync(ids_d, ids.data(), ids.size() * 4, hipMemcpyHostToDevice, st));
    B_TRY_HIP(hipMemsetAsync(flags, 0, (size_t)(nbmax + 1) * sizeof(int32_t), st));

    // a1: scaling, face masses, Q_1
    B_LAUNCH(node_scale_kernel, (int64_t)nb * N, g, vel_dev, t.ncell[0], t.ncell[1], org_d, N, nb, Sd, flags + nbmax);
    B_LAUNCH(face_mass_kernel, (int64_t)nb * p, g, Sd, mask_d, N, nb, Hb);
    std::vector<double> Hbat((size_t)nb * p);
    B_TRY_HIP(hipMemcpyAsync(Hbat.data(), Hb, Hbat.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    B_TRY_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < nb; ++b) std::copy(Hbat.begin() + (size_t)b * p, Hbat.begin() + (size_t)(b + 1) * p, Hall.begin() + (size_t)ids[b] * p);
    std::vector<double> thr_h(nb);
    for (int b = 0; b < nb; ++b) {
      double hm = 0.0;
      for (int q = 0; q < p; ++q) {
        const double hv = Hall[(size_t)ids[b] * p + q];
        if (!(hv > 0.0))
          return c->fail(SFM_EBREAKDOWN, "subdomain " + std::to_string(ids[b]) + ": empty boundary patch " +
                                             std::to_string(q) + " (rank-deficient start block)");
        hm = std::max(hm, hv);
      }
      thr_h[b] = 1e-24 * hm;   // |diag B| < 1e-12 |B_1|
    }
    B_TRY_HIP(hipMemcpyAsync(thr, thr_h.data(), nb * sizeof(double), hipMemcpyHostToDevice, st));
    B_LAUNCH(init_q1_kernel, (int64_t)nb * N * p, g, Sd, mask_d, Hb, N, kp, nb, Z);
    B_LAUNCH(diag_kernel, (int64_t)nb * pp, Hb, p, nb, Bt, (int64_t)k * pp, 0);   // B_1^T = diag(H^{1/2})

    // a2: block Lanczos (three-term recurrence + one full CGS pass) and two-pass Cholesky QR on a
    // basis Zb of `rows` rows
    // (node-major, ld kp).  apply(jj, W, ldw, sW) writes the operator applied to block jj.
    // Steps jj < nsteps; the step jj = k - 1 only forms A_k.
    auto lanczos = [&](double* Zb, int64_t rows, int nsteps, const double* thrp, auto&& apply) -> sfm_status {
      const int64_t sZb = rows * kp;
      for (int jj = 0; jj < nsteps; ++jj) {
        const bool last = jj + 1 == kb;
        double* W = last ? Wl : Zb + (int64_t)(jj + 1) * p;
        const int ldw = last ? p : kp;
        const int64_t sW = last ? rows * p : sZb;
        const sfm_status ra = apply(jj, W, ldw, sW);
        if (ra != SFM_OK) return ra;
        const int nprev = (jj + 1) * p;
        // Projection coefficients in column-major p x ncols form: C[r + c p] = (Z^T W)[c][r];
        // W -= Z C is then the product C (p x ncols) Z^T on the node-major W.
        // Three-term recurrence first: C2 block j = Q_j^T W, W -= Q_j C2_j (and, from the second
        // block on, W -= Q_{j-1} B_j^T with B_j from the previous step's QR), then one pass of
        // classical Gram-Schmidt against every block so far (C1), which removes only the rounding
        // drift left after the recurrence; A_j = sym(C2_j + C1_j).
        double* C2j = C2 + (int64_t)jj * p * p;
        B_TRY_HIP(dgemm_batched(NN, TT, p, p, (int)rows, one, W, ldw, sW, Zb + (int64_t)jj * p, kp, sZb, zero, last ? C1 + (int64_t)jj * p * p : C2j, p, (int64_t)kp * p, nb, st, gw, kGemmWorkBytes));
        if (last) {
          B_LAUNCH(accum_a_kernel, (int64_t)nb * pp, C1, (const double*)nullptr, p, (int64_t)kp * p, jj * p,
                   A + (int64_t)jj * pp, (int64_t)k * pp, nb);
          break;
        }
        if (jj == 0) {
          B_TRY_HIP(dgemm_batched(NN, NN, p, (int)rows, p, mone, C2j, p, (int64_t)kp * p, Zb, kp, sZb, one, W, ldw, sW,
                                  nb, st, gw, kGemmWorkBytes));
        } else {
          // W -= Q_{j-1} B_j^T + Q_j A_j as one product over the adjacent blocks (Q_{j-1}^T A Q_j = B_j^T: in
          // the C form its transpose, B_j; Bt holds B_j^T column-major)
          B_LAUNCH(recurrence_coef_kernel, (int64_t)nb * 2 * pp, Bt + (int64_t)jj * pp, (int64_t)k * pp, C2j,
                   (int64_t)kp * p, p, nb, Af);
          B_TRY_HIP(dgemm_batched(NN, NN, p, (int)rows, 2 * p, mone, Af, p, 2 * pp, Zb + (int64_t)(jj - 1) * p, kp, sZb,
                                  one, W, ldw, sW, nb, st, gw, kGemmWorkBytes));
        }
        B_TRY_HIP(dgemm_batched(NN, TT, p, nprev, (int)rows, one, W, ldw, sW, Zb, kp, sZb, zero, C1, p, (int64_t)kp * p, nb, st, gw, kGemmWorkBytes));
        B_TRY_HIP(dgemm_batched(NN, NN, p, (int)rows, nprev, mone, C1, p, (int64_t)kp * p, Zb, kp, sZb, one, W, ldw, sW, nb, st, gw, kGemmWorkBytes));
        B_LAUNCH(accum_a_kernel, (int64_t)nb * pp, C1, C2, p, (int64_t)kp * p, jj * p, A + (int64_t)jj * pp,
                 (int64_t)k * pp, nb);
        // Cholesky QR, twice: W = Q (L1 L2)^T.  Each pass multiplies by the inverse of its
        // Cholesky factor (a batched triangular inverse and one batched DGEMM; a batched
        // triangular solve with `rows` right-hand sides runs as many small products), out of
        // place through Wl: pass 1 W -> Wl, pass 2 Wl -> W.
        double* Ls[2] = {L1, L2};
        for (int pass = 0; pass < 2; ++pass) {
          const double* src = pass == 0 ? W : Wl;
          const int lsrc = pass == 0 ? ldw : p;
          const int64_t ssrc = pass == 0 ? sW : rows * p;
          double* dst = pass == 0 ? Wl : W;
          const int ldst = pass == 0 ? p : ldw;
          const int64_t sdst = pass == 0 ? rows * p : sW;
          B_TRY_HIP(dgemm_batched(NN, TT, p, p, (int)rows, one, src, lsrc, ssrc, src, lsrc, ssrc, zero, Ls[pass], p, pp, nb, st, gw, kGemmWorkBytes));
          hipLaunchKernelGGL(cholesky_kernel, dim3(nb), dim3(256), 0, st, Ls[pass], p, pp,
                             pass == 0 ? thrp : (const double*)nullptr, kGramRelTol, flags);
          B_TRY_HIP(hipGetLastError());
          B_TRY_HIP(trtri_lower_batched(Ls[pass], pp, T1, pp, p, nb, st));
          B_LAUNCH(zero_upper_kernel, (int64_t)nb * pp, T1, p, pp, nb);
          B_TRY_HIP(dgemm_batched(NN, NN, p, (int)rows, p, one, T1, p, pp, src, lsrc, ssrc, zero, dst, ldst, sdst, nb, st, gw, kGemmWorkBytes));   // dst^T = L^{-1} src^T
        }
        // B_{j+1}^T = L1 L2
        B_TRY_HIP(dgemm_batched(NN, NN, p, p, p, one, L1, p, pp, L2, p, pp, zero, Bt + (int64_t)(jj + 1) * pp, p, (int64_t)k * pp, nb, st, gw, kGemmWorkBytes));
      }
      return SFM_OK;
    };

    if (!finite) {
      // polynomial space: block Lanczos on (A_+, F)
      rc = lanczos(Z, N, kb, thr, [&](int jj, double* W, int ldw, int64_t sW) -> sfm_status {
        B_LAUNCH(stencil_kernel, (int64_t)nb * (N / g.n[2]) * p, g, Sd, N, nb, Z + (int64_t)jj * p, kp, sZ, W, ldw, sW, 0.0);
        return SFM_OK;
      });
      if (rc != SFM_OK) return rc;
    } else {
      // rational space: V = orthonormal basis of {F, (A_+ + sigma)^{-1} F, ...} from block Lanczos on
      // ((A_+ + sigma I)^{-1}, F) with batched Jacobi-PCG solves (the tridiagonal blocks of this
      // recurrence are not needed), then the reduced pair (V^T A_+ V, V^T F = E_1 B_1) is
      // tridiagonalised by a second block Lanczos in the kp-dimensional space, Z = V Z~.
      const CgVec cv{N, p, nchunk, nb};
      const int64_t sN = N * p;
      const dim3 cgrid(nchunk, nb);
      const unsigned sgrid = (unsigned)((nb * p + 255) / 256);
      B_LAUNCH(shifted_diag_kernel, (int64_t)nb * N, g, Sd, N, nb, shift.sigma, Dinv);
      const double rtol2 = shift.rtol * shift.rtol;
      rc = lanczos(Z, N, k - 1, nullptr, [&](int jj, double* X, int ldx, int64_t sx) -> sfm_status {
        const double* Bv = Z + (int64_t)jj * p;
        hipLaunchKernelGGL(cg_init_kernel, cgrid, dim3(256), 0, st, cv, Bv, kp, sZ, Dinv, X, ldx, sx, Rv, Pv, part);
        B_TRY_HIP(hipGetLastError());
        hipLaunchKernelGGL(cg_start_kernel, dim3(sgrid), dim3(256), 0, st, cv, part, cgs, active);
        B_TRY_HIP(hipGetLastError());
        int it = 0;
        for (;;) {
          for (int q = 0; q < kCgCheck; ++q, ++it) {
            B_LAUNCH(stencil_kernel, (int64_t)nb * (N / g.n[2]) * p, g, Sd, N, nb, Pv, p, sN, Qv, p, sN, shift.sigma);
            hipLaunchKernelGGL(cg_dot_kernel, cgrid, dim3(256), 0, st, cv, Pv, Qv, part);
            B_TRY_HIP(hipGetLastError());
            hipLaunchKernelGGL(cg_alpha_kernel, dim3(sgrid), dim3(256), 0, st, cv, part, cgs, active);
            B_TRY_HIP(hipGetLastError());
            hipLaunchKernelGGL(cg_update_kernel, cgrid, dim3(256), 0, st, cv, cgs + 2 * nb * p, Dinv, Pv, Qv, X, ldx,
                               sx, Rv, part);
            B_TRY_HIP(hipGetLastError());
            hipLaunchKernelGGL(cg_beta_kernel, dim3(sgrid), dim3(256), 0, st, cv, part, cgs, active, rtol2);
            B_TRY_HIP(hipGetLastError());
            B_LAUNCH(cg_dir_kernel, (int64_t)nb * N * p, cv, Dinv, Rv, cgs + 3 * nb * p, Pv);
          }
          hipLaunchKernelGGL(count_active_kernel, dim3(1), dim3(256), 0, st, active, nb * p, count);
          B_TRY_HIP(hipGetLastError());
          int na = 0;
          B_TRY_HIP(hipMemcpyAsync(&na, count, sizeof(int), hipMemcpyDeviceToHost, st));
          B_TRY_HIP(hipStreamSynchronize(st));
          if (na == 0) break;
          if (it >= shift.max_iter)
            return c->fail(SFM_ENOCONV, "shifted solve of Lanczos block " + std::to_string(jj + 1) + " (build batch " +
                                            std::to_string(bidx) + ", subdomains " + std::to_string(ids.front()) +
                                            ".." + std::to_string(ids.back()) + "): " +
                                            std::to_string(na) + " columns above rtol after " + std::to_string(it) +
                                            " iterations");
        }
        cg_iters_max = std::max(cg_iters_max, it);
        if (verbose) {
          std::fprintf(stderr, "[sfm] shifted build: block %d of batch %d, %d CG iterations\n", jj + 1, bidx, it);
          std::fflush(stderr);
        }
        return SFM_OK;
      });
      if (rc != SFM_OK) return rc;
      // A~ = V^T A_+ V, one block row at a time (symmetric: rows jj*p.. of the column-major kp x kp)
      for (int jj = 0; jj < k; ++jj) {
        B_LAUNCH(stencil_kernel, (int64_t)nb * (N / g.n[2]) * p, g, Sd, N, nb, Z + (int64_t)jj * p, kp, sZ, Wl, p, N * p, 0.0);
        B_TRY_HIP(dgemm_batched(NN, TT, p, kp, (int)N, one, Wl, p, N * p, Z, kp, sZ, zero, At + (int64_t)jj * p, kp, kpkp, nb, st, gw, kGemmWorkBytes));
      }
      B_LAUNCH(symmetrize_kernel, (int64_t)nb * kpkp, At, kp, kpkp, nb);
      // block Lanczos on (A~, E_1 B_1): Q~_1 = E_1, same B_1^T = diag(H^{1/2})
      B_LAUNCH(eye_block_kernel, (int64_t)nb * kp * p, kp, p, nb, Zh, kpkp);
      rc = lanczos(Zh, kp, k, thr, [&](int jj, double* W, int ldw, int64_t sW) -> sfm_status {
        // W^T = Q~_j^T A~ (column-major p x kp)
        B_TRY_HIP(dgemm_batched(NN, NN, p, kp, kp, one, Zh + (int64_t)jj * p, kp, kpkp, At, kp, kpkp, zero, W, ldw, sW, nb, st, gw, kGemmWorkBytes));
        return SFM_OK;
      });
      if (rc != SFM_OK) return rc;
      // Z = V Z~ in node chunks staged through Wl (column-major: Z^T = Z~^T V^T)
      const int64_t nc = std::max<int64_t>(1, (N * p) / kp);
      for (int64_t n0 = 0; n0 < N; n0 += nc) {
        const int64_t nn = std::min(nc, N - n0);
        B_LAUNCH(copy_blocks_kernel, (int64_t)nb * nn * kp, Z + n0 * kp, sZ, Wl, N * p, nn * kp, nb, 1.0);
        B_TRY_HIP(dgemm_batched(NN, NN, kp, (int)nn, kp, one, Zh, kp, kpkp, Wl, kp, N * p, zero, Z + n0 * kp, kp, sZ, nb, st, gw, kGemmWorkBytes));
      }
    }
    // a3: S-fraction
    const int64_t sk = (int64_t)k * pp;
    B_LAUNCH(diag_kernel, (int64_t)nb * pp, Hb, p, nb, G, sk, 0);
    B_LAUNCH(diag_kernel, (int64_t)nb * pp, Hb, p, nb, Gi, sk, 1);
    for (int jj = 0; jj < kb; ++jj) {
      double* Gj = G + jj * pp;
      double* Gij = Gi + jj * pp;
      double* Gamj = Gam + jj * pp;
      B_TRY_HIP(dgemm_batched(NN, TT, p, p, p, one, Gj, p, sk, Gj, p, sk, zero, Gh + jj * pp, p, sk, nb, st, gw, kGemmWorkBytes));
      B_LAUNCH(symmetrize_kernel, (int64_t)nb * pp, Gh + jj * pp, p, sk, nb);
      if (jj > 0) {   // Gamma-hat_j = G_j G_j^T must be positive definite at the FP64 level (kGammaRelTol)
        B_LAUNCH(copy_blocks_kernel, (int64_t)nb * pp, Gh + jj * pp, sk, L2, pp, pp, nb, 1.0);
        hipLaunchKernelGGL(cholesky_kernel, dim3(nb), dim3(256), 0, st, L2, p, pp, (const double*)nullptr,
                           kGammaRelTol, flags);
        B_TRY_HIP(hipGetLastError());
      }
      B_TRY_HIP(dgemm_batched(NN, NN, p, p, p, one, A + jj * pp, p, sk, Gij, p, sk, zero, T1, p, pp, nb, st, gw, kGemmWorkBytes));
      if (jj == 0) {
        B_TRY_HIP(dgemm_batched(TT, NN, p, p, p, one, Gij, p, sk, T1, p, pp, zero, Gamj, p, sk, nb, st, gw, kGemmWorkBytes));
      } else {
        B_LAUNCH(copy_blocks_kernel, (int64_t)nb * pp, Gam + (jj - 1) * pp, sk, Gamj, sk, pp, nb, 1.0);
        B_TRY_HIP(dgemm_batched(TT, NN, p, p, p, one, Gij, p, sk, T1, p, pp, mone, Gamj, p, sk, nb, st, gw, kGemmWorkBytes));
      }
      B_LAUNCH(symmetrize_kernel, (int64_t)nb * pp, Gamj, p, sk, nb);
      if (jj + 1 == kb) break;
      // Cholesky of Gamma_j (must be SPD for j < k)
      B_LAUNCH(copy_blocks_kernel, (int64_t)nb * pp, Gamj, sk, L1, pp, pp, nb, 1.0);
      hipLaunchKernelGGL(cholesky_kernel, dim3(nb), dim3(256), 0, st, L1, p, pp, (const double*)nullptr, kGammaRelTol,
                         flags);
      B_TRY_HIP(hipGetLastError());
      double* Gn = G + (jj + 1) * pp;
      double* Gin = Gi + (jj + 1) * pp;
      double* Btn = Bt + (jj + 1) * pp;
      // G_{j+1} = -Gamma_j^{-1} G_j^{-T} B_{j+1}^T
      B_TRY_HIP(dgemm_batched(TT, NN, p, p, p, one, Gij, p, sk, Btn, p, sk, zero, Gn, p, sk, nb, st, gw, kGemmWorkBytes));
      B_TRY_HIP(trsm_lower_batched(false, -1.0, L1, pp, Gn, sk, p, nb, st));
      B_TRY_HIP(trsm_lower_batched(true, 1.0, L1, pp, Gn, sk, p, nb, st));
      // G_{j+1}^{-1} = -B_{j+1}^{-T} G_j^T Gamma_j
      B_TRY_HIP(dgemm_batched(TT, NN, p, p, p, one, Gj, p, sk, Gamj, p, sk, zero, Gin, p, sk, nb, st, gw, kGemmWorkBytes));
      B_TRY_HIP(trsm_lower_batched(false, -1.0, Btn, sk, Gin, sk, p, nb, st));
    }
    // coefficients to the FP64 store [S][2][k][p][p] (symmetric: column-major = row-major)
    B_LAUNCH(scatter_blocks_kernel, (int64_t)nb * kb * pp, Gam, sk, c->coef64_d, 2 * sk, (int64_t)kb * pp, nb, ids_d);
    B_LAUNCH(scatter_blocks_kernel, (int64_t)nb * kb * pp, Gh, sk, c->coef64_d + sk, 2 * sk, (int64_t)kb * pp, nb, ids_d);

    // a4: projections of the points of this batch
    for (int mode = 0; mode < 2; ++mode) {
      const std::vector<int32_t>& sub = mode == 0 ? src_sub : rec_sub;
      const std::vector<int32_t>& loc = mode == 0 ? src_local : rec_local;
      std::vector<int32_t> pb, pn, pid;
      for (size_t i = 0; i < sub.size(); ++i)
        if (batch_of[sub[i]] == bidx) {
          pb.push_back(pos_of[sub[i]]);
          pn.push_back(loc[i]);
          pid.push_back((int32_t)i);
        }
      const int npts = (int)pb.size();
      if (npts == 0) continue;
      std::vector<int32_t> packed;
      packed.insert(packed.end(), pb.begin(), pb.end());
      packed.insert(packed.end(), pn.begin(), pn.end());
      packed.insert(packed.end(), pid.begin(), pid.end());
      B_TRY_HIP(hipMemcpyAsync(pts, packed.data(), packed.size() * 4, hipMemcpyHostToDevice, st));
      B_LAUNCH(project_points_kernel, (int64_t)npts * kp, Z, Sd, N, k, kb, p, G, Gi, sk, pts, pts + npts, pts + 2 * npts,
               npts, mode, mode == 0 ? c->src_vec64_d : c->rec_rows64_d);
      B_TRY_HIP(hipStreamSynchronize(st));   // pts is reused
    }
    if (ic) {
      const float* fields[2] = {u0_dev, v0_dev};
      float* outs[2] = {c->U0_d, c->V0_d};
      for (int fi = 0; fi < 2; ++fi) {
        if (!fields[fi]) continue;
        hipLaunchKernelGGL(project_field_kernel, dim3((nb * kp + 255) / 256), dim3(256), 0, st, g, Z, Sd, N, kp, nb,
                           fields[fi], t.ncell[0], t.ncell[1], org_d, ybuf);
        B_TRY_HIP(hipGetLastError());
        B_LAUNCH(apply_g_kernel, (int64_t)nb * kp, ybuf, G, sk, k, kb, p, P16, nb, ids_d, outs[fi]);
      }
    }
    // breakdown flags of this batch
    std::vector<int32_t> fl(nbmax + 1);
    B_TRY_HIP(hipMemcpyAsync(fl.data(), flags, fl.size() * 4, hipMemcpyDeviceToHost, st));
    B_TRY_HIP(hipStreamSynchronize(st));
    if (verbose) {
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
      std::fprintf(stderr, "[sfm] ROM build: batch %d (%d subdomains of %dx%dx%d cells) of %d subdomains done, %.2f s\n",
                   bidx, nb, w[0], w[1], w[2], S, el);
      std::fflush(stderr);
    }
    if (fl[nbmax]) status = c->fail(SFM_EINVAL, "sound speed must be positive and finite at every node");
    for (int b = 0; b < nb && status == SFM_OK; ++b)
      if (fl[b])
        status = c->fail(SFM_EBREAKDOWN, "subdomain " + std::to_string(ids[b]) +
                                             ": block Lanczos breakdown, or an S-fraction level that is not positive definite "
                                             "at the FP64 level");
  }
  if (status != SFM_OK) {
    release_roms(c);
    return status;
  }
  std::vector<double> sv;
  if (nsrc > 0) {
    sv.resize((size_t)nsrc * kp);
    B_TRY_HIP(hipMemcpy(sv.data(), c->src_vec64_d, sv.size() * sizeof(double), hipMemcpyDeviceToHost));
  }
  if (ic) {
    // Both sides of a shared face projected the same trace; keep one copy so the shared
    // boundary entries start (and stay) bit-identical.
    for (int fi = 0; fi < 2; ++fi) {
      float* arr = fi == 0 ? c->U0_d : c->V0_d;
      B_LAUNCH(unify_ports_kernel, (int64_t)S * p, c->nbr_d, S, k, p, t.m, P16, arr);
    }
  }
  rc = finalize_roms(c, Hall, src_sub, sv, rec_sub, st);
  if (rc != SFM_OK) return rc;
  if (cg_iters_out) *cg_iters_out = cg_iters_max;
  c->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return SFM_OK;
}

}  // namespace

extern "C" sfm_status sfm_build_roms(sfm_ctx c, const float* vel_dev, int32_t nsrc, const int32_t* src_ijk,
                                     int32_t nrec, const int32_t* rec_ijk, const float* u0_dev,
                                     const float* v0_dev, void* stream) {
  if (!c) return SFM_EINVAL;
  const ShiftSpec spec{INFINITY, 0.0, 0};
  const sfm_status rc = build_roms(c, spec, vel_dev, nsrc, src_ijk, nrec, rec_ijk, u0_dev, v0_dev, nullptr, stream);
  if (rc != SFM_OK) release_roms(c);
  return rc;
}

extern "C" sfm_status sfm_build_roms_levels(sfm_ctx c, const int32_t* k_per_sub, const float* vel_dev, int32_t nsrc,
                                            const int32_t* src_ijk, int32_t nrec, const int32_t* rec_ijk,
                                            const float* u0_dev, const float* v0_dev, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!k_per_sub) return c->fail(SFM_EINVAL, "k_per_sub is NULL");
  const Topology& t = c->topo;
  for (int s = 0; s < t.S; ++s)
    if (k_per_sub[s] < 2 || k_per_sub[s] > t.k)
      return c->fail(SFM_EINVAL, "subdomain " + std::to_string(s) + ": levels " + std::to_string(k_per_sub[s]) +
                                     " outside [2, " + std::to_string(t.k) + "]");
  const ShiftSpec spec{INFINITY, 0.0, 0};
  sfm_status rc = build_roms(c, spec, vel_dev, nsrc, src_ijk, nrec, rec_ijk, u0_dev, v0_dev, nullptr, stream, k_per_sub);
  if (rc == SFM_OK) rc = sfm_set_levels(c, k_per_sub);
  if (rc != SFM_OK) release_roms(c);
  return rc;
}

extern "C" sfm_status sfm_build_roms_shifted(sfm_ctx c, double sigma, double cg_rtol, int32_t cg_max_iter,
                                             const float* vel_dev, int32_t nsrc, const int32_t* src_ijk, int32_t nrec,
                                             const int32_t* rec_ijk, const float* u0_dev, const float* v0_dev,
                                             int32_t* cg_iters, void* stream) {
  if (!c) return SFM_EINVAL;
  c->err.clear();
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return c->fail(SFM_EINVAL, "sigma must be positive and finite");
  if (!(cg_rtol > 0.0 && cg_rtol < 1.0)) return c->fail(SFM_EINVAL, "cg_rtol must lie in (0, 1)");
  if (cg_max_iter < 1) return c->fail(SFM_EINVAL, "cg_max_iter must be at least 1");
  if (c->cfg.precision != SFM_PREC_FP64)
    return c->fail(SFM_EINVAL, "finite-shift ROMs need FP64 coefficient storage (SFM_PREC_FP64): their last "
                               "S-fraction level is singular along the subdomain's constant mode and FP32 or "
                               "BF16 rounding makes it indefinite");
  const ShiftSpec spec{sigma, cg_rtol, cg_max_iter};
  const sfm_status rc = build_roms(c, spec, vel_dev, nsrc, src_ijk, nrec, rec_ijk, u0_dev, v0_dev, cg_iters, stream);
  if (rc != SFM_OK) release_roms(c);
  return rc;
}
