// FP64 Cholesky factorisation H = L L^T of the Newton matrix and the solve x = -H^{-1} g (the linear
// system of each Newton step, section 4, "Primal optimization": second-order steps expressed as dense
// linear algebra).
//
// Right-looking blocked algorithm with 64-wide panels. Per panel k:
//   1. one workgroup factors the 64 x 64 diagonal block in LDS and writes its inverse (for the panel solve
//      and for the triangular solves later);
//   2. the rows below are multiplied by the inverse transpose (independent 64-row blocks);
//   3. the trailing lower triangle is updated, H_ij -= L_ik L_jk^T, one 64 x 64 tile per workgroup on FP64 MFMA.
// A non-positive or non-finite pivot sets a failure flag; the host then retries with a diagonal jitter.
#include "common.h"
#include "launch.h"

namespace spsvm {

constexpr int NB = kCholNB;
constexpr int NB_LD = NB + 1;

// Factor the 64 x 64 diagonal block in LDS and write L_kk and its inverse. Thread t owns column t & 63 and
// rows (t >> 6) + 4 r, so every step is one parallel sweep followed by one barrier:
//  factor step j:  A[i][l] -= A[i][j] A[l][j] / A[j][j]  for j < l <= i (column j itself is scaled at the end);
//  inverse step p: X[i][c] -= L[i][p] X[p][c] / L[p][p]   for i > p      (rows of X are scaled at the end).
__global__ __launch_bounds__(256) void k_potrf_diag(double* __restrict__ H, int64_t ldh, int m, int k0,
                                                    double* __restrict__ Linv, NewtonScalars* sc) {
  __shared__ double A[NB][NB_LD];
  __shared__ double X[NB][NB_LD];
  __shared__ double dg[NB];
  const int nb = m - k0 < NB ? m - k0 : NB;
  const int tid = threadIdx.x, col = tid & 63, r0 = tid >> 6;
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    A[r][c] = (r < nb && c <= r) ? H[(int64_t)(k0 + r) * ldh + k0 + c] : (r == c ? 1.0 : 0.0);
    X[r][c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  bool bad = false;
  for (int j = 0; j < NB; ++j) {
    const double piv = A[j][j];
    if (tid == 0) bad |= !(piv > 0.0) || !(piv < __builtin_huge_val());
    const double rp = (piv > 0.0 && piv < __builtin_huge_val()) ? 1.0 / piv : 0.0;
    if (col > j) {
      // all LDS reads of the step first, then the writes (keeps the reads pipelined)
      double aij[16], aic[16];
      const double alj = A[col][j] * rp;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        aij[q] = A[r0 + 4 * q][j];
        aic[q] = A[r0 + 4 * q][col];
      }
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (r0 + 4 * q >= col) A[r0 + 4 * q][col] = aic[q] - aij[q] * alj;
    }
    __syncthreads();
  }
  if (tid < NB) {
    const double p = A[tid][tid];
    dg[tid] = (p > 0.0 && p < __builtin_huge_val()) ? sqrt(p) : 1.0;
  }
  __syncthreads();
  // L[i][c] = A[i][c] / sqrt(A[c][c]) below the diagonal, sqrt(A[c][c]) on it
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int i = r0 + 4 * q;
    if (i > col) A[i][col] /= dg[col];
  }
  __syncthreads();
  if (tid < NB) A[tid][tid] = dg[tid];
  __syncthreads();
  // inverse of the lower-triangular L: column-oriented forward substitution on X = I
  for (int p = 0; p < NB; ++p) {
    const double xp = X[p][col] / A[p][p];
    double aip[16], xic[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      aip[q] = A[r0 + 4 * q][p];
      xic[q] = X[r0 + 4 * q][col];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (r0 + 4 * q > p) X[r0 + 4 * q][col] = xic[q] - aip[q] * xp;
    __syncthreads();
  }
  double* Lo = Linv + (int64_t)(k0 / NB) * NB * NB;
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    Lo[e] = (c <= r) ? X[r][c] / A[r][r] : 0.0;
    if (r < nb && c <= r) H[(int64_t)(k0 + r) * ldh + k0 + c] = A[r][c];
  }
  if (tid == 0 && bad) sc->fail = 1;
}

// Rows r >= k0 + 64: L[r, panel] = H[r, panel] Linv^T, a 64 x 64 x 64 product per workgroup on FP64 MFMA.
constexpr int TU_LD = NB + 4;

__global__ __launch_bounds__(256) void k_trsm_panel(double* __restrict__ H, int64_t ldh, int m, int k0,
                                                    const double* __restrict__ Linv) {
  __shared__ __attribute__((aligned(32))) double Bm[NB][TU_LD];
  __shared__ __attribute__((aligned(32))) double Li[NB][TU_LD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, i16 = lane & 15;
  const int r0 = k0 + NB + blockIdx.x * NB;
  const double* Lo = Linv + (int64_t)(k0 / NB) * NB * NB;
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e >> 6, c = e & 63;
    Li[r][c] = Lo[e];
    Bm[r][c] = (r0 + r < m) ? H[(int64_t)(r0 + r) * ldh + k0 + c] : 0.0;
  }
  __syncthreads();
  const int wr = w >> 1, wc = w & 1;
  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0, 0, 0, 0};
#pragma unroll
  for (int kk = 0; kk < NB; kk += 16) {
    doublex4 av[2], bv[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) av[i] = *(const doublex4*)&Bm[wr * 32 + i * 16 + i16][kk + 4 * g];
#pragma unroll
    for (int j = 0; j < 2; ++j) bv[j] = *(const doublex4*)&Li[wc * 32 + j * 16 + i16][kk + 4 * g];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][s], bv[j][s], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = r0 + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
        const int cc = wc * 32 + j * 16 + i16;
        if (rr < m) H[(int64_t)rr * ldh + k0 + cc] = acc[i][j][r];
      }
}

// Trailing update of the lower tiles at or below the diagonal of the remaining matrix.
__device__ __forceinline__ void tri_tile(int t, int& tr, int& tc) {
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  tr = r;
  tc = t - r * (r + 1) / 2;
}

__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ H, int64_t ldh, int m, int k0) {
  __shared__ __attribute__((aligned(32))) double Pa[NB][TU_LD];
  __shared__ __attribute__((aligned(32))) double Pb[NB][TU_LD];
  int tr, tc;
  tri_tile(blockIdx.x, tr, tc);
  const int base = k0 + NB;
  const int ra = base + tr * NB, rb = base + tc * NB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, i16 = lane & 15;
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    Pa[r][c] = (ra + r < m) ? H[(int64_t)(ra + r) * ldh + k0 + c] : 0.0;
    Pb[r][c] = (rb + r < m) ? H[(int64_t)(rb + r) * ldh + k0 + c] : 0.0;
  }
  __syncthreads();
  const int wr = w >> 1, wc = w & 1;
  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0, 0, 0, 0};
#pragma unroll
  for (int kk = 0; kk < NB; kk += 16) {
    doublex4 av[2], bv[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) av[i] = *(const doublex4*)&Pa[wr * 32 + i * 16 + i16][kk + 4 * g];
#pragma unroll
    for (int j = 0; j < 2; ++j) bv[j] = *(const doublex4*)&Pb[wc * 32 + j * 16 + i16][kk + 4 * g];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][s], bv[j][s], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = ra + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
        const int gc = rb + wc * 32 + j * 16 + i16;
        if (gr < m && gc < m && gc <= gr) H[(int64_t)gr * ldh + gc] -= acc[i][j][r];
      }
}

void launch_cholesky(double* H, int64_t ldh, int m, double* Linv, NewtonScalars* sc, hipStream_t s) {
  for (int k0 = 0; k0 < m; k0 += NB) {
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, H, ldh, m, k0, Linv, sc);
    SPSVM_LAUNCHED();
    const int rest = m - k0 - NB;
    if (rest <= 0) break;
    const int nblk = (int)ceil_div(rest, NB);
    hipLaunchKernelGGL(k_trsm_panel, dim3(nblk), dim3(256), 0, s, H, ldh, m, k0, Linv);
    SPSVM_LAUNCHED();
    hipLaunchKernelGGL(k_chol_update, dim3(nblk * (nblk + 1) / 2), dim3(256), 0, s, H, ldh, m, k0);
    SPSVM_LAUNCHED();
  }
}

// ----------------------------------------------------------------------------------- triangular solves
// One workgroup of 1024 threads. Forward: z_b = Linv_b (g_b - L[b, <b] z_<b); backward:
// x_b = Linv_b^T (z_b - L[>b, b]^T x_>b); the result is negated (x = -H^{-1} g).
__global__ __launch_bounds__(1024) void k_chol_solve(const double* __restrict__ L, int64_t ldh, int m,
                                                     const double* __restrict__ Linv, const double* __restrict__ g,
                                                     double* __restrict__ x, double* __restrict__ z) {
  __shared__ double part[16][NB];
  __shared__ double rhs[NB];
  const int tid = threadIdx.x;
  const int nblk = (int)((m + NB - 1) / NB);
  // forward
  for (int b = 0; b < nblk; ++b) {
    const int b0 = b * NB;
    const int r = tid >> 4, p0 = tid & 15;
    double s = 0.0;
    if (b0 + r < m)
      for (int p = p0; p < b0; p += 16) s += L[(int64_t)(b0 + r) * ldh + p] * z[p];
    part[p0][r] = s;
    __syncthreads();
    if (tid < NB) {
      double t = 0.0;
      for (int q = 0; q < 16; ++q) t += part[q][tid];
      rhs[tid] = (b0 + tid < m) ? g[b0 + tid] - t : 0.0;
    }
    __syncthreads();
    if (tid < NB && b0 + tid < m) {
      const double* Lo = Linv + (int64_t)b * NB * NB + (int64_t)tid * NB;
      double t = 0.0;
      for (int p = 0; p <= tid; ++p) t += Lo[p] * rhs[p];
      z[b0 + tid] = t;
    }
    __syncthreads();
  }
  // backward
  for (int b = nblk - 1; b >= 0; --b) {
    const int b0 = b * NB;
    const int c = tid & 63, p0 = tid >> 6;
    double s = 0.0;
    if (b0 + c < m)
      for (int i = b0 + NB + p0; i < m; i += 16) s += L[(int64_t)i * ldh + b0 + c] * x[i];
    part[p0][c] = s;
    __syncthreads();
    if (tid < NB) {
      double t = 0.0;
      for (int q = 0; q < 16; ++q) t += part[q][tid];
      rhs[tid] = (b0 + tid < m) ? z[b0 + tid] - t : 0.0;
    }
    __syncthreads();
    if (tid < NB && b0 + tid < m) {
      const double* Lo = Linv + (int64_t)b * NB * NB;
      double t = 0.0;
      for (int p = tid; p < NB; ++p) t += Lo[(int64_t)p * NB + tid] * rhs[p];
      x[b0 + tid] = t;
    }
    __syncthreads();
  }
  for (int k = tid; k < m; k += 1024) x[k] = -x[k];
}

void launch_chol_solve(const double* L, int64_t ldh, int m, const double* Linv, const double* g, double* x,
                       double* work, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_solve, dim3(1), dim3(1024), 0, s, L, ldh, m, Linv, g, x, work);
  SPSVM_LAUNCHED();
}

}  // namespace spsvm
