// FP64 Cholesky factorisation H = L L^T of the Newton matrix and the solve x = -H^{-1} g (the linear
// system of each Newton step, section 4, "Primal optimization": second-order steps expressed as dense
// linear algebra).
//
// Right-looking blocked algorithm in two levels: outer panels of 256 columns, each factored as four inner panels
// of 64. Per inner panel k:
//   1. one workgroup factors the 64 x 64 diagonal block in LDS and writes its inverse (for the panel solve
//      and for the triangular solves later);
//   2. the rows below are multiplied by the inverse transpose (independent 64-row blocks);
//   3. the rest of the outer panel (its columns right of k, every row below) is updated, H_ij -= L_ik L_jk^T,
//      one 64 x 64 tile per workgroup on FP64 MFMA.
// After the fourth inner panel the trailing lower triangle right of the outer panel is updated once with all
// 256 of its columns (H_ij -= L_i,K L_j,K^T, K the outer panel): each tile of the trailing matrix is read and
// written once per 256 columns instead of once per 64, and its MFMA chain is four times longer.
// A non-positive or non-finite pivot sets a failure flag; the host then retries with a diagonal jitter.
#include <mutex>
#include <string>

#include "common.h"
#include "launch.h"

namespace spsvm {

constexpr int NB = kCholNB;
constexpr int NB_LD = NB + 1;

// Factor the 64 x 64 diagonal block in LDS and write L_kk and its inverse. The block is itself processed in
// four 16-wide column blocks: wave 0 factors the 16 x 16 diagonal sub-block and inverts it (no barriers
// inside one wave), then all threads solve the sub-panel below it and update the trailing sub-matrix. The
// inverse of the 64 x 64 factor is assembled from the 16 x 16 inverses by block forward substitution:
// X_bb = D_b^{-1}, X_bc = -D_b^{-1} sum_{k=c}^{b-1} L_bk X_kc.
constexpr int SB = 16;

// Grid z = slot of the batch.
__global__ __launch_bounds__(256) void k_potrf_diag(const CholBatch bt, int64_t ldh, int m, int k0) {
  double* __restrict__ H = bt.H[blockIdx.z];
  double* __restrict__ Linv = bt.Linv[blockIdx.z];
  NewtonScalars* sc = bt.sc[blockIdx.z];
  __shared__ double A[NB][NB_LD];
  __shared__ double X[NB][NB_LD];
  __shared__ double Rd[SB];
  __shared__ __attribute__((aligned(16))) double Cj[SB];  // column j of the sub-block being factored
  __shared__ int bad;
  const int nb = m - k0 < NB ? m - k0 : NB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, i16 = lane & 15;
  if (tid == 0) bad = 0;
  {
    // all 16 loads of this thread in flight before the LDS stores
    double v[NB * NB / 256];
#pragma unroll
    for (int q = 0; q < NB * NB / 256; ++q) {
      const int e = tid + q * 256, r = e >> 6, c = e & 63;
      v[q] = (r < nb && c <= r) ? H[(int64_t)(k0 + r) * ldh + k0 + c] : (r == c ? 1.0 : 0.0);
    }
#pragma unroll
    for (int q = 0; q < NB * NB / 256; ++q) {
      const int e = tid + q * 256, r = e >> 6, c = e & 63;
      A[r][c] = v[q];
      X[r][c] = 0.0;
    }
  }
  __syncthreads();
  for (int kb = 0; kb < NB / SB; ++kb) {
    const int c0 = kb * SB;
    if (w == 0) {
      // Unblocked Cholesky factorisation and inversion of the 16 x 16 diagonal sub-block: lane l < 16 holds row l
      // (r[i] = A[c0 + l][c0 + i], i <= l). Step j: every lane puts its column-j entry in LDS and the wave reads
      // the column back as broadcasts (one store and eight 16-byte reads, no lane reads); the rows below j take
      // L[l][j] = r[j] / L[j][j] and subtract L[l][j] L[i][j] from every r[i], i > j. For i > l that entry is in
      // the unused upper triangle, so the update needs no test; lanes 16..63 shadow row 0 and write nothing.
      const int lr = lane < SB ? lane : 0;
      double r[SB], x[SB];
#pragma unroll
      for (int i = 0; i < SB; ++i) r[i] = A[c0 + lr][c0 + i];
      bool badl = false;
      double rdl = 1.0;  // 1 / L[lane][lane]
#pragma unroll
      for (int j = 0; j < SB; ++j) {
        if (lane < SB) Cj[lane] = r[j];
        __builtin_amdgcn_wave_barrier();
        double cj[SB];
#pragma unroll
        for (int i = 0; i < SB; ++i) cj[i] = Cj[i];
        __builtin_amdgcn_wave_barrier();
        const double piv = cj[j];
        // a pivot must be a positive normal number (a subnormal one is as good as zero here, and the hardware
        // estimate below need not take it): else the factorisation is reported as not positive definite
        const bool ok = piv >= 2.2250738585072014e-308 && piv < __builtin_huge_val();
        badl |= !ok;
        // 1 / sqrt(piv) from the hardware estimate and one Newton step (relative error squared, far below FP64
        // rounding), then L[j][j] = piv / sqrt(piv): four dependent operations instead of a sqrt and a division
        const double pv = ok ? piv : 1.0, y0 = __builtin_amdgcn_rsq(pv);
        const double rd = y0 * __fma_rn(-0.5 * pv * y0, y0, 1.5), d = pv * rd;
        const double lj = r[j] * rd;  // L[lane][j] for the rows below j
#pragma unroll
        for (int i = j + 1; i < SB; ++i) r[i] = __fma_rn(-lj, cj[i] * rd, r[i]);
        r[j] = lane == j ? d : lj;
        rdl = lane == j ? rd : rdl;
      }
      // L's row `lane` goes to LDS; then column lane of the inverse, x_i = (e_lane[i] - sum_{q < i} L[i][q]
      // x_q) / L[i][i], with L read back at addresses common to the wave (LDS broadcasts; one wave, in order)
      if (lane < SB) {
#pragma unroll
        for (int i = 0; i < SB; ++i)
          if (i <= lane) A[c0 + lane][c0 + i] = r[i];
        Rd[lane] = rdl;
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int i = 0; i < SB; ++i) {
        double t = (lane == i) ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < i; ++q) t -= A[c0 + i][c0 + q] * x[q];
        x[i] = (i >= lane) ? t * Rd[i] : 0.0;
      }
      if (lane < SB) {
#pragma unroll
        for (int i = 0; i < SB; ++i) X[c0 + i][c0 + lane] = x[i];
      }
      if (lane == 0 && badl) bad = 1;
    }
    __syncthreads();
    const int nr = NB / SB - 1 - kb;  // 16-row blocks below this sub-block
    if (nr > 0) {
      // sub-panel on FP64 MFMA, one wave per 16-row block i: L_ik = A_ik D_k^{-T}. In a step lane (g, i16)
      // supplies P[i16][4g + s] and Q[i16][4g + s]; acc[r] ends as (P Q^T)[g + 4r][i16]. Results stay in
      // registers until every wave has read its block.
      doublex4 pacc = {0.0, 0.0, 0.0, 0.0};
      const int ib = kb + 1 + w;
      if (w < nr) {
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
          pacc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[ib * SB + i16][c0 + 4 * g + s2],
                                                      X[c0 + i16][c0 + 4 * g + s2], pacc, 0, 0, 0);
      }
      __syncthreads();
      if (w < nr) {
#pragma unroll
        for (int r = 0; r < 4; ++r) A[ib * SB + g + 4 * r][c0 + i16] = pacc[r];
      }
      __syncthreads();
      // trailing blocks A_ij -= L_ik L_jk^T for kb < j <= i, round robin over the waves (they write columns
      // right of the sub-panel, which is only read). Diagonal blocks are updated whole; their upper halves
      // are never read.
      const int npairs = nr * (nr + 1) / 2;
      for (int p = w; p < npairs; p += 4) {
        int ii = 0, jj = p;
        while (jj > ii) {
          jj -= ii + 1;
          ++ii;
        }
        const int bi = kb + 1 + ii, bj = kb + 1 + jj;
        doublex4 t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
          t = __builtin_amdgcn_mfma_f64_16x16x4f64(A[bi * SB + i16][c0 + 4 * g + s2],
                                                   A[bj * SB + i16][c0 + 4 * g + s2], t, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) A[bi * SB + g + 4 * r][bj * SB + i16] -= t[r];
      }
      __syncthreads();
    }
  }
  // off-diagonal 16 x 16 blocks of the inverse, one block row b at a time, wave c for block column c:
  // T_bc = sum_{k=c}^{b-1} L_bk X_kc (written in place of X_bc, which nobody reads yet), then
  // X_bc = -D_b^{-1} T_bc. For a product P Q lane (g, i16) supplies P[i16][4g + s] and Q[4g + s][i16].
  for (int b = 1; b < NB / SB; ++b) {
    if (w < b) {
      const int c = w;
      doublex4 t = {0.0, 0.0, 0.0, 0.0};
      for (int k = c; k < b; ++k) {
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
          t = __builtin_amdgcn_mfma_f64_16x16x4f64(A[b * SB + i16][k * SB + 4 * g + s2],
                                                   X[k * SB + 4 * g + s2][c * SB + i16], t, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) X[b * SB + g + 4 * r][c * SB + i16] = t[r];
    }
    __syncthreads();
    doublex4 u = {0.0, 0.0, 0.0, 0.0};
    if (w < b) {
      const int c = w;
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2)
        u = __builtin_amdgcn_mfma_f64_16x16x4f64(X[b * SB + i16][b * SB + 4 * g + s2],
                                                 X[b * SB + 4 * g + s2][c * SB + i16], u, 0, 0, 0);
    }
    __syncthreads();
    if (w < b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) X[b * SB + g + 4 * r][w * SB + i16] = -u[r];
    }
    __syncthreads();
  }
  double* Lo = Linv + (int64_t)(k0 / NB) * NB * NB;
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e >> 6, c = e & 63;
    Lo[e] = (c <= r) ? X[r][c] : 0.0;
    if (r < nb && c <= r) H[(int64_t)(k0 + r) * ldh + k0 + c] = A[r][c];
  }
  if (tid == 0 && bad) sc->fail = 1;
}

// Rows r >= k0 + 64: L[r, panel] = H[r, panel] Linv^T, a 64 x 64 x 64 product per workgroup on FP64 MFMA.
constexpr int TU_LD = NB + 4;

__global__ __launch_bounds__(256) void k_trsm_panel(const CholBatch bt, int64_t ldh, int m, int k0) {
  double* __restrict__ H = bt.H[blockIdx.z];
  const double* __restrict__ Linv = bt.Linv[blockIdx.z];
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

// Tile (tr, tc) of a launch over the lower triangle (ctiles = 0: tri_tile of the workgroup index) or over a strip
// of ctiles tile columns and every tile row at or below each (the rest of an outer panel). False: no tile.
__device__ __forceinline__ bool update_tile(int ctiles, int& tr, int& tc) {
  if (ctiles == 0) {
    tri_tile(blockIdx.x, tr, tc);
    return true;
  }
  tr = blockIdx.x / ctiles;
  tc = blockIdx.x - tr * ctiles;
  return tc <= tr;
}

// Operands come straight from global memory (no LDS, no barrier): wave (wr, wc) owns a 32 x 32 block and lane
// group g takes the columns kp + 64 q + 16 g .. + 15 of each 64-column chunk q of the panel [kp, kp + kw), so in
// MFMA step s the four lane groups supply four distinct columns and every column enters the sum once; each lane
// loads its rows' 16 values of a chunk as four 32-byte vectors. The tiles start at row and column `base`; the
// strictly upper block of a diagonal tile is skipped.
__global__ __launch_bounds__(256) void k_chol_update(const CholBatch bt, int64_t ldh, int m, int kp, int kw, int base,
                                                     int ctiles) {
  double* __restrict__ H = bt.H[blockIdx.z];
  int tr, tc;
  if (!update_tile(ctiles, tr, tc)) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, i16 = lane & 15;
  const int wr = w >> 1, wc = w & 1;
  if (tr == tc && wr < wc) return;  // wave-uniform
  const int ra = base + tr * NB + wr * 32, rb = base + tc * NB + wc * 32;
  if (ra >= m || rb >= m) return;
  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0, 0, 0, 0};
  for (int k0 = kp; k0 < kp + kw; k0 += NB) {
    double av[2][16], bv[2][16];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = ra + i * 16 + i16;
      const double* p = H + (int64_t)(row < m ? row : k0) * ldh + k0 + 16 * g;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const doublex4 v = row < m ? *(const doublex4*)(p + 4 * h) : doublex4{0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < 4; ++e) av[i][4 * h + e] = v[e];
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int row = rb + j * 16 + i16;
      const double* p = H + (int64_t)(row < m ? row : k0) * ldh + k0 + 16 * g;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const doublex4 v = row < m ? *(const doublex4*)(p + 4 * h) : doublex4{0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < 4; ++e) bv[j][4 * h + e] = v[e];
      }
    }
#pragma unroll
    for (int st = 0; st < 16; ++st)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][st], bv[j][st], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = ra + i * 16 + g + 4 * r;
        const int gc = rb + j * 16 + i16;
        if (gr < m && gc < m && gc <= gr) H[(int64_t)gr * ldh + gc] -= acc[i][j][r];
      }
}

// The same update with 128 x 128 tiles for large trailing matrices: each wave owns a 64 x 64 block (4 x 4
// MFMA tiles), half the loads per MFMA of the 64 x 64 tiles. The panel's columns are taken in quarters of
// 16 (lane group g: columns 4 g .. 4 g + 3 of the quarter, one 32-byte load per row).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_chol_update128(
    const CholBatch bt, int64_t ldh, int m, int kp, int kw, int base) {
  double* __restrict__ H = bt.H[blockIdx.z];
  int tr, tc;
  tri_tile(blockIdx.x, tr, tc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, i16 = lane & 15;
  const int wr = w >> 1, wc = w & 1;
  if (tr == tc && wr < wc) return;  // wave-uniform
  const int ra = base + tr * 128 + wr * 64, rb = base + tc * 128 + wc * 64;
  if (ra >= m || rb >= m) return;
  doublex4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = doublex4{0, 0, 0, 0};
  for (int qt = 0; qt < kw / 16; ++qt) {  // quarters of 16 columns: lane group g takes columns 16 qt + 4 g .. + 3
    double av[4][4], bv[4][4];
    const int kc = kp + 16 * qt + 4 * g;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = ra + i * 16 + i16;
      const doublex4 v = row < m ? *(const doublex4*)(H + (int64_t)row * ldh + kc) : doublex4{0, 0, 0, 0};
#pragma unroll
      for (int e = 0; e < 4; ++e) av[i][e] = v[e];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = rb + j * 16 + i16;
      const doublex4 v = row < m ? *(const doublex4*)(H + (int64_t)row * ldh + kc) : doublex4{0, 0, 0, 0};
#pragma unroll
      for (int e = 0; e < 4; ++e) bv[j][e] = v[e];
    }
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][st], bv[j][st], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = ra + i * 16 + g + 4 * r;
        const int gc = rb + j * 16 + i16;
        if (gr < m && gc < m && gc <= gr) H[(int64_t)gr * ldh + gc] -= acc[i][j][r];
      }
}

// Columns of an outer panel (four inner panels of 64).
constexpr int kCholOuter = 4 * NB;

// The panel chain of one group of problems: each panel step is one launch per kernel for the whole group.
static void cholesky_chain(const CholBatch& b, int64_t ldh, int m, hipStream_t s) {
  const unsigned nz = (unsigned)b.count;
  for (int K0 = 0; K0 < m; K0 += kCholOuter) {
    const int kend = std::min(K0 + kCholOuter, m);
    for (int k0 = K0; k0 < kend; k0 += NB) {
      hipLaunchKernelGGL(k_potrf_diag, dim3(1, 1, nz), dim3(256), 0, s, b, ldh, m, k0);
      SPSVM_LAUNCHED();
      const int rest = m - k0 - NB;
      if (rest <= 0) return;
      const int nblk = (int)ceil_div(rest, NB);
      hipLaunchKernelGGL(k_trsm_panel, dim3(nblk, 1, nz), dim3(256), 0, s, b, ldh, m, k0);
      SPSVM_LAUNCHED();
      const int ct = (int)ceil_div(std::max(kend - k0 - NB, 0), NB);  // tile columns left in the outer panel
      if (ct > 0) {
        hipLaunchKernelGGL(k_chol_update, dim3(nblk * ct, 1, nz), dim3(256), 0, s, b, ldh, m, k0, NB, k0 + NB, ct);
        SPSVM_LAUNCHED();
      }
    }
    const int rest = m - kend;  // the trailing matrix right of the outer panel, all of its columns at once
    if (rest <= 0) return;
    if (rest >= 512 && nz >= 4) {  // many problems: the larger tiles; one problem: more, smaller workgroups
      const int nb2 = (int)ceil_div(rest, 128);
      hipLaunchKernelGGL(k_chol_update128, dim3(nb2 * (nb2 + 1) / 2, 1, nz), dim3(256), 0, s, b, ldh, m, K0,
                         kend - K0, kend);
    } else {
      const int nblk = (int)ceil_div(rest, NB);
      hipLaunchKernelGGL(k_chol_update, dim3(nblk * (nblk + 1) / 2, 1, nz), dim3(256), 0, s, b, ldh, m, K0,
                         kend - K0, kend, 0);
    }
    SPSVM_LAUNCHED();
  }
}

// Side streams for batched factorisations. A panel chain is a sequence of dependent launches whose diagonal-block
// step runs one workgroup per problem, so most of the chip idles during it; a batch is therefore split into up to
// kCholStreams groups whose chains run at the same time on their own streams (default priority), forked from and
// joined back to the caller's stream with events, and each group's diagonal steps overlap the others' updates.
// The streams and events are created once per device and kept until the process ends; the enqueueing is
// serialised by a mutex (a later call may reuse the events once its predecessor's waits are enqueued).
constexpr int kCholStreams = 4;
struct CholStreams {
  hipStream_t st[kCholStreams - 1];
  hipEvent_t fork, join[kCholStreams - 1];
};
static std::mutex g_cs_mu;
static CholStreams* g_cs[256];

static CholStreams* chol_streams_locked() {  // g_cs_mu held
  int dev = 0;
  SPSVM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 256) throw Failure(1, "Cholesky streams: device index out of range");
  if (!g_cs[dev]) {
    CholStreams* c = new CholStreams();
    for (int i = 0; i < kCholStreams - 1; ++i) {
      SPSVM_HIP(hipStreamCreateWithFlags(&c->st[i], hipStreamNonBlocking));
      SPSVM_HIP(hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming));
    }
    SPSVM_HIP(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
    g_cs[dev] = c;
  }
  return g_cs[dev];
}

// All slots share m and ldh. Batches of 8 or more problems run as up to kCholStreams concurrent groups.
void launch_cholesky_batch(const CholBatch& b, int64_t ldh, int m, hipStream_t s) {
  if (b.count <= 0 || m <= 0) return;
  if (b.count > kMaxBatch) throw Failure(1, "Cholesky batch: too many slots");
  const int groups = b.count >= 8 ? std::min(kCholStreams, b.count / 4) : 1;
  if (groups <= 1) {
    cholesky_chain(b, ldh, m, s);
    return;
  }
  std::lock_guard<std::mutex> lock(g_cs_mu);
  CholStreams* cs = chol_streams_locked();
  SPSVM_HIP(hipEventRecord(cs->fork, s));
  for (int g = 0; g < groups; ++g) {
    CholBatch sub{};
    for (int q = g * b.count / groups; q < (g + 1) * b.count / groups; ++q) {
      sub.H[sub.count] = b.H[q];
      sub.Linv[sub.count] = b.Linv[q];
      sub.sc[sub.count] = b.sc[q];
      ++sub.count;
    }
    hipStream_t gs = g == 0 ? s : cs->st[g - 1];
    if (g > 0) SPSVM_HIP(hipStreamWaitEvent(gs, cs->fork, 0));
    cholesky_chain(sub, ldh, m, gs);
    if (g > 0) SPSVM_HIP(hipEventRecord(cs->join[g - 1], gs));
  }
  for (int g = 1; g < groups; ++g) SPSVM_HIP(hipStreamWaitEvent(s, cs->join[g - 1], 0));
}

void launch_cholesky(double* H, int64_t ldh, int m, double* Linv, NewtonScalars* sc, hipStream_t s) {
  CholBatch b{};
  b.H[0] = H;
  b.Linv[0] = Linv;
  b.sc[0] = sc;
  b.count = 1;
  launch_cholesky_batch(b, ldh, m, s);
}

// ----------------------------------------------------------------------------------- triangular solves
// Largest m solved by one workgroup per problem: z and x (16 m bytes of LDS) plus the partial sums fit in 64 KB.
constexpr int kSolveOneMax = 3328;

// One workgroup of 1024 threads. Forward: z_b = Linv_b (g_b - L[b, <b] z_<b); backward:
// x_b = Linv_b^T (z_b - L[>b, b]^T x_>b); the result is negated (x = -H^{-1} g).
__global__ __launch_bounds__(1024) void k_chol_solve(const SolveBatch bt, int64_t ldh, int m) {
  const double* __restrict__ L = bt.L[blockIdx.z];
  const double* __restrict__ Linv = bt.Linv[blockIdx.z];
  const double* __restrict__ g = bt.g[blockIdx.z];
  double* __restrict__ x = bt.x[blockIdx.z];
  __shared__ double part[16][NB];
  __shared__ double rhs[NB];
  extern __shared__ double zx[];  // z = L^-1 g and x = L^-T z stay in LDS: 2 m doubles (m <= kSolveOneMax)
  double* zs = zx;
  double* xs = zx + m;
  const int tid = threadIdx.x;
  const int nblk = (int)((m + NB - 1) / NB);
  // forward; the inner sums keep their order (unrolled so that several rows' loads are in flight)
  for (int b = 0; b < nblk; ++b) {
    const int b0 = b * NB;
    const int r = tid >> 4, p0 = tid & 15;
    double s = 0.0;
    if (b0 + r < m) {
      const double* __restrict__ Lr = L + (int64_t)(b0 + r) * ldh;
#pragma unroll 8
      for (int p = p0; p < b0; p += 16) s += Lr[p] * zs[p];
    }
    part[p0][r] = s;
    __syncthreads();
    if (tid < NB) {
      double t = 0.0;
      for (int q = 0; q < 16; ++q) t += part[q][tid];
      rhs[tid] = (b0 + tid < m) ? g[b0 + tid] - t : 0.0;
    }
    __syncthreads();
    if (tid < NB && b0 + tid < m) {
      const double* __restrict__ Lo = Linv + (int64_t)b * NB * NB + (int64_t)tid * NB;
      double t = 0.0;
#pragma unroll 8
      for (int p = 0; p <= tid; ++p) t += Lo[p] * rhs[p];
      zs[b0 + tid] = t;
    }
    __syncthreads();
  }
  // backward
  for (int b = nblk - 1; b >= 0; --b) {
    const int b0 = b * NB;
    const int c = tid & 63, p0 = tid >> 6;
    double s = 0.0;
    if (b0 + c < m) {
#pragma unroll 8
      for (int i = b0 + NB + p0; i < m; i += 16) s += L[(int64_t)i * ldh + b0 + c] * xs[i];
    }
    part[p0][c] = s;
    __syncthreads();
    if (tid < NB) {
      double t = 0.0;
      for (int q = 0; q < 16; ++q) t += part[q][tid];
      rhs[tid] = (b0 + tid < m) ? zs[b0 + tid] - t : 0.0;
    }
    __syncthreads();
    if (tid < NB && b0 + tid < m) {
      const double* __restrict__ Lo = Linv + (int64_t)b * NB * NB;
      double t = 0.0;
#pragma unroll 8
      for (int p = tid; p < NB; ++p) t += Lo[(int64_t)p * NB + tid] * rhs[p];
      xs[b0 + tid] = t;
    }
    __syncthreads();
  }
  for (int k = tid; k < m; k += 1024) x[k] = -xs[k];
}

// m > kSolveOneMax: one launch per 64-row block step, the remaining blocks updated in parallel (right-looking).
// Forward, step b: every workgroup forms z_b = Linv_b r_b (r: right-hand side, held in x); the one for
// block b stores z_b, the others update their own block r_rb -= L[rb, b] z_b. Backward, step b: every
// workgroup forms x_b = Linv_b^T z_b; the one for block b stores -x_b, the others update z_rb -= L[b, rb]^T x_b.
// Right-hand side blocks are read only in their own step and written only by their own workgroup.
__global__ __launch_bounds__(64) void k_solve_copy(const SolveBatch bt, int m) {
  const double* g = bt.g[blockIdx.z];
  double* x = bt.x[blockIdx.z];
  for (int k = blockIdx.x * 64 + threadIdx.x; k < m; k += gridDim.x * 64) x[k] = g[k];
}

__global__ __launch_bounds__(256) void k_trsv_fwd(const SolveBatch bt, int64_t ldh, int m, int b) {
  const int rb = b + blockIdx.x;
  const int b0 = b * NB, r0 = rb * NB;
  if (r0 >= m) return;
  const double* __restrict__ L = bt.L[blockIdx.z];
  const double* __restrict__ Lo = bt.Linv[blockIdx.z] + (int64_t)b * NB * NB;
  double* __restrict__ r = bt.x[blockIdx.z];
  double* __restrict__ z = bt.work[blockIdx.z];
  __shared__ double zb[NB];
  __shared__ double rhs[NB];
  const int t = threadIdx.x;
  if (t < NB) rhs[t] = b0 + t < m ? r[b0 + t] : 0.0;
  __syncthreads();
  if (t < NB) {
    double a = 0.0;
    const double* row = Lo + (int64_t)t * NB;
    for (int p = 0; p <= t; ++p) a += row[p] * rhs[p];
    zb[t] = a;
  }
  __syncthreads();
  if (rb == b) {
    if (t < NB && b0 + t < m) z[b0 + t] = zb[t];
    return;
  }
  // rows r0 + i, four threads per row, sixteen columns each
  const int i = t >> 2, q = t & 3;
  double a = 0.0;
  if (r0 + i < m) {
    const double* row = L + (int64_t)(r0 + i) * ldh + b0;
#pragma unroll
    for (int p = q * 16; p < q * 16 + 16; ++p) a += (b0 + p < m ? row[p] : 0.0) * zb[p];
  }
  a += __shfl_xor(a, 1, kWave);
  a += __shfl_xor(a, 2, kWave);
  if (q == 0 && r0 + i < m) r[r0 + i] -= a;
}

__global__ __launch_bounds__(256) void k_trsv_bwd(const SolveBatch bt, int64_t ldh, int m, int b) {
  const int rb = blockIdx.x;  // 0 .. b
  const int b0 = b * NB, r0 = rb * NB;
  const double* __restrict__ L = bt.L[blockIdx.z];
  const double* __restrict__ Lo = bt.Linv[blockIdx.z] + (int64_t)b * NB * NB;
  double* __restrict__ z = bt.work[blockIdx.z];
  double* __restrict__ x = bt.x[blockIdx.z];
  __shared__ double xb[NB];
  __shared__ double rhs[NB];
  __shared__ double part[4][NB];
  const int t = threadIdx.x;
  if (t < NB) rhs[t] = b0 + t < m ? z[b0 + t] : 0.0;
  __syncthreads();
  if (t < NB) {
    double a = 0.0;
    for (int p = t; p < NB; ++p) a += Lo[(int64_t)p * NB + t] * rhs[p];
    xb[t] = a;
  }
  __syncthreads();
  if (rb == b) {
    if (t < NB && b0 + t < m) x[b0 + t] = -xb[t];
    return;
  }
  // columns r0 + j of L's rows b0 + i: thread (q, j) sums rows i = q, q + 4, ...
  const int j = t & 63, q = t >> 6;
  double a = 0.0;
  for (int i = q; i < NB; i += 4)
    if (b0 + i < m) a += L[(int64_t)(b0 + i) * ldh + r0 + j] * xb[i];
  part[q][j] = a;
  __syncthreads();
  if (t < NB) z[r0 + t] -= part[0][t] + part[1][t] + part[2][t] + part[3][t];
}

void launch_chol_solve_batch(const SolveBatch& b, int64_t ldh, int m, hipStream_t s) {
  if (b.count <= 0 || m <= 0) return;
  if (b.count > kMaxBatch) throw Failure(1, "solve batch: too many slots");
  const unsigned nz = (unsigned)b.count;
  if (m <= kSolveOneMax) {  // one workgroup per problem: no launch per block step
    hipLaunchKernelGGL(k_chol_solve, dim3(1, 1, nz), dim3(1024), (size_t)2 * m * sizeof(double), s, b, ldh, m);
    SPSVM_LAUNCHED();
    return;
  }
  const int nb = (int)ceil_div(m, NB);
  hipLaunchKernelGGL(k_solve_copy, dim3((unsigned)std::min<int64_t>(ceil_div(m, 64), 64), 1, nz), dim3(64), 0, s, b, m);
  SPSVM_LAUNCHED();
  for (int k = 0; k < nb; ++k) {
    hipLaunchKernelGGL(k_trsv_fwd, dim3((unsigned)(nb - k), 1, nz), dim3(256), 0, s, b, ldh, m, k);
    SPSVM_LAUNCHED();
  }
  for (int k = nb - 1; k >= 0; --k) {
    hipLaunchKernelGGL(k_trsv_bwd, dim3((unsigned)(k + 1), 1, nz), dim3(256), 0, s, b, ldh, m, k);
    SPSVM_LAUNCHED();
  }
}

void launch_chol_solve(const double* L, int64_t ldh, int m, const double* Linv, const double* g, double* x,
                       double* work, hipStream_t s) {
  SolveBatch b{};
  b.L[0] = L;
  b.Linv[0] = Linv;
  b.g[0] = g;
  b.x[0] = x;
  b.work[0] = work;
  b.count = 1;
  launch_chol_solve_batch(b, ldh, m, s);
}


// ------------------------------------------------------------------------ allocation-free Newton solve
// The scratch of one Newton solve (the inverses of L's 64 x 64 diagonal blocks, the forward-solve vector and the
// status scalars) for systems up to kNoAllocMaxM, in a static device array: each GPU the library runs on holds its
// own copy (2.1 MiB) until the process ends. Host code never uses the array's name as an address: the pointer
// comes from hipGetSymbolAddress, once per device, with that device current. Calls that overlap on one GPU share
// the array and race.
constexpr int kNoAllocMaxM = 4096;
constexpr size_t kNoAllocLinv = (size_t)(kNoAllocMaxM / kCholNB) * kCholNB * kCholNB * sizeof(double);
constexpr size_t kNoAllocZ = (size_t)kNoAllocMaxM * sizeof(double);
constexpr size_t kNoAllocBytes = kNoAllocLinv + kNoAllocZ + 256;
static_assert(sizeof(NewtonScalars) <= 256, "status scalars fit the scratch tail");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_at[256];  // device address of `scratch` per device index

static char* scratch_for_current_device() {
  int dev = 0;
  SPSVM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 256) throw Failure(3, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* ptr = nullptr;
    SPSVM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw Failure(3, "hipGetSymbolAddress returned a null address for the scratch array");
    g_scratch_at[dev] = ptr;
  }
  return (char*)g_scratch_at[dev];
}

__global__ void k_clear_fail(NewtonScalars* sc) {
  if (threadIdx.x == 0) sc->fail = 0;
}

int newton_solve_noalloc_max() { return kNoAllocMaxM; }

void newton_solve_noalloc(double* H, int64_t ldh, int m, const double* g, double* x, hipStream_t st) {
  if (m < 1 || m > kNoAllocMaxM)
    throw Failure(1, "m = " + std::to_string(m) + " is outside [1, " + std::to_string(kNoAllocMaxM) +
                         "], the largest system the allocation-free solve's static scratch holds");
  char* base = scratch_for_current_device();
  double* Linv = (double*)base;
  double* z = (double*)(base + kNoAllocLinv);
  NewtonScalars* sc = (NewtonScalars*)(base + kNoAllocLinv + kNoAllocZ);
  hipLaunchKernelGGL(k_clear_fail, dim3(1), dim3(64), 0, st, sc);  // the last call's flag stays in the array
  SPSVM_LAUNCHED();
  launch_cholesky(H, ldh, m, Linv, sc, st);
  launch_chol_solve(H, ldh, m, Linv, g, x, z, st);
  int32_t fl = 0;
  SPSVM_HIP(hipMemcpyAsync(&fl, &sc->fail, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SPSVM_HIP(hipStreamSynchronize(st));
  if (fl) throw Failure(4, "Cholesky met a non-positive or non-finite pivot");
}

}  // namespace spsvm
