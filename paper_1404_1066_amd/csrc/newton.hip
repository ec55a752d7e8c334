// Newton re-optimisation of Eq. 4 on a fixed basis J (section 4, "Sparse primal optimization"; Newton's
// method on the squared-hinge primal of section 4, "Primal optimization"):
//   f(beta) = lambda/2 beta^T K_JJ beta + 1/2 sum_i max(0, a_i)^2,  a_i = 1 - y_i o_i,  o = K_XJ beta,
//   grad f  = lambda K_JJ beta + K_I^T (o_I - y_I),     H = lambda K_JJ + K_I^T K_I,   I = {i : a_i > 0}.
// K_JJ is kept as its own FP64 matrix (computed from the basis rows), so the regulariser stays positive
// definite whatever precision the n x |J| block K_XJ is stored in.
// Kernels: GEMV o = K_XJ x (one wave per row), violator compaction (wave ballot + block prefix sums),
// gradient (GEMV^T over the compacted rows), the SYRK of H over the compacted rows with MFMA, and the
// exact line search along d (bracketed semismooth Newton on the piecewise-linear derivative).
// All reductions run in a fixed order, so results are bitwise reproducible.
#include "common.h"
#include "launch.h"

namespace spsvm {

// ------------------------------------------------------------------------------------------------ GEMV
template <typename TK>
__global__ __launch_bounds__(256) void k_gemv(const TK* __restrict__ K, int64_t ldk, int64_t n, int m,
                                              const double* __restrict__ x, double* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= n) return;
  const TK* k = K + row * ldk;
  double s = 0.0;
  for (int j = lane; j < m; j += kWave) s += (double)k[j] * x[j];
  s = wave_sum(s);
  if (lane == 0) out[row] = s;
}

template <typename TK>
void launch_gemv(const TK* K, int64_t ldk, int64_t n, int m, const double* x, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_gemv<TK>), dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, s, K, ldk, n, m, x, out);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------------------------------ compaction
constexpr int kCompactRows = 4096;  // rows per block: 16 chunks of 256

// a_i = 1 - y_i o_i with explicit rounding (no contraction), so every kernel draws the same I.
__device__ __forceinline__ double margin_gap(float y, double o) { return __dadd_rn(1.0, -__dmul_rn((double)y, o)); }

__global__ __launch_bounds__(256) void k_compact_count(const double* __restrict__ o, const float* __restrict__ y,
                                                       int64_t n, const uint8_t* __restrict__ act_ref,
                                                       int32_t* __restrict__ cnt, double* __restrict__ bsum,
                                                       int32_t* __restrict__ bflips) {
  __shared__ double rd[4];
  __shared__ int ri[4];
  const int64_t lo = (int64_t)blockIdx.x * kCompactRows;
  int c = 0, fl = 0;
  double s = 0.0;
  for (int j = 0; j < kCompactRows / 256; ++j) {
    const int64_t i = lo + j * 256 + threadIdx.x;
    if (i < n) {
      const double a = margin_gap(y[i], o[i]);
      const int v = a > 0.0;
      c += v;
      if (v) s += a * a;
      if (act_ref) fl += (v != (int)act_ref[i]);
    }
  }
  c = block_sum_int(c, ri);
  fl = block_sum_int(fl, ri);
  s = block_sum(s, rd);
  if (threadIdx.x == 0) {
    cnt[blockIdx.x] = c;
    bsum[blockIdx.x] = s;
    bflips[blockIdx.x] = fl;
  }
}

__global__ __launch_bounds__(256) void k_compact_write(const double* __restrict__ o, const float* __restrict__ y,
                                                       int64_t n, const int32_t* __restrict__ cnt,
                                                       const double* __restrict__ bsum,
                                                       const int32_t* __restrict__ bflips, int nblk,
                                                       uint8_t* __restrict__ act_out, int32_t* __restrict__ I,
                                                       NewtonScalars* sc) {
  __shared__ int ri[4];
  __shared__ int wc[4];
  int part = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += 256) part += cnt[b];
  int offset = block_sum_int(part, ri);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t lo = (int64_t)blockIdx.x * kCompactRows;
  for (int j = 0; j < kCompactRows / 256; ++j) {
    const int64_t i = lo + j * 256 + threadIdx.x;
    int v = 0;
    if (i < n) {
      v = margin_gap(y[i], o[i]) > 0.0;
      act_out[i] = (uint8_t)v;
    }
    const unsigned long long mask = __ballot(v);
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wc[w] = __popcll(mask);
    __syncthreads();
    int base = offset;
    for (int q = 0; q < w; ++q) base += wc[q];
    if (v) I[base + rank] = (int32_t)i;
    offset += wc[0] + wc[1] + wc[2] + wc[3];
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int tot = 0, fl = 0;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) {
      tot += cnt[b];
      fl += bflips[b];
      s += bsum[b];
    }
    sc->n_sv = tot;
    sc->flips = fl;
    sc->sum_a2 = s;
  }
}

int compact_blocks(int64_t n) { return (int)std::max<int64_t>(1, ceil_div(n, kCompactRows)); }

void launch_compact(const double* o, const float* y, int64_t n, const uint8_t* act_ref, uint8_t* act_out, int32_t* I,
                    int32_t* blk_count, double* blk_sum, int32_t* blk_flips, NewtonScalars* sc, hipStream_t s) {
  const int nblk = compact_blocks(n);
  hipLaunchKernelGGL(k_compact_count, dim3(nblk), dim3(256), 0, s, o, y, n, act_ref, blk_count, blk_sum, blk_flips);
  SPSVM_LAUNCHED();
  hipLaunchKernelGGL(k_compact_write, dim3(nblk), dim3(256), 0, s, o, y, n, blk_count, blk_sum, blk_flips, nblk,
                     act_out, I, sc);
  SPSVM_LAUNCHED();
}

// -------------------------------------------------------------------------------------------- gradient
template <typename TK>
__global__ __launch_bounds__(256) void k_grad_partial(const TK* __restrict__ K, int64_t ldk, int m,
                                                      const int32_t* __restrict__ I, int n_sv, int rows_per_chunk,
                                                      const double* __restrict__ o, const float* __restrict__ y,
                                                      double* __restrict__ partial) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  const int lo = blockIdx.y * rows_per_chunk;
  const int hi = lo + rows_per_chunk < n_sv ? lo + rows_per_chunk : n_sv;
  if (k >= m) return;
  double acc = 0.0;
  for (int r = lo; r < hi; ++r) {
    const int64_t i = I[r];
    acc += (double)K[i * ldk + k] * (o[i] - (double)y[i]);
  }
  partial[(int64_t)blockIdx.y * m + k] = acc;
}

// g = lambda v + sum of the chunk partials, with v = K_JJ beta; also |g|^2 and beta . v = beta^T K_JJ beta.
__global__ __launch_bounds__(1024) void k_grad_finish(int m, const double* __restrict__ partial, int nchunk,
                                                      const double* __restrict__ v, const double* __restrict__ beta,
                                                      double lam, double* __restrict__ g, NewtonScalars* sc) {
  __shared__ double rd[16];
  double gn = 0.0, bo = 0.0;
  for (int k = threadIdx.x; k < m; k += 1024) {
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += partial[(int64_t)c * m + k];
    s += lam * v[k];
    g[k] = s;
    gn += s * s;
    bo += beta[k] * v[k];
  }
  gn = block_sum(gn, rd);
  bo = block_sum(bo, rd);
  if (threadIdx.x == 0) {
    sc->gnorm2 = gn;
    sc->beta_oJ = bo;
  }
}

int gradient_chunks(int m, int n_sv) {
  const int colblocks = (int)ceil_div(std::max(m, 1), 256);
  int c = std::max(1, 1024 / colblocks);
  c = std::min<int>(c, (int)std::max<int64_t>(1, ceil_div(n_sv, 64)));
  return c;
}

template <typename TK>
void launch_gradient(const TK* K, int64_t ldk, int m, const int32_t* I, int n_sv, const double* o, const float* y,
                     const double* v, const double* beta, double lam, double* partial, int nchunk, double* g,
                     NewtonScalars* sc, hipStream_t s) {
  const int rows = (int)std::max<int64_t>(1, ceil_div(n_sv, nchunk));
  hipLaunchKernelGGL((k_grad_partial<TK>), dim3((unsigned)ceil_div(m, 256), nchunk), dim3(256), 0, s, K, ldk, m, I,
                     n_sv, rows, o, y, partial);
  SPSVM_LAUNCHED();
  hipLaunchKernelGGL(k_grad_finish, dim3(1), dim3(1024), 0, s, m, partial, nchunk, v, beta, lam, g, sc);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------------------------------------ SYRK
// Partial H tiles over a range of violator rows: P[split][tile] = sum_{r in split} K[I_r, T_r]^T K[I_r, T_c]
// for the lower tiles (T_r >= T_c) of 64 x 64. Rows are staged 32 at a time, converted to FP64 and
// transposed into LDS so that each MFMA operand fetch is a 4-wide read along the row index (the contraction
// dimension). The products run on FP64 MFMA: a product of two FP32 values is exact in FP64, so the Gram
// part of H is accumulated to FP64 accuracy and stays positive semi-definite even when the basis columns are
// nearly dependent (FP32 accumulation loses that).
constexpr int SY_T = 64, SY_BK = 32, SY_LD = SY_BK + 4;

__device__ __forceinline__ void tile_of(int t, int& tr, int& tc) {
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  tr = r;
  tc = t - r * (r + 1) / 2;
}

template <typename TK>
__global__ __launch_bounds__(256) void k_syrk(const TK* __restrict__ K, int64_t ldk, int m,
                                              const int32_t* __restrict__ I, int n_sv, int rows_per_split, int ntiles,
                                              double* __restrict__ partial) {
  __shared__ __attribute__((aligned(32))) double At[SY_T][SY_LD];
  __shared__ __attribute__((aligned(32))) double Bt[SY_T][SY_LD];
  int tr, tc;
  tile_of(blockIdx.x, tr, tc);
  const bool diag = tr == tc;
  const int lo = blockIdx.y * rows_per_split;
  const int hi = lo + rows_per_split < n_sv ? lo + rows_per_split : n_sv;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, i16 = lane & 15;
  const int wr = w >> 1, wc = w & 1;
  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0, 0, 0, 0};
  const int ca = tr * SY_T, cb = tc * SY_T;
  for (int r0 = lo; r0 < hi; r0 += SY_BK) {
    double va[8], vb[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid + e * 256, rr = idx >> 6, cc = idx & 63;
      const int rrow = r0 + rr;
      const int64_t row = rrow < hi ? (int64_t)I[rrow] : -1;
      va[e] = (row >= 0 && ca + cc < m) ? (double)K[row * ldk + ca + cc] : 0.0;
      vb[e] = (!diag && row >= 0 && cb + cc < m) ? (double)K[row * ldk + cb + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid + e * 256, rr = idx >> 6, cc = idx & 63;
      At[cc][rr] = va[e];
      if (!diag) Bt[cc][rr] = vb[e];
    }
    __syncthreads();
    double(*Bp)[SY_LD] = diag ? At : Bt;
#pragma unroll
    for (int kk = 0; kk < SY_BK; kk += 16) {
      doublex4 av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = *(const doublex4*)&At[wr * 32 + i * 16 + i16][kk + 4 * g];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = *(const doublex4*)&Bp[wc * 32 + j * 16 + i16][kk + 4 * g];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][s], bv[j][s], acc[i][j], 0, 0, 0);
    }
  }
  double* out = partial + ((int64_t)blockIdx.y * ntiles + blockIdx.x) * (SY_T * SY_T);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = wr * 32 + i * 16 + (lane >> 4) + 4 * r, cc = wc * 32 + j * 16 + i16;
        out[rr * SY_T + cc] = acc[i][j][r];
      }
}

int syrk_tiles(int m) {
  const int t = (int)ceil_div(m, SY_T);
  return t * (t + 1) / 2;
}

int syrk_splits(int m, int n_sv) {
  const int nt = syrk_tiles(m);
  int s = (int)ceil_div(1024, nt);
  s = std::min<int>(s, (int)std::max<int64_t>(1, ceil_div(n_sv, 256)));
  return std::max(1, std::min(s, 64));
}

size_t syrk_partial_doubles(int m_max) {
  size_t best = 0;
  // the split count only shrinks as m grows, so the bound over m <= m_max is reached at some tile count
  for (int t = 1; t <= ceil_div(std::max(m_max, 1), SY_T); ++t) {
    const int nt = t * (t + 1) / 2;
    const int s = std::max(1, std::min<int>((int)ceil_div(1024, nt), 64));
    best = std::max(best, (size_t)s * nt * SY_T * SY_T);
  }
  return best;
}

template <typename TK>
void launch_syrk(const TK* K, int64_t ldk, int m, const int32_t* I, int n_sv, int nsplit, double* partial,
                 hipStream_t s) {
  const int nt = syrk_tiles(m);
  const int rows = (int)std::max<int64_t>(1, ceil_div(n_sv, nsplit));
  hipLaunchKernelGGL((k_syrk<TK>), dim3(nt, nsplit), dim3(256), 0, s, K, ldk, m, I, n_sv, rows, nt, partial);
  SPSVM_LAUNCHED();
}

// H (lower triangle) = lambda K_JJ + sum of the split partials (+ diag_add on the diagonal); K_JJ is the FP64
// kernel matrix of the basis rows (row-major, leading dimension ldh).
__global__ __launch_bounds__(256) void k_syrk_reduce(const double* __restrict__ KJJ, int m, double lam,
                                                     const double* __restrict__ partial, int nsplit, int ntiles,
                                                     double diag_add, double* __restrict__ H, int64_t ldh) {
  int tr, tc;
  tile_of(blockIdx.x, tr, tc);
  for (int e = 0; e < 16; ++e) {
    const int idx = threadIdx.x + e * 256, r = idx >> 6, c = idx & 63;
    const int gr = tr * SY_T + r, gc = tc * SY_T + c;
    if (gr >= m || gc >= m || gc > gr) continue;
    double s = lam * KJJ[(int64_t)gr * ldh + gc];
    for (int p = 0; p < nsplit; ++p) s += partial[((int64_t)p * ntiles + blockIdx.x) * (SY_T * SY_T) + idx];
    if (gr == gc) s += diag_add;
    H[(int64_t)gr * ldh + gc] = s;
  }
}

void launch_syrk_reduce(const double* KJJ, int m, double lam, const double* partial, int nsplit, double diag_add,
                        double* H, int64_t ldh, hipStream_t s) {
  const int nt = syrk_tiles(m);
  hipLaunchKernelGGL(k_syrk_reduce, dim3(nt), dim3(256), 0, s, KJJ, m, lam, partial, nsplit, nt, diag_add, H, ldh);
  SPSVM_LAUNCHED();
}

__global__ __launch_bounds__(256) void k_trace(const double* __restrict__ H, int64_t ldh, int m, NewtonScalars* sc) {
  __shared__ double rd[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < m; k += 256) s += H[(int64_t)k * ldh + k];
  s = block_sum(s, rd);
  if (threadIdx.x == 0) sc->trace = s;
}

void launch_trace(const double* H, int64_t ldh, int m, NewtonScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, s, H, ldh, m, sc);
  SPSVM_LAUNCHED();
}

// ---------------------------------------------------------------------------------------- line search
// phi(t) = f(beta + t d) = const + lambda (t c1 + t^2 c2 / 2) + 1/2 sum max(0, a_i - t b_i)^2,
// a_i = 1 - y_i o_i, b_i = y_i delta_i, delta = K_XJ d, c1 = beta^T K_JJ d, c2 = d^T K_JJ d (from w = K_JJ d).
__global__ __launch_bounds__(256) void k_c1c2(const double* __restrict__ beta, const double* __restrict__ dvec,
                                              const double* __restrict__ w, int m, LineState* ls) {
  __shared__ double rd[4];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < m; k += 256) {
    a += beta[k] * w[k];
    b += dvec[k] * w[k];
  }
  a = block_sum(a, rd);
  b = block_sum(b, rd);
  if (threadIdx.x == 0) {
    LineState s;
    s.c1 = a;
    s.c2 = b;
    s.t = 1.0;
    s.t_prev = 0.0;
    s.lo = 0.0;
    s.hi = __builtin_huge_val();
    s.dec = 0.0;
    s.status = 0;
    s.newton = 0;
    s.passes = 0;
    s.pad = 0;
    *ls = s;
  }
}

void launch_c1c2(const double* beta, const double* dvec, const double* w, int m, LineState* ls, hipStream_t s) {
  hipLaunchKernelGGL(k_c1c2, dim3(1), dim3(256), 0, s, beta, dvec, w, m, ls);
  SPSVM_LAUNCHED();
}

// Pass 0 evaluates t = 0 and t = 1 (slots A and B); later passes evaluate t (slot B) with flips against t_prev.
// Partial record per block: {P_A, Q_A, P_B, Q_B, V_B, flips}.
__global__ __launch_bounds__(256) void k_ls_pass(const double* __restrict__ o, const double* __restrict__ delta,
                                                 const float* __restrict__ y, int64_t n, int64_t rows_per_blk,
                                                 const LineState* __restrict__ ls, double* __restrict__ partial) {
  __shared__ double rd[4];
  if (ls->status != 0) return;
  const bool first = ls->passes == 0;
  const double t = ls->t, tp = ls->t_prev;
  const int64_t lo = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t hi = lo + rows_per_blk < n ? lo + rows_per_blk : n;
  double pa = 0.0, qa = 0.0, pb = 0.0, qb = 0.0, vb = 0.0;
  int fl = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const double yi = (double)y[i];
    const double a = 1.0 - yi * o[i];
    const double b = yi * delta[i];
    const double ep = a - tp * b, e = a - t * b;
    if (first && ep > 0.0) {
      pa += a * b;
      qa += b * b;
    }
    if (e > 0.0) {
      pb += a * b;
      qb += b * b;
    }
    const double u = fmax(a, 0.0), w = fmax(e, 0.0);
    vb += (w - u) * (w + u);
    fl += ((e > 0.0) != (ep > 0.0)) ? 1 : 0;
  }
  double v[6] = {pa, qa, pb, qb, vb, (double)fl};
  for (int k = 0; k < 6; ++k) {
    const double r = block_sum(v[k], rd);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * 6 + k] = r;
  }
}

__global__ void k_ls_update(LineState* ls, const double* __restrict__ partial, int nblk, double lam) {
  if (threadIdx.x != 0) return;
  LineState s = *ls;
  if (s.status != 0) return;
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int b = 0; b < nblk; ++b)
    for (int k = 0; k < 6; ++k) v[k] += partial[(int64_t)b * 6 + k];
  const double P = v[2], Q = v[3], V = v[4], F = v[5];
  const double lc1 = lam * s.c1, lc2 = lam * s.c2;
  bool done = false;
  if (s.passes == 0) {
    const double P0 = v[0], Q0 = v[1];
    s.passes = 1;
    const double g0 = lc1 - P0;
    if (g0 >= 0.0) {  // no descent along d
      s.t = 0.0;
      s.dec = 0.0;
      s.status = 1;
      *ls = s;
      return;
    }
    if (F == 0.0) {  // active set constant on [0, 1]: phi' is one linear piece there
      const double r = (P0 - lc1) / (lc2 + Q0);
      if (r >= 0.0 && r <= 1.0) {
        s.t = r;
        s.dec = -(r * lc1 + 0.5 * r * r * lc2) + r * P0 - 0.5 * r * r * Q0;
        s.status = 1;
        *ls = s;
        return;
      }
    }
    const double g1 = lc1 + lc2 - (P - Q);
    if (g1 < 0.0)
      s.lo = 1.0;
    else
      s.hi = 1.0;
    const double r1 = (P - lc1) / (lc2 + Q);
    const double r0 = (P0 - lc1) / (lc2 + Q0);
    if (r1 > s.lo && r1 < s.hi) {
      s.t_prev = 1.0;
      s.t = r1;
      s.newton = 1;
    } else if (r0 > s.lo && r0 < s.hi) {
      s.t_prev = 0.0;
      s.t = r0;
      s.newton = 1;
    } else {
      s.t_prev = 1.0;
      s.newton = 0;
      s.t = s.hi < __builtin_huge_val() ? 0.5 * (s.lo + s.hi) : s.lo + fmax(1.0, s.lo);
    }
    *ls = s;
    return;
  }
  s.passes += 1;
  const double g = lc1 + s.t * lc2 - (P - s.t * Q);
  done = (s.newton && F == 0.0) || g == 0.0;
  if (!done) {
    if (g < 0.0)
      s.lo = s.t;
    else
      s.hi = s.t;
    const double r = (P - lc1) / (lc2 + Q);
    double nx;
    int nw;
    if (r > s.lo && r < s.hi) {
      nx = r;
      nw = 1;
    } else {
      nw = 0;
      nx = s.hi < __builtin_huge_val() ? 0.5 * (s.lo + s.hi) : s.lo + fmax(1.0, s.lo);
    }
    if (nx > s.lo && nx < s.hi && s.passes < 64) {
      s.t_prev = s.t;
      s.t = nx;
      s.newton = nw;
    } else {
      done = true;
    }
  }
  if (done) {
    s.status = 1;
    s.dec = -(s.t * lc1 + 0.5 * s.t * s.t * lc2) - 0.5 * V;
  }
  *ls = s;
}

void launch_ls_round(const double* o, const double* delta, const float* y, int64_t n, double lam, LineState* ls,
                     double* partial, int nblk, hipStream_t s) {
  const int64_t rows = ceil_div(n, nblk);
  hipLaunchKernelGGL(k_ls_pass, dim3(nblk), dim3(256), 0, s, o, delta, y, n, rows, ls, partial);
  SPSVM_LAUNCHED();
  hipLaunchKernelGGL(k_ls_update, dim3(1), dim3(64), 0, s, ls, partial, nblk, lam);
  SPSVM_LAUNCHED();
}

__global__ __launch_bounds__(256) void k_apply_step(const LineState* __restrict__ ls, double* __restrict__ beta,
                                                    const double* __restrict__ dvec, int m, double* __restrict__ o,
                                                    const double* __restrict__ delta, int64_t n) {
  const double t = ls->t;
  if (t == 0.0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) o[i] += t * delta[i];
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += stride) beta[k] += t * dvec[k];
}

void launch_apply_step(const LineState* ls, double* beta, const double* dvec, int m, double* o, const double* delta,
                       int64_t n, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(ceil_div(std::max<int64_t>(n, m), 256), 2048);
  hipLaunchKernelGGL(k_apply_step, dim3((unsigned)blocks), dim3(256), 0, s, ls, beta, dvec, m, o, delta, n);
  SPSVM_LAUNCHED();
}

__global__ void k_scale(double* v, int m, double a) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < m; k += gridDim.x * blockDim.x) v[k] *= a;
}
void launch_scale(double* v, int m, double a, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(m, 256), 64))),
                     dim3(256), 0, s, v, m, a);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------------------------ instantiations
template void launch_gemv<float>(const float*, int64_t, int64_t, int, const double*, double*, hipStream_t);
template void launch_gemv<double>(const double*, int64_t, int64_t, int, const double*, double*, hipStream_t);
template void launch_gradient<float>(const float*, int64_t, int, const int32_t*, int, const double*, const float*,
                                     const double*, const double*, double, double*, int, double*, NewtonScalars*,
                                     hipStream_t);
template void launch_gradient<double>(const double*, int64_t, int, const int32_t*, int, const double*, const float*,
                                      const double*, const double*, double, double*, int, double*, NewtonScalars*,
                                      hipStream_t);
template void launch_syrk<float>(const float*, int64_t, int, const int32_t*, int, int, double*, hipStream_t);
template void launch_syrk<double>(const double*, int64_t, int, const int32_t*, int, int, double*, hipStream_t);

}  // namespace spsvm
