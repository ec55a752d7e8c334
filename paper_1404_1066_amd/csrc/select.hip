// Greedy basis selection (section 4, "Sparse primal optimization": score a random candidate subset by the
// loss reduction each candidate would bring, add the best to J).
//
// Score of candidate c (row x_c, kernel column k = K(X, x_c)): the exact decrease of
//   f(beta) = lambda/2 beta^T K_JJ beta + 1/2 sum_i max(0, 1 - y_i o_i)^2
// when only the new coefficient s is optimised:
//   psi(s) - f = lambda (s o_c + s^2/2) + 1/2 sum_i [max(0, a_i - s b_i)^2 - max(0, a_i)^2],
//   a_i = 1 - y_i o_i, b_i = y_i k_i.
// psi' is continuous, increasing and piecewise linear. Each pass over the n rows evaluates, for all 64
// candidate slots at once, the sums P = sum_A a_i b_i, Q = sum_A b_i^2 over the active set A(s) = {a_i - s b_i > 0},
// the value sum V, and the number of rows whose activity differs from the previous point. The update then
// takes the Newton root of the current linear piece, (P - lambda o_c) / (lambda + Q), inside a bracket of the
// root (bisection when it falls outside). When a Newton root has the same active set as the point it came
// from, psi' is linear between them and the root is exact.
#include "common.h"
#include "launch.h"

namespace spsvm {

__device__ __forceinline__ bool hash_in(uint64_t h, const uint64_t* __restrict__ list, int cnt) {
  for (int q = 0; q < cnt; ++q)
    if (list[q] == h) return true;
  return false;
}

// 64 threads: one per slot.
__global__ void k_score_init(const int32_t* __restrict__ cand, const double* __restrict__ o,
                             const uint64_t* __restrict__ hash, const uint64_t* __restrict__ stage_hash, int n_stage,
                             CandState* __restrict__ st, NewtonScalars* sc) {
  __shared__ int red[1];
  const int c = threadIdx.x;
  CandState s;
  s.idx = cand[c];
  s.s = 0.0;
  s.s_prev = 0.0;
  s.lo = -__builtin_huge_val();
  s.hi = __builtin_huge_val();
  s.oc = 0.0;
  s.score = -__builtin_huge_val();
  s.newton = 0;
  s.passes = 0;
  if (s.idx < 0 || hash_in(hash[s.idx], stage_hash, n_stage)) {
    s.status = 2;
  } else {
    s.status = 0;
    s.oc = o[s.idx];
  }
  st[c] = s;
  const int na = block_sum_int(s.status == 0 ? 1 : 0, red);
  if (c == 0) sc->n_active_sel = na;
}

void launch_score_init(const int32_t* cand, const double* o, const uint64_t* hash, const uint64_t* stage_hash,
                       int n_stage, CandState* st, NewtonScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_score_init, dim3(1), dim3(kCandSlots), 0, s, cand, o, hash, stage_hash, n_stage, st, sc);
  SPSVM_LAUNCHED();
}

// One pass: thread (wave q, lane c) handles slot c on rows lo + q, lo + q + 4, ... of this block's range.
template <typename TK>
__global__ __launch_bounds__(256) void k_score_pass(const TK* __restrict__ Kc, const float* __restrict__ y,
                                                    const double* __restrict__ o, int64_t n, int64_t rows_per_blk,
                                                    const CandState* __restrict__ st, double* __restrict__ partial,
                                                    const NewtonScalars* __restrict__ sc) {
  if (sc->n_active_sel == 0) return;
  __shared__ double sh[4][4][kCandSlots];
  const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int status = st[c].status;
  double P = 0.0, Q = 0.0, V = 0.0, F = 0.0;
  if (status == 0) {
    const double s = st[c].s, sp = st[c].s_prev;
    const bool chk = st[c].passes > 0;
    const int64_t lo = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t hi = lo + rows_per_blk < n ? lo + rows_per_blk : n;
    int fl = 0;
    for (int64_t i = lo + q; i < hi; i += 4) {
      const double yi = (double)y[i];
      const double a = 1.0 - yi * o[i];
      const double b = yi * (double)Kc[i * kCandSlots + c];
      const double e = a - s * b;
      if (e > 0.0) {
        P += a * b;
        Q += b * b;
      }
      const double u = fmax(a, 0.0), w = fmax(e, 0.0);
      V += (w - u) * (w + u);
      if (chk) fl += ((e > 0.0) != (a - sp * b > 0.0)) ? 1 : 0;
    }
    F = (double)fl;
  }
  sh[q][0][c] = P;
  sh[q][1][c] = Q;
  sh[q][2][c] = V;
  sh[q][3][c] = F;
  __syncthreads();
  if (q == 0) {
    double* out = partial + ((int64_t)blockIdx.x * kCandSlots + c) * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = sh[0][k][c] + sh[1][k][c] + sh[2][k][c] + sh[3][k][c];
  }
}

// Next point of a bracketed semismooth Newton iteration on an increasing piecewise-linear function.
// g: value at the current point x; r: Newton root of the current piece. Returns false when the bracket
// cannot be split any further (then x is kept).
__device__ __forceinline__ bool bracket_next(double x, double g, double r, double& lo, double& hi, double& nx,
                                             int& newton) {
  if (g < 0.0)
    lo = x;
  else
    hi = x;
  if (r > lo && r < hi) {
    nx = r;
    newton = 1;
  } else {
    newton = 0;
    const bool flo = lo > -__builtin_huge_val(), fhi = hi < __builtin_huge_val();
    if (flo && fhi)
      nx = 0.5 * (lo + hi);
    else if (flo)
      nx = lo + fmax(1.0, fabs(lo));
    else
      nx = hi - fmax(1.0, fabs(hi));
  }
  return nx > lo && nx < hi;
}

constexpr int kMaxPasses = 64;

// 64 threads: reduce the partials of each active slot in block order and advance it.
__global__ void k_score_update(CandState* __restrict__ st, const double* __restrict__ partial, int nblk, double lam,
                               NewtonScalars* sc) {
  __shared__ int red[1];
  if (sc->n_active_sel == 0) return;
  const int c = threadIdx.x;
  CandState s = st[c];
  int still = 0;
  if (s.status == 0) {
    double P = 0.0, Q = 0.0, V = 0.0, F = 0.0;
    for (int b = 0; b < nblk; ++b) {
      const double* p = partial + ((int64_t)b * kCandSlots + c) * 4;
      P += p[0];
      Q += p[1];
      V += p[2];
      F += p[3];
    }
    s.passes += 1;
    const double g = lam * (s.oc + s.s) - (P - s.s * Q);
    bool done = (s.newton && F == 0.0) || g == 0.0;
    if (!done) {
      const double r = (P - lam * s.oc) / (lam + Q);
      double nx;
      int nw;
      if (bracket_next(s.s, g, r, s.lo, s.hi, nx, nw) && s.passes < kMaxPasses) {
        s.s_prev = s.s;
        s.s = nx;
        s.newton = nw;
        still = 1;
      } else {
        done = true;  // bracket exhausted or pass cap: keep the current point
      }
    }
    if (done) {
      s.status = 1;
      s.score = -(lam * (s.s * s.oc + 0.5 * s.s * s.s) + 0.5 * V);
    }
    st[c] = s;
  }
  const int na = block_sum_int(still, red);
  if (c == 0) sc->n_active_sel = na;
}

int score_blocks(int64_t n) {
  int64_t b = ceil_div(n, 512);
  return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

template <typename TK>
void launch_score_round(const TK* Kc, const float* y, const double* o, int64_t n, double lam, CandState* st,
                        double* partial, int nblk, NewtonScalars* sc, hipStream_t s) {
  const int64_t rows = round_up(ceil_div(n, nblk), 4);
  hipLaunchKernelGGL((k_score_pass<TK>), dim3(nblk), dim3(256), 0, s, Kc, y, o, n, rows, st, partial, sc);
  SPSVM_LAUNCHED();
  hipLaunchKernelGGL(k_score_update, dim3(1), dim3(kCandSlots), 0, s, st, partial, nblk, lam, sc);
  SPSVM_LAUNCHED();
}

// Argmax over the scored slots (strictly larger score wins, equal scores go to the lower training row),
// then append the winner to J and beta.
__global__ void k_select(const CandState* __restrict__ st, const uint64_t* __restrict__ hash,
                         uint64_t* __restrict__ stage_hash, int q, int64_t* __restrict__ J, double* __restrict__ beta,
                         int32_t* __restrict__ m_dev, Selection* __restrict__ sel) {
  const int c = threadIdx.x;
  const CandState s = st[c];
  const bool ok = s.status == 1 && s.idx >= 0 && !(s.score != s.score);
  double best = ok ? s.score : -__builtin_huge_val();
  int bidx = ok ? s.idx : 0x7fffffff;
  int bslot = c;
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, kWave);
    const int oi = __shfl_xor(bidx, off, kWave);
    const int os = __shfl_xor(bslot, off, kWave);
    if (ob > best || (ob == best && oi < bidx)) {
      best = ob;
      bidx = oi;
      bslot = os;
    }
  }
  if (c == 0) {
    Selection r;
    r.valid = bidx != 0x7fffffff;
    r.slot = bslot;
    r.idx = bidx;
    r.score = best;
    r.s = 0.0;
    r.pos = *m_dev;
    if (r.valid) {
      r.s = st[bslot].s;
      J[r.pos] = bidx;
      beta[r.pos] = r.s;
      stage_hash[q] = hash[bidx];
      *m_dev = r.pos + 1;
    }
    *sel = r;
  }
}

// o += s * k_winner; K_XJ[:, pos] = k_winner.
template <typename TK>
__global__ __launch_bounds__(256) void k_append(const Selection* __restrict__ sel, const TK* __restrict__ Kc, int64_t n,
                                                double* __restrict__ o, TK* __restrict__ KXJ, int64_t ldk) {
  const Selection s = *sel;
  if (!s.valid) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const TK k = Kc[i * kCandSlots + s.slot];
    o[i] += s.s * (double)k;
    KXJ[i * ldk + s.pos] = k;
  }
}

template <typename TK>
void launch_select_append(const CandState* st, const uint64_t* hash, uint64_t* stage_hash, int q, const TK* Kc,
                          int64_t n, double* o, TK* KXJ, int64_t ldk, int64_t* J, double* beta, int32_t* m_dev,
                          Selection* sel, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(1), dim3(kCandSlots), 0, s, st, hash, stage_hash, q, J, beta, m_dev, sel);
  SPSVM_LAUNCHED();
  const int64_t blocks = std::min<int64_t>(ceil_div(n, 256), 2048);
  hipLaunchKernelGGL((k_append<TK>), dim3((unsigned)blocks), dim3(256), 0, s, sel, Kc, n, o, KXJ, ldk);
  SPSVM_LAUNCHED();
}

template void launch_score_round<float>(const float*, const float*, const double*, int64_t, double, CandState*,
                                        double*, int, NewtonScalars*, hipStream_t);
template void launch_score_round<double>(const double*, const float*, const double*, int64_t, double, CandState*,
                                         double*, int, NewtonScalars*, hipStream_t);
template void launch_select_append<float>(const CandState*, const uint64_t*, uint64_t*, int, const float*, int64_t,
                                          double*, float*, int64_t, int64_t*, double*, int32_t*, Selection*,
                                          hipStream_t);
template void launch_select_append<double>(const CandState*, const uint64_t*, uint64_t*, int, const double*, int64_t,
                                           double*, double*, int64_t, int64_t*, double*, int32_t*, Selection*,
                                           hipStream_t);

}  // namespace spsvm
