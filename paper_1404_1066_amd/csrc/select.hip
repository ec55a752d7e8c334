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
// from, psi' is linear between them and the root is exact. A pass also lists, per slot, the rows whose
// activity changes inside a window of |s| / 256 around its point s (usually none or a handful); when the root
// lies in that window the update finds it exactly by walking those rows' breakpoints in order, without the
// pass that would otherwise confirm it.
#include "common.h"
#include "launch.h"

namespace spsvm {

constexpr int kMaxStageHash = 256;
constexpr int kScoreWaves = 8;  // waves per scoring workgroup  // stage winners staged in LDS by the score init (the default stage cap)

__device__ __forceinline__ bool hash_in(uint64_t h, const uint64_t* __restrict__ list, int cnt) {
  for (int q = 0; q < cnt; ++q)
    if (list[q] == h) return true;
  return false;
}

__device__ __forceinline__ void clear_bounds(CandState& s) {
  s.phi_lo = s.g_lo = s.phi_hi = s.g_hi = 0.0;
  s.lb = 0.0;  // psi(0) - psi(0)
  s.ub = __builtin_huge_val();
}

// Largest decrease psi(0) - min psi still possible given what the passes have seen. psi'' >= lambda everywhere
// (the regulariser's curvature; the loss terms only add to it), so at an evaluated point x
//   psi(z) - psi(0) >= T_x(z) = phi_x + g_x (z - x) + lambda/2 (z - x)^2
// for all z, and the minimiser lies in the bracket [lo, hi]. The minimum of max(T_lo, T_hi) over the bracket is
// attained at a bracket end, at the unconstrained minimiser of T_lo or T_hi, or where the two cross; the bound
// is minus the smallest of max(T_lo, T_hi) over those points (exact in real arithmetic, no iteration).
__device__ __forceinline__ double score_upper(const CandState& s, double lam) {
  const bool hl = s.lo > -__builtin_huge_val(), hh = s.hi < __builtin_huge_val();
  if (!hl && !hh) return __builtin_huge_val();
  auto L = [&](double z) {
    double v = -__builtin_huge_val();
    if (hl) {
      const double u = z - s.lo;
      v = fmax(v, s.phi_lo + s.g_lo * u + 0.5 * lam * u * u);
    }
    if (hh) {
      const double u = z - s.hi;
      v = fmax(v, s.phi_hi + s.g_hi * u + 0.5 * lam * u * u);
    }
    return v;
  };
  double m = __builtin_huge_val();
  if (hl) {
    m = fmin(m, L(s.lo));
    const double z = s.lo - s.g_lo / lam;
    if (!hh || z <= s.hi) m = fmin(m, L(z));
  }
  if (hh) {
    m = fmin(m, L(s.hi));
    const double z = s.hi - s.g_hi / lam;
    if (!hl || z >= s.lo) m = fmin(m, L(z));
  }
  if (hl && hh) {  // T_lo - T_hi is linear in u = z - lo: zero at u = -c0 / c1
    const double h = s.hi - s.lo;
    const double c0 = s.phi_lo - s.phi_hi + s.g_hi * h - 0.5 * lam * h * h;
    const double c1 = s.g_lo - s.g_hi + lam * h;
    if (c1 != 0.0) {
      const double u = -c0 / c1;
      if (u >= 0.0 && u <= h) m = fmin(m, L(s.lo + u));
    }
  }
  return -m;
}

// A slot is dropped when even its largest possible decrease is below the best decrease another slot has already
// reached: it cannot win the argmax. The relative margin keeps rounding in the sums (far below it) from ever
// dropping a slot whose computed final score could reach the winner's.
constexpr double kDropMargin = 1e-7;

// 64 threads: one per slot. bias (may be null): the model's offset b, which o includes; a candidate's regulariser
// cross term needs (K beta)_c = o_c - b.
__global__ void k_score_init(const int32_t* __restrict__ cand, const double* __restrict__ o,
                             const uint64_t* __restrict__ hash, const uint64_t* __restrict__ stage_hash, int n_stage,
                             CandState* __restrict__ st, NewtonScalars* sc, const double* __restrict__ bias) {
  __shared__ int red[1];
  __shared__ uint64_t sh[kMaxStageHash];
  const int c = threadIdx.x;
  // hashes of this stage's earlier winners, staged in LDS (every slot scans all of them)
  const int ns = n_stage < kMaxStageHash ? n_stage : kMaxStageHash;
  for (int q = c; q < ns; q += kCandSlots) sh[q] = stage_hash[q];
  __syncthreads();
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
  clear_bounds(s);
  if (s.idx < 0 || hash_in(hash[s.idx], sh, ns) || (n_stage > ns && hash_in(hash[s.idx], stage_hash + ns, n_stage - ns))) {
    s.status = 2;
  } else {
    s.status = 0;
    s.oc = bias ? o[s.idx] - *bias : o[s.idx];
  }
  st[c] = s;
  cand_win_count(st)[c] = 0;
  const int na = block_sum_int(s.status == 0 ? 1 : 0, red);
  if (c == 0) sc->n_active_sel = na;
}

void launch_score_init(const int32_t* cand, const double* o, const uint64_t* hash, const uint64_t* stage_hash,
                       int n_stage, CandState* st, NewtonScalars* sc, const double* bias, hipStream_t s) {
  hipLaunchKernelGGL(k_score_init, dim3(1), dim3(kCandSlots), 0, s, cand, o, hash, stage_hash, n_stage, st, sc, bias);
  SPSVM_LAUNCHED();
}

// a_i - z b_i with one rounding; every kernel that classifies rows as active (> 0) uses this form, so the
// pass sums, the flip counts and the window lists agree row by row.
__device__ __forceinline__ double gap_at(double a, double b, double z) { return __fma_rn(-z, b, a); }

// For a label y = +-1 (the entry points reject any other value), y o and y k are o and k with their sign
// flipped when y < 0, exactly: a_i = 1 - y_i o_i as margin_gap gives it, with the sign taken by integer
// operations (scalar ones where y and o are the same for the whole wave) instead of a conversion and an FP64
// product, and b_i = y_i k_i from an exact FP32 product (FP64 values: the sign flipped).
__device__ __forceinline__ double gap_pm1(float y, double o) {
  const long long sign = (long long)(__float_as_uint(y) & 0x80000000u) << 32;
  return __dadd_rn(1.0, -__longlong_as_double(__double_as_longlong(o) ^ sign));
}
__device__ __forceinline__ double signed_pm1(float y, float k) { return (double)(y * k); }
__device__ __forceinline__ double signed_pm1(float y, double k) {
  const long long sign = (long long)(__float_as_uint(y) & 0x80000000u) << 32;
  return __longlong_as_double(__double_as_longlong(k) ^ sign);
}

constexpr double kWinFrac = 1.0 / 256.0;  // window half-width relative to |s|

struct WinRoot {
  bool found;
  double r, phi;  // root and psi(r) - psi(0)
};

// Exact root of psi' inside the window [s - w, s + w], from the sums at s (P, Q over the rows active at s, V)
// and the cnt window rows sorted by breakpoint along the direction of descent (ra, rb). Segment k has the rows
// of the first k breakpoints toggled; its linear root is accepted when it lies in the window and every window
// row is active there exactly as segment k assumes (then no other row changes either: each row's activity is
// monotone in z, and rows off the list keep theirs over the window). psi(r) is continued from psi(s) with the
// exact change of each row's term.
__device__ WinRoot window_root(const CandState& st, double P, double Q, double V, double lam, const double* ra,
                               const double* rb, int cnt, double w) {
  WinRoot out{false, 0.0, 0.0};
  const double s = st.s, zl = s - w, zh = s + w;
  double Pc = P, Qc = Q;
  for (int k = 0; k <= cnt; ++k) {
    const double r = (Pc - lam * st.oc) / (lam + Qc);
    if (r >= zl && r <= zh) {
      bool ok = true;
      for (int j = 0; j < cnt && ok; ++j) {
        const bool flips = (gap_at(ra[j], rb[j], s) > 0.0) != (gap_at(ra[j], rb[j], r) > 0.0);
        ok = flips == (j < k);
      }
      if (ok) {
        // rows active at both points: the sums at s without the rows that went inactive
        double Pb = P, Qb = Q, dv = 0.0;
        for (int j = 0; j < k; ++j) {
          const double es = gap_at(ra[j], rb[j], s), er = gap_at(ra[j], rb[j], r);
          if (es > 0.0) {
            Pb -= ra[j] * rb[j];
            Qb -= rb[j] * rb[j];
            dv -= es * es;
          } else {
            dv += er * er;
          }
        }
        dv += (s - r) * (2.0 * Pb - (s + r) * Qb);
        out.found = true;
        out.r = r;
        out.phi = lam * (r * st.oc + 0.5 * r * r) + 0.5 * (V + dv);
        return out;
      }
    }
    if (k < cnt) {
      if (gap_at(ra[k], rb[k], s) > 0.0) {
        Pc -= ra[k] * rb[k];
        Qc -= rb[k] * rb[k];
      } else {
        Pc += ra[k] * rb[k];
        Qc += rb[k] * rb[k];
      }
    }
  }
  return out;
}

// Advance one slot after a pass (sums P, Q, V and the flip count F at the slot's current point s).
__device__ __forceinline__ bool bracket_next(double x, double g, double r, double& lo, double& hi, double& nx,
                                             int& newton);
constexpr int kMaxPasses = 64;

__device__ __forceinline__ int advance_slot(CandState& s, double P, double Q, double V, double F, double lam,
                                            const WinRoot* wr = nullptr) {
  s.passes += 1;
  const double g = lam * (s.oc + s.s) - (P - s.s * Q);
  double phi = lam * (s.s * s.oc + 0.5 * s.s * s.s) + 0.5 * V;  // psi(s) - psi(0)
  s.lb = fmax(s.lb, -phi);
  bool done = (s.newton && F == 0.0) || g == 0.0;
  if (!done && wr && wr->found) {  // exact root inside the window of this pass
    s.s = wr->r;
    phi = wr->phi;
    done = true;
  }
  int still = 0;
  if (!done) {
    const double r = (P - lam * s.oc) / (lam + Q);
    // A Newton step below 1e-10 of |s| changes the score only in the second order of the step (the
    // derivative is already ~0 there), i.e. far below FP64 rounding of the score: stop at s.
    if (s.newton && fabs(r - s.s) <= 1e-10 * fabs(s.s)) done = true;
  }
  if (!done) {
    const double r = (P - lam * s.oc) / (lam + Q);
    double nx;
    int nw;
    if (g < 0.0) {  // the bracket end bracket_next moves to s
      s.phi_lo = phi;
      s.g_lo = g;
    } else {
      s.phi_hi = phi;
      s.g_hi = g;
    }
    if (bracket_next(s.s, g, r, s.lo, s.hi, nx, nw) && s.passes < kMaxPasses) {
      s.s_prev = s.s;
      s.s = nx;
      s.newton = nw;
      s.ub = fmax(score_upper(s, lam), s.lb);
      still = 1;
    } else {
      done = true;  // bracket exhausted or pass cap: keep the current point
    }
  }
  if (done) {
    s.status = 1;
    s.score = -phi;
    s.lb = s.ub = s.score;
  }
  return still;
}

// One pass over the rows for the slots still being scored (na of the 64). The candidate block is column-major
// (column stride ldc), so a live slot's values are one contiguous column. The live slots are packed onto the
// lanes: with R = 64 / na, lane r * na + a (r < R) of wave q takes live slot a on the chunks of 8 consecutive rows
// starting at lo + 8 (q R + r) + m 8 kScoreWaves R of its workgroup's range; a pass thus reads one column per
// live slot. The per-lane sums are added over the waves, then over r, in a fixed order, and written as this
// workgroup's record {P, Q, V, flips} of each live slot.
template <typename TK>
__global__ __launch_bounds__(64 * kScoreWaves, 5) void k_score_pass(const TK* __restrict__ Kc, int64_t ldc,
                                                                  const float* __restrict__ y,
                                                                  const double* __restrict__ o, int64_t n,
                                                                  int64_t rows_per_blk,
                                                                  const CandState* __restrict__ st,
                                                                  int32_t* __restrict__ drop,
                                                                  int32_t* __restrict__ wcnt,
                                                                  double* __restrict__ wrows,
                                                                  double* __restrict__ partial, int nodrop) {
  __shared__ double sh[kScoreWaves][4][kCandSlots];
  __shared__ double red[4][kCandSlots];
  __shared__ int act[kCandSlots];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  // Lane = slot. Slots that cannot win any more (their upper bound below the best lower bound of all slots)
  // are dropped before the pass; every wave takes the same decision from the same states, workgroup 0 records
  // it for the update that follows.
  const int status = st[lane].status;
  double best = status == 1 ? st[lane].score : (status == 0 ? st[lane].lb : -__builtin_huge_val());
  for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off, kWave));
  const bool dropped = !nodrop && status == 0 && st[lane].ub < best - kDropMargin * fabs(best);
  if (blockIdx.x == 0 && q == 0) drop[lane] = dropped ? 1 : 0;
  const bool live = status == 0 && !dropped;
  const unsigned long long mask = __ballot(live);
  const int na = __popcll(mask);
  if (na == 0) return;  // every slot is settled (same answer in every wave and workgroup)
  if (q == 0 && live) act[__popcll(mask & ((1ull << lane) - 1ull))] = lane;
  __syncthreads();
  const int R = kCandSlots / na, r = lane / na, a = lane - r * na;
  double P = 0.0, Q = 0.0, V = 0.0, F = 0.0;
  if (r < R) {
    const int c = act[a];
    const TK* __restrict__ kc = Kc + (int64_t)c * ldc;  // the slot's candidate column
    const double s = st[c].s, sp = st[c].s_prev;
    const bool chk = st[c].passes > 0;
    // A row's activity changes inside [s - w, s + w] only if |a_i - s b_i| <= w |b_i| (exactly; the gap is one
    // correctly rounded fma, so its sign is exact, and s -+ w and the product add relative errors near 2^-52):
    // the test below with a 1e-4 relative margin lists every such row, and possibly a few more, which the
    // walk classifies exactly.
    const double wt = 1.0001 * kWinFrac * fabs(s);
    const bool win = wt > 0.0;
    int32_t* __restrict__ cnt = wcnt + c;
    double* __restrict__ rows = wrows + (int64_t)c * kWinCap * 2;
    const int64_t lo = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t hi = lo + rows_per_blk < n ? lo + rows_per_blk : n;
    constexpr int U = 8;
    const int64_t step = (int64_t)kScoreWaves * R * U;
    double P2 = 0.0, Q2 = 0.0, V2 = 0.0;
    int fl = 0, fl2 = 0;
    auto one = [&](double av, double b, double& Pa, double& Qa, double& Va, int& fa) {
      const double e = gap_at(av, b, s);
      const double ua = fmax(av, 0.0), we = fmax(e, 0.0);
      // b where the row is active at s, else an exact zero (whose products add nothing): one select, not a
      // branch, so that no control flow keeps the compiler from issuing a chunk's loads together, feeds both
      // sums, each one fused multiply-add (the pass is bound by its vector ALU instructions)
      const double bm = e > 0.0 ? b : 0.0;
      Pa = __fma_rn(av, bm, Pa);
      Qa = __fma_rn(bm, bm, Qa);
      Va += (we - ua) * (we + ua);
      fa += chk && ((e > 0.0) != (gap_at(av, b, sp) > 0.0)) ? 1 : 0;
      // rows whose activity changes inside the window (rare): every one is counted, so a list that ran out of
      // room (count above kWinCap) is seen as incomplete by the update; the first kWinCap are stored
      if (win && fabs(e) <= wt * fabs(b)) {
        const int k = atomicAdd(cnt, 1);
        if (k < kWinCap) {
          rows[2 * k] = av;
          rows[2 * k + 1] = b;
        }
      }
    };
    // chunks of U consecutive rows per lane (contiguous loads from the column), even rows summed apart from odd
    // (uniform: y and o are the same in every lane, where the sign of a_i is best taken by scalar operations)
    auto chunk = [&](auto uniform, const float* yv, const double* ov, const TK* kv) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double av = decltype(uniform)::value ? gap_pm1(yv[u], ov[u]) : margin_gap(yv[u], ov[u]);
        const double b = signed_pm1(yv[u], kv[u]);
        if (u & 1)
          one(av, b, P2, Q2, V2, fl2);
        else
          one(av, b, P, Q, V, fl);
      }
    };
    int64_t i = lo + (int64_t)(q * R + r) * U;
    if (R == 1) {
      // more than 32 live slots: every live lane of the wave takes the same rows, so y and o are read with
      // scalar loads (the row offset made wave-uniform) and the vector loads carry candidate values only
      int64_t iu = lo + (int64_t)__builtin_amdgcn_readfirstlane(q) * U;
      for (; iu + U - 1 < hi; iu += step) {
        float yv[U];
        double ov[U];
        TK kv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          yv[u] = y[iu + u];
          ov[u] = o[iu + u];
          kv[u] = kc[iu + u];
        }
        chunk(std::true_type{}, yv, ov, kv);
      }
      i = iu;
    } else {
      for (; i + U - 1 < hi; i += step) {
        float yv[U];
        double ov[U];
        TK kv[U];  // converted where used: a conversion here would wait for the load
#pragma unroll
        for (int u = 0; u < U; ++u) {
          yv[u] = y[i + u];
          ov[u] = o[i + u];
          kv[u] = kc[i + u];
        }
        chunk(std::false_type{}, yv, ov, kv);
      }
    }
    for (; i < hi; ++i) one(margin_gap(y[i], o[i]), signed_pm1(y[i], kc[i]), P, Q, V, fl);  // partial chunk
    P += P2;
    Q += Q2;
    V += V2;
    F = (double)(fl + fl2);
  }
  sh[q][0][lane] = P;
  sh[q][1][lane] = Q;
  sh[q][2][lane] = V;
  sh[q][3][lane] = F;
  __syncthreads();
  if (threadIdx.x < 4 * kCandSlots) {  // over the waves, per lane and component
    const int l = threadIdx.x & 63, k = threadIdx.x >> 6;
    double t = sh[0][k][l];
#pragma unroll
    for (int v = 1; v < kScoreWaves; ++v) t += sh[v][k][l];
    red[k][l] = t;
  }
  __syncthreads();
  if (threadIdx.x < 4 * kCandSlots) {  // over r, per live slot and component
    const int aa = threadIdx.x & 63, k = threadIdx.x >> 6;
    if (aa < na) {
      double t = red[k][aa];
      for (int rr = 1; rr < R; ++rr) t += red[k][rr * na + aa];
      partial[((int64_t)act[aa] * gridDim.x + blockIdx.x) * 4 + k] = t;  // slot-major: [slot][record][4]
    }
  }
}

// One workgroup per slot: reduce the slot's partial records over the workgroups of the pass with a fixed
// tree, then advance the slot.
__global__ __launch_bounds__(256) void k_score_update(CandState* __restrict__ st, const double* __restrict__ partial,
                                                      int nblk, double lam, int32_t* __restrict__ live) {
  __shared__ double red[4][4];
  const int c = blockIdx.x;
  if (st[c].status != 0) return;
  if (cand_drop_flags(st)[c]) {  // dropped by the pass: not read, retired without a score
    __syncthreads();  // every thread has read the status before it changes
    if (threadIdx.x == 0) st[c].status = 3;
    return;
  }
  __shared__ double wa[kWinCap], wb[kWinCap];
  if (threadIdx.x == 0 && live) atomicAdd(live, 1);  // slot-passes: this slot was read by the pass
  double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int b = threadIdx.x; b < nblk; b += 256) {  // in order; several records in flight
    const doublex4 p = *(const doublex4*)(partial + ((int64_t)c * nblk + b) * 4);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += p[k];
  }
  // fixed order: xor butterflies inside each wave, then the four waves in order
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = wave_sum(v[k]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) red[w][k] = v[k];
  __syncthreads();
  // wave 0: the window rows sorted by breakpoint along the descent direction (rank sort over the lanes; equal
  // keys ordered by value, so the order never depends on the order the pass appended them), then lane 0 walks
  // them and advances the slot
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    double t[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
    CandState cs = st[c];
    int32_t* cntp = cand_win_count(st) + c;
    const int cnt = *cntp;
    const double w = kWinFrac * fabs(cs.s);
    const bool usable = w > 0.0 && cnt <= kWinCap;  // a longer list is incomplete: no window root this pass
    const bool any = cnt > 0;
    WinRoot wr{false, 0.0, 0.0};
    if (usable) {
      const double g = lam * (cs.oc + cs.s) - (t[0] - cs.s * t[1]);
      const double dir = g < 0.0 ? 1.0 : -1.0;
      const bool real = lane < cnt;
      const double* rows = cand_win_rows(st) + (int64_t)c * kWinCap * 2;
      const double a = real ? rows[2 * lane] : 0.0, b = real ? rows[2 * lane + 1] : 0.0;
      double key = real ? dir * (a / b - cs.s) : 0.0;
      if (!(key >= 0.0)) key = __builtin_huge_val();  // breakpoints behind s are never crossed
      int rank = 0;
      for (int j = 0; any && j < cnt; ++j) {  // only real entries can come before a real one
        const bool rj = __shfl((int)real, j, kWave) != 0;
        const double kj = __shfl(key, j, kWave), aj = __shfl(a, j, kWave), bj = __shfl(b, j, kWave);
        const bool before = (rj && !real) ||
                            (rj == real && (kj < key || (kj == key && (aj < a || (aj == a && (bj < b || (bj == b && j < lane)))))));
        rank += before ? 1 : 0;
      }
      if (real) {
        wa[rank] = a;
        wb[rank] = b;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      __builtin_amdgcn_wave_barrier();
      if (lane == 0 && cs.status == 0) wr = window_root(cs, t[0], t[1], t[2], lam, wa, wb, cnt, w);
    }
    if (lane == 0) {
      advance_slot(cs, t[0], t[1], t[2], t[3], lam, &wr);
      st[c] = cs;
      *cntp = 0;  // the next pass lists the window of the slot's next point
    }
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

// Workgroups of the scoring pass that the device holds at once (CUs x resident workgroups per CU of the
// heavier instance); 256 x 2 on MI355X (five waves per SIMD: two 8-wave workgroups per CU), also the value
// taken when no device can be queried.
static int score_resident() {
  static const int v = [] {
    int dev = 0, cus = 0, pf = 0, pd = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&pf, k_score_pass<float>, 64 * kScoreWaves, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&pd, k_score_pass<double>, 64 * kScoreWaves, 0) != hipSuccess ||
        cus <= 0 || std::min(pf, pd) <= 0) {
      (void)hipGetLastError();  // leave no error behind for the next launch check
      return 512;
    }
    return cus * std::min(pf, pd);
  }();
  return v;
}

// 128 rows per workgroup, but no more workgroups than the device holds at once: a pass is then one round of
// workgroups (a second, nearly empty round costs about as much as the first), and longer passes give each
// workgroup more rows.
int score_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 128), score_resident())); }

template <typename TK>
void launch_score_pass(const TK* Kc, int64_t ldc, const float* y, const double* o, int64_t n, CandState* st,
                       double* partial, int nblk, hipStream_t s, bool nodrop) {
  const int64_t rows = round_up(ceil_div(n, nblk), kScoreWaves);
  hipLaunchKernelGGL((k_score_pass<TK>), dim3(nblk), dim3(64 * kScoreWaves), 0, s, Kc, ldc, y, o, n, rows, st,
                     cand_drop_flags(st), cand_win_count(st), cand_win_rows(st), partial, nodrop ? 1 : 0);
  SPSVM_LAUNCHED();
}

void launch_score_update(CandState* st, const double* partial, int nblk, double lam, int32_t* live, hipStream_t s) {
  hipLaunchKernelGGL(k_score_update, dim3(kCandSlots), dim3(256), 0, s, st, partial, nblk, lam, live);
  SPSVM_LAUNCHED();
}

// Slot set-up and the update after a first pass that came with the kernel block, in one launch: workgroup c
// sets slot c up as the initialisation kernel does (its 256 threads scan the stage's earlier winners at once),
// then reduces the slot's partial records and advances it as the update kernel does.
__global__ __launch_bounds__(256) void k_score_init_update(const int32_t* __restrict__ cand,
                                                           const double* __restrict__ o,
                                                           const uint64_t* __restrict__ hash,
                                                           const uint64_t* __restrict__ stage_hash, int n_stage,
                                                           CandState* __restrict__ st,
                                                           const double* __restrict__ partial, int nblk,
                                                           double lam, const double* __restrict__ bias) {
  __shared__ double red[4][4];
  __shared__ int taken;
  const int c = blockIdx.x;
  const int idx = cand[c];
  if (threadIdx.x == 0) {
    taken = 0;
    cand_win_count(st)[c] = 0;  // no window list for the first pass, which came with the kernel block
  }
  __syncthreads();
  if (idx >= 0) {
    const uint64_t h = hash[idx];
    for (int q = threadIdx.x; q < n_stage; q += 256)
      if (stage_hash[q] == h) taken = 1;
  }
  __syncthreads();
  CandState s;
  s.idx = idx;
  s.s = 0.0;
  s.s_prev = 0.0;
  s.lo = -__builtin_huge_val();
  s.hi = __builtin_huge_val();
  s.oc = 0.0;
  s.score = -__builtin_huge_val();
  s.newton = 0;
  s.passes = 0;
  clear_bounds(s);
  if (idx < 0 || taken) {
    s.status = 2;
    if (threadIdx.x == 0) st[c] = s;
    return;
  }
  s.status = 0;
  s.oc = bias ? o[idx] - *bias : o[idx];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int b = threadIdx.x; b < nblk; b += 256) {  // in order; several records in flight
    const doublex4 p = *(const doublex4*)(partial + ((int64_t)c * nblk + b) * 4);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += p[k];
  }
  // the update kernel's order: xor butterflies inside each wave, then the four waves in order
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = wave_sum(v[k]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) red[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
    advance_slot(s, t[0], t[1], t[2], t[3], lam);
    st[c] = s;
  }
}

void launch_score_init_update(const int32_t* cand, const double* o, const uint64_t* hash, const uint64_t* stage_hash,
                              int n_stage, CandState* st, const double* partial, int nblk, double lam,
                              const double* bias, hipStream_t s) {
  hipLaunchKernelGGL(k_score_init_update, dim3(kCandSlots), dim3(256), 0, s, cand, o, hash, stage_hash, n_stage, st,
                     partial, nblk, lam, bias);
  SPSVM_LAUNCHED();
}


// Argmax over the scored slots (strictly larger score wins, equal scores go to the lower training row), then
// the append: o += s * k_winner and K_XJ[:, pos] = k_winner over all rows. Every workgroup takes the same
// argmax from the slot states; workgroup 0 alone records it (J, beta, the stage hash, the pass counters and
// the next basis size). The basis size is double-buffered by step parity: step q reads m_dev[q & 1] and
// writes m_dev[(q + 1) & 1], so no workgroup reads a value another one has already advanced.
// A step whose slots did not all settle within the launched passes selects nothing, sets incomplete[0] and
// records its index in incomplete[4]; every later step of the same launch sequence then selects nothing
// either (incomplete[0] is already set when it starts), so o, J and the basis size stay as they were after the
// last complete step and the stage can be resumed from the recorded step.
// The basis row's index goes to J[pos] (and J32[pos]); its coefficient and kernel column to position pos + off
// of beta and K_XJ (off = 1 when the first coordinate is the offset b). write_col = 0 leaves K_XJ alone (its column
// is formed later from the stage's winners at a higher precision than the candidate block's).
template <typename TK>
__global__ __launch_bounds__(256) void k_select_append(const CandState* __restrict__ st,
                                                       const uint64_t* __restrict__ hash,
                                                       uint64_t* __restrict__ stage_hash, int q,
                                                       int64_t* __restrict__ J, int32_t* __restrict__ J32,
                                                       double* __restrict__ beta,
                                                       int32_t* __restrict__ m_dev, Selection* __restrict__ sel,
                                                       int32_t* __restrict__ incomplete, int fused0,
                                                       const TK* __restrict__ Kc, int64_t ldc, int64_t n,
                                                       double* __restrict__ o, TK* __restrict__ KXJ, int64_t ldk,
                                                       int off, int write_col) {
  __shared__ Selection choice;
  if (threadIdx.x < kWave) {
    const int c = threadIdx.x;
    const CandState s = st[c];
    // an earlier step of this sequence did not settle (read before this step's own flag can be set; a workgroup
    // that sees this step's flag instead is in a step that selects nothing anyway)
    const bool after_fail = incomplete[0] != 0;
    const int pending = __any(s.status == 0);  // a slot still being scored: this step must be redone
    const bool ok = !pending && !after_fail && s.status == 1 && s.idx >= 0 && !(s.score != s.score);
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
    const double s_best = __shfl(s.s, bslot, kWave);
    if (c == 0) {
      Selection r;
      r.valid = bidx != 0x7fffffff;
      r.slot = bslot;
      r.idx = bidx;
      r.score = best;
      r.s = r.valid ? s_best : 0.0;
      r.pos = m_dev[q & 1];
      choice = r;
      if (blockIdx.x == 0) {
        if (pending && !after_fail) {
          incomplete[0] = 1;
          incomplete[4] = q;  // the first step to redo
        }
        if (r.valid) {
          J[r.pos] = bidx;
          J32[r.pos] = bidx;
          beta[r.pos + off] = r.s;
          stage_hash[q] = hash[bidx];
        }
        m_dev[(q + 1) & 1] = r.pos + (r.valid ? 1 : 0);
        *sel = r;
      }
    }
    if (blockIdx.x == 0) {
      int mp = s.passes;
      for (int off = 32; off > 0; off >>= 1) mp = max(mp, __shfl_xor(mp, off, kWave));
      if (c == 0) {
        atomicMax(&incomplete[1], mp);  // largest number of passes any slot needed in this stage
        atomicAdd(&incomplete[2], mp > fused0 ? mp - fused0 : 0);  // launched passes of this step that did
                                                                    // work (fused0: the first came with the block)
      }
    }
  }
  __syncthreads();
  const Selection r = choice;
  if (!r.valid) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const TK k = Kc[(int64_t)r.slot * ldc + i];  // column-major candidate block
    o[i] += r.s * (double)k;
    if (write_col) KXJ[i * ldk + r.pos + off] = k;
  }
}

template <typename TK>
void launch_select_append(const CandState* st, const uint64_t* hash, uint64_t* stage_hash, int q, const TK* Kc,
                          int64_t ldc, int64_t n, double* o, TK* KXJ, int64_t ldk, int64_t* J, int32_t* J32,
                          double* beta, int32_t* m_dev, Selection* sel, int32_t* incomplete, int fused0, int off,
                          bool write_col, hipStream_t s) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 2048));
  hipLaunchKernelGGL((k_select_append<TK>), dim3((unsigned)blocks), dim3(256), 0, s, st, hash, stage_hash, q, J, J32,
                     beta, m_dev, sel, incomplete, fused0, Kc, ldc, n, o, KXJ, ldk, off, write_col ? 1 : 0);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------ one basis shared by a batch of problems
// Argmax over the slots of the sum of P problems' exact scores (problem p's slot states at st0 + p * stride bytes;
// every problem scored the same candidates, no slot dropped). A slot counts only when every problem finished it;
// the sum runs in problem order; the largest sum wins, the lower row on ties. The winner's row goes to J[pos] and
// J32[pos], its hash to the stage list; the pending / incomplete protocol is that of k_select_append.
__global__ __launch_bounds__(kCandSlots) void k_shared_select(const char* __restrict__ st0, int64_t stride, int P,
                                                              const uint64_t* __restrict__ hash,
                                                              uint64_t* __restrict__ stage_hash, int q,
                                                              int64_t* __restrict__ J, int32_t* __restrict__ J32,
                                                              int32_t* __restrict__ m_dev,
                                                              Selection* __restrict__ sel,
                                                              int32_t* __restrict__ incomplete) {
  const int c = threadIdx.x;
  const bool after_fail = incomplete[0] != 0;
  const int idx = reinterpret_cast<const CandState*>(st0)[c].idx;
  bool all_done = true, any_active = false;
  double total = 0.0;
  int mp = 0, work = 0;
  for (int p = 0; p < P; ++p) {
    const CandState& s = reinterpret_cast<const CandState*>(st0 + (int64_t)p * stride)[c];
    all_done = all_done && s.status == 1;
    any_active = any_active || s.status == 0;
    total += s.status == 1 ? s.score : 0.0;
    mp = max(mp, s.passes);
    work += s.passes;
  }
  const int pending = __any(any_active);
  const bool ok = !pending && !after_fail && all_done && idx >= 0 && !(total != total);
  double best = ok ? total : -__builtin_huge_val();
  int bidx = ok ? idx : 0x7fffffff;
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
  for (int off = 32; off > 0; off >>= 1) {
    mp = max(mp, __shfl_xor(mp, off, kWave));
    work += __shfl_xor(work, off, kWave);
  }
  if (c == 0) {
    Selection r;
    r.valid = bidx != 0x7fffffff;
    r.slot = bslot;
    r.idx = bidx;
    r.score = best;
    r.s = 0.0;  // per problem: the slot's point in that problem's state
    r.pos = m_dev[q & 1];
    if (pending && !after_fail) {
      incomplete[0] = 1;
      incomplete[4] = q;
    }
    if (r.valid) {
      J[r.pos] = bidx;
      J32[r.pos] = bidx;
      stage_hash[q] = hash[bidx];
    }
    m_dev[(q + 1) & 1] = r.pos + (r.valid ? 1 : 0);
    *sel = r;
    atomicMax(&incomplete[1], mp);  // largest number of passes any slot of any problem needed in this stage
    atomicAdd(&incomplete[2], work);
  }
}

void launch_shared_select(const CandState* st0, int64_t stride, int P, const uint64_t* hash, uint64_t* stage_hash,
                          int q, int64_t* J, int32_t* J32, int32_t* m_dev, Selection* sel, int32_t* incomplete,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_shared_select, dim3(1), dim3(kCandSlots), 0, s, (const char*)st0, stride, P, hash, stage_hash,
                     q, J, J32, m_dev, sel, incomplete);
  SPSVM_LAUNCHED();
}

// One problem's append of the shared winner: its coefficient (the problem's one-dimensional optimum, the point
// of the winning slot in its state) to beta[pos], and o += s k_winner.
template <typename TK>
__global__ __launch_bounds__(256) void k_shared_append(const Selection* __restrict__ sel,
                                                       const CandState* __restrict__ st,
                                                       const TK* __restrict__ Kc, int64_t ldc, int64_t n,
                                                       double* __restrict__ o, double* __restrict__ beta) {
  const Selection r = *sel;
  if (!r.valid) return;
  const double s = st[r.slot].s;
  if (blockIdx.x == 0 && threadIdx.x == 0) beta[r.pos] = s;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    o[i] += s * (double)Kc[(int64_t)r.slot * ldc + i];
}

// The winner's column of one gamma's candidate block into that gamma's K_XJ (column pos).
template <typename TK>
__global__ __launch_bounds__(256) void k_shared_column(const Selection* __restrict__ sel, const TK* __restrict__ Kc,
                                                       int64_t ldc, int64_t n, TK* __restrict__ KXJ, int64_t ldk) {
  const Selection r = *sel;
  if (!r.valid) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    KXJ[i * ldk + r.pos] = Kc[(int64_t)r.slot * ldc + i];
}

template <typename TK>
void launch_shared_append(const Selection* sel, const CandState* st, const TK* Kc, int64_t ldc, int64_t n, double* o,
                          double* beta, hipStream_t s) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 2048));
  hipLaunchKernelGGL((k_shared_append<TK>), dim3((unsigned)blocks), dim3(256), 0, s, sel, st, Kc, ldc, n, o, beta);
  SPSVM_LAUNCHED();
}

template <typename TK>
void launch_shared_column(const Selection* sel, const TK* Kc, int64_t ldc, int64_t n, TK* KXJ, int64_t ldk,
                          hipStream_t s) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 2048));
  hipLaunchKernelGGL((k_shared_column<TK>), dim3((unsigned)blocks), dim3(256), 0, s, sel, Kc, ldc, n, KXJ, ldk);
  SPSVM_LAUNCHED();
}

template void launch_shared_append<float>(const Selection*, const CandState*, const float*, int64_t, int64_t, double*,
                                          double*, hipStream_t);
template void launch_shared_append<double>(const Selection*, const CandState*, const double*, int64_t, int64_t,
                                           double*, double*, hipStream_t);
template void launch_shared_column<float>(const Selection*, const float*, int64_t, int64_t, float*, int64_t,
                                          hipStream_t);
template void launch_shared_column<double>(const Selection*, const double*, int64_t, int64_t, double*, int64_t,
                                           hipStream_t);

template void launch_score_pass<float>(const float*, int64_t, const float*, const double*, int64_t, CandState*,
                                       double*, int, hipStream_t, bool);
template void launch_score_pass<double>(const double*, int64_t, const float*, const double*, int64_t, CandState*,
                                        double*, int, hipStream_t, bool);
template void launch_select_append<float>(const CandState*, const uint64_t*, uint64_t*, int, const float*, int64_t,
                                          int64_t, double*, float*, int64_t, int64_t*, int32_t*, double*, int32_t*,
                                          Selection*, int32_t*, int, int, bool, hipStream_t);
template void launch_select_append<double>(const CandState*, const uint64_t*, uint64_t*, int, const double*, int64_t,
                                           int64_t, double*, double*, int64_t, int64_t*, int32_t*, double*, int32_t*,
                                           Selection*, int32_t*, int, int, bool, hipStream_t);

}  // namespace spsvm
