// Host orchestration of SP-SVM training (section 4, "Sparse primal optimization"): stages of greedy
// basis additions, each followed by Newton re-optimisation of Eq. 4. Every O(n) or larger step is a
// kernel; the host draws candidate indices, launches, and reads back a few scalars per iteration.
#include "trainer.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <type_traits>

#include "launch.h"

spsvm_model::~spsvm_model() {
  if (XJ) (void)hipFree(XJ);
  if (XJnorm) (void)hipFree(XJnorm);
  if (beta_dev) (void)hipFree(beta_dev);
}

namespace spsvm {

// ------------------------------------------------------------------------------------ candidate draws
static constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

static inline uint64_t splitmix_finalise(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void draw_step(uint64_t seed, int64_t t, int64_t n, int kappa, const std::vector<uint64_t>& row_hash,
               const std::vector<uint64_t>& blocked_sorted, int32_t* out64) {
  for (int c = 0; c < kCandSlots; ++c) out64[c] = -1;
  uint64_t state = seed ^ ((uint64_t)(t + 1) * kGolden);
  int got = 0;
  for (int attempt = 0; attempt < 64 * kappa && got < kappa; ++attempt) {
    state += kGolden;
    const uint64_t z = splitmix_finalise(state);
    const int32_t idx = (int32_t)(((z >> 32) * (uint64_t)n) >> 32);
    bool seen = false;
    for (int c = 0; c < got; ++c) seen |= out64[c] == idx;
    if (seen) continue;
    if (std::binary_search(blocked_sorted.begin(), blocked_sorted.end(), row_hash[idx])) continue;
    out64[got++] = idx;
  }
}

int64_t stage_size(int64_t J, int64_t J_max, double growth, int64_t cap) {
  const int64_t g = (int64_t)std::floor(growth * (double)J);
  return std::min<int64_t>(J_max - J, std::max<int64_t>(1, std::min<int64_t>(cap, g)));
}

// ------------------------------------------------------------------------------------------ workspace
Plan make_plan(int64_t n, int64_t d, int64_t J_max, const spsvm_options& opt, bool with_selection, bool x_double,
               bool x_aligned, bool batch) {
  Plan p;
  const int64_t xe = x_double ? 8 : 4;
  p.ldx = round_up(d, 16 / xe);
  p.pad_x = p.ldx != d || !x_aligned;
  p.ldj = padded_ld<double>(d);
  p.n = n;
  p.d = d;
  p.J_max = J_max;
  p.tk_double = opt.precision == SPSVM_F64;
  p.ldk = round_up(J_max, 4);
  p.ldh = round_up(J_max, 4);
  const size_t tk = p.tk_double ? 8 : 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (size_t)round_up((int64_t)std::max<size_t>(bytes, 1), 256);
    return at;
  };
  const int64_t nb_c = compact_blocks(n), nb_s = score_blocks(n);
  const int64_t cap = with_selection ? opt.chunk_cap : 1;
  p.xnorm = take(n * tk);
  p.hash = take(n * 8);
  p.KXJ = take((size_t)n * p.ldk * tk);
  p.Kc = take(with_selection ? (size_t)n * kCandSlots * tk : 0);
  p.o = take(n * 8);
  p.delta = take(n * 8);
  p.act0 = take(n);
  p.act1 = take(n);
  p.I = take(n * 4);
  p.cblk_cnt = take(nb_c * 4);
  p.cblk_sum = take(nb_c * 8);
  p.cblk_flips = take(nb_c * 4);
  p.J = take(J_max * 8);
  p.J32 = take(J_max * 4);
  p.beta = take(J_max * 8);
  p.dvec = take(J_max * 8);
  p.g = take(J_max * 8);
  p.z = take(J_max * 8);
  p.H = take((size_t)J_max * p.ldh * 8);
  p.Linv = take((size_t)ceil_div(J_max, kCholNB) * kCholNB * kCholNB * 8);
  p.syrk_part = take(syrk_partial_doubles((int)J_max) * 8);
  p.grad_part = take((size_t)1024 * 256 * 8);
  p.cand_state = take(kCandSlots * sizeof(CandState));
  p.sel = take(sizeof(Selection));
  p.ls = take(sizeof(LineState));
  p.scalars = take(sizeof(NewtonScalars));
  p.score_part = take((size_t)nb_s * kCandSlots * 4 * 8);
  p.ls_part = take((size_t)nb_s * 6 * 8);
  p.cand_table = take((size_t)cap * kCandSlots * 4);
  p.stage_hash = take(cap * 8);
  p.m_dev = take(4);
  p.flags = take(16);
  p.XJ64 = take((size_t)J_max * p.ldj * 8);
  p.xjnorm = take(J_max * 8);
  p.KJJ = take((size_t)J_max * p.ldh * 8);
  p.vJ = take(J_max * 8);
  p.wJ = take(J_max * 8);
  p.iota = take(J_max * 4);
  p.incomplete = take(8);
  p.o_stage = take(with_selection ? n * 8 : 0);
  p.Hf = take((size_t)J_max * p.ldh * 8);
  p.F_in = take(n * 4);
  p.F_out = take(n * 4);
  p.fcnt_in = take(nb_c * 4);
  p.fcnt_out = take(nb_c * 4);
  p.Xp = take(p.pad_x ? (size_t)n * p.ldx * xe : 0);
  p.D = take(batch ? (size_t)n * p.ldk * tk : 0);
  p.DJJ = take(batch ? (size_t)J_max * p.ldh * 8 : 0);
  p.bytes = off;
  return p;
}

// ----------------------------------------------------------------------------------------- the trainer
namespace {

struct Pinned {
  void* p = nullptr;
  explicit Pinned(size_t bytes) { SPSVM_HIP(hipHostMalloc(&p, bytes, hipHostMallocDefault)); }
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};

using clk = std::chrono::steady_clock;
constexpr size_t kPinnedScalars = 16384;  // bytes of pinned memory for scalar read-backs
static double secs(clk::time_point a, clk::time_point b) { return std::chrono::duration<double>(b - a).count(); }

// HIP-event timing of selected kernels on the training stream. Pairs of events bracket each timed launch;
// elapsed times are collected after the stream has been synchronised.
struct Profiler {
  hipStream_t st = nullptr;
  int mask = 0;
  struct Pending {
    hipEvent_t a, b;
    int cat;
    double work;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  double seconds[4] = {0, 0, 0, 0}, work[4] = {0, 0, 0, 0};
  int64_t count[4] = {0, 0, 0, 0};

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    SPSVM_HIP(hipEventCreate(&e));
    return e;
  }
  template <class F>
  void timed(int cat, double w, F&& launch) {
    if (!(mask & (1 << cat))) {
      launch();
      return;
    }
    hipEvent_t a = get(), b = get();
    SPSVM_HIP(hipEventRecord(a, st));
    launch();
    SPSVM_HIP(hipEventRecord(b, st));
    pending.push_back({a, b, cat, w});
    if (pending.size() >= 2048) {
      SPSVM_HIP(hipStreamSynchronize(st));
      flush();
    }
  }
  void flush() {  // the stream must have been synchronised
    for (const Pending& p : pending) {
      float ms = 0.f;
      SPSVM_HIP(hipEventElapsedTime(&ms, p.a, p.b));
      seconds[p.cat] += 1e-3 * ms;
      work[p.cat] += p.work;
      count[p.cat] += 1;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  ~Profiler() {
    for (const Pending& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};
enum { kProfKblock = 0, kProfSyrk = 1, kProfScore = 2, kProfChol = 3 };

template <typename TX, typename TK>
struct Impl {
  const TX* X;   // caller's n x d matrix
  const TX* Xk;  // the matrix the kernel-block GEMMs read: X itself or its padded copy (row stride p.ldx)
  const float* y;
  int64_t n, d, J_max;
  double C, gamma, lam;
  spsvm_options opt;
  hipStream_t st;
  Plan p;
  char* base;
  Pinned pin;
  spsvm_stats stats{};
  Profiler prof;

  TK *xnorm, *KXJ, *Kc;
  uint64_t *hash, *stage_hash;
  double *o, *delta, *beta, *dvec, *g, *z, *H, *Linv, *syrk_part, *grad_part, *score_part, *ls_part, *cblk_sum;
  double *XJ64, *xjnorm, *KJJ, *vJ, *wJ, *o_stage, *Hf;
  int32_t *iota, *incomplete, *F_in, *F_out, *fcnt_in, *fcnt_out;
  bool bf16_exact = false;  // every X value is exactly a BF16 number (split-BF16 lo parts are all zero)
  bool hb_valid = false;  // H (unfactored) holds lambda K_JJ + K_I^T K_I for the first m_fact basis vectors and
  int m_fact = 0;         // the violator status in act_fact
  uint8_t *act_fact, *act_cur;
  int32_t *I, *cblk_cnt, *cblk_flips, *cand_table, *m_dev, *flags, *J32;
  int64_t* J;
  CandState* cst;
  Selection* sel;
  LineState* ls;
  NewtonScalars* sc;
  std::vector<uint64_t> hash_host;

  template <typename T>
  T* at(size_t off) {
    return reinterpret_cast<T*>(base + off);
  }

  Impl(const TX* X_, const float* y_, int64_t n_, int64_t d_, double C_, double g_, int64_t Jm, const spsvm_options& o_,
       void* ws, hipStream_t s, const Plan& plan)
      : X(X_), y(y_), n(n_), d(d_), J_max(Jm), C(C_), gamma(g_), lam(1.0 / C_), opt(o_), st(s), p(plan),
        base((char*)ws), pin(kPinnedScalars + (size_t)o_.chunk_cap * kCandSlots * 4) {
    prof.st = s;
    prof.mask = o_.profile;
    Xk = p.pad_x ? at<TX>(p.Xp) : X;
    xnorm = at<TK>(p.xnorm);
    KXJ = at<TK>(p.KXJ);
    Kc = at<TK>(p.Kc);
    hash = at<uint64_t>(p.hash);
    stage_hash = at<uint64_t>(p.stage_hash);
    o = at<double>(p.o);
    delta = at<double>(p.delta);
    beta = at<double>(p.beta);
    dvec = at<double>(p.dvec);
    g = at<double>(p.g);
    z = at<double>(p.z);
    H = at<double>(p.H);
    Linv = at<double>(p.Linv);
    syrk_part = at<double>(p.syrk_part);
    grad_part = at<double>(p.grad_part);
    score_part = at<double>(p.score_part);
    ls_part = at<double>(p.ls_part);
    cblk_sum = at<double>(p.cblk_sum);
    act_fact = at<uint8_t>(p.act0);
    act_cur = at<uint8_t>(p.act1);
    I = at<int32_t>(p.I);
    cblk_cnt = at<int32_t>(p.cblk_cnt);
    cblk_flips = at<int32_t>(p.cblk_flips);
    cand_table = at<int32_t>(p.cand_table);
    m_dev = at<int32_t>(p.m_dev);
    flags = at<int32_t>(p.flags);
    J32 = at<int32_t>(p.J32);
    J = at<int64_t>(p.J);
    cst = at<CandState>(p.cand_state);
    sel = at<Selection>(p.sel);
    ls = at<LineState>(p.ls);
    sc = at<NewtonScalars>(p.scalars);
    XJ64 = at<double>(p.XJ64);
    xjnorm = at<double>(p.xjnorm);
    KJJ = at<double>(p.KJJ);
    vJ = at<double>(p.vJ);
    wJ = at<double>(p.wJ);
    iota = at<int32_t>(p.iota);
    incomplete = at<int32_t>(p.incomplete);
    o_stage = at<double>(p.o_stage);
    Hf = at<double>(p.Hf);
    F_in = at<int32_t>(p.F_in);
    F_out = at<int32_t>(p.F_out);
    fcnt_in = at<int32_t>(p.fcnt_in);
    fcnt_out = at<int32_t>(p.fcnt_out);
  }

  // The n x N kernel block in the training precision (split-BF16 products in MIXED mode).
  void kblock(const int32_t* cols, int ncols, TK* out, int64_t ldo) {
    if constexpr (std::is_same<TK, float>::value) {
      if (opt.precision == SPSVM_MIXED) {
        launch_kblock_split<TX>(Xk, p.ldx, n, d, xnorm, cols, ncols, out, ldo, gamma, bf16_exact, st);
        return;
      }
    }
    launch_kblock<TX, TK>(Xk, p.ldx, n, d, xnorm, cols, ncols, out, ldo, gamma, st);
  }

  // Basis rows m0..m1 of J gathered into XJ64 (FP64), then the FP64 kernel matrix K_JJ of the first m1 rows.
  void update_basis(int m0, int m1) {
    if (m1 <= m0) return;
    launch_gather_rows<TX, double>(X, d, J + m0, m1 - m0, XJ64 + (size_t)m0 * p.ldj, p.ldj, st);
    launch_row_norms<double, double>(XJ64 + (size_t)m0 * p.ldj, m1 - m0, d, p.ldj, xjnorm + m0, st);
    launch_kblock<double, double>(XJ64, p.ldj, m1, d, xjnorm, iota, m1, KJJ, p.ldh, gamma, st);
  }

  void sync() {
    SPSVM_HIP(hipStreamSynchronize(st));
    prof.flush();
  }

  template <typename T>
  T read(const T* dev) {
    SPSVM_HIP(hipMemcpyAsync(pin.p, dev, sizeof(T), hipMemcpyDeviceToHost, st));
    sync();
    T v;
    std::memcpy(&v, pin.p, sizeof(T));
    return v;
  }

  // ---------------------------------------------------------------------------------------- preparation
  void prepare() {
    SPSVM_HIP(hipMemsetAsync(flags, 0, 12, st));
    launch_iota(iota, J_max, st);
    if (p.pad_x) launch_pad_rows<TX>(X, n, d, at<TX>(p.Xp), p.ldx, st);
    launch_check_inputs<TX>(X, n * d, y, n, flags, st);
    launch_row_hash<TX>(X, n, d, hash, st);
    launch_row_norms<TX, TK>(X, n, d, d, xnorm, st);
    hash_host.resize(n);
    SPSVM_HIP(hipMemcpyAsync(hash_host.data(), hash, n * 8, hipMemcpyDeviceToHost, st));
    SPSVM_HIP(hipMemcpyAsync(pin.p, flags, 12, hipMemcpyDeviceToHost, st));
    sync();
    int32_t f[3];
    std::memcpy(f, pin.p, 12);
    if (f[0]) throw Failure(SPSVM_E_INVALID_ARG, "X holds NaN or Inf");
    bf16_exact = f[2] == 0;
    if (f[1]) throw Failure(SPSVM_E_INVALID_ARG, "labels must be exactly +1 or -1");
    std::vector<uint64_t> hs = hash_host;
    std::sort(hs.begin(), hs.end());
    const int64_t distinct = std::unique(hs.begin(), hs.end()) - hs.begin();
    if (J_max > distinct)
      throw Failure(SPSVM_E_INVALID_ARG, "J_max (" + std::to_string(J_max) + ") exceeds the number of distinct rows (" +
                                             std::to_string(distinct) + ")");
  }

  // prepare() for a batch: the label check covers all P label vectors (ny values).
  void prepare_batch(const float* Y, int64_t ny) {
    const float* keep = y;
    y = nullptr;
    prepare();
    y = keep;
    SPSVM_HIP(hipMemsetAsync(flags, 0, 8, st));
    launch_check_inputs<TX>(X, 0, Y, ny, flags, st);
    SPSVM_HIP(hipMemcpyAsync(pin.p, flags, 8, hipMemcpyDeviceToHost, st));
    sync();
    int32_t f[2];
    std::memcpy(f, pin.p, 8);
    if (f[1]) throw Failure(SPSVM_E_INVALID_ARG, "labels must be exactly +1 or -1");
  }

  // ------------------------------------------------------------------------------------ Newton at fixed J
  // Returns the number of iterations.
  int newton(int m) {
    if (m <= 0) return 0;
    launch_gemv<TK>(KXJ, p.ldk, n, m, beta, o, st);
    bool fact_valid = false;
    double g0 = 0.0;
    int it = 0;
    for (; it < opt.newton_max_iter; ++it) {
      launch_compact(o, y, n, hb_valid ? act_fact : nullptr, act_cur, I, cblk_cnt, cblk_sum, cblk_flips, sc, st);
      NewtonScalars s = read(sc);
      const int nchunk = gradient_chunks(m, s.n_sv);
      launch_gemv<double>(KJJ, p.ldh, m, m, beta, vJ, st);
      launch_gradient<TK>(KXJ, p.ldk, m, I, s.n_sv, o, y, vJ, beta, lam, grad_part, nchunk, g, sc, st);
      s = read(sc);
      const double gn = std::sqrt(s.gnorm2);
      const double f = 0.5 * lam * s.beta_oJ + 0.5 * s.sum_a2;
      if (!std::isfinite(f) || !std::isfinite(gn))
        throw Failure(SPSVM_E_NO_CONVERGENCE, "non-finite objective or gradient in Newton (m=" + std::to_string(m) + ")");
      if (it == 0) g0 = gn;
      if (opt.log_level >= 2)
        std::fprintf(stderr, "[spsvm]   newton it=%d m=%d f=%.15e |g|=%.3e n_sv=%d flips=%d\n", it, m, f, gn, s.n_sv,
                     s.flips);
      if (gn <= opt.newton_tol * std::max(1.0, g0)) break;
      if (!fact_valid || s.flips > opt.refactor_frac * std::max(1, s.n_sv)) {
        factorize(m, s.n_sv);
        fact_valid = true;
        std::swap(act_fact, act_cur);
      }
      launch_chol_solve(Hf, p.ldh, m, Linv, g, dvec, z, st);
      launch_gemv<TK>(KXJ, p.ldk, n, m, dvec, delta, st);
      launch_gemv<double>(KJJ, p.ldh, m, m, dvec, wJ, st);
      launch_c1c2(beta, dvec, wJ, m, ls, st);
      const int nblk = score_blocks(n);
      LineState L;
      int rounds = 0;
      for (;;) {
        for (int r = 0; r < 3; ++r) launch_ls_round(o, delta, y, n, lam, ls, ls_part, nblk, st);
        rounds += 3;
        L = read(ls);
        if (L.status != 0 || rounds >= 66) break;
      }
      stats.ls_passes += L.passes;
      launch_apply_step(ls, beta, dvec, m, o, delta, n, st);
      if (L.t == 0.0) {
        ++it;
        break;
      }
      if (L.dec <= opt.newton_ftol * f) {
        ++it;
        break;
      }
    }
    if (it >= opt.newton_max_iter) stats.iter_cap_hits += 1;
    stats.newton_iters += it;
    return it;
  }

  // Forms H = lambda K_JJ + K_I^T K_I for the current basis (m) and violator status (act_cur), then factors a
  // copy. Tile rows of H that already existed at the last factorisation are updated with the rows that joined
  // or left the violator set (exact FP64 products, so the update loses nothing); the remaining tile rows are
  // recomputed over all violators. A full recomputation is chosen when it is cheaper.
  void factorize(int m, int n_sv) {
    const int B = syrk_tile_size();
    const int T = syrk_tile_rows(m), ntile = T * (T + 1) / 2;
    int tr0 = 0, n_in = 0, n_out = 0;
    if (hb_valid) {
      launch_flip_lists(act_cur, act_fact, n, fcnt_in, fcnt_out, F_in, F_out, sc, st);
      const NewtonScalars s = read(sc);
      n_in = s.n_in;
      n_out = s.n_out;
      const int t0 = m_fact / B;
      const double r0 = (double)t0 * B;
      const double cost_inc = (double)(n_in + n_out) * r0 * r0 + (double)n_sv * ((double)m * m - r0 * r0);
      const double cost_full = (double)n_sv * m * m;
      if (cost_inc < 0.8 * cost_full) tr0 = t0;
    }
    const int t_old = tr0 * (tr0 + 1) / 2;
    const double r0 = (double)tr0 * B;
    auto syrk_part = [&](const int32_t* rows, int nrows, int lo, int hi, int mode, double work) {
      if (nrows <= 0 || hi <= lo) return;
      const int ns = syrk_splits(hi - lo, nrows);
      prof.timed(kProfSyrk, work, [&] { launch_syrk<TK>(KXJ, p.ldk, m, rows, nrows, lo, hi, ns, this->syrk_part, st); });
      launch_syrk_reduce(KJJ, m, lam, this->syrk_part, ns, lo, hi, mode, H, p.ldh, st);
    };
    if (tr0 > 0) {
      syrk_part(F_in, n_in, 0, t_old, +1, (double)n_in * r0 * (r0 + 1.0));
      syrk_part(F_out, n_out, 0, t_old, -1, (double)n_out * r0 * (r0 + 1.0));
      stats.incremental_factorizations += 1;
    }
    if (t_old < ntile) {
      if (n_sv > 0) {
        syrk_part(I, n_sv, t_old, ntile, 0, (double)n_sv * ((double)m * (m + 1.0) - r0 * (r0 + 1.0)));
      } else {  // no violators: H = lambda K_JJ on the recomputed tiles
        launch_syrk<TK>(KXJ, p.ldk, m, I, 0, t_old, ntile, 1, this->syrk_part, st);
        launch_syrk_reduce(KJJ, m, lam, this->syrk_part, 1, t_old, ntile, 0, H, p.ldh, st);
      }
    }
    hb_valid = true;
    m_fact = m;
    // factor a copy of H (H itself is kept for the next update)
    SPSVM_HIP(hipMemcpyAsync(Hf, H, (size_t)m * p.ldh * 8, hipMemcpyDeviceToDevice, st));
    SPSVM_HIP(hipMemsetAsync(&sc->fail, 0, 4, st));
    prof.timed(kProfChol, (double)m * m * m / 3.0, [&] { launch_cholesky(Hf, p.ldh, m, Linv, sc, st); });
    stats.factorizations += 1;
    if (read(&sc->fail) == 0) return;
    // jitter retries: H + mu * mean(diag H) * I
    launch_trace(H, p.ldh, m, sc, st);
    const double mean_diag = read(&sc->trace) / m;
    for (double mu : {1e-14, 1e-12, 1e-10, 1e-8}) {
      SPSVM_HIP(hipMemcpyAsync(Hf, H, (size_t)m * p.ldh * 8, hipMemcpyDeviceToDevice, st));
      launch_add_diag(Hf, p.ldh, m, mu * mean_diag, st);
      SPSVM_HIP(hipMemsetAsync(&sc->fail, 0, 4, st));
      launch_cholesky(Hf, p.ldh, m, Linv, sc, st);
      stats.factorizations += 1;
      if (read(&sc->fail) == 0) return;
    }
    throw Failure(SPSVM_E_NOT_PD, "Newton matrix not positive definite after jitter retries (m=" + std::to_string(m) + ")");
  }

  // Objective and residual statistics at the current beta (o is recomputed).
  void final_eval(int m, double* F, NewtonScalars* out) {
    if (m == 0) {
      *F = C * 0.5 * (double)n;
      return;
    }
    launch_gemv<TK>(KXJ, p.ldk, n, m, beta, o, st);
    launch_compact(o, y, n, nullptr, act_cur, I, cblk_cnt, cblk_sum, cblk_flips, sc, st);
    NewtonScalars s = read(sc);
    launch_gemv<double>(KJJ, p.ldh, m, m, beta, vJ, st);
    launch_gradient<TK>(KXJ, p.ldk, m, I, s.n_sv, o, y, vJ, beta, lam, grad_part, gradient_chunks(m, s.n_sv), g, sc, st);
    s = read(sc);
    *out = s;
    *F = C * (0.5 * lam * s.beta_oJ + 0.5 * s.sum_a2);
  }

  // ------------------------------------------------------------------------------------ greedy training
  int select_and_optimise() {
    int m = 0;
    int64_t t = 0;
    std::vector<uint64_t> blocked;  // sorted hashes of J's rows
    std::vector<int32_t> table((size_t)opt.chunk_cap * kCandSlots);
    SPSVM_HIP(hipMemsetAsync(o, 0, n * 8, st));
    SPSVM_HIP(hipMemsetAsync(m_dev, 0, 4, st));
    const int nblk = score_blocks(n);
    int first_rounds = 4;
    while (m < J_max) {
      const auto t0 = clk::now();
      const int cs = (int)stage_size(m, J_max, opt.growth, opt.chunk_cap);
      for (int q = 0; q < cs; ++q) draw_step(opt.seed, t + q, n, opt.kappa, hash_host, blocked, &table[(size_t)q * kCandSlots]);
      int32_t* tp = (int32_t*)((char*)pin.p + kPinnedScalars);
      std::memcpy(tp, table.data(), (size_t)cs * kCandSlots * 4);
      SPSVM_HIP(hipMemcpyAsync(cand_table, tp, (size_t)cs * kCandSlots * 4, hipMemcpyHostToDevice, st));
      // One attempt runs every step of the stage without host synchronisation. A step whose slots did not all
      // converge within the launched passes selects nothing and flags the stage, which is then rerun from its
      // saved start state with more passes (64 passes always suffice: the update stops every slot by then).
      SPSVM_HIP(hipMemcpyAsync(o_stage, o, n * 8, hipMemcpyDeviceToDevice, st));
      for (int attempt = 0;; ++attempt) {
        // passes launched per step: one more than the most any step of the previous stage needed
        const int rounds = attempt == 0 ? first_rounds : (attempt == 1 ? std::max(2 * first_rounds, 12) : 64);
        if (attempt > 0) {
          SPSVM_HIP(hipMemcpyAsync(o, o_stage, n * 8, hipMemcpyDeviceToDevice, st));
          int32_t* mh = (int32_t*)((char*)pin.p + 8192);
          *mh = m;
          SPSVM_HIP(hipMemcpyAsync(m_dev, mh, 4, hipMemcpyHostToDevice, st));
          stats.stage_redos += 1;
        }
        SPSVM_HIP(hipMemsetAsync(incomplete, 0, 8, st));
        for (int q = 0; q < cs; ++q) {
          const int32_t* cq = cand_table + (size_t)q * kCandSlots;
          int ncand = 0;
          for (int c = 0; c < kCandSlots; ++c) ncand += table[(size_t)q * kCandSlots + c] >= 0;
          prof.timed(kProfKblock, 2.0 * n * ncand * d,
                     [&] { kblock(cq, kCandSlots, Kc, kCandSlots); });
          launch_score_init(cq, o, hash, stage_hash, q, cst, sc, st);
          for (int r = 0; r < rounds; ++r) {
            prof.timed(kProfScore, (double)n * (opt.kappa * sizeof(TK) + 12.0),
                       [&] { launch_score_pass<TK>(Kc, y, o, n, cst, score_part, nblk, st); });
            launch_score_update(cst, score_part, nblk, lam, st);
          }
          stats.score_passes += rounds;
          launch_select_append<TK>(cst, hash, stage_hash, q, Kc, n, o, KXJ, p.ldk, J, beta, m_dev, sel, incomplete, st);
        }
        int32_t flags2[2];
        SPSVM_HIP(hipMemcpyAsync(pin.p, incomplete, 8, hipMemcpyDeviceToHost, st));
        sync();
        std::memcpy(flags2, pin.p, 8);
        first_rounds = std::min(64, std::max(3, flags2[1] + 1));
        if (flags2[0] == 0 || rounds >= 64) break;
      }
      t += cs;
      const int m_new = read(m_dev);
      stats.additions += m_new - m;
      if (m_new > m) {
        std::vector<int64_t> jn(m_new - m);
        SPSVM_HIP(hipMemcpyAsync(jn.data(), J + m, (m_new - m) * 8, hipMemcpyDeviceToHost, st));
        sync();
        for (int64_t j : jn) blocked.push_back(hash_host[j]);
        std::sort(blocked.begin(), blocked.end());
      }
      const auto t1 = clk::now();
      stats.seconds_select += secs(t0, t1);
      if (m_new == m) break;
      update_basis(m, m_new);
      m = m_new;
      const int its = newton(m);
      stats.stages += 1;
      const auto t2 = clk::now();
      stats.seconds_newton += secs(t1, t2);
      if (opt.log_level >= 1)
        std::fprintf(stderr, "[spsvm] stage %lld |J|=%d added=%d newton_iters=%d select=%.3fs newton=%.3fs\n",
                     (long long)stats.stages, m, cs, its, secs(t0, t1), secs(t1, t2));
    }
    return m;
  }

  int fixed_basis(const int64_t* Jh, int64_t m) {
    std::vector<uint64_t> hs(m);
    for (int64_t k = 0; k < m; ++k) {
      if (Jh[k] < 0 || Jh[k] >= n) throw Failure(SPSVM_E_INVALID_ARG, "basis index out of range");
      hs[k] = hash_host[Jh[k]];
    }
    std::sort(hs.begin(), hs.end());
    if (std::unique(hs.begin(), hs.end()) != hs.end())
      throw Failure(SPSVM_E_INVALID_ARG, "basis rows must be pairwise distinct in value");
    std::vector<int32_t> j32(Jh, Jh + m);
    SPSVM_HIP(hipMemcpyAsync(J, Jh, m * 8, hipMemcpyHostToDevice, st));
    SPSVM_HIP(hipMemcpyAsync(J32, j32.data(), m * 4, hipMemcpyHostToDevice, st));
    const auto t0 = clk::now();
    prof.timed(kProfKblock, 2.0 * n * m * d,
               [&] { kblock(J32, (int)m, KXJ, p.ldk); });
    update_basis(0, (int)m);
    SPSVM_HIP(hipMemsetAsync(beta, 0, m * 8, st));
    sync();
    const auto t1 = clk::now();
    stats.seconds_select += secs(t0, t1);
    newton((int)m);
    stats.stages = 1;
    stats.seconds_newton += secs(t1, clk::now());
    return (int)m;
  }

  // ------------------------------------------------------------------------- batched problems, shared J
  // The squared distances D(X, X_J) (n x m) and D_JJ (FP64) are computed once; for each distinct gamma the
  // kernel block K = exp(-gamma D) and K_JJ are formed once, then each problem with that gamma runs the
  // Newton re-optimisation from beta = 0 with its own labels and C.
  void batch(int64_t P, const float* Y, const double* Cs, const double* gs, const int64_t* Jh, int64_t m,
             spsvm_model** outs) {
    std::vector<uint64_t> hs(m);
    for (int64_t k = 0; k < m; ++k) {
      if (Jh[k] < 0 || Jh[k] >= n) throw Failure(SPSVM_E_INVALID_ARG, "basis index out of range");
      hs[k] = hash_host[Jh[k]];
    }
    std::sort(hs.begin(), hs.end());
    if (std::unique(hs.begin(), hs.end()) != hs.end())
      throw Failure(SPSVM_E_INVALID_ARG, "basis rows must be pairwise distinct in value");
    std::vector<int32_t> j32(Jh, Jh + m);
    SPSVM_HIP(hipMemcpyAsync(J, Jh, m * 8, hipMemcpyHostToDevice, st));
    SPSVM_HIP(hipMemcpyAsync(J32, j32.data(), m * 4, hipMemcpyHostToDevice, st));
    TK* D = at<TK>(p.D);
    double* DJJ = at<double>(p.DJJ);
    const auto t0 = clk::now();
    // distances once: n x m block (training precision) and the basis block in FP64
    {
      const double keep = gamma;
      gamma = 0.0;
      prof.timed(kProfKblock, 2.0 * n * m * d, [&] { kblock(J32, (int)m, D, p.ldk); });
      gamma = keep;
    }
    launch_gather_rows<TX, double>(X, d, J, m, XJ64, p.ldj, st);
    launch_row_norms<double, double>(XJ64, m, d, p.ldj, xjnorm, st);
    launch_kblock<double, double>(XJ64, p.ldj, m, d, xjnorm, iota, (int)m, DJJ, p.ldh, 0.0, st);
    sync();
    const double dist_s = secs(t0, clk::now());
    std::vector<char> done(P, 0);
    for (int64_t a = 0; a < P; ++a) {
      if (done[a]) continue;
      const double g = gs[a];
      launch_rbf_from_dist<TK>(D, n, (int)m, p.ldk, KXJ, g, st);
      launch_rbf_from_dist<double>(DJJ, m, (int)m, p.ldh, KJJ, g, st);
      for (int64_t q = a; q < P; ++q) {
        if (done[q] || gs[q] != g) continue;
        done[q] = 1;
        const auto t1 = clk::now();
        stats = spsvm_stats{};
        y = Y + q * n;
        C = Cs[q];
        lam = 1.0 / C;
        gamma = g;
        hb_valid = false;
        SPSVM_HIP(hipMemsetAsync(beta, 0, m * 8, st));
        newton((int)m);
        stats.stages = 1;
        stats.seconds_select = dist_s / P;  // share of the distance block
        stats.seconds_newton = secs(t1, clk::now());
        outs[q] = build_model((int)m);
      }
    }
  }

  spsvm_model* build_model(int m) {
    double F = 0.0;
    NewtonScalars s{};
    final_eval(m, &F, &s);
    stats.n_sv = s.n_sv;
    stats.grad_norm = std::sqrt(s.gnorm2);
    sync();
    stats.kblock_launches = prof.count[kProfKblock];
    stats.kblock_seconds = prof.seconds[kProfKblock];
    stats.kblock_flops = prof.work[kProfKblock];
    stats.syrk_launches = prof.count[kProfSyrk];
    stats.syrk_seconds = prof.seconds[kProfSyrk];
    stats.syrk_flops = prof.work[kProfSyrk];
    stats.score_launches = prof.count[kProfScore];
    stats.score_seconds = prof.seconds[kProfScore];
    stats.score_bytes = prof.work[kProfScore];
    stats.chol_calls = prof.count[kProfChol];
    stats.chol_seconds = prof.seconds[kProfChol];
    stats.chol_flops = prof.work[kProfChol];
    auto* md = new spsvm_model();
    try {
      md->m = m;
      md->d = d;
      md->tk_double = std::is_same<TK, double>::value;
      md->C = C;
      md->gamma = gamma;
      md->objective = F;
      md->stats = stats;
      md->J.resize(m);
      md->beta.resize(m);
      if (m > 0) {
        SPSVM_HIP(hipMemcpyAsync(md->J.data(), J, m * 8, hipMemcpyDeviceToHost, st));
        SPSVM_HIP(hipMemcpyAsync(md->beta.data(), beta, m * 8, hipMemcpyDeviceToHost, st));
        md->ldz = padded_ld<TK>(d);
        SPSVM_HIP(hipMalloc(&md->XJ, (size_t)m * md->ldz * sizeof(TK)));
        SPSVM_HIP(hipMalloc(&md->XJnorm, (size_t)m * sizeof(TK)));
        SPSVM_HIP(hipMalloc(&md->beta_dev, (size_t)m * 8));
        launch_gather_rows<TX, TK>(X, d, J, m, (TK*)md->XJ, md->ldz, st);
        launch_row_norms<TK, TK>((const TK*)md->XJ, m, d, md->ldz, (TK*)md->XJnorm, st);
        SPSVM_HIP(hipMemcpyAsync(md->beta_dev, beta, m * 8, hipMemcpyDeviceToDevice, st));
        sync();
      }
    } catch (...) {
      delete md;
      throw;
    }
    return md;
  }
};

template <typename TX, typename TK>
spsvm_model* train_typed(const TX* X, const float* y, int64_t n, int64_t d, double C, double gamma, int64_t J_max,
                         const spsvm_options& opt, void* ws, const Plan& plan, hipStream_t st, const int64_t* J_fixed) {
  Impl<TX, TK> im(X, y, n, d, C, gamma, J_max, opt, ws, st, plan);
  im.prepare();
  const int m = J_fixed ? im.fixed_basis(J_fixed, J_max) : im.select_and_optimise();
  return im.build_model(m);
}

}  // namespace

spsvm_model* run_train(const void* X, bool x_double, const float* y, int64_t n, int64_t d, double C, double gamma,
                       int64_t J_max, const spsvm_options& opt, void* ws, size_t ws_bytes, hipStream_t stream,
                       const int64_t* J_fixed) {
  const Plan plan = make_plan(n, d, J_max, opt, J_fixed == nullptr, x_double, ((uintptr_t)X & 15u) == 0);
  if (!ws || ((uintptr_t)ws & 255u)) throw Failure(SPSVM_E_WORKSPACE, "workspace must be a 256-byte aligned device pointer");
  if (ws_bytes < plan.bytes)
    throw Failure(SPSVM_E_WORKSPACE, "workspace too small: need " + std::to_string(plan.bytes) + " bytes, got " +
                                         std::to_string(ws_bytes));
  const bool tk_double = opt.precision == SPSVM_F64;
  if (x_double)
    return tk_double ? train_typed<double, double>((const double*)X, y, n, d, C, gamma, J_max, opt, ws, plan, stream, J_fixed)
                     : train_typed<double, float>((const double*)X, y, n, d, C, gamma, J_max, opt, ws, plan, stream, J_fixed);
  return tk_double ? train_typed<float, double>((const float*)X, y, n, d, C, gamma, J_max, opt, ws, plan, stream, J_fixed)
                   : train_typed<float, float>((const float*)X, y, n, d, C, gamma, J_max, opt, ws, plan, stream, J_fixed);
}

template <typename TX, typename TK>
static void predict_typed(const spsvm_model* md, const TX* Xt, int64_t n_t, double* out, hipStream_t st) {
  const int64_t d = md->d, ld = padded_ld<TX>(d);
  const TX* A = Xt;
  void* tmp = nullptr;
  if (ld != d || ((uintptr_t)Xt & 15u)) {  // rows must start on 16-byte boundaries: use a padded copy
    SPSVM_HIP(hipMalloc(&tmp, (size_t)n_t * ld * sizeof(TX)));
    launch_pad_rows<TX>(Xt, n_t, d, (TX*)tmp, ld, st);
    A = (const TX*)tmp;
  }
  try {
    launch_predict<TX, TK>(A, ld, n_t, d, (const TK*)md->XJ, md->ldz, (const TK*)md->XJnorm, (int)md->m, md->beta_dev,
                           out, md->gamma, st);
    SPSVM_HIP(hipStreamSynchronize(st));
  } catch (...) {
    if (tmp) (void)hipFree(tmp);
    throw;
  }
  if (tmp) SPSVM_HIP(hipFree(tmp));
}

template <typename TX, typename TK>
static void batch_typed(const TX* X, int64_t n, int64_t d, int64_t P, const float* Y, const double* C,
                        const double* gamma, const int64_t* J, int64_t m, const spsvm_options& opt, void* ws,
                        const Plan& plan, hipStream_t st, spsvm_model** out) {
  Impl<TX, TK> im(X, Y, n, d, C[0], gamma[0], m, opt, ws, st, plan);
  im.prepare_batch(Y, n * P);
  try {
    im.batch(P, Y, C, gamma, J, m, out);
  } catch (...) {
    for (int64_t p = 0; p < P; ++p) {
      delete out[p];
      out[p] = nullptr;
    }
    throw;
  }
}

void run_train_batch(const void* X, bool x_double, int64_t n, int64_t d, int64_t P, const float* Y, const double* C,
                     const double* gamma, const int64_t* J, int64_t m, const spsvm_options& opt, void* ws,
                     size_t ws_bytes, hipStream_t stream, spsvm_model** out) {
  const Plan plan = make_plan(n, d, m, opt, false, x_double, ((uintptr_t)X & 15u) == 0, true);
  if (!ws || ((uintptr_t)ws & 255u)) throw Failure(SPSVM_E_WORKSPACE, "workspace must be a 256-byte aligned device pointer");
  if (ws_bytes < plan.bytes)
    throw Failure(SPSVM_E_WORKSPACE, "workspace too small: need " + std::to_string(plan.bytes) + " bytes, got " +
                                         std::to_string(ws_bytes));
  for (int64_t p = 0; p < P; ++p) out[p] = nullptr;
  const bool tk_double = opt.precision == SPSVM_F64;
  if (x_double) {
    if (tk_double)
      batch_typed<double, double>((const double*)X, n, d, P, Y, C, gamma, J, m, opt, ws, plan, stream, out);
    else
      batch_typed<double, float>((const double*)X, n, d, P, Y, C, gamma, J, m, opt, ws, plan, stream, out);
  } else {
    if (tk_double)
      batch_typed<float, double>((const float*)X, n, d, P, Y, C, gamma, J, m, opt, ws, plan, stream, out);
    else
      batch_typed<float, float>((const float*)X, n, d, P, Y, C, gamma, J, m, opt, ws, plan, stream, out);
  }
}

void run_predict(const spsvm_model* md, const void* Xt, bool x_double, int64_t n_t, double* out, hipStream_t st) {
  if (md->m == 0) {
    SPSVM_HIP(hipMemsetAsync(out, 0, n_t * 8, st));
    SPSVM_HIP(hipStreamSynchronize(st));
  } else if (md->tk_double) {
    if (x_double)
      predict_typed<double, double>(md, (const double*)Xt, n_t, out, st);
    else
      predict_typed<float, double>(md, (const float*)Xt, n_t, out, st);
  } else {
    if (x_double)
      predict_typed<double, float>(md, (const double*)Xt, n_t, out, st);
    else
      predict_typed<float, float>(md, (const float*)Xt, n_t, out, st);
  }
}

}  // namespace spsvm
