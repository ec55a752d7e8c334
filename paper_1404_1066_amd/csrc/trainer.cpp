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
  // step t starts 2^32 states after step t - 1 (before the seed is mixed in): a step makes at most 64 kappa
  // draws, so the streams of different steps never share a state and each step draws a fresh subset
  uint64_t state = seed ^ ((((uint64_t)t << 32) + 1) * kGolden);
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

// Steps whose candidate columns come from one kernel-block launch. For wide rows every launch streams all of X
// once, and the column tiles of the steps of a stage (all drawn at its start) share each row slab of it through
// L2; launches of more column tiles spread that stream over more products (2 000 000 x 2000 rows, single-pass
// BF16: 3, 4, 6, 9 and 12 tiles of 256 columns per launch ran at 815, 787-815, 866, 881 and 894 TFLOP/s). A
// launch takes only the valid candidates of its steps, each written to its own slot, so a group is as many steps
// as fill twelve such tiles (52 at kappa = 59: 3068 columns), at most 52: the candidate buffer keeps 64 slots
// per step, n x 64 x 52 values. The first scoring pass is launched for all but the first step.
// Gradient contraction per Newton step below which an older factor is formed again (see newton_slots).
constexpr double kReuseContraction = 100.0;

int cand_group(int64_t d, int64_t chunk_cap, int kappa) {
  const int64_t fill = std::max<int64_t>(1, 3072 / std::max(1, std::min(kappa, kCandSlots)));
  return (int)std::min<int64_t>(d >= 256 ? std::min<int64_t>(52, fill) : 1, std::max<int64_t>(chunk_cap, 1));
}

int64_t stage_size(int64_t J, int64_t J_max, double growth, int64_t cap) {
  const int64_t g = (int64_t)std::floor(growth * (double)J);
  return std::min<int64_t>(J_max - J, std::max<int64_t>(1, std::min<int64_t>(cap, g)));
}

// ------------------------------------------------------------------------------------------ workspace
Plan make_plan(int64_t n, int64_t d, int64_t J_max, const spsvm_options& opt, bool with_selection, bool x_double,
               bool x_aligned, bool batch, int64_t problems, bool csr, int shared_gammas) {
  Plan p;
  p.csr = csr;
  const int64_t xe = x_double ? 8 : 4;
  p.ldx = round_up(d, 16 / xe);
  // FP32 / FP64 kernel blocks read X with 16-byte vector loads, so rows must start on 16-byte boundaries (else a
  // padded copy); the mixed-precision blocks read the split BF16 copies instead and never need it
  p.pad_x = !csr && opt.precision != SPSVM_MIXED && (p.ldx != d || !x_aligned);
  p.ldj = padded_ld<double>(d);
  p.n = n;
  p.d = d;
  p.J_max = J_max;
  p.tk_double = opt.precision == SPSVM_F64;
  p.batch = batch;
  p.slots = batch ? (int)std::max<int64_t>(1, std::min<int64_t>(problems, kBatchSlots)) : 1;
  p.off = opt.bias ? 1 : 0;
  const int64_t Ms = J_max + p.off;  // largest Newton system: the basis vectors and the offset
  p.ldk = round_up(Ms, 4);
  p.ldh = round_up(Ms, 4);
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
  p.kxj_host = opt.kxj_host != 0;
  p.KXJ = take(p.kxj_host ? 0 : (size_t)n * p.ldk * tk);
  p.Kc = take(with_selection ? (size_t)round_up(n, 4) * kCandSlots * (csr ? 1 : cand_group(d, opt.chunk_cap, opt.kappa)) * tk
                             : 0);
  p.J = take(J_max * 8);
  p.J32 = take(J_max * 4);
  p.cand_state = take(kCandStateBytes);
  p.sel = take(sizeof(Selection));
  p.ls = take(p.slots * sizeof(LineState));
  p.scalars = take(p.slots * sizeof(NewtonScalars));
  p.score_part = take((size_t)std::max<int64_t>(nb_s, ceil_div(n, kKblockRows)) * kCandSlots * 4 * 8);
  p.cand_table = take((size_t)cap * kCandSlots * 4);
  p.cand_cols = take(with_selection && !csr ? (size_t)2 * cap * kCandSlots * 4 : 0);  // launch rows, then slots
  p.stage_hash = take(cap * 8);
  p.m_dev = take(8);  // basis size, double-buffered by step parity
  p.flags = take(16);
  p.XJ64 = take((size_t)J_max * p.ldj * 8);
  p.xjnorm = take(J_max * 8);
  p.KJJ = take((size_t)Ms * p.ldh * 8);
  p.iota = take(J_max * 4);
  p.incomplete = take(32);  // [0] a step did not settle, [1] most passes needed, [2] working passes, [3] slot-passes, [4] first step to redo
  p.Xp = take(p.pad_x ? (size_t)n * p.ldx * xe : 0);
  const bool fixed_batch = batch && shared_gammas == 0;  // the distances and K^T K of a given shared basis
  p.D = take(fixed_batch ? (size_t)n * p.ldk * tk : 0);
  p.DJJ = take(fixed_batch ? (size_t)J_max * p.ldh * 8 : 0);
  p.G = take(fixed_batch ? (size_t)Ms * p.ldh * 8 : 0);
  if (shared_gammas > 0) {
    p.shared_gammas = shared_gammas;
    p.problems = problems;
    auto arr = [&](size_t each, int64_t count, size_t* stride) {
      *stride = (size_t)round_up((int64_t)std::max<size_t>(each, 1), 256);
      return take(*stride * (size_t)std::max<int64_t>(count, 1));
    };
    p.sh_K = arr((size_t)n * p.ldk * tk, shared_gammas - 1, &p.sh_K_stride);
    p.sh_KJJ = arr((size_t)Ms * p.ldh * 8, shared_gammas - 1, &p.sh_KJJ_stride);
    p.sh_Kc = arr((size_t)round_up(n, 4) * kCandSlots * tk, shared_gammas - 1, &p.sh_Kc_stride);
    p.sh_o = arr((size_t)n * 8, problems, &p.sh_o_stride);
    p.sh_beta = arr((size_t)Ms * 8, problems, &p.sh_beta_stride);
    p.sh_cst = arr(kCandStateBytes, problems, &p.sh_cst_stride);
  }
  const bool mixed = opt.precision == SPSVM_MIXED;
  p.ldb = split_ld(d);
  p.Xhi = take(mixed ? (size_t)n * p.ldb * 2 : 0);
  p.Xlo = take(mixed ? (size_t)n * p.ldb * 2 : 0);
  p.Zc = take(csr ? (size_t)kCandSlots * d * 4 : 0);
  // one problem's Newton state
  {
    size_t so = 0;
    auto st = [&](size_t bytes) {
      const size_t at = so;
      so += (size_t)round_up((int64_t)std::max<size_t>(bytes, 1), 256);
      return at;
    };
    SlotPlan& q = p.slot;
    q.o = st(n * 8);
    q.delta = st(n * 8);
    q.act0 = st(n);
    q.act1 = st(n);
    q.I = st(n * 4);
    q.cblk_cnt = st(nb_c * 4);
    q.cblk_sum = st(nb_c * 8);
    q.cblk_flips = st(nb_c * 4);
    q.beta = st(Ms * 8);
    q.dvec = st(Ms * 8);
    q.g = st(Ms * 8);
    q.z = st(Ms * 8);
    q.H = st((size_t)Ms * p.ldh * 8);
    q.Hf = st((size_t)Ms * p.ldh * 8);
    q.Linv = st((size_t)ceil_div(Ms, kCholNB) * kCholNB * kCholNB * 8);
    q.syrk_part = st((batch ? syrk_partial_doubles_batch((int)Ms) : syrk_partial_doubles((int)Ms)) * 8);
    q.grad_part = st((size_t)1024 * 256 * 8);
    q.ls_part = st((size_t)ls_blocks(n) * 6 * 8);
    q.vJ = st(Ms * 8);
    q.wJ = st(Ms * 8);
    q.F_in = st(n * 4);
    q.F_out = st(n * 4);
    q.fcnt_in = st(nb_c * 4);
    q.fcnt_out = st(nb_c * 4);
    q.bytes = so;
  }
  p.slots_at = take((size_t)p.slots * p.slot.bytes);
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
  int stride = 1;  // time every stride-th launch of a category
  int64_t seen[4] = {0, 0, 0, 0};
  struct Pending {
    hipEvent_t a, b;
    int cat;
    double work, work2;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  double seconds[4] = {0, 0, 0, 0}, work[4] = {0, 0, 0, 0}, work2[4] = {0, 0, 0, 0};
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
  // w: algorithmic work of the launch; w2: a second figure (the MFMA flops a kernel block issues)
  template <class F>
  void timed(int cat, double w, F&& launch, double w2 = 0.0) {
    if (!(mask & (1 << cat)) || (seen[cat]++ % stride) != 0) {
      launch();
      return;
    }
    hipEvent_t a = get(), b = get();
    SPSVM_HIP(hipEventRecord(a, st));
    launch();
    SPSVM_HIP(hipEventRecord(b, st));
    pending.push_back({a, b, cat, w, w2});
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
      work2[p.cat] += p.work2;
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
  const TX* X;   // caller's n x d matrix (null for CSR rows)
  CsrX csr;      // CSR rows (indptr null for a dense X)
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
  double *XJ64, *xjnorm, *KJJ, *vJ, *wJ, *Hf;
  int32_t *iota, *incomplete, *F_in, *F_out, *fcnt_in, *fcnt_out;
  bool bf16_exact = false;  // every X value is exactly a BF16 number (split-BF16 lo parts are all zero)
  uint8_t *act_fact, *act_cur;
  int32_t *I, *cblk_cnt, *cblk_flips, *cand_table, *m_dev, *flags, *J32;
  int64_t* J;
  CandState* cst;
  Selection* sel;
  LineState* ls;
  NewtonScalars* sc;
  std::vector<uint64_t> hash_host;

  // One problem's Newton state. A training run uses slot 0 (its buffers are also the members above); a batch
  // runs up to kBatchSlots problems in lockstep, one per slot.
  struct Slot {
    const float* y = nullptr;
    double C = 1.0, lam = 1.0;
    const TK* K = nullptr;         // n x ldk kernel block of the basis
    const double* KJJ = nullptr;   // FP64 kernel matrix of the basis (ldh)
    double *o, *delta, *beta, *dvec, *g, *z, *H, *Hf, *Linv, *syrk_part, *grad_part, *ls_part, *cblk_sum, *vJ, *wJ;
    uint8_t *act_fact, *act_cur;
    int32_t *I, *cblk_cnt, *cblk_flips, *F_in, *F_out, *fcnt_in, *fcnt_out;
    NewtonScalars* sc;
    LineState* ls;
    spsvm_stats* stats = nullptr;  // counters this slot's solves add to
    spsvm_stats own{};
    bool hb_valid = false;  // H (unfactored) holds lambda K_JJ + K_I^T K_I for the first m_fact basis vectors and
    int m_fact = 0;         // the violator status in act_fact
    // the current solve
    bool fact_valid = false;
    bool reused = false;  // the last step solved with a factor formed before an earlier step
    double g0 = 0.0, f = 0.0, g_step = 0.0;  // g_step: ||grad f|| before the last step
    int it = 0, tr0 = 0, n_in = 0, n_out = 0;
    NewtonScalars s{};
    LineState L{};
  };
  std::vector<Slot> slots;
  Pinned pin_slots;
  void* host_k = nullptr;  // pinned host memory holding K_XJ (kxj_host)
  ~Impl() {
    if (host_k) {
      (void)hipStreamSynchronize(st);
      (void)hipHostFree(host_k);
    }
  }
  Impl(const Impl&) = delete;
  Impl& operator=(const Impl&) = delete;

  template <typename T>
  T* at(size_t off) {
    return reinterpret_cast<T*>(base + off);
  }

  Impl(const TX* X_, const float* y_, int64_t n_, int64_t d_, double C_, double g_, int64_t Jm, const spsvm_options& o_,
       void* ws, hipStream_t s, const Plan& plan)
      : X(X_), y(y_), n(n_), d(d_), J_max(Jm), C(C_), gamma(g_), lam(1.0 / C_), opt(o_), st(s), p(plan),
        base((char*)ws), pin(kPinnedScalars + (size_t)3 * o_.chunk_cap * kCandSlots * 4),
        pin_slots((size_t)plan.slots * (sizeof(NewtonScalars) + sizeof(LineState))) {
    prof.st = s;
    prof.mask = o_.profile & 0xF;
    prof.stride = std::max(1, (o_.profile >> 8) & 0xFF);
    Xk = p.pad_x ? at<TX>(p.Xp) : X;
    xnorm = at<TK>(p.xnorm);
    if (p.kxj_host) {  // K_XJ beyond the workspace: pinned host memory, mapped for the kernels
      SPSVM_HIP(hipHostMalloc(&host_k, (size_t)n * p.ldk * sizeof(TK), hipHostMallocDefault));
      KXJ = (TK*)host_k;
    } else {
      KXJ = at<TK>(p.KXJ);
    }
    Kc = at<TK>(p.Kc);
    hash = at<uint64_t>(p.hash);
    stage_hash = at<uint64_t>(p.stage_hash);
    score_part = at<double>(p.score_part);
    cand_table = at<int32_t>(p.cand_table);
    m_dev = at<int32_t>(p.m_dev);
    flags = at<int32_t>(p.flags);
    J32 = at<int32_t>(p.J32);
    J = at<int64_t>(p.J);
    cst = at<CandState>(p.cand_state);
    sel = at<Selection>(p.sel);
    XJ64 = at<double>(p.XJ64);
    xjnorm = at<double>(p.xjnorm);
    KJJ = at<double>(p.KJJ);
    iota = at<int32_t>(p.iota);
    incomplete = at<int32_t>(p.incomplete);
    slots.resize(p.slots);
    for (int q = 0; q < p.slots; ++q) {
      Slot& S = slots[q];
      char* b = base + p.slots_at + (size_t)q * p.slot.bytes;
      const SlotPlan& sp = p.slot;
      S.o = (double*)(b + sp.o);
      S.delta = (double*)(b + sp.delta);
      S.beta = (double*)(b + sp.beta);
      S.dvec = (double*)(b + sp.dvec);
      S.g = (double*)(b + sp.g);
      S.z = (double*)(b + sp.z);
      S.H = (double*)(b + sp.H);
      S.Hf = (double*)(b + sp.Hf);
      S.Linv = (double*)(b + sp.Linv);
      S.syrk_part = (double*)(b + sp.syrk_part);
      S.grad_part = (double*)(b + sp.grad_part);
      S.ls_part = (double*)(b + sp.ls_part);
      S.cblk_sum = (double*)(b + sp.cblk_sum);
      S.vJ = (double*)(b + sp.vJ);
      S.wJ = (double*)(b + sp.wJ);
      S.act_fact = (uint8_t*)(b + sp.act0);
      S.act_cur = (uint8_t*)(b + sp.act1);
      S.I = (int32_t*)(b + sp.I);
      S.cblk_cnt = (int32_t*)(b + sp.cblk_cnt);
      S.cblk_flips = (int32_t*)(b + sp.cblk_flips);
      S.F_in = (int32_t*)(b + sp.F_in);
      S.F_out = (int32_t*)(b + sp.F_out);
      S.fcnt_in = (int32_t*)(b + sp.fcnt_in);
      S.fcnt_out = (int32_t*)(b + sp.fcnt_out);
      S.sc = at<NewtonScalars>(p.scalars) + q;
      S.ls = at<LineState>(p.ls) + q;
      S.stats = p.batch ? &S.own : &stats;
    }
    Slot& s0 = slots[0];
    s0.y = y;
    s0.C = C;
    s0.lam = lam;
    s0.K = KXJ;
    s0.KJJ = KJJ;
    o = s0.o;
    delta = s0.delta;
    beta = s0.beta;
    dvec = s0.dvec;
    g = s0.g;
    z = s0.z;
    H = s0.H;
    Hf = s0.Hf;
    Linv = s0.Linv;
    syrk_part = s0.syrk_part;
    grad_part = s0.grad_part;
    ls_part = s0.ls_part;
    cblk_sum = s0.cblk_sum;
    vJ = s0.vJ;
    wJ = s0.wJ;
    act_fact = s0.act_fact;
    act_cur = s0.act_cur;
    I = s0.I;
    cblk_cnt = s0.cblk_cnt;
    cblk_flips = s0.cblk_flips;
    F_in = s0.F_in;
    F_out = s0.F_out;
    fcnt_in = s0.fcnt_in;
    fcnt_out = s0.fcnt_out;
    sc = s0.sc;
    ls = s0.ls;
  }

  // The n x N kernel block in the training precision (split-BF16 products in MIXED mode; single-pass BF16 products,
  // hi.hi' only, when single_pass is set).
  void kblock(const int32_t* cols, int ncols, TK* out, int64_t ldo, const Score0& s0 = Score0{},
              bool colmajor = false, bool single_pass = false) {
    if constexpr (std::is_same<TX, float>::value && std::is_same<TK, float>::value) {
      if (csr.indptr) {  // sparse rows against the candidate rows made dense (column-major, no fused first pass)
        if (!colmajor || ncols > kCandSlots) throw Failure(SPSVM_E_INVALID_ARG, "sparse rows: column-major blocks of <= 64");
        float* Zc = at<float>(p.Zc);
        launch_csr_gather<int32_t, float>(csr.indptr, csr.indices, csr.values, cols, ncols, Zc, d, st);
        launch_csr_kblock(csr.indptr, csr.indices, csr.values, n, d, xnorm, Zc, d, nullptr, cols, ncols, out, ldo,
                          gamma, 0, nullptr, st);
        return;
      }
    }
    if constexpr (std::is_same<TK, float>::value) {
      if (opt.precision == SPSVM_MIXED) {
        launch_kblock_bf16(at<unsigned short>(p.Xhi), bf16_exact || single_pass ? nullptr : at<unsigned short>(p.Xlo),
                           p.ldb, n, xnorm, cols, ncols, out, ldo, gamma, st, s0, colmajor);
        return;
      }
    }
    launch_kblock<TX, TK>(Xk, p.ldx, n, d, xnorm, cols, ncols, out, ldo, gamma, st, s0, colmajor);
  }

  // Kernel a candidate block of ncols columns runs on: in MIXED precision the split-BF16 block's tile variant (one
  // kernel each), else the path's one kernel (-1).
  int cand_kernel(int64_t ncols, bool single_pass) const {
    if constexpr (std::is_same<TK, float>::value) {
      if (opt.precision == SPSVM_MIXED && !csr.indptr)
        return kblock_bf16_variant(n, p.ldb, ncols, !bf16_exact && !single_pass, true);
    }
    return -1;
  }

  // MFMA flops kblock() issues for ncols columns.
  double kblock_issued(int64_t ncols, bool single_pass = false, bool candidates = false) const {
    if constexpr (std::is_same<TK, float>::value) {
      if (opt.precision == SPSVM_MIXED)
        return kblock_bf16_issued_flops(n, p.ldb, ncols, !bf16_exact && !single_pass, candidates);
    }
    return kblock_issued_flops(n, d, ncols);
  }

  // MIXED precision on values that are not all BF16 numbers: the candidate columns, which only feed the selection
  // heuristic's scores, come from single-pass BF16 products; the columns of the stage's winners, which enter K_XJ
  // and the Newton system, are formed again with the split correction once the stage is complete.
  bool single_pass_candidates() const {
    return std::is_same<TK, float>::value && opt.precision == SPSVM_MIXED && !bf16_exact;
  }

  // Basis rows m0..m1 of J gathered into XJ64 (FP64), then the FP64 kernel matrix K_JJ of the first m1 rows.
  void update_basis(int m0, int m1) {
    if (m1 <= m0) return;
    if (csr.indptr)
      launch_csr_gather<int64_t, double>(csr.indptr, csr.indices, csr.values, J + m0, m1 - m0,
                                         XJ64 + (size_t)m0 * p.ldj, p.ldj, st);
    else
      launch_gather_rows<TX, double>(X, d, J + m0, m1 - m0, XJ64 + (size_t)m0 * p.ldj, p.ldj, st);
    launch_row_norms<double, double>(XJ64 + (size_t)m0 * p.ldj, m1 - m0, d, p.ldj, xjnorm + m0, st);
    launch_kblock<double, double>(XJ64, p.ldj, m1, d, xjnorm, iota, m1, KJJ + (size_t)p.off * (p.ldh + 1), p.ldh,
                                  gamma, st);
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
    SPSVM_HIP(hipMemsetAsync(flags, 0, 16, st));
    launch_iota(iota, J_max, st);
    if (csr.indptr) {
      if constexpr (std::is_same<TX, float>::value) {
        launch_check_inputs<float>(csr.values, csr.nnz, y, n, flags, st);
        launch_csr_check(csr.indptr, csr.indices, n, d, flags + 3, st);
        launch_csr_row_hash(csr.indptr, csr.indices, csr.values, n, d, hash, st);
        launch_csr_row_norms<TK>(csr.indptr, csr.values, n, xnorm, st);
      }
    } else {
      if (p.pad_x) launch_pad_rows<TX>(X, n, d, at<TX>(p.Xp), p.ldx, st);
      launch_check_inputs<TX>(X, n * d, y, n, flags, st);
      launch_row_hash<TX>(X, n, d, hash, st);
      launch_row_norms<TX, TK>(X, n, d, d, xnorm, st);
    }
    hash_host.resize(n);
    SPSVM_HIP(hipMemcpyAsync(hash_host.data(), hash, n * 8, hipMemcpyDeviceToHost, st));
    SPSVM_HIP(hipMemcpyAsync(pin.p, flags, 16, hipMemcpyDeviceToHost, st));
    sync();
    int32_t f[4];
    std::memcpy(f, pin.p, 16);
    if (f[0]) throw Failure(SPSVM_E_INVALID_ARG, "X holds NaN or Inf");
    if (f[3]) throw Failure(SPSVM_E_INVALID_ARG, "sparse rows: feature indices must lie in [0, d) and increase within a row");
    bf16_exact = f[2] == 0;
    if (opt.precision == SPSVM_MIXED)
      launch_split_bf16<TX>(X, n, d, d, at<unsigned short>(p.Xhi), bf16_exact ? nullptr : at<unsigned short>(p.Xlo),
                            p.ldb, st);
    if (f[1]) throw Failure(SPSVM_E_INVALID_ARG, "labels must be exactly +1 or -1");
    if (p.off) {  // the offset's coordinate: a column of ones in K_XJ, a zero row and column in K_JJ
      launch_fill_column<TK>(KXJ, n, p.ldk, 0, 1.0, st);
      SPSVM_HIP(hipMemsetAsync(KJJ, 0, (size_t)(J_max + 1) * p.ldh * 8, st));
    }
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

  // Reads every slot's NewtonScalars (or LineState) back in one copy.
  void read_slots() {
    const size_t b = slots.size() * sizeof(NewtonScalars);
    SPSVM_HIP(hipMemcpyAsync(pin_slots.p, slots[0].sc, b, hipMemcpyDeviceToHost, st));
    sync();
    for (size_t q = 0; q < slots.size(); ++q) std::memcpy(&slots[q].s, (char*)pin_slots.p + q * sizeof(NewtonScalars), sizeof(NewtonScalars));
  }
  void read_slot_lines() {
    const size_t b = slots.size() * sizeof(LineState);
    SPSVM_HIP(hipMemcpyAsync(pin_slots.p, slots[0].ls, b, hipMemcpyDeviceToHost, st));
    sync();
    for (size_t q = 0; q < slots.size(); ++q) std::memcpy(&slots[q].L, (char*)pin_slots.p + q * sizeof(LineState), sizeof(LineState));
  }

  // ------------------------------------------------------------------------------------ Newton at fixed J
  // Newton re-optimisation of beta at a fixed basis of m vectors, for the given slots in lockstep: each phase
  // is launched for every unfinished slot before the host reads their scalars back in one copy, and the SYRK,
  // Cholesky and triangular solves of all slots are batched launches. Every slot takes exactly the decisions
  // and kernel calls of a solve on its own. Returns the iterations of the first slot.
  int newton(int m) { return newton_slots(m, {0}); }

  // out = K x (the slot's n x m kernel block) for the given slots; in a batch one MFMA launch serves up to
  // kMaxBatch slots with a single read of the shared block.
  void gemv_slots(int m, const std::vector<int>& ids, double* Slot::*x, double* Slot::*out) {
    if (!p.batch) {
      for (int q : ids) launch_gemv<TK>(slots[q].K, p.ldk, n, m, slots[q].*x, slots[q].*out, st);
      return;
    }
    for (size_t a = 0; a < ids.size(); a += kMaxBatch) {
      GemvBatch gb{};
      const TK* K = slots[ids[a]].K;
      for (size_t k = a; k < ids.size() && k < a + kMaxBatch; ++k) {
        const Slot& S = slots[ids[k]];
        if (S.K != K) throw Failure(SPSVM_E_INVALID_ARG, "batched GEMV: slots must share the kernel block");
        gb.x[gb.count] = S.*x;
        gb.out[gb.count] = S.*out;
        gb.count++;
      }
      launch_gemv_batch<TK>(K, p.ldk, n, m, gb, st);
    }
  }

  // out = K_JJ x (FP64, m x m) for the given slots, batched like gemv_slots.
  void gemv_kjj_slots(int m, const std::vector<int>& ids, double* Slot::*x, double* Slot::*out) {
    if (!p.batch) {
      for (int q : ids) launch_gemv<double>(slots[q].KJJ, p.ldh, m, m, slots[q].*x, slots[q].*out, st);
      return;
    }
    for (size_t a = 0; a < ids.size(); a += kMaxBatch) {
      GemvBatch gb{};
      const double* KJJ = slots[ids[a]].KJJ;
      for (size_t k = a; k < ids.size() && k < a + kMaxBatch; ++k) {
        const Slot& S = slots[ids[k]];
        if (S.KJJ != KJJ) throw Failure(SPSVM_E_INVALID_ARG, "batched GEMV: slots must share K_JJ");
        gb.x[gb.count] = S.*x;
        gb.out[gb.count] = S.*out;
        gb.count++;
      }
      launch_gemv_batch<double>(KJJ, p.ldh, m, m, gb, st);
    }
  }

  // Gradient, |g|^2 and beta . K_JJ beta for the given slots (their violator sets compacted on the device). A
  // batch takes the dense form, one read of K for up to kMaxBatch slots.
  void gradient_slots(int m, const std::vector<int>& ids) {
    gemv_kjj_slots(m, ids, &Slot::beta, &Slot::vJ);
    if (!p.batch) {
      for (int q : ids) {
        Slot& S = slots[q];
        launch_gradient<TK>(S.K, p.ldk, m, S.I, S.o, S.y, S.vJ, S.beta, S.lam, S.grad_part,
                            gradient_chunks(m, (int)n), S.g, S.sc, st);
      }
      return;
    }
    for (size_t a = 0; a < ids.size(); a += kMaxBatch) {
      GradBatch gb{};
      const TK* K = slots[ids[a]].K;
      for (size_t k = a; k < ids.size() && k < a + kMaxBatch; ++k) {
        const Slot& S = slots[ids[k]];
        if (S.K != K) throw Failure(SPSVM_E_INVALID_ARG, "batched gradient: slots must share the kernel block");
        const int c = gb.count++;
        gb.o[c] = S.o;
        gb.y[c] = S.y;
        gb.partial[c] = S.grad_part;
        gb.v[c] = S.vJ;
        gb.beta[c] = S.beta;
        gb.g[c] = S.g;
        gb.sc[c] = S.sc;
        gb.lam[c] = S.lam;
      }
      launch_gradient_batch<TK>(K, p.ldk, n, m, gb, st);
    }
  }

  int newton_slots(int m, const std::vector<int>& ids) {
    if (m <= 0 || ids.empty()) return 0;
    std::vector<int> act;
    gemv_slots(m, ids, &Slot::beta, &Slot::o);
    for (int q : ids) {
      Slot& S = slots[q];
      S.fact_valid = false;
      S.reused = false;
      S.g0 = 0.0;
      S.it = 0;
      act.push_back(q);
    }
    auto finish = [&](Slot& S) {
      if (S.it >= opt.newton_max_iter) S.stats->iter_cap_hits += 1;
      S.stats->newton_iters += S.it;
    };
    const int first = ids[0];
    int first_its = 0;
    while (!act.empty()) {
      for (size_t a = 0; a < act.size(); a += kMaxBatch) {
        CompactBatch cb{};
        for (size_t k = a; k < act.size() && k < a + kMaxBatch; ++k) {
          Slot& S = slots[act[k]];
          const int c = cb.count++;
          cb.o[c] = S.o;
          cb.y[c] = S.y;
          cb.act_ref[c] = S.hb_valid ? S.act_fact : nullptr;
          cb.act_out[c] = S.act_cur;
          cb.I[c] = S.I;
          cb.cnt[c] = S.cblk_cnt;
          cb.bsum[c] = S.cblk_sum;
          cb.bflips[c] = S.cblk_flips;
          cb.sc[c] = S.sc;
        }
        launch_compact_batch(cb, n, st);
      }
      gradient_slots(m, act);  // takes |I| from the device
      read_slots();
      std::vector<int> go, refac;
      for (int q : act) {
        Slot& S = slots[q];
        const double gn = std::sqrt(S.s.gnorm2);
        S.f = 0.5 * S.lam * S.s.beta_oJ + 0.5 * S.s.sum_a2;
        if (!std::isfinite(S.f) || !std::isfinite(gn))
          throw Failure(SPSVM_E_NO_CONVERGENCE, "non-finite objective or gradient in Newton (m=" + std::to_string(m) + ")");
        if (S.it == 0) S.g0 = gn;
        if (opt.log_level >= 2)
          std::fprintf(stderr, "[spsvm]   newton slot=%d it=%d m=%d f=%.15e |g|=%.3e n_sv=%d flips=%d\n", q, S.it, m,
                       S.f, gn, S.s.n_sv, S.s.flips);
        if (gn <= opt.newton_tol * std::max(1.0, S.g0)) {
          finish(S);
          if (q == first) first_its = S.it;
          continue;
        }
        go.push_back(q);
        // An older factor is kept while few violators changed since it was formed and each step solved with it
        // cut ||grad f|| at least kReuseContraction-fold (Newton-like); a slower step means the matrix drifted
        // too far, and the remaining steps would only converge linearly.
        const bool slow = S.reused && gn * kReuseContraction > S.g_step;
        if (!S.fact_valid || slow || S.s.flips > opt.refactor_frac * std::max(1, S.s.n_sv)) {
          refac.push_back(q);
          S.reused = false;
        } else {
          S.reused = true;
        }
        S.g_step = gn;
      }
      if (go.empty()) break;
      factorize_slots(m, refac);
      for (int q : refac) {
        Slot& S = slots[q];
        S.fact_valid = true;
        std::swap(S.act_fact, S.act_cur);
      }
      for (size_t a = 0; a < go.size(); a += kMaxBatch) {
        SolveBatch sb{};
        for (size_t k = a; k < go.size() && k < a + kMaxBatch; ++k) {
          const Slot& S = slots[go[k]];
          const int c = sb.count++;
          sb.L[c] = S.Hf;
          sb.Linv[c] = S.Linv;
          sb.g[c] = S.g;
          sb.x[c] = S.dvec;
          sb.work[c] = S.z;
        }
        launch_chol_solve_batch(sb, p.ldh, m, st);
      }
      gemv_slots(m, go, &Slot::dvec, &Slot::delta);
      gemv_kjj_slots(m, go, &Slot::dvec, &Slot::wJ);
      // line search: all unfinished slots in each launch (up to kMaxBatch)
      auto ls_batch = [&](const std::vector<int>& ids, size_t a) {
        LsBatch b{};
        for (size_t k = a; k < ids.size() && k < a + kMaxBatch; ++k) {
          Slot& S = slots[ids[k]];
          const int c = b.count++;
          b.o[c] = S.o;
          b.delta[c] = S.delta;
          b.y[c] = S.y;
          b.ls[c] = S.ls;
          b.partial[c] = S.ls_part;
          b.lam[c] = S.lam;
          b.beta[c] = S.beta;
          b.dvec[c] = S.dvec;
          b.w[c] = S.wJ;
        }
        return b;
      };
      for (size_t a = 0; a < go.size(); a += kMaxBatch) launch_c1c2_batch(ls_batch(go, a), m, st);
      const int nblk = ls_blocks(n);
      std::vector<int> lsq = go;
      int rounds = 0;
      while (!lsq.empty()) {
        for (size_t a = 0; a < lsq.size(); a += kMaxBatch) {
          const LsBatch b = ls_batch(lsq, a);
          for (int r = 0; r < 3; ++r) launch_ls_round_batch(b, n, nblk, st);
        }
        rounds += 3;
        read_slot_lines();
        std::vector<int> keep;
        for (int q : lsq)
          if (slots[q].L.status == 0 && rounds < 66) keep.push_back(q);
        lsq.swap(keep);
      }
      for (size_t a = 0; a < go.size(); a += kMaxBatch) launch_apply_step_batch(ls_batch(go, a), m, n, st);
      act.clear();
      for (int q : go) {
        Slot& S = slots[q];
        S.stats->ls_passes += S.L.passes;
        S.it += 1;
        if (S.L.t == 0.0 || S.L.dec <= opt.newton_ftol * S.f || S.it >= opt.newton_max_iter) {
          finish(S);
          if (q == first) first_its = S.it;
        } else {
          act.push_back(q);
        }
      }
    }
    return first_its;
  }

  // For the given slots: forms H = lambda K_JJ + K_I^T K_I for the current basis (m) and violator status
  // (act_cur), then factors a copy. Tile rows of H that already existed at the slot's last factorisation are
  // updated with the rows that joined or left the violator set (exact FP64 products, so the update loses
  // nothing); the remaining tile rows are recomputed over all violators. A full recomputation is chosen when it
  // is cheaper.
  void factorize(int m) { factorize_slots(m, {0}); }

  void factorize_slots(int m, const std::vector<int>& ids) {
    if (ids.empty()) return;
    const int B = syrk_tile_size();
    const int T = syrk_tile_rows(m), ntile = T * (T + 1) / 2;
    std::vector<int> fl;
    for (int q : ids)
      if (slots[q].hb_valid) fl.push_back(q);
    for (size_t a = 0; a < fl.size(); a += kMaxBatch) {
      FlipBatch fb{};
      for (size_t k = a; k < fl.size() && k < a + kMaxBatch; ++k) {
        Slot& S = slots[fl[k]];
        const int c = fb.count++;
        fb.act_new[c] = S.act_cur;
        fb.act_old[c] = S.act_fact;
        fb.cnt_in[c] = S.fcnt_in;
        fb.cnt_out[c] = S.fcnt_out;
        fb.F_in[c] = S.F_in;
        fb.F_out[c] = S.F_out;
        fb.sc[c] = S.sc;
      }
      launch_flip_lists_batch(fb, n, st);
    }
    if (!fl.empty()) read_slots();
    for (int q : ids) {
      Slot& S = slots[q];
      S.tr0 = 0;
      S.n_in = S.n_out = 0;
      if (!S.hb_valid) continue;
      S.n_in = S.s.n_in;
      S.n_out = S.s.n_out;
      // tile rows of H that are complete: all of them when the basis has not grown since, else those below
      // the last factorisation's partial tile row
      const int t0 = S.m_fact == m ? T : S.m_fact / B;
      const double r0 = std::min<double>((double)t0 * B, m);
      const double cost_inc = (double)(S.n_in + S.n_out) * r0 * r0 + (double)S.s.n_sv * ((double)m * m - r0 * r0);
      const double cost_full = (double)S.s.n_sv * m * m;
      if (cost_inc < 0.8 * cost_full) S.tr0 = t0;
    }
    // The three row sets (joined, left, recomputed tiles) run as batched SYRK launches, each followed by its
    // reduction into H (a slot's partial buffer is reused by the next set).
    for (int kind : {+1, -1, 0}) {
      std::vector<int> use;
      for (int q : ids) {
        const Slot& S = slots[q];
        const int t_old = S.tr0 * (S.tr0 + 1) / 2;
        if (kind != 0 && (S.tr0 == 0 || (kind > 0 ? S.n_in : S.n_out) <= 0)) continue;
        if (kind == 0 && t_old >= ntile) continue;
        use.push_back(q);
      }
      for (size_t a = 0; a < use.size(); a += kMaxBatch) {
        SyrkBatch<TK> sb{};
        ReduceBatch rb{};
        double work = 0.0;
        const int cnt = (int)std::min<size_t>(kMaxBatch, use.size() - a);
        for (int k = 0; k < cnt; ++k) {
          Slot& S = slots[use[a + k]];
          const int t_old = S.tr0 * (S.tr0 + 1) / 2;
          const double r0 = std::min<double>((double)S.tr0 * B, m);
          const int32_t* rows = kind > 0 ? S.F_in : (kind < 0 ? S.F_out : S.I);
          const int nrows = kind > 0 ? S.n_in : (kind < 0 ? S.n_out : S.s.n_sv);
          const int lo = kind == 0 ? t_old : 0, hi = kind == 0 ? ntile : t_old;
          const int ns = nrows <= 0 ? 1 : (p.batch ? syrk_splits_batch(hi - lo, nrows) : syrk_splits(hi - lo, nrows));
          sb.K[k] = S.K;
          sb.rows[k] = rows;
          sb.partial[k] = S.syrk_part;
          sb.n_rows[k] = std::max(nrows, 0);
          sb.nsplit[k] = ns;
          sb.tile_lo[k] = lo;
          sb.tile_hi[k] = hi;
          rb.KJJ[k] = S.KJJ;
          rb.partial[k] = S.syrk_part;
          rb.H[k] = S.H;
          rb.lam[k] = S.lam;
          rb.nsplit[k] = ns;
          rb.tile_lo[k] = lo;
          rb.tile_hi[k] = hi;
          rb.mode[k] = kind;
          work += kind == 0 ? (double)nrows * ((double)m * (m + 1.0) - r0 * (r0 + 1.0)) : (double)nrows * r0 * (r0 + 1.0);
        }
        sb.count = rb.count = cnt;
        if (work > 0.0)
          prof.timed(kProfSyrk, work, [&] { launch_syrk_batch<TK>(sb, p.ldk, m, st); });
        else
          launch_syrk_batch<TK>(sb, p.ldk, m, st);
        launch_syrk_reduce_batch(rb, m, p.ldh, st);
      }
    }
    for (int q : ids) {
      Slot& S = slots[q];
      if (S.tr0 > 0) S.stats->incremental_factorizations += 1;
      S.hb_valid = true;
      S.m_fact = m;
      // factor a copy of H (H itself is kept for the next update)
      SPSVM_HIP(hipMemcpyAsync(S.Hf, S.H, (size_t)m * p.ldh * 8, hipMemcpyDeviceToDevice, st));
      SPSVM_HIP(hipMemsetAsync(&S.sc->fail, 0, 4, st));
      S.stats->factorizations += 1;
    }
    for (size_t a = 0; a < ids.size(); a += kMaxBatch) {
      CholBatch cb{};
      for (size_t k = a; k < ids.size() && k < a + kMaxBatch; ++k) {
        const Slot& S = slots[ids[k]];
        const int c = cb.count++;
        cb.H[c] = S.Hf;
        cb.Linv[c] = S.Linv;
        cb.sc[c] = S.sc;
      }
      prof.timed(kProfChol, cb.count * (double)m * m * m / 3.0, [&] { launch_cholesky_batch(cb, p.ldh, m, st); });
    }
    read_slots();
    for (int q : ids) {
      Slot& S = slots[q];
      if (S.s.fail == 0) continue;
      // jitter retries: H + mu * mean(diag H) * I
      launch_trace(S.H, p.ldh, m, S.sc, st);
      const double mean_diag = read(&S.sc->trace) / m;
      bool ok = false;
      for (double mu : {1e-14, 1e-12, 1e-10, 1e-8}) {
        SPSVM_HIP(hipMemcpyAsync(S.Hf, S.H, (size_t)m * p.ldh * 8, hipMemcpyDeviceToDevice, st));
        launch_add_diag(S.Hf, p.ldh, m, mu * mean_diag, st);
        SPSVM_HIP(hipMemsetAsync(&S.sc->fail, 0, 4, st));
        launch_cholesky(S.Hf, p.ldh, m, S.Linv, S.sc, st);
        S.stats->factorizations += 1;
        S.stats->jitter_retries += 1;
        if (read(&S.sc->fail) == 0) {
          ok = true;
          break;
        }
      }
      if (!ok)
        throw Failure(SPSVM_E_NOT_PD,
                      "Newton matrix not positive definite after jitter retries (m=" + std::to_string(m) + ")");
    }
  }

  // Objective and residual statistics at the slot's current beta (o is recomputed unless the caller just did).
  void final_eval(Slot& S, int m, double* F, NewtonScalars* out, bool o_fresh = false) {
    if (m == 0) {
      *F = S.C * 0.5 * (double)n;
      return;
    }
    if (!o_fresh) launch_gemv<TK>(S.K, p.ldk, n, m, S.beta, S.o, st);
    launch_compact(S.o, S.y, n, nullptr, S.act_cur, S.I, S.cblk_cnt, S.cblk_sum, S.cblk_flips, S.sc, st);
    NewtonScalars s = read(S.sc);
    S.s = s;
    gradient_slots(m, {(int)(&S - slots.data())});
    s = read(S.sc);
    *out = s;
    *F = S.C * (0.5 * S.lam * s.beta_oJ + 0.5 * s.sum_a2);
  }

  // ------------------------------------------------------------------------------------ greedy training
  int select_and_optimise() {
    int m = 0;
    int64_t t = 0;
    std::vector<uint64_t> blocked;  // sorted hashes of J's rows
    std::vector<int32_t> table((size_t)opt.chunk_cap * kCandSlots);
    SPSVM_HIP(hipMemsetAsync(o, 0, n * 8, st));
    SPSVM_HIP(hipMemsetAsync(m_dev, 0, 8, st));
    SPSVM_HIP(hipMemsetAsync(beta, 0, (J_max + p.off) * 8, st));  // with the offset: b = 0 before the first stage
    const int nblk = score_blocks(n);
    const bool approx = single_pass_candidates();
    const double* bias_dev = p.off ? beta : nullptr;  // b (coefficient 0) when it is fitted
    double err_prev = 1.0;  // training error at o = 0: every y_i o_i = 0 counts as an error
    int first_rounds = 4;
    while (m < J_max) {
      const auto t0 = clk::now();
      const int cs = (int)stage_size(m, J_max, opt.growth, opt.chunk_cap);
      for (int q = 0; q < cs; ++q) draw_step(opt.seed, t + q, n, opt.kappa, hash_host, blocked, &table[(size_t)q * kCandSlots]);
      int32_t* tp = (int32_t*)((char*)pin.p + kPinnedScalars);
      std::memcpy(tp, table.data(), (size_t)cs * kCandSlots * 4);
      SPSVM_HIP(hipMemcpyAsync(cand_table, tp, (size_t)cs * kCandSlots * 4, hipMemcpyHostToDevice, st));
      // One attempt runs the steps of the stage without host synchronisation. A step whose slots did not all
      // converge within the launched passes selects nothing, and so does every later step of the attempt; the
      // stage then resumes from that step (o, J and the basis size are as the last complete step left them)
      // with more passes (64 passes always suffice: the update stops every slot by then).
      const int G = csr.indptr ? 1 : cand_group(d, opt.chunk_cap, opt.kappa);
      const int full_cols = G > 1 ? G * std::min(opt.kappa, kCandSlots) : kCandSlots;  // columns of a full group
      const bool fused = !csr.indptr;  // the dense blocks yield the first scoring pass of their first step
      int qstart = 0, m_q = m;  // first step of the attempt and the basis size it starts from
      for (int attempt = 0;; ++attempt) {
        const int rounds = attempt == 0   ? first_rounds
                           : attempt == 1 ? std::min(64, first_rounds + 2)
                           : attempt == 2 ? std::min(64, std::max(12, 2 * first_rounds + 4))
                                          : 64;
        {
          // the stage's steps read the basis size at m_dev[q & 1] and leave the next one at m_dev[(q + 1) & 1]
          int32_t* mh = (int32_t*)((char*)pin.p + 8192);
          *mh = m_q;
          SPSVM_HIP(hipMemcpyAsync(m_dev + (qstart & 1), mh, 4, hipMemcpyHostToDevice, st));
        }
        if (attempt > 0) stats.stage_redos += 1;
        SPSVM_HIP(hipMemsetAsync(incomplete, 0, 32, st));
        // Launches of several steps take only their valid candidates: per launch, the rows and their slots
        // (step within the launch x kCandSlots + slot), laid out launch after launch in cand_cols (rows, then
        // slots at cap x kCandSlots). draw_step fills a prefix of each step's slots, so the first step's
        // candidates keep launch column = slot, which the fused first scoring pass relies on.
        std::vector<int> g_off, g_cnt;
        int32_t* ccols = at<int32_t>(p.cand_cols);
        const size_t slots_cap = (size_t)opt.chunk_cap * kCandSlots;
        if (G > 1) {
          int32_t* rows_h = (int32_t*)((char*)pin.p + kPinnedScalars + slots_cap * 4);
          int32_t* dst_h = rows_h + slots_cap;
          int tot = 0;
          for (int q0 = qstart; q0 < cs; q0 += G) {
            const int gsz = std::min(G, cs - q0);
            g_off.push_back(tot);
            for (int j = 0; j < gsz; ++j)
              for (int c = 0; c < kCandSlots; ++c) {
                const int32_t v = table[(size_t)(q0 + j) * kCandSlots + c];
                if (v < 0) continue;
                rows_h[tot] = v;
                dst_h[tot] = j * kCandSlots + c;
                ++tot;
              }
            g_cnt.push_back(tot - g_off.back());
          }
          if (tot > 0) {
            SPSVM_HIP(hipMemcpyAsync(ccols, rows_h, (size_t)tot * 4, hipMemcpyHostToDevice, st));
            SPSVM_HIP(hipMemcpyAsync(ccols + slots_cap, dst_h, (size_t)tot * 4, hipMemcpyHostToDevice, st));
          }
        }
        for (int q0 = qstart, gi = 0; q0 < cs; q0 += G, ++gi) {
          const int gsz = std::min(G, cs - q0);  // steps sharing this kernel-block launch
          const int64_t ldc = round_up(n, 4);     // candidate columns, column-major (one contiguous column each)
          int ncand = 0;
          for (int c = 0; c < kCandSlots * gsz; ++c) ncand += table[(size_t)q0 * kCandSlots + c] >= 0;
          // the candidate block also yields the first scoring pass (at s = 0) of its first step
          Score0 s0;
          s0.y = y;
          s0.o = o;
          s0.partial = fused ? score_part : nullptr;
          s0.dst = G > 1 ? ccols + slots_cap + g_off[gi] : nullptr;
          const int32_t* cols = G > 1 ? ccols + g_off[gi] : cand_table + (size_t)q0 * kCandSlots;
          const int ncols = G > 1 ? g_cnt[gi] : kCandSlots * gsz;
          // timed: the launches on the kernel a full group runs on, so that the timings describe one kernel
          if (cand_kernel(ncols, approx) == cand_kernel(full_cols, approx))
            prof.timed(
                kProfKblock, 2.0 * n * ncand * d, [&] { kblock(cols, ncols, Kc, ldc, s0, true, approx); },
                kblock_issued(ncols, approx, true));
          else
            kblock(cols, ncols, Kc, ldc, s0, true, approx);
          for (int j = 0; j < gsz; ++j) {
            const int q = q0 + j;
            const int32_t* cq = cand_table + (size_t)q * kCandSlots;
            const TK* Kq = Kc + (size_t)j * kCandSlots * ldc;
            if (j == 0 && fused) {
              launch_score_init_update(cq, o, hash, stage_hash, q, cst, score_part, (int)ceil_div(n, kKblockRows),
                                       lam, bias_dev, st);
            } else {
              launch_score_init(cq, o, hash, stage_hash, q, cst, sc, bias_dev, st);
              prof.timed(kProfScore, (double)n * (opt.kappa * sizeof(TK) + 12.0),
                         [&] { launch_score_pass<TK>(Kq, ldc, y, o, n, cst, score_part, nblk, st); });
              launch_score_update(cst, score_part, nblk, lam, incomplete + 3, st);
            }
            for (int r = 1; r < rounds; ++r) {
              prof.timed(kProfScore, (double)n * (opt.kappa * sizeof(TK) + 12.0),
                         [&] { launch_score_pass<TK>(Kq, ldc, y, o, n, cst, score_part, nblk, st); });
              launch_score_update(cst, score_part, nblk, lam, incomplete + 3, st);
            }
            stats.score_passes += rounds - (j == 0 && fused ? 1 : 0);
            launch_select_append<TK>(cst, hash, stage_hash, q, Kq, ldc, n, o, KXJ, p.ldk, J, J32, beta, m_dev, sel,
                                     incomplete, j == 0 && fused ? 1 : 0, p.off, !approx, st);
          }
        }
        int32_t flags2[8];
        SPSVM_HIP(hipMemcpyAsync(pin.p, incomplete, 32, hipMemcpyDeviceToHost, st));
        sync();
        std::memcpy(flags2, pin.p, 32);
        stats.score_passes_active += flags2[2];
        stats.score_slot_passes += flags2[3];
        // passes for the next stage: as many as the most any step needed, plus one in reserve unless every step
        // of this attempt needed exactly that many (one kernel-block launch per step, so each step's count is
        // its own: a uniform stage predicts the next one well, and a miss only resumes from the step concerned)
        const bool uniform = G == 1 && flags2[0] == 0 && flags2[2] == (cs - qstart) * (flags2[1] - (fused ? 1 : 0));
        first_rounds = std::min(64, std::max(2, flags2[1] + (uniform ? 0 : 1)));
        if (flags2[0] == 0 || rounds >= 64) break;
        qstart = flags2[4];
        m_q = read(m_dev + (cs & 1));  // the steps after the incomplete one left the size unchanged
      }
      t += cs;
      const int m_new = read(m_dev + (cs & 1));
      stats.additions += m_new - m;
      if (m_new > m) {
        std::vector<int64_t> jn(m_new - m);
        SPSVM_HIP(hipMemcpyAsync(jn.data(), J + m, (m_new - m) * 8, hipMemcpyDeviceToHost, st));
        sync();
        for (int64_t j : jn) blocked.push_back(hash_host[j]);
        std::sort(blocked.begin(), blocked.end());
      }
      if (approx && m_new > m)  // the winners' columns, split-BF16
        kblock(J32 + m, m_new - m, KXJ + p.off + m, p.ldk);
      const auto t1 = clk::now();
      stats.seconds_select += secs(t0, t1);
      if (m_new == m) {
        stats.stop_reason = 2;
        break;
      }
      update_basis(m, m_new);
      const int added = m_new - m;
      m = m_new;
      const int its = newton(m + p.off);
      stats.stages += 1;
      bool stop = false;
      if (opt.eps_stop > 0.0) {  // the stopping rule of section 4, after the re-optimisation
        launch_count_errors(o, y, n, sc, st);
        const double err = (double)read(&sc->n_err) / (double)n;
        stats.train_error = err;
        stop = (err_prev - err) / added < opt.eps_stop;
        err_prev = err;
      }
      const auto t2 = clk::now();
      stats.seconds_newton += secs(t1, t2);
      if (opt.log_level >= 1)
        std::fprintf(stderr, "[spsvm] stage %lld |J|=%d added=%d newton_iters=%d select=%.3fs newton=%.3fs\n",
                     (long long)stats.stages, m, cs, its, secs(t0, t1), secs(t1, t2));
      if (stop) {
        stats.stop_reason = 1;
        break;
      }
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
    prof.timed(kProfKblock, 2.0 * n * m * d, [&] { kblock(J32, (int)m, KXJ + p.off, p.ldk); }, kblock_issued(m));
    update_basis(0, (int)m);
    SPSVM_HIP(hipMemsetAsync(beta, 0, (m + p.off) * 8, st));
    sync();
    const auto t1 = clk::now();
    stats.seconds_select += secs(t0, t1);
    newton((int)m + p.off);
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
      prof.timed(kProfKblock, 2.0 * n * m * d, [&] { kblock(J32, (int)m, D, p.ldk); }, kblock_issued(m));
      gamma = keep;
    }
    launch_gather_rows<TX, double>(X, d, J, m, XJ64, p.ldj, st);
    launch_row_norms<double, double>(XJ64, m, d, p.ldj, xjnorm, st);
    launch_kblock<double, double>(XJ64, p.ldj, m, d, xjnorm, iota, (int)m, DJJ, p.ldh, 0.0, st);
    sync();
    const double dist_s = secs(t0, clk::now());
    // Problems with the same gamma share the kernel block; they run in lockstep, up to one per slot.
    std::vector<char> done(P, 0);
    const int Q = (int)slots.size();
    for (int64_t a = 0; a < P; ++a) {
      if (done[a]) continue;
      const double g = gs[a];
      launch_rbf_from_dist<TK>(D, n, (int)m, p.ldk, KXJ + p.off, g, st);
      launch_rbf_from_dist<double>(DJJ, m, (int)m, p.ldh, KJJ + (size_t)p.off * (p.ldh + 1), g, st);
      gamma = g;
      std::vector<int64_t> group;
      for (int64_t q = a; q < P; ++q)
        if (!done[q] && gs[q] == g) {
          done[q] = 1;
          group.push_back(q);
        }
      // At beta = 0 every row is a violator, so every problem of the group starts from H = lambda K_JJ + K^T K
      // with the same K^T K (labels do not enter it): it is formed once over all n rows.
      double* G = at<double>(p.G);
      {
        Slot& S0 = slots[0];
        const int ms = (int)m + p.off;  // Newton system: the basis vectors and the offset
        const int T = syrk_tile_rows(ms), ntile = T * (T + 1) / 2;
        launch_iota(S0.I, n, st);
        const int ns = syrk_splits_batch(ntile, (int)n);
        prof.timed(kProfSyrk, (double)n * ms * (ms + 1.0),
                   [&] { launch_syrk<TK>(KXJ, p.ldk, ms, S0.I, (int)n, 0, ntile, ns, S0.syrk_part, st); });
        launch_syrk_reduce(KJJ, ms, 0.0, S0.syrk_part, ns, 0, ntile, 0, G, p.ldh, st);
      }
      for (size_t c0 = 0; c0 < group.size(); c0 += Q) {
        const auto t1 = clk::now();
        std::vector<int> ids;
        for (size_t k = c0; k < group.size() && k < c0 + Q; ++k) {
          const int64_t q = group[k];
          Slot& S = slots[ids.size()];
          S.own = spsvm_stats{};
          S.y = Y + q * n;
          S.C = Cs[q];
          S.lam = 1.0 / Cs[q];
          S.K = KXJ;
          S.KJJ = KJJ;
          launch_scaled_sum_lower(S.H, KJJ, G, S.lam, (int)m + p.off, p.ldh, st);
          SPSVM_HIP(hipMemsetAsync(S.act_fact, 1, n, st));  // every row a violator, as at beta = 0
          S.hb_valid = true;
          S.m_fact = (int)m + p.off;
          SPSVM_HIP(hipMemsetAsync(S.beta, 0, (m + p.off) * 8, st));
          ids.push_back((int)ids.size());
        }
        newton_slots((int)m + p.off, ids);
        gemv_slots((int)m + p.off, ids, &Slot::beta, &Slot::o);  // o at the final beta, for the models' statistics
        sync();
        const double share = secs(t1, clk::now()) / ids.size();
        for (size_t k = 0; k < ids.size(); ++k) {
          Slot& S = slots[ids[k]];
          S.own.stages = 1;
          S.own.seconds_select = dist_s / P;  // share of the distance block
          S.own.seconds_newton = share;       // share of the lockstep solve
          outs[group[c0 + k]] = build_model(S, (int)m, true);
        }
      }
    }
  }

  // ------------------------------------------------------------- batched problems, one greedy basis for all
  // The selection of section 4 for P problems on the same rows at once. Each step draws one candidate set (as for
  // one problem); every problem scores every candidate exactly with its own kernel column (one candidate block per
  // distinct gamma), labels, C and outputs, and no candidate is dropped (one that cannot win a problem may win the
  // sum); the largest sum of the problems' decreases wins (lower row on ties) and enters every problem with that
  // problem's one-dimensional optimum. After each stage every problem is re-optimised by Newton, the problems of
  // one gamma in lockstep on that gamma's kernel block, each from a freshly formed H.
  int shared(int64_t P, const float* Y, const double* Cs, const double* gs, spsvm_model** outs) {
    std::vector<double> gam;
    std::vector<int> gof(P);
    for (int64_t q = 0; q < P; ++q) {
      int g = 0;
      while (g < (int)gam.size() && gam[g] != gs[q]) ++g;
      if (g == (int)gam.size()) gam.push_back(gs[q]);
      gof[q] = g;
    }
    const int G = (int)gam.size();
    if (G != p.shared_gammas || P != p.problems) throw Failure(SPSVM_E_INVALID_ARG, "shared basis: plan mismatch");
    auto Kg = [&](int g) { return g == 0 ? KXJ : at<TK>(p.sh_K + (size_t)(g - 1) * p.sh_K_stride); };
    auto KJJg = [&](int g) { return g == 0 ? KJJ : at<double>(p.sh_KJJ + (size_t)(g - 1) * p.sh_KJJ_stride); };
    auto Kcg = [&](int g) { return g == 0 ? Kc : at<TK>(p.sh_Kc + (size_t)(g - 1) * p.sh_Kc_stride); };
    auto op = [&](int64_t q) { return at<double>(p.sh_o + (size_t)q * p.sh_o_stride); };
    auto bp = [&](int64_t q) { return at<double>(p.sh_beta + (size_t)q * p.sh_beta_stride); };
    auto cp = [&](int64_t q) { return at<CandState>(p.sh_cst + (size_t)q * p.sh_cst_stride); };
    for (int64_t q = 0; q < P; ++q) {
      SPSVM_HIP(hipMemsetAsync(op(q), 0, n * 8, st));
      SPSVM_HIP(hipMemsetAsync(bp(q), 0, J_max * 8, st));
    }
    SPSVM_HIP(hipMemsetAsync(m_dev, 0, 8, st));
    std::vector<spsvm_stats> pstats(P);
    int m = 0;
    int64_t t = 0;
    std::vector<uint64_t> blocked;
    std::vector<int32_t> table((size_t)opt.chunk_cap * kCandSlots);
    const int nblk = score_blocks(n);
    const int64_t ldc = round_up(n, 4);
    int first_rounds = 4;
    while (m < J_max) {
      const auto t0 = clk::now();
      const int cs = (int)stage_size(m, J_max, opt.growth, opt.chunk_cap);
      for (int q = 0; q < cs; ++q) draw_step(opt.seed, t + q, n, opt.kappa, hash_host, blocked, &table[(size_t)q * kCandSlots]);
      int32_t* tp = (int32_t*)((char*)pin.p + kPinnedScalars);
      std::memcpy(tp, table.data(), (size_t)cs * kCandSlots * 4);
      SPSVM_HIP(hipMemcpyAsync(cand_table, tp, (size_t)cs * kCandSlots * 4, hipMemcpyHostToDevice, st));
      // attempts and resumption as in the single-problem selection: a step whose slots did not all settle in any
      // problem selects nothing, nor do the later steps of the attempt, and the stage resumes from it
      int qstart = 0, m_q = m;
      for (int attempt = 0;; ++attempt) {
        const int rounds = attempt == 0   ? first_rounds
                           : attempt == 1 ? std::min(64, first_rounds + 2)
                           : attempt == 2 ? std::min(64, std::max(12, 2 * first_rounds + 4))
                                          : 64;
        {
          int32_t* mh = (int32_t*)((char*)pin.p + 8192);
          *mh = m_q;
          SPSVM_HIP(hipMemcpyAsync(m_dev + (qstart & 1), mh, 4, hipMemcpyHostToDevice, st));
        }
        if (attempt > 0) stats.stage_redos += 1;
        SPSVM_HIP(hipMemsetAsync(incomplete, 0, 32, st));
        for (int q = qstart; q < cs; ++q) {
          const int32_t* cq = cand_table + (size_t)q * kCandSlots;
          for (int g = 0; g < G; ++g) {
            gamma = gam[g];
            prof.timed(kProfKblock, 2.0 * n * kCandSlots * d, [&] { kblock(cq, kCandSlots, Kcg(g), ldc, Score0{}, true); },
                       kblock_issued(kCandSlots));
          }
          for (int64_t pq = 0; pq < P; ++pq) {
            const float* yq = Y + pq * n;
            launch_score_init(cq, op(pq), hash, stage_hash, q, cp(pq), sc, nullptr, st);
            for (int r = 0; r < rounds; ++r) {
              prof.timed(kProfScore, (double)n * (opt.kappa * sizeof(TK) + 12.0),
                         [&] { launch_score_pass<TK>(Kcg(gof[pq]), ldc, yq, op(pq), n, cp(pq), score_part, nblk, st, true); });
              launch_score_update(cp(pq), score_part, nblk, 1.0 / Cs[pq], incomplete + 3, st);
            }
          }
          stats.score_passes += (int64_t)rounds * P;
          launch_shared_select(cp(0), (int64_t)p.sh_cst_stride, (int)P, hash, stage_hash, q, J, J32, m_dev, sel,
                               incomplete, st);
          for (int64_t pq = 0; pq < P; ++pq)
            launch_shared_append<TK>(sel, cp(pq), Kcg(gof[pq]), ldc, n, op(pq), bp(pq), st);
          for (int g = 0; g < G; ++g) launch_shared_column<TK>(sel, Kcg(g), ldc, n, Kg(g), p.ldk, st);
        }
        int32_t flags2[8];
        SPSVM_HIP(hipMemcpyAsync(pin.p, incomplete, 32, hipMemcpyDeviceToHost, st));
        sync();
        std::memcpy(flags2, pin.p, 32);
        first_rounds = std::min(64, std::max(2, flags2[1] + 1));
        if (flags2[0] == 0 || rounds >= 64) break;
        qstart = flags2[4];
        m_q = read(m_dev + (qstart & 1));
      }
      t += cs;
      const int m_new = read(m_dev + (cs & 1));
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
      if (m_new == m) {
        stats.stop_reason = 2;
        break;
      }
      // basis rows in FP64 and each gamma's K_JJ
      launch_gather_rows<TX, double>(X, d, J + m, m_new - m, XJ64 + (size_t)m * p.ldj, p.ldj, st);
      launch_row_norms<double, double>(XJ64 + (size_t)m * p.ldj, m_new - m, d, p.ldj, xjnorm + m, st);
      for (int g = 0; g < G; ++g)
        launch_kblock<double, double>(XJ64, p.ldj, m_new, d, xjnorm, iota, m_new, KJJg(g), p.ldh, gam[g], st);
      m = m_new;
      // Newton for every problem, the problems of one gamma in lockstep
      const int Q = (int)slots.size();
      for (int g = 0; g < G; ++g) {
        std::vector<int64_t> group;
        for (int64_t q = 0; q < P; ++q)
          if (gof[q] == g) group.push_back(q);
        for (size_t c0 = 0; c0 < group.size(); c0 += Q) {
          std::vector<int> ids;
          for (size_t k = c0; k < group.size() && k < c0 + Q; ++k) {
            const int64_t q = group[k];
            Slot& S = slots[ids.size()];
            S.y = Y + q * n;
            S.C = Cs[q];
            S.lam = 1.0 / Cs[q];
            S.K = Kg(g);
            S.KJJ = KJJg(g);
            S.hb_valid = false;
            S.stats = &pstats[q];
            SPSVM_HIP(hipMemcpyAsync(S.beta, bp(q), m * 8, hipMemcpyDeviceToDevice, st));
            ids.push_back((int)ids.size());
          }
          newton_slots(m, ids);
          for (size_t k = 0; k < ids.size(); ++k) {
            const int64_t q = group[c0 + k];
            Slot& S = slots[ids[k]];
            SPSVM_HIP(hipMemcpyAsync(bp(q), S.beta, m * 8, hipMemcpyDeviceToDevice, st));
            SPSVM_HIP(hipMemcpyAsync(op(q), S.o, n * 8, hipMemcpyDeviceToDevice, st));
          }
        }
      }
      sync();
      stats.stages += 1;
      stats.seconds_newton += secs(t1, clk::now());
    }
    // models: every problem on the shared basis, with its coefficients and outputs
    for (int64_t q = 0; q < P; ++q) {
      const int g = gof[q];
      Slot& S = slots[0];
      S.y = Y + q * n;
      S.C = Cs[q];
      S.lam = 1.0 / Cs[q];
      S.K = Kg(g);
      S.KJJ = KJJg(g);
      gamma = gam[g];
      spsvm_stats own = stats;  // the shared selection's counters, then this problem's Newton counters
      own.newton_iters = pstats[q].newton_iters;
      own.factorizations = pstats[q].factorizations;
      own.incremental_factorizations = pstats[q].incremental_factorizations;
      own.ls_passes = pstats[q].ls_passes;
      own.iter_cap_hits = pstats[q].iter_cap_hits;
      own.jitter_retries = pstats[q].jitter_retries;
      S.own = own;
      S.stats = &S.own;
      SPSVM_HIP(hipMemcpyAsync(S.beta, bp(q), (size_t)std::max(m, 1) * 8, hipMemcpyDeviceToDevice, st));
      SPSVM_HIP(hipMemcpyAsync(S.o, op(q), n * 8, hipMemcpyDeviceToDevice, st));
      outs[q] = build_model(S, m, true);
    }
    return m;
  }

  spsvm_model* build_model(int m) { return build_model(slots[0], m); }

  spsvm_model* build_model(Slot& S, int m, bool o_fresh = false) {
    double F = 0.0;
    NewtonScalars s{};
    final_eval(S, m > 0 ? m + p.off : 0, &F, &s, o_fresh);  // with the offset the system has one more coordinate
    spsvm_stats& stats = *S.stats;
    stats.n_sv = s.n_sv;
    stats.grad_norm = std::sqrt(s.gnorm2);
    if (m > 0) {  // training error at the returned model (o is current after final_eval)
      launch_count_errors(S.o, S.y, n, S.sc, st);
      stats.train_error = (double)read(&S.sc->n_err) / (double)n;
    } else {
      stats.train_error = 1.0;  // o = 0: every row counts as an error
    }
    sync();
    stats.kblock_launches = prof.count[kProfKblock];
    stats.kblock_seconds = prof.seconds[kProfKblock];
    stats.kblock_flops = prof.work[kProfKblock];
    stats.kblock_mfma_flops = prof.work2[kProfKblock];
    stats.syrk_launches = prof.count[kProfSyrk];
    stats.syrk_seconds = prof.seconds[kProfSyrk];
    stats.syrk_flops = prof.work[kProfSyrk];
    stats.score_launches = prof.count[kProfScore];
    stats.score_seconds = prof.seconds[kProfScore];
    // the timed passes' share of what all launched passes read: y and o (12 bytes per row) in every pass that
    // did work, and one candidate column per slot still being scored
    stats.score_bytes = stats.score_passes > 0
                            ? (double)prof.count[kProfScore] / (double)stats.score_passes * (double)n *
                                  (12.0 * (double)stats.score_passes_active + (double)sizeof(TK) * (double)stats.score_slot_passes)
                            : 0.0;
    stats.chol_calls = prof.count[kProfChol];
    stats.chol_seconds = prof.seconds[kProfChol];
    stats.chol_flops = prof.work[kProfChol];
    auto* md = new spsvm_model();
    try {
      md->m = m;
      md->d = d;
      md->tk_double = std::is_same<TK, double>::value;
      md->C = S.C;
      md->gamma = gamma;
      md->objective = F;
      md->stats = stats;
      md->J.resize(m);
      md->beta.resize(m);
      if (m > 0) {
        if (p.off) md->bias = read(S.beta);  // coefficient 0 is b
        SPSVM_HIP(hipMemcpyAsync(md->J.data(), J, m * 8, hipMemcpyDeviceToHost, st));
        SPSVM_HIP(hipMemcpyAsync(md->beta.data(), S.beta + p.off, m * 8, hipMemcpyDeviceToHost, st));
        md->ldz = padded_ld<TK>(d);
        SPSVM_HIP(hipMalloc(&md->XJ, (size_t)m * md->ldz * sizeof(TK)));
        SPSVM_HIP(hipMalloc(&md->XJnorm, (size_t)m * sizeof(TK)));
        SPSVM_HIP(hipMalloc(&md->beta_dev, (size_t)m * 8));
        if (csr.indptr) {
          if constexpr (std::is_same<TK, float>::value)
            launch_csr_gather<int64_t, float>(csr.indptr, csr.indices, csr.values, J, m, (float*)md->XJ, md->ldz, st);
        } else {
          launch_gather_rows<TX, TK>(X, d, J, m, (TK*)md->XJ, md->ldz, st);
        }
        launch_row_norms<TK, TK>((const TK*)md->XJ, m, d, md->ldz, (TK*)md->XJnorm, st);
        SPSVM_HIP(hipMemcpyAsync(md->beta_dev, S.beta + p.off, m * 8, hipMemcpyDeviceToDevice, st));
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

spsvm_model* run_train_csr(const CsrX& Xc, const float* y, int64_t n, int64_t d, double C, double gamma,
                           int64_t J_max, const spsvm_options& opt, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (opt.precision != SPSVM_F32) throw Failure(SPSVM_E_INVALID_ARG, "sparse rows train in SPSVM_F32 precision");
  const Plan plan = make_plan(n, d, J_max, opt, true, false, true, false, 1, true);
  if (!ws || ((uintptr_t)ws & 255u)) throw Failure(SPSVM_E_WORKSPACE, "workspace must be a 256-byte aligned device pointer");
  if (ws_bytes < plan.bytes)
    throw Failure(SPSVM_E_WORKSPACE, "workspace too small: need " + std::to_string(plan.bytes) + " bytes, got " +
                                         std::to_string(ws_bytes));
  Impl<float, float> im(nullptr, y, n, d, C, gamma, J_max, opt, ws, stream, plan);
  im.csr = Xc;
  im.prepare();
  const int m = im.select_and_optimise();
  return im.build_model(m);
}

void run_predict_csr(const spsvm_model* md, const CsrX& Xt, int64_t n_t, double* out, hipStream_t st) {
  if (n_t <= 0) return;
  if (md->tk_double) throw Failure(SPSVM_E_INVALID_ARG, "sparse prediction needs a model with FP32 kernel values");
  SPSVM_HIP(hipMemsetAsync(out, 0, n_t * 8, st));
  if (md->m > 0) {
    float* xn = nullptr;
    SPSVM_HIP(hipMalloc(&xn, (size_t)n_t * sizeof(float)));
    try {
      launch_csr_row_norms<float>(Xt.indptr, Xt.values, n_t, xn, st);
      for (int64_t c0 = 0; c0 < md->m; c0 += kCandSlots) {  // 64 basis rows per launch, sums added in order
        const int nc = (int)std::min<int64_t>(kCandSlots, md->m - c0);
        launch_csr_kblock(Xt.indptr, Xt.indices, Xt.values, n_t, md->d, xn, (const float*)md->XJ + c0 * md->ldz,
                          md->ldz, (const float*)md->XJnorm + c0, nullptr, nc, out, 0, md->gamma, 1,
                          md->beta_dev + c0, st);
      }
      launch_add_scalar(out, n_t, md->bias, st);
      SPSVM_HIP(hipStreamSynchronize(st));
    } catch (...) {
      (void)hipFree(xn);
      throw;
    }
    SPSVM_HIP(hipFree(xn));
  }
  SPSVM_HIP(hipStreamSynchronize(st));
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
                           out, md->gamma, md->bias, st);
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
  const Plan plan = make_plan(n, d, m, opt, false, x_double, ((uintptr_t)X & 15u) == 0, true, P);
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

int distinct_gammas(const double* gamma, int64_t P) {
  std::vector<double> g;
  for (int64_t q = 0; q < P; ++q)
    if (std::find(g.begin(), g.end(), gamma[q]) == g.end()) g.push_back(gamma[q]);
  return (int)g.size();
}

template <typename TX, typename TK>
static void shared_typed(const TX* X, int64_t n, int64_t d, int64_t P, const float* Y, const double* C,
                         const double* gamma, int64_t J_max, const spsvm_options& opt, void* ws, const Plan& plan,
                         hipStream_t st, spsvm_model** out) {
  Impl<TX, TK> im(X, Y, n, d, C[0], gamma[0], J_max, opt, ws, st, plan);
  im.prepare_batch(Y, n * P);
  try {
    im.shared(P, Y, C, gamma, out);
  } catch (...) {
    for (int64_t p = 0; p < P; ++p) {
      delete out[p];
      out[p] = nullptr;
    }
    throw;
  }
}

void run_train_shared(const void* X, bool x_double, int64_t n, int64_t d, int64_t P, const float* Y, const double* C,
                      const double* gamma, int64_t J_max, const spsvm_options& opt, void* ws, size_t ws_bytes,
                      hipStream_t stream, spsvm_model** out) {
  const Plan plan = make_plan(n, d, J_max, opt, true, x_double, ((uintptr_t)X & 15u) == 0, true, P, false,
                              distinct_gammas(gamma, P));
  if (!ws || ((uintptr_t)ws & 255u)) throw Failure(SPSVM_E_WORKSPACE, "workspace must be a 256-byte aligned device pointer");
  if (ws_bytes < plan.bytes)
    throw Failure(SPSVM_E_WORKSPACE, "workspace too small: need " + std::to_string(plan.bytes) + " bytes, got " +
                                         std::to_string(ws_bytes));
  for (int64_t p = 0; p < P; ++p) out[p] = nullptr;
  const bool tk_double = opt.precision == SPSVM_F64;
  if (x_double) {
    if (tk_double)
      shared_typed<double, double>((const double*)X, n, d, P, Y, C, gamma, J_max, opt, ws, plan, stream, out);
    else
      shared_typed<double, float>((const double*)X, n, d, P, Y, C, gamma, J_max, opt, ws, plan, stream, out);
  } else {
    if (tk_double)
      shared_typed<float, double>((const float*)X, n, d, P, Y, C, gamma, J_max, opt, ws, plan, stream, out);
    else
      shared_typed<float, float>((const float*)X, n, d, P, Y, C, gamma, J_max, opt, ws, plan, stream, out);
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

// ------------------------------------------------------------------------------------------ one-vs-one
// Workspace of a one-vs-one training: a pair's gathered rows (pair_rows x d), their labels and row indices, then
// the training workspace of pair_rows rows.
static size_t ovo_head_bytes(int64_t pair_rows, int64_t d, bool x_double) {
  const size_t xb = (size_t)round_up(pair_rows * d * (x_double ? 8 : 4), 256);
  return xb + (size_t)round_up(pair_rows * 4, 256) + (size_t)round_up(pair_rows * 8, 256);
}

size_t ovo_workspace_bytes(int64_t pair_rows, int64_t d, int64_t J_max, const spsvm_options& opt, bool x_double) {
  return ovo_head_bytes(pair_rows, d, x_double) + make_plan(pair_rows, d, J_max, opt, true, x_double, true).bytes;
}

void run_train_ovo(const void* X, bool x_double, const int32_t* classes, int64_t n, int64_t d, int K, double C,
                   double gamma, int64_t J_max, const spsvm_options& opt, void* ws, size_t ws_bytes, hipStream_t st,
                   spsvm_model** out) {
  const int P = K * (K - 1) / 2;
  for (int p = 0; p < P; ++p) out[p] = nullptr;
  if (!ws || ((uintptr_t)ws & 255u)) throw Failure(SPSVM_E_WORKSPACE, "workspace must be a 256-byte aligned device pointer");
  std::vector<int32_t> cls((size_t)n);
  SPSVM_HIP(hipMemcpyAsync(cls.data(), classes, n * 4, hipMemcpyDeviceToHost, st));
  SPSVM_HIP(hipStreamSynchronize(st));
  std::vector<int64_t> count(K, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (cls[i] < 0 || cls[i] >= K) throw Failure(SPSVM_E_INVALID_ARG, "class ids must lie in [0, K)");
    count[cls[i]] += 1;
  }
  int64_t pair_max = 0;
  for (int a = 0; a < K; ++a)
    for (int b = a + 1; b < K; ++b) pair_max = std::max(pair_max, count[a] + count[b]);
  const size_t head = ovo_head_bytes(pair_max, d, x_double);
  const size_t need = head + make_plan(pair_max, d, J_max, opt, true, x_double, true).bytes;
  if (ws_bytes < need)
    throw Failure(SPSVM_E_WORKSPACE, "workspace too small for the largest class pair: need " + std::to_string(need) +
                                         " bytes, got " + std::to_string(ws_bytes));
  char* base = (char*)ws;
  void* Xp = base;
  float* yp = (float*)(base + round_up(pair_max * d * (x_double ? 8 : 4), 256));
  int64_t* rows_dev = (int64_t*)((char*)yp + round_up(pair_max * 4, 256));
  void* tws = base + head;
  std::vector<int64_t> rows;
  std::vector<float> y;
  int p = 0;
  try {
    for (int a = 0; a < K; ++a)
      for (int b = a + 1; b < K; ++b, ++p) {
        rows.clear();
        y.clear();
        for (int64_t i = 0; i < n; ++i)
          if (cls[i] == a || cls[i] == b) {
            rows.push_back(i);
            y.push_back(cls[i] == a ? 1.0f : -1.0f);
          }
        const int64_t m = (int64_t)rows.size();
        if (count[a] == 0 || count[b] == 0)
          throw Failure(SPSVM_E_INVALID_ARG, "class pair (" + std::to_string(a) + ", " + std::to_string(b) +
                                                 ") has a class without rows");
        SPSVM_HIP(hipMemcpyAsync(rows_dev, rows.data(), m * 8, hipMemcpyHostToDevice, st));
        SPSVM_HIP(hipMemcpyAsync(yp, y.data(), m * 4, hipMemcpyHostToDevice, st));
        if (x_double)
          launch_gather_pair<double>((const double*)X, d, rows_dev, m, (double*)Xp, st);
        else
          launch_gather_pair<float>((const float*)X, d, rows_dev, m, (float*)Xp, st);
        spsvm_model* md = nullptr;
        try {
          md = run_train(Xp, x_double, yp, m, d, C, gamma, std::min<int64_t>(J_max, m), opt, tws, ws_bytes - head, st,
                         nullptr);
        } catch (const Failure& e) {
          throw Failure(e.status, "class pair (" + std::to_string(a) + ", " + std::to_string(b) + "): " + e.what());
        }
        for (int64_t& j : md->J) j = rows[j];  // pair rows back to rows of X
        out[p] = md;
      }
  } catch (...) {
    for (int q = 0; q < P; ++q) {
      delete out[q];
      out[q] = nullptr;
    }
    throw;
  }
}

size_t ovo_predict_workspace_bytes(int64_t n_t, int K) {
  return (size_t)round_up(n_t * 8, 256) + (size_t)round_up(n_t * K * 4, 256);
}

void run_predict_ovo(const spsvm_model* const* models, int K, const void* Xt, bool x_double, int64_t n_t,
                     int32_t* classes, void* ws, size_t ws_bytes, hipStream_t st) {
  if (n_t <= 0) return;
  if (!ws || ((uintptr_t)ws & 255u) || ws_bytes < ovo_predict_workspace_bytes(n_t, K))
    throw Failure(SPSVM_E_WORKSPACE, "workspace must be 256-byte aligned with >= spsvm_predict_ovo_workspace_bytes");
  double* dec = (double*)ws;
  int32_t* votes = (int32_t*)((char*)ws + round_up(n_t * 8, 256));
  SPSVM_HIP(hipMemsetAsync(votes, 0, (size_t)n_t * K * 4, st));
  int p = 0;
  for (int a = 0; a < K; ++a)
    for (int b = a + 1; b < K; ++b, ++p) {
      if (!models[p]) throw Failure(SPSVM_E_INVALID_ARG, "model pointer of pair " + std::to_string(p) + " is NULL");
      run_predict(models[p], Xt, x_double, n_t, dec, st);
      launch_ovo_vote(dec, n_t, a, b, K, votes, st);
    }
  launch_ovo_argmax(votes, n_t, K, classes, st);
  SPSVM_HIP(hipStreamSynchronize(st));
}

}  // namespace spsvm
