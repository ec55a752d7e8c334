// Launchers of the SP-SVM kernels (host side). All launches go to the given stream; none synchronises.
#pragma once

#include "common.h"

namespace spsvm {

// ------------------------------------------------------------------------------ shared device structs
// One candidate slot of a selection step (exact one-dimensional minimisation, see select.hip).
struct CandState {
  double s, s_prev, lo, hi;  // evaluation point, previous point, bracket of the root of psi'
  double oc;                 // o at the candidate's row
  double score;              // exact decrease of f when done
  double phi_lo, g_lo;       // psi - psi(0) and psi' at lo (when lo is finite)
  double phi_hi, g_hi;       // the same at hi
  double lb, ub;             // bounds on the score: best decrease seen so far; largest decrease still possible
  int32_t idx;               // training row, -1 for an empty slot
  int32_t status;            // 0 active, 1 done, 2 skipped, 3 dropped (cannot win: ub below another slot's lb)
  int32_t newton;            // s is the Newton root of the previous point's segment
  int32_t passes;
};
constexpr int kCandSlots = 64;
// The slot states are followed by kCandSlots int32 drop flags (a pass marks the slots it dropped, the update
// that follows it retires them), kCandSlots int32 window counts and, per slot, kWinCap window rows (a_i, b_i):
// the rows whose violator status changes inside the window around the slot's point of the pass.
constexpr int kWinCap = 64;
constexpr size_t kCandStateBytes = kCandSlots * sizeof(CandState) + 2 * kCandSlots * sizeof(int32_t) +
                                   (size_t)kCandSlots * kWinCap * 2 * sizeof(double);
__host__ __device__ inline int32_t* cand_drop_flags(CandState* st) { return reinterpret_cast<int32_t*>(st + kCandSlots); }
__host__ __device__ inline int32_t* cand_win_count(CandState* st) { return cand_drop_flags(st) + kCandSlots; }
__host__ __device__ inline double* cand_win_rows(CandState* st) {
  return reinterpret_cast<double*>(cand_win_count(st) + kCandSlots);
}

// Batched launches: up to kMaxBatch independent problems (slots) per launch, one grid z-index per slot; the
// per-slot operands travel by value in the kernel arguments. 48 covers the 40 problems of one kernel width in
// a one-vs-rest x C sweep with a single launch per step, and keeps the largest argument block near 3 KB.
constexpr int kMaxBatch = 48;

// Result of a selection step.
struct Selection {
  double s;       // coefficient of the new basis vector
  double score;   // decrease of f
  int32_t valid;  // 0 when no candidate could be scored
  int32_t slot;   // candidate slot (column of the candidate block)
  int32_t idx;    // training row
  int32_t pos;    // position in J (column of K_XJ)
};

// Line-search state along d (exact minimisation of f(beta + t d), t >= 0).
struct LineState {
  double t, t_prev, lo, hi;
  double c1, c2;   // beta . delta_J, d . delta_J (delta = K_XJ d)
  double dec;      // f(beta) - f(beta + t d) when done
  int32_t status;  // 0 active, 1 done
  int32_t newton;
  int32_t passes;
  int32_t pad;
};

// Per-iteration scalars of the Newton loop, copied to the host.
struct NewtonScalars {
  double sum_a2;   // sum_i max(0, 1 - y_i o_i)^2
  double gnorm2;   // ||grad f||^2
  double beta_oJ;  // beta^T K_JJ beta
  double trace;    // trace of H (jitter scale)
  int32_t n_sv;    // |I|
  int32_t flips;   // rows whose violator status differs from the last factorisation
  int32_t fail;    // Cholesky met a non-positive pivot
  int32_t n_active_sel;  // candidates still being scored
  int32_t n_in, n_out;   // rows that joined / left the violator set since the last Newton matrix
  int32_t n_err;         // rows with y_i o_i <= 0 (training errors), counted by launch_count_errors
  int32_t pad_;
};

// ----------------------------------------------------------------------------------------- kblock.hip
template <typename TX, typename TK>
void launch_row_norms(const TX* X, int64_t n, int64_t d, int64_t ldx, TK* out, hipStream_t st);
template <typename TX>
void launch_row_hash(const TX* X, int64_t n, int64_t d, uint64_t* out, hipStream_t st);
// First scoring pass (at s = 0) fused into the candidate block: for every 128-row tile t (of T = ceil(n / 128))
// and column c of the first 64 columns the epilogue writes partial[(c * T + t) * 4 + {0, 1, 2, 3}] =
// {P, Q, 0, 0}, the sums of a_i b_i and b_i^2 over the rows of the tile with a_i = 1 - y_i o_i > 0
// (b_i = y_i k_ic), in the slot-major layout of a scoring pass. Only with column-major out (the launchers
// reject it otherwise).
// dst (column-major out only): launch column c is written to column dst[c] of out, so the valid candidates of
// several steps can share tiles while each keeps its slot; the fused records stay keyed by launch column, which
// is the slot of the first step when that step's candidates come first and fill a prefix of its slots.
struct Score0 {
  const float* y = nullptr;
  const double* o = nullptr;
  double* partial = nullptr;  // nullptr: no fused pass
  const int32_t* dst = nullptr;  // nullptr: launch column c goes to column c
};
constexpr int kKblockRows = 128;  // rows per kernel-block tile (the fused pass writes one record per tile)

// X rows start at multiples of ldx elements; ldx * sizeof(TX) and X must be 16-byte aligned.
// gamma > 0 writes exp(-gamma d2); gamma == 0 writes the squared distances d2.
template <typename TX, typename TK>
// colmajor: out[c * ldo + i] (columns 16-byte aligned, ldo a multiple of 4) instead of out[i * ldo + c].
void launch_kblock(const TX* X, int64_t ldx, int64_t n, int64_t d, const TK* xnorm, const int32_t* cidx, int ncols,
                   TK* out, int64_t ldo, double gamma, hipStream_t st, const Score0& s0 = Score0{},
                   bool colmajor = false);
// out = sum_k beta_k exp(-gamma |xt - z_k|^2) + bias per row of Xt.
template <typename TX, typename TK>
void launch_predict(const TX* Xt, int64_t ldxt, int64_t n, int64_t d, const TK* Z, int64_t ldz, const TK* znorm, int m,
                    const double* beta, double* out, double gamma, double bias, hipStream_t st);
// Split-BF16 copies of X for the mixed kernel block: hi = bf16(x), lo = bf16(x - hi) (round to nearest even),
// n x ldb each with ldb = split_ld(d) (d rounded up to 32, zero padded); lo may be null (not needed).
int64_t split_ld(int64_t d);
template <typename TX>
void launch_split_bf16(const TX* X, int64_t n, int64_t d, int64_t ldx, unsigned short* hi, unsigned short* lo,
                       int64_t ldb, hipStream_t st);
// The kernel block with split-BF16 products x.z ~ hi.hi' + hi.lo' + lo.hi' from the split copies, FP32 results
// (same output and fused pass as launch_kblock). lo = nullptr: every X value is a BF16 number (lo = 0), so only
// hi.hi' is issued (identical result).
// MFMA flops one launch issues (whole tiles of the variant the launcher picks; three products per multiply-add
// with the split correction), for the roofline next to the algorithmic 2 n ncols d.
double kblock_issued_flops(int64_t n, int64_t d, int64_t ncols);
double kblock_bf16_issued_flops(int64_t n, int64_t ldb, int64_t ncols, bool split, bool candidates);
// Tile variant (one kernel each) that launch_kblock_bf16 runs for this shape: the forced one, the tuned one, else
// the shape rule; candidate blocks are column-major with the fused first pass.
int kblock_bf16_variant(int64_t n, int64_t ldb, int64_t ncols, bool split, bool candidates);
void launch_kblock_bf16(const unsigned short* hi, const unsigned short* lo, int64_t ldb, int64_t n,
                        const float* xnorm, const int32_t* cidx, int ncols, float* out, int64_t ldo, double gamma,
                        hipStream_t st, const Score0& s0 = Score0{}, bool colmajor = false);
template <typename TK>
void launch_rbf_from_dist(const TK* D, int64_t rows, int ncols, int64_t ld, TK* K, double gamma, hipStream_t st);
template <typename TX>
void launch_pad_rows(const TX* X, int64_t n, int64_t d, TX* out, int64_t ldo, hipStream_t st);
// Row stride (elements) that makes every row start on a 16-byte boundary.
template <typename TX>
inline int64_t padded_ld(int64_t d) {
  return round_up(d, 16 / (int64_t)sizeof(TX));
}
template <typename TX>
void launch_check_inputs(const TX* X, int64_t total, const float* y, int64_t n, int32_t* flags, hipStream_t st);
template <typename TX, typename TK>
void launch_gather_rows(const TX* X, int64_t d, const int64_t* idx, int64_t m, TK* out, int64_t ldo, hipStream_t st);
void launch_iota(int32_t* out, int64_t m, hipStream_t st);
// K[i * ld + col] = v for rows 0 .. rows - 1.
template <typename TK>
void launch_fill_column(TK* K, int64_t rows, int64_t ld, int64_t col, double v, hipStream_t st);

// ----------------------------------------------------------------------------------------- select.hip
// Score slots for step `step` of the candidate table (kCandSlots indices per step, -1 = empty).
// bias (device, may be null): the offset b included in o; the slots take o_c - b as (K beta)_c.
void launch_score_init(const int32_t* cand, const double* o, const uint64_t* hash, const uint64_t* stage_hash,
                       int n_stage, CandState* st, NewtonScalars* sc, const double* bias, hipStream_t s);
// One scoring pass over the n rows for all active slots (candidate block Kc column-major, column stride ldc;
// partial sums per workgroup), then one workgroup per
// slot reduces them and advances the slot. Both kernels return at once when every slot is settled.
// nodrop: no slot is dropped (every score is exact: the shared-basis selection sums them over problems).
template <typename TK>
void launch_score_pass(const TK* Kc, int64_t ldc, const float* y, const double* o, int64_t n, CandState* st,
                       double* partial, int nblk, hipStream_t s, bool nodrop = false);
// live (may be null): incremented once per slot that the pass scored (for the byte count of the passes).
void launch_score_update(CandState* st, const double* partial, int nblk, double lam, int32_t* live, hipStream_t s);
// launch_score_init followed by launch_score_update on the nblk records of a first pass that came with the
// kernel block, as one launch.
void launch_score_init_update(const int32_t* cand, const double* o, const uint64_t* hash, const uint64_t* stage_hash,
                              int n_stage, CandState* st, const double* partial, int nblk, double lam,
                              const double* bias, hipStream_t s);
// Argmax of the scored slots and its append (one launch). Kc: the step's candidate columns, column-major
// (column stride ldc); fused0: its first scoring pass came with the block; m_dev: two ints, step q reads the basis size at
// m_dev[q & 1] and writes the next at m_dev[(q + 1) & 1]. The row index goes to J[pos] and J32[pos], the coefficient
// to beta[pos + off] and (write_col) the column to K_XJ column pos + off.
template <typename TK>
void launch_select_append(const CandState* st, const uint64_t* hash, uint64_t* stage_hash, int q, const TK* Kc,
                          int64_t ldc, int64_t n, double* o, TK* KXJ, int64_t ldk, int64_t* J, int32_t* J32,
                          double* beta, int32_t* m_dev, Selection* sel, int32_t* incomplete, int fused0, int off,
                          bool write_col, hipStream_t s);
int score_blocks(int64_t n);
// One basis shared by P problems: argmax over the slots of the sum of the problems' scores (problem p's slot states
// at st0 + p * stride bytes), appended to J / J32 like launch_select_append; then per problem its coefficient and
// o += s k (launch_shared_append), and per gamma the winner's column into its K_XJ (launch_shared_column).
void launch_shared_select(const CandState* st0, int64_t stride, int P, const uint64_t* hash, uint64_t* stage_hash,
                          int q, int64_t* J, int32_t* J32, int32_t* m_dev, Selection* sel, int32_t* incomplete,
                          hipStream_t s);
template <typename TK>
void launch_shared_append(const Selection* sel, const CandState* st, const TK* Kc, int64_t ldc, int64_t n, double* o,
                          double* beta, hipStream_t s);
template <typename TK>
void launch_shared_column(const Selection* sel, const TK* Kc, int64_t ldc, int64_t n, TK* KXJ, int64_t ldk,
                          hipStream_t s);

// ----------------------------------------------------------------------------------------- newton.hip
template <typename TK>
void launch_gemv(const TK* K, int64_t ldk, int64_t n, int m, const double* x, double* out, hipStream_t s);
void launch_compact(const double* o, const float* y, int64_t n, const uint8_t* act_ref, uint8_t* act_out,
                    int32_t* I, int32_t* blk_count, double* blk_sum, int32_t* blk_flips, NewtonScalars* sc,
                    hipStream_t s);
// The same for up to kMaxBatch problems per launch (grid y = slot), one entry per problem.
struct CompactBatch {
  const double* o[kMaxBatch];
  const float* y[kMaxBatch];
  const uint8_t* act_ref[kMaxBatch];
  uint8_t* act_out[kMaxBatch];
  int32_t* I[kMaxBatch];
  int32_t* cnt[kMaxBatch];
  double* bsum[kMaxBatch];
  int32_t* bflips[kMaxBatch];
  NewtonScalars* sc[kMaxBatch];
  int count;
};
void launch_compact_batch(const CompactBatch& b, int64_t n, hipStream_t s);
int compact_blocks(int64_t n);
// sc->n_err = number of rows with y_i o_i <= 0 (misclassified; a zero output counts).
void launch_count_errors(const double* o, const float* y, int64_t n, NewtonScalars* sc, hipStream_t s);
// Workgroups of a line-search pass over n rows (partial records per workgroup).
int ls_blocks(int64_t n);
template <typename TK>
void launch_gradient(const TK* K, int64_t ldk, int m, const int32_t* I, const double* o, const float* y,
                     const double* v, const double* beta, double lam, double* partial, int nchunk, double* g,
                     NewtonScalars* sc, hipStream_t s);
int gradient_chunks(int m, int n_sv);

// out_q = K x_q for up to kMaxBatch vectors x_q (m FP64 values each, 32-byte aligned) with one read of K
// (n x m, leading dimension ldk a multiple of 4, rows 16-byte aligned). FP64 MFMA, exact products.
struct GemvBatch {
  const double* x[kMaxBatch];
  double* out[kMaxBatch];
  int count;
};
template <typename TK>
void launch_gemv_batch(const TK* K, int64_t ldk, int64_t n, int m, const GemvBatch& b, hipStream_t s);

// Gradients of up to kMaxBatch problems sharing K, in dense form: for each slot the chunk partials
// partial[c * m + j] = sum_{i in chunk c, a_i > 0} K[i][j] (o_i - y_i) (a_i = 1 - y_i o_i), one read of K for
// all slots; then, per slot, g = lambda v + sum of the partials and the norms (as the single-problem gradient).
struct GradBatch {
  const double* o[kMaxBatch];
  const float* y[kMaxBatch];
  double* partial[kMaxBatch];
  const double* v[kMaxBatch];
  const double* beta[kMaxBatch];
  double* g[kMaxBatch];
  NewtonScalars* sc[kMaxBatch];
  double lam[kMaxBatch];
  int count;
};
int gradient_chunks_dense(int64_t n, int m);
template <typename TK>
void launch_gradient_batch(const TK* K, int64_t ldk, int64_t n, int m, const GradBatch& b, hipStream_t s);

// SYRK partials over the rows rows[0..n_rows) for the lower 128 x 128 tiles tile_lo..tile_hi-1 (tiles numbered
// row by row: tile t = tr (tr + 1) / 2 + tc), split into nsplit row ranges.
template <typename TK>
struct SyrkBatch {
  const TK* K[kMaxBatch];
  const int32_t* rows[kMaxBatch];
  double* partial[kMaxBatch];
  int n_rows[kMaxBatch], nsplit[kMaxBatch], tile_lo[kMaxBatch], tile_hi[kMaxBatch];
  int count;
};
template <typename TK>
void launch_syrk_batch(const SyrkBatch<TK>& b, int64_t ldk, int m, hipStream_t s);
template <typename TK>
void launch_syrk(const TK* K, int64_t ldk, int m, const int32_t* I, int n_rows, int tile_lo, int tile_hi, int nsplit,
                 double* partial, hipStream_t s);
// mode 0: H = lambda K_JJ + partials; +1: H += partials; -1: H -= partials (same tile range as the SYRK).
struct ReduceBatch {
  const double* KJJ[kMaxBatch];
  const double* partial[kMaxBatch];
  double* H[kMaxBatch];
  double lam[kMaxBatch];
  int nsplit[kMaxBatch], tile_lo[kMaxBatch], tile_hi[kMaxBatch], mode[kMaxBatch];
  int count;
};
void launch_syrk_reduce_batch(const ReduceBatch& b, int m, int64_t ldh, hipStream_t s);
void launch_syrk_reduce(const double* KJJ, int m, double lam, const double* partial, int nsplit, int tile_lo,
                        int tile_hi, int mode, double* H, int64_t ldh, hipStream_t s);
void launch_add_diag(double* H, int64_t ldh, int m, double v, hipStream_t s);
// Lower triangle: H = lam * KJJ + G (all m x m, leading dimension ldh).
void launch_scaled_sum_lower(double* H, const double* KJJ, const double* G, double lam, int m, int64_t ldh,
                             hipStream_t s);
// Rows that joined (act_new and not act_old) and left the violator set, listed in ascending order, for up to
// kMaxBatch problems per launch; per-workgroup counts in cnt_in / cnt_out (compact_blocks(n) each), totals in
// the scalars (n_in, n_out).
struct FlipBatch {
  const uint8_t* act_new[kMaxBatch];
  const uint8_t* act_old[kMaxBatch];
  int32_t* cnt_in[kMaxBatch];
  int32_t* cnt_out[kMaxBatch];
  int32_t* F_in[kMaxBatch];
  int32_t* F_out[kMaxBatch];
  NewtonScalars* sc[kMaxBatch];
  int count;
};
void launch_flip_lists_batch(const FlipBatch& b, int64_t n, hipStream_t s);
void launch_trace(const double* H, int64_t ldh, int m, NewtonScalars* sc, hipStream_t s);
int syrk_tiles(int m);
int syrk_tile_rows(int m);
int syrk_tile_size();
int syrk_splits(int ntiles, int n_rows);
// Split count of one problem in a batched Newton solve (at most kSyrkBatchSplits).
int syrk_splits_batch(int ntiles, int n_rows);
constexpr int kSyrkBatchSplits = 2;
size_t syrk_partial_doubles(int m_max);
size_t syrk_partial_doubles_batch(int m_max);
// Exact line search of up to kMaxBatch problems per launch (grid dimension = slot): per slot the margins o, the
// step delta = K_XJ d, the labels, the line state, the pass partials (ls_blocks(n) x 6 doubles), lambda, and for
// the set-up and the step: beta, d and w = K_JJ d (the step updates beta and o in place).
struct LsBatch {
  double* o[kMaxBatch];
  const double* delta[kMaxBatch];
  const float* y[kMaxBatch];
  LineState* ls[kMaxBatch];
  double* partial[kMaxBatch];
  double lam[kMaxBatch];
  double* beta[kMaxBatch];
  const double* dvec[kMaxBatch];
  const double* w[kMaxBatch];
  int count;
};
// c1 = beta . w, c2 = d . w and a fresh line state.
void launch_c1c2_batch(const LsBatch& b, int m, hipStream_t s);
// One pass over the rows and one update of the line state.
void launch_ls_round_batch(const LsBatch& b, int64_t n, int nblk, hipStream_t s);
// beta += t d, o += t delta with the final step t.
void launch_apply_step_batch(const LsBatch& b, int m, int64_t n, hipStream_t s);
void launch_scale(double* v, int m, double a, hipStream_t s);

// ------------------------------------------------------------------------------------------- chol.hip
constexpr int kCholNB = 64;
// In-place lower Cholesky of H (m x m, leading dimension ldh); Linv receives the inverses of the diagonal
// blocks (ceil(m/64) blocks of 64 x 64). Sets sc->fail on a non-positive or non-finite pivot.
void launch_cholesky(double* H, int64_t ldh, int m, double* Linv, NewtonScalars* sc, hipStream_t s);
struct CholBatch {
  double* H[kMaxBatch];
  double* Linv[kMaxBatch];
  NewtonScalars* sc[kMaxBatch];
  int count;
};
void launch_cholesky_batch(const CholBatch& b, int64_t ldh, int m, hipStream_t s);
// x = -L^{-T} L^{-1} g using the factor and the diagonal-block inverses.
void launch_chol_solve(const double* L, int64_t ldh, int m, const double* Linv, const double* g, double* x,
                       double* work, hipStream_t s);
struct SolveBatch {
  const double* L[kMaxBatch];
  const double* Linv[kMaxBatch];
  const double* g[kMaxBatch];
  double* x[kMaxBatch];
  double* work[kMaxBatch];
  int count;
};
void launch_chol_solve_batch(const SolveBatch& b, int64_t ldh, int m, hipStream_t s);
// Cholesky and x = -H^{-1} g (as launch_cholesky + launch_chol_solve) with the scratch in a static device array
// (no device allocation); m <= newton_solve_noalloc_max(). Throws on a non-positive pivot; synchronises the stream.
int newton_solve_noalloc_max();
void newton_solve_noalloc(double* H, int64_t ldh, int m, const double* g, double* x, hipStream_t st);

// ------------------------------------------------------------------------------------- multiclass.hip
// out = the rows rows[0 .. m) of X (n x d, dense), dense m x d.
template <typename TX>
void launch_gather_pair(const TX* X, int64_t d, const int64_t* rows, int64_t m, TX* out, hipStream_t st);
// One-vs-one votes of pair (a, b) from its decision values (votes: n x K int32), then the winning class per row.
void launch_ovo_vote(const double* dec, int64_t n, int a, int b, int K, int32_t* votes, hipStream_t st);
void launch_ovo_argmax(const int32_t* votes, int64_t n, int K, int32_t* classes, hipStream_t st);

// ----------------------------------------------------------------------------------------- sparse.hip
// CSR feature matrices (row i: values[indptr[i] .. indptr[i + 1]) at increasing features indices[...], FP32).
template <typename TK>
void launch_csr_row_norms(const int64_t* indptr, const float* values, int64_t n, TK* out, hipStream_t st);
void launch_csr_row_hash(const int64_t* indptr, const int32_t* indices, const float* values, int64_t n, int64_t d,
                         uint64_t* out, hipStream_t st);
// flags[0] |= a feature index outside [0, d) or not increasing within its row.
void launch_csr_check(const int64_t* indptr, const int32_t* indices, int64_t n, int64_t d, int32_t* flags,
                      hipStream_t st);
// Dense copies (m x ldo) of the rows idx[0 .. m) (a negative index gives a zero row).
template <typename TI, typename TK>
void launch_csr_gather(const int64_t* indptr, const int32_t* indices, const float* values, const TI* idx, int64_t m,
                       TK* out, int64_t ldo, hipStream_t st);
// Kernel block of the sparse rows against up to 64 dense rows Z (ncols x ldz): mode 0 writes column-major FP32
// out[c * ldo + i] (norms xnorm[cidx[c]]; negative cidx: column untouched); mode 1 adds sum_c beta[c] K_ic to the
// FP64 out[i] (norms znorm[c], cidx null).
void launch_csr_kblock(const int64_t* indptr, const int32_t* indices, const float* values, int64_t n, int64_t d,
                       const float* xnorm, const float* Z, int64_t ldz, const float* znorm, const int32_t* cidx,
                       int ncols, void* out, int64_t ldo, double gamma, int mode, const double* beta, hipStream_t st);
void launch_add_scalar(double* out, int64_t n, double v, hipStream_t st);

}  // namespace spsvm
