/*
 * spsvm.h - C ABI of the SP-SVM training library for AMD Instinct MI355X (gfx950).
 *
 * The library trains the sparse primal SVM of section 4 of "Parallel Support Vector Machines in
 * Practice" ("Sparse primal optimization", Eq. 4) with the RBF kernel of section 2:
 *
 *   min_beta  F(beta) = 1/2 beta^T K_JJ beta + C/2 sum_i max(0, 1 - y_i sum_k beta_k k(x_i, x_{J_k}))^2,
 *   k(x, z) = exp(-gamma ||x - z||^2),
 *
 * over a basis J of training rows that is grown greedily (random candidate subsets, each candidate
 * scored by the loss reduction it brings) and re-optimised by Newton's method after each stage of
 * additions. The bias term is omitted, as section 2 allows, unless spsvm_options.bias asks for it; growth
 * stops at a given |J| or by the training-error rule of section 4. Every step runs in HIP kernels on the GPU;
 * the host only orchestrates launches.
 *
 * Conventions for every call:
 *  - Pointers named "device" are HIP device pointers; the caller owns them and keeps them alive and
 *    unmodified for the duration of the call. "host" pointers are ordinary CPU memory.
 *  - Matrices are row-major and dense, with rows contiguous (row i of X starts at X + i * d).
 *  - The stream argument is a hipStream_t passed as void*; NULL means the default stream. Calls are
 *    synchronous with respect to the host: they return after their GPU work has finished.
 *  - Every call returns a status code; no C++ exception crosses this interface. On failure, any
 *    output model pointer is set to NULL and spsvm_last_error() describes the failure.
 *  - Results are deterministic: the same inputs, options and device give bitwise-identical outputs
 *    (fixed reduction orders, no floating-point atomics).
 */
#ifndef SPSVM_H
#define SPSVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPSVM_OK = 0,
  SPSVM_E_INVALID_ARG = 1,    /* an argument is out of range; nothing was launched */
  SPSVM_E_OUT_OF_MEMORY = 2,  /* a model or host staging allocation failed */
  SPSVM_E_HIP = 3,            /* a HIP runtime call failed; the message carries hipGetErrorString */
  SPSVM_E_NOT_PD = 4,         /* the Newton matrix stayed non positive definite after the jitter retries */
  SPSVM_E_NO_CONVERGENCE = 5, /* the objective or gradient became non-finite (Newton hitting its iteration
                                 cap is not an error; it is counted in spsvm_stats.iter_cap_hits) */
  SPSVM_E_WORKSPACE = 6       /* workspace pointer missing, misaligned (256 B) or smaller than required */
} spsvm_status;

/* Arithmetic used for the kernel values and the Newton matrix.
 *  SPSVM_F64: everything in FP64 (distances, kernel block, Newton matrix).
 *  SPSVM_F32: distances and the n x |J| kernel block in FP32 (FP32 MFMA); the Newton matrix is
 *             accumulated on FP64 MFMA from the FP32 kernel values (their products are exact in FP64);
 *             the |J| x |J| regulariser K_JJ, Cholesky, solves, line search, scores and objective in FP64.
 *  SPSVM_MIXED: as F32, but squared distances from BF16 MFMA products with a hi/lo split
 *             correction (x = hi + lo, both BF16; x.z ~ hi.hi + hi.lo + lo.hi). */
typedef enum { SPSVM_F64 = 0, SPSVM_F32 = 1, SPSVM_MIXED = 2 } spsvm_precision;

/* Element type of a feature matrix handed to the library. */
typedef enum { SPSVM_DT_F32 = 0, SPSVM_DT_F64 = 1 } spsvm_dtype;

typedef struct {
  uint32_t struct_size;    /* sizeof(spsvm_options); set by spsvm_options_default */
  uint64_t seed;           /* candidate-sampling seed (SplitMix64 streams, one per addition step) */
  int32_t kappa;           /* candidates drawn per addition step, 1..64; default 59 */
  double growth;           /* stage size = max(1, min(chunk_cap, floor(growth * |J|))); default 0.25 */
  int32_t chunk_cap;       /* upper bound of the stage size, 1..4096; default 256 */
  double newton_tol;       /* stop when ||grad f|| <= tol * max(1, ||grad f at entry||); default 1e-10 */
  double newton_ftol;      /* stop when an exact step lowers f by <= ftol * f; default 1e-14 */
  int32_t newton_max_iter; /* Newton iterations per re-optimisation, >= 1; default 50 */
  spsvm_precision precision; /* default SPSVM_F32 */
  int32_t log_level;       /* 0 silent; 1 one line per stage on stderr; 2 one line per Newton iteration */
  int32_t profile;         /* bits 0-3: kernels to time with HIP events on the call's stream (results in
                              spsvm_stats): 1 kernel block (the candidate blocks that run on the kernel a full
                              group of candidate steps runs on, so that the times describe one kernel; the basis
                              block of the fixed-basis and batched calls), 2 Newton-matrix SYRK, 4 candidate-score
                              passes, 8 Cholesky factorisations; 0 (default) records nothing. Bits 8-15: k, time only
                              every k-th launch of a kernel (0 or 1: every launch); each timed launch is
                              bracketed by two events, which delay the stream a few microseconds */
  double refactor_frac;    /* the Newton matrix is re-formed and re-factorised when more than this fraction of
                              the violator set changed since the last factorisation, or when a step solved with
                              an older factor cut ||grad f|| less than 100-fold (else the last factor is reused;
                              the exact line search keeps every step a descent step); default 0.002 */
  int32_t bias;            /* 1: fit the offset b of Eq. 4 (decision k_i^T beta + b, b not regularised), solved with
                              beta in every Newton re-optimisation and held fixed while candidates are scored;
                              0 (default): b = 0, as section 2 allows */
  double eps_stop;         /* > 0: the stopping rule of section 4 (implementation paragraph; section 5 uses 5e-6):
                              after each re-optimisation, training stops when the decrease of the training error
                              (fraction of rows with y_i o_i <= 0; 1 before the first stage) divided by the number
                              of vectors the stage added is below eps_stop (an unchanged or larger error stops it);
                              J_max stays an upper bound. 0 (default): grow J to J_max */
  int32_t kxj_host;        /* 1: hold the n x |J| kernel block K_XJ in pinned host memory, which the call allocates
                              and frees before it returns, instead of in the workspace: for n |J| beyond the GPU's
                              memory (the method needs O(|J| n) memory, section 4). Every pass over K_XJ (outputs,
                              gradient, Newton matrix, appended columns) then streams it over the host link; the
                              kernels and results are those of 0. The batched calls (spsvm_train_batch,
                              spsvm_train_shared) reject it. 0 (default): K_XJ in the workspace */
} spsvm_options;

typedef struct spsvm_model spsvm_model; /* opaque, owned by the library */

/* Training statistics of a model (filled by spsvm_model_stats). */
typedef struct {
  int64_t stages;           /* re-optimisation stages run */
  int64_t additions;        /* basis vectors added by greedy selection */
  int64_t newton_iters;     /* Newton iterations over all stages */
  int64_t factorizations;   /* Cholesky factorisations of the Newton matrix (incl. jitter retries) */
  int64_t score_passes;     /* O(n) scoring passes launched after the first, which the candidate block computes
                               (a pass whose slots are all settled exits at once) */
  int64_t score_passes_active; /* launched scoring passes in which some slot was still being scored */
  int64_t score_slot_passes;   /* sum over those passes of the slots still being scored */
  int64_t ls_passes;        /* O(n) passes spent in exact line searches */
  int64_t iter_cap_hits;    /* re-optimisations stopped by newton_max_iter */
  int64_t stage_redos;      /* selection stages rerun with more scoring passes */
  int64_t incremental_factorizations; /* Newton matrices updated from the rows that joined or left the
                                         violator set instead of being recomputed */
  int64_t n_sv;             /* margin violators (y_i o_i < 1) at the returned solution */
  double grad_norm;         /* ||grad f|| at the returned solution (f = F / C) */
  double seconds_select;    /* wall time in greedy selection */
  double seconds_newton;    /* wall time in Newton re-optimisation */
  /* Per-kernel GPU time (HIP events) and algorithmic work of the timed launches of the kernels selected by
   * spsvm_options.profile (every k-th launch with a stride k); zero otherwise. */
  int64_t kblock_launches;  /* timed kernel-block GEMMs (candidate blocks on the kernel of a full group of steps,
                               basis blocks) */
  double kblock_seconds;
  double kblock_flops;      /* 2 n N d per launch, N = columns computed */
  int64_t syrk_launches;    /* timed Newton-matrix SYRKs */
  double syrk_seconds;
  double syrk_flops;        /* n_sv m (m + 1) per launch (lower triangle, multiply-add = 2) */
  int64_t score_launches;   /* timed candidate-score passes over the n rows */
  double score_seconds;
  double score_bytes;       /* bytes the timed passes had to read: their share (timed / launched) of
                               n (12 score_passes_active + sizeof(K) score_slot_passes), i.e. o (FP64) and y (FP32)
                               in every active pass and one candidate column per slot still being scored */
  int64_t chol_calls;       /* timed Cholesky factorisations (all panel kernels of one factorisation) */
  double chol_seconds;
  double chol_flops;        /* m^3 / 3 per factorisation */
  double kblock_mfma_flops; /* MFMA flops the timed kernel blocks issued: whole tiles, the feature dimension padded
                               to the k chunk, three products per multiply-add with the split-BF16 correction */
  int64_t jitter_retries;   /* factorisations repeated with a diagonal shift mu * mean(diag H), mu = 1e-14, 1e-12,
                               1e-10, 1e-8 in turn, because the Newton matrix was not numerically positive definite */
  int64_t stop_reason;      /* 0: |J| reached J_max; 1: the eps_stop rule; 2: no candidate could be added */
  double train_error;       /* fraction of rows with y_i o_i <= 0 at the returned model (1 with an empty basis) */
} spsvm_stats;

/* Fills *opt with the defaults listed above. */
void spsvm_options_default(spsvm_options* opt);

/* Bytes of device workspace spsvm_train needs for n rows, d features of type xdt and up to J_max basis
 * vectors with these options (NULL = defaults). The kernel block n x J_max and the candidate block n x 64
 * dominate. In SPSVM_F32 and SPSVM_F64 the figure includes a copy of X with rows padded to 16-byte
 * boundaries, which training uses when d is not a multiple of 4 (FP32) or 2 (FP64) or X does not start on a
 * 16-byte boundary (the query cannot see X, so it always reserves it in those modes); SPSVM_MIXED reads
 * split BF16 copies of X instead (also in the workspace) and needs no padded copy. */
spsvm_status spsvm_train_workspace_bytes(int64_t n, int64_t d, int64_t J_max, spsvm_dtype xdt,
                                         const spsvm_options* opt, size_t* bytes);

/* Greedy SP-SVM training (section 4, Eq. 4): grows J to J_max rows and returns J and beta.
 *  X:   device, n x d, element type xdt, finite values.
 *  y:   device, n labels, each exactly +1.0f or -1.0f.
 *  C, gamma: finite and > 0. J_max: 1 <= J_max <= number of distinct rows of X.
 *  workspace: device, at least spsvm_train_workspace_bytes(...) bytes, 256-byte aligned; its
 *    contents on entry do not matter and are undefined on return. No other device memory is
 *    allocated except the returned model (X_J and beta copies).
 *  out: receives the model; free it with spsvm_model_free.
 * Rows with identical feature vectors (compared by a 64-bit hash of their values) never both
 * enter J. If fewer than J_max rows can be added (all candidates blocked), training stops early
 * and the model holds fewer basis vectors. */
spsvm_status spsvm_train(const void* X, spsvm_dtype xdt, const float* y, int64_t n, int64_t d, double C,
                         double gamma, int64_t J_max, const spsvm_options* opt, void* workspace,
                         size_t ws_bytes, void* stream, spsvm_model** out);

/* Bytes of device workspace spsvm_train_fixed_basis needs (m basis vectors); as above. */
spsvm_status spsvm_fixed_workspace_bytes(int64_t n, int64_t d, int64_t m, spsvm_dtype xdt, const spsvm_options* opt,
                                         size_t* bytes);

/* Newton re-optimisation of Eq. 4 on a given basis (no selection): computes the kernel block
 * K(X, X_J) for all n rows and the m given rows, then minimises F from beta = 0.
 *  J: host, m distinct row indices in [0, n), rows pairwise distinct in value.
 * Other arguments as for spsvm_train. */
spsvm_status spsvm_train_fixed_basis(const void* X, spsvm_dtype xdt, const float* y, int64_t n, int64_t d,
                                     double C, double gamma, const int64_t* J, int64_t m,
                                     const spsvm_options* opt, void* workspace, size_t ws_bytes, void* stream,
                                     spsvm_model** out);

/* Bytes of device workspace spsvm_train_batch needs for P problems on m shared basis vectors. The
 * workspace holds the Newton state of min(P, 64) problems, which are solved in lockstep; as above. */
spsvm_status spsvm_batch_workspace_bytes(int64_t n, int64_t d, int64_t P, int64_t m, spsvm_dtype xdt,
                                         const spsvm_options* opt, size_t* bytes);

/* P independent Newton re-optimisations of Eq. 4 that share X and one basis J (e.g. one-vs-rest classes
 * crossed with a (C, gamma) grid). Problem p has labels Y + p n, C[p] and gamma[p]. The squared distances
 * between all rows and the basis rows are computed once; the kernel block exp(-gamma D) once per distinct
 * gamma; each problem then runs the Newton solve from beta = 0. Model p equals what
 * spsvm_train_fixed_basis returns for problem p (same kernels, same arithmetic).
 *  Y: device, P x n labels (+1 / -1). C, gamma: host, P values each, finite and > 0.
 *  J: host, m row indices, rows pairwise distinct in value. out: host array of P model pointers; on
 *  failure every entry is NULL. Other arguments as for spsvm_train. */
spsvm_status spsvm_train_batch(const void* X, spsvm_dtype xdt, int64_t n, int64_t d, int64_t P, const float* Y,
                               const double* C, const double* gamma, const int64_t* J, int64_t m,
                               const spsvm_options* opt, void* workspace, size_t ws_bytes, void* stream,
                               spsvm_model** out);

/* Greedy growth of one basis shared by P problems on the same rows (the selection of section 4, "Sparse primal
 * optimization", applied to a one-vs-rest x (C, gamma) batch), each problem re-optimised by Newton after every
 * stage. Every step draws one candidate set as spsvm_train does (same stream and rules); each problem scores every
 * candidate exactly (the decrease of its f_p = F_p / C_p when only the new coefficient is optimised, with its own
 * labels, C and gamma), and the candidate with the largest sum of the problems' scores (added in problem order)
 * joins the basis of every problem, each with its own one-dimensional optimum as the starting coefficient.
 *  Y: device, P x n labels (+1 / -1). C, gamma: host, P values each, finite and > 0. J_max: basis size to reach,
 *  1 .. number of distinct rows. opt: as for spsvm_train; the offset (bias) and the stopping rule (eps_stop) are
 *  not available here (SPSVM_E_INVALID_ARG). out: host array of P model pointers, all on the same basis; on
 *  failure every entry is NULL. Other arguments as for spsvm_train. */
spsvm_status spsvm_train_shared(const void* X, spsvm_dtype xdt, int64_t n, int64_t d, int64_t P, const float* Y,
                                const double* C, const double* gamma, int64_t J_max, const spsvm_options* opt,
                                void* workspace, size_t ws_bytes, void* stream, spsvm_model** out);

/* Bytes of device workspace spsvm_train_shared needs: per distinct value of gamma (host, P values) an n x J_max
 * kernel block, its K_JJ and a candidate block; per problem its outputs, coefficients and candidate-scoring state;
 * the Newton state of min(P, 64) problems solved in lockstep. */
spsvm_status spsvm_train_shared_workspace_bytes(int64_t n, int64_t d, int64_t P, const double* gamma, int64_t J_max,
                                                spsvm_dtype xdt, const spsvm_options* opt, size_t* bytes);

/* Feature matrices as compressed sparse rows (CSR), for data whose dense form is mostly zeros (section 5: the dense
 * GPU implementation could not hold KDDCup99): row i holds the FP32 values values[indptr[i] .. indptr[i + 1]) at
 * the features indices[...], which must lie in [0, d) and increase strictly within the row. indptr: device, n + 1
 * int64 (indptr[0] = 0); indices: device, int32; values: device, FP32, finite. Training runs in SPSVM_F32: the
 * candidate rows are made dense, and each row's nonzeros meet them in FP32 products; the model keeps dense
 * copies of its basis rows, so spsvm_predict (dense rows) and spsvm_predict_csr both apply. */

/* Bytes of device workspace spsvm_train_csr needs (n rows, d features, up to J_max basis vectors). */
spsvm_status spsvm_train_csr_workspace_bytes(int64_t n, int64_t d, int64_t J_max, const spsvm_options* opt,
                                             size_t* bytes);

/* Greedy SP-SVM training on CSR rows; as spsvm_train otherwise (opt->precision must be SPSVM_F32; the offset and
 * the stopping rule apply). Rows are duplicates when their nonzero values and features agree. */
spsvm_status spsvm_train_csr(const int64_t* indptr, const int32_t* indices, const float* values, int64_t n,
                             int64_t d, const float* y, double C, double gamma, int64_t J_max,
                             const spsvm_options* opt, void* workspace, size_t ws_bytes, void* stream,
                             spsvm_model** out);

/* Decision values of CSR rows (d as in training): out[i] = sum_k beta_k exp(-gamma ||x_i - x_{J_k}||^2) + b, FP32
 * kernel values and FP64 sums, for a model with FP32 kernel values. out: device, n_t doubles. Allocates n_t floats of
 * row norms for the call. */
spsvm_status spsvm_predict_csr(const spsvm_model* model, const int64_t* indptr, const int32_t* indices,
                               const float* values, int64_t n_t, double* out, void* stream);

/* Bytes of device workspace spsvm_train_ovo needs when the largest class pair has pair_rows rows (the count of
 * class a plus the count of class b, largest over the pairs): that pair's gathered rows, labels and row indices,
 * and the training workspace of pair_rows rows (as spsvm_train_workspace_bytes). */
spsvm_status spsvm_ovo_workspace_bytes(int64_t pair_rows, int64_t d, int64_t J_max, spsvm_dtype xdt,
                                       const spsvm_options* opt, size_t* bytes);

/* One-vs-one multiclass training, as section 5 trains MNIST8M: one greedy SP-SVM per pair of classes (a, b), a < b,
 * in the order (0, 1), (0, 2), ..., (K - 2, K - 1), each on the rows of classes a (label +1) and b (label -1) only,
 * in their order in X, with C, gamma, J_max and the options shared (the candidate draws of every pair use
 * opt->seed). The pairs run one after another, each on the whole GPU; a pair's rows are gathered into the
 * workspace first.
 *  classes: device, n int32 class ids in [0, K); K >= 2; every class must have rows.
 *  J_max: per pair; a pair with fewer rows trains to its row count (fewer distinct rows: SPSVM_E_INVALID_ARG).
 *  out: host array of K (K - 1) / 2 model pointers; model J indices are rows of X. On failure all are NULL.
 * Other arguments as for spsvm_train. */
spsvm_status spsvm_train_ovo(const void* X, spsvm_dtype xdt, const int32_t* classes, int64_t n, int64_t d, int32_t K,
                             double C, double gamma, int64_t J_max, const spsvm_options* opt, void* workspace,
                             size_t ws_bytes, void* stream, spsvm_model** out);

/* Bytes of device workspace spsvm_predict_ovo needs for n_t rows and K classes. */
spsvm_status spsvm_predict_ovo_workspace_bytes(int64_t n_t, int32_t K, size_t* bytes);

/* One-vs-one prediction: each pair model of spsvm_train_ovo (same order) votes for a when its decision value is
 * positive and for b otherwise; classes[i] is the class with the most votes, the lowest class on ties.
 *  models: host array of K (K - 1) / 2 models. Xt: device, n_t x d. classes: device, n_t int32. */
spsvm_status spsvm_predict_ovo(const spsvm_model* const* models, int32_t K, const void* Xt, spsvm_dtype xdt,
                               int64_t n_t, int32_t* classes, void* workspace, size_t ws_bytes, void* stream);

/* Reads a model. Any output pointer may be NULL.
 *  m: number of basis vectors. J_idx: host, capacity >= m, receives the training-row indices of J in
 *  the order they were added. beta: host, capacity >= m. objective: F(beta) of Eq. 4 (paper scale),
 *  evaluated by the GPU at the returned beta. */
spsvm_status spsvm_model_get(const spsvm_model* model, int64_t* m, int64_t* J_idx, double* beta,
                             double* objective);

/* The offset b of a model (0 unless trained with spsvm_options.bias = 1; batched models share the option). */
spsvm_status spsvm_model_bias(const spsvm_model* model, double* b);

/* Copies the training statistics of a model into *stats. */
spsvm_status spsvm_model_stats(const spsvm_model* model, spsvm_stats* stats);

/* Decision values out[i] = sum_k beta_k exp(-gamma ||xt_i - x_{J_k}||^2) + b (the classifier of Eq. 4; b = 0
 * unless the model was trained with the offset), evaluated in the model's precision with FP64 accumulation.
 *  Xt: device, n_t x d, element type xdt. out: device, n_t doubles. The n_t x m kernel block is never
 *  stored. The model keeps its own copy of X_J, so the training X need not be alive. When d is not a
 *  multiple of 4 (FP32) or 2 (FP64), or Xt is not 16-byte aligned, a padded copy of Xt is allocated for
 *  the call and freed before it returns. */
spsvm_status spsvm_predict(const spsvm_model* model, const void* Xt, spsvm_dtype xdt, int64_t n_t, double* out,
                           void* stream);

/* Releases a model; NULL is allowed. */
void spsvm_model_free(spsvm_model* model);

/* Static text for a status code. */
const char* spsvm_status_string(spsvm_status s);

/* Detail of the last failure on the calling thread ("" if none). Valid until the next call. */
const char* spsvm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPSVM_H */
