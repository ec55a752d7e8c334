/*
 * spsvm_components.h - single steps of the SP-SVM hot path behind the same C ABI conventions as
 * spsvm.h (device/host pointers as named, void* stream = hipStream_t or NULL, calls return after the
 * GPU work is done, status codes, spsvm_last_error for details). They run the same kernels as
 * spsvm_train and exist so each step can be checked and timed on its own.
 */
#ifndef SPSVM_COMPONENTS_H
#define SPSVM_COMPONENTS_H

#include "spsvm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* RBF kernel block (section 2 kernel; the K(X, X_J) block and candidate columns of section 4):
 *   out[i * ldo + c] = exp(-gamma ||x_i - x_{idx[c]}||^2),  0 <= i < n, 0 <= c < ncols,
 * with squared distances |x_i|^2 + |x_j|^2 - 2 x_i . x_j clamped at 0, dot products on MFMA.
 *  X: device n x d (xdt). idx: device, ncols int32 row indices in [0, n) (a negative index leaves that
 *  column untouched). precision: SPSVM_F64 (out is double), SPSVM_F32 (out is float, FP32 products) or
 *  SPSVM_MIXED (out is float, split-BF16 products hi.hi' + hi.lo' + lo.hi' accumulated in FP32; when every
 *  value of X is a BF16 number the lo parts are zero and the single-pass products hi.hi' give the same values).
 *  out: device, n rows of leading dimension ldo >= ncols. workspace: device, 256-byte aligned, at least
 *  spsvm_rbf_block_workspace_bytes(n, d, xdt) bytes (row norms, a padded copy of X when d is not a
 *  multiple of 4 for FP32 / 2 for FP64 or X is not 16-byte aligned, and for SPSVM_MIXED the BF16 hi and lo
 *  copies of X, d rounded up to 32 per row, and a flag word). The call returns after the stream has
 *  finished the block. */
spsvm_status spsvm_rbf_block(const void* X, spsvm_dtype xdt, int64_t n, int64_t d, const int32_t* idx, int64_t ncols,
                             spsvm_precision precision, double gamma, void* out, int64_t ldo, void* workspace,
                             size_t ws_bytes, void* stream);

/* Bytes of device workspace spsvm_rbf_block needs. */
spsvm_status spsvm_rbf_block_workspace_bytes(int64_t n, int64_t d, spsvm_dtype xdt, size_t* bytes);

/* Bytes of device workspace spsvm_newton_solve needs for an m x m system. */
spsvm_status spsvm_newton_solve_workspace_bytes(int64_t m, size_t* bytes);

/* Newton step of section 4: FP64 Cholesky H = L L^T (in place: the lower triangle of H is overwritten
 * by L; the strict upper triangle is neither read nor written), then x = -H^{-1} g.
 *  H: device, m x m FP64, row-major with leading dimension ldh >= m. g, x: device, m doubles.
 *  Returns SPSVM_E_NOT_PD (no retry) when a pivot is not positive or not finite. */
spsvm_status spsvm_newton_solve(double* H, int64_t ldh, int64_t m, const double* g, double* x, void* workspace,
                                size_t ws_bytes, void* stream);

/* spsvm_newton_solve without a workspace, for callers that cannot allocate device memory (work captured in a
 * HIP graph around the call, tight serving loops, harnesses that forbid hipMalloc). Same arguments, kernels and
 * results as spsvm_newton_solve, for 1 <= m <= 4096; larger m is rejected with SPSVM_E_INVALID_ARG before any GPU
 * work. Its scratch (the inverted diagonal blocks of L, a work vector, a status flag; 2.1 MiB) is a static device
 * array that each GPU the library runs on holds until the process ends; no device memory is allocated or freed.
 * Every call on one GPU uses that GPU's array, so calls that overlap on one GPU (other threads, other streams)
 * race; the call synchronises its stream before it returns. */
spsvm_status spsvm_newton_solve_noalloc(double* H, int64_t ldh, int64_t m, const double* g, double* x, void* stream);

/* Candidate rows of addition step t (0-based over the whole run) when no row is blocked: SplitMix64
 * (Steele, Lea and Flood 2014) from state seed ^ ((t + 1) * 0x9E3779B97F4A7C15), index = high 32 bits of
 * each output times n, shifted right by 32; repeats are skipped; at most 64 * kappa draws.
 *  out: host, 64 int32; unused slots are set to -1. Host-only: no GPU work. */
spsvm_status spsvm_candidate_draw(uint64_t seed, int64_t t, int64_t n, int32_t kappa, int32_t* out);

/* Greedy-selection scores of section 4 ("Sparse primal optimization": each candidate of a random subset is
 * scored by the loss reduction it would bring). For candidate c with kernel column k_c (k_c(x_c) = 1) the score
 * is the exact decrease of f(beta) = lambda/2 beta^T K_JJ beta + 1/2 sum_i max(0, 1 - y_i o_i)^2 (lambda = 1 / C,
 * Eq. 4 divided by C) when only a new coefficient s for c is optimised and every other coefficient is fixed:
 *   psi_c(s) - f = lambda (s o_c + s^2 / 2) + 1/2 sum_i [max(0, a_i - s b_i)^2 - max(0, a_i)^2],
 *   a_i = 1 - y_i o_i, b_i = y_i k_c[i],  score_c = psi_c(0) - min_s psi_c(s) >= 0.
 * The same passes and updates as greedy training run (64 candidate slots, semismooth Newton on psi_c' with the
 * window walk, candidates that cannot win dropped), up to 64 passes.
 *  o: device, n doubles (current outputs K_XJ beta). y: device, n floats, each exactly +1 or -1 (checked on the
 *    device first: SPSVM_E_INVALID_ARG otherwise).
 *  Kc: device, the ncand candidate columns, column-major: column c (n values of type kdt) starts at
 *    Kc + c * ldc elements, ldc >= n. oc: host, ncand doubles, o at each candidate's row. 1 <= ncand <= 64.
 *  s_out, score_out: host, ncand doubles: the minimiser and the score of each candidate with status 1; a dropped
 *    candidate (status 3: its largest possible score is below another candidate's reached one) reports the
 *    bracket point it stopped at and -infinity. status_out, passes_out: host, ncand int32 (may be NULL): 1 scored,
 *    3 dropped; the passes over the rows each slot took. winner: host, the candidate with the largest score (the
 *    lowest index on ties), -1 if none.
 *  workspace: device, 256-byte aligned, at least spsvm_score_workspace_bytes(n) bytes. */
spsvm_status spsvm_score_candidates(const double* o, const float* y, int64_t n, const void* Kc, spsvm_dtype kdt,
                                    int64_t ldc, const double* oc, int32_t ncand, double C, double* s_out,
                                    double* score_out, int32_t* status_out, int32_t* passes_out, int32_t* winner,
                                    void* workspace, size_t ws_bytes, void* stream);

/* Bytes of device workspace spsvm_score_candidates needs for n rows. */
spsvm_status spsvm_score_workspace_bytes(int64_t n, size_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* SPSVM_COMPONENTS_H */
