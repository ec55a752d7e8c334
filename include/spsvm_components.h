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
 *  SPSVM_MIXED (out is float, split-BF16 products hi.hi' + hi.lo' + lo.hi' accumulated in FP32).
 *  out: device, n rows of leading dimension ldo >= ncols. workspace: device, 256-byte aligned, at least
 *  spsvm_rbf_block_workspace_bytes(n, d, xdt) bytes (row norms, a padded copy of X when d is not a
 *  multiple of 4 for FP32 / 2 for FP64 or X is not 16-byte aligned, and for SPSVM_MIXED the BF16 hi and lo
 *  copies of X, d rounded up to 32 per row). */
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

/* Candidate rows of addition step t (0-based over the whole run) when no row is blocked: SplitMix64
 * (Steele, Lea and Flood 2014) from state seed ^ ((t + 1) * 0x9E3779B97F4A7C15), index = high 32 bits of
 * each output times n, shifted right by 32; repeats are skipped; at most 64 * kappa draws.
 *  out: host, 64 int32; unused slots are set to -1. Host-only: no GPU work. */
spsvm_status spsvm_candidate_draw(uint64_t seed, int64_t t, int64_t n, int32_t kappa, int32_t* out);

#ifdef __cplusplus
}
#endif

#endif /* SPSVM_COMPONENTS_H */
