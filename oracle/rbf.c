/*
 * FP64 RBF kernel block for the SP-SVM oracle (test infrastructure only: tests, the smoke check and
 * the benchmark's CPU-baseline leg use it; the GPU library never does).
 *
 * out[i*m + k] = exp(-gamma * sum_t (X[i,t] - Z[k,t])^2)
 *
 * This is the RBF kernel as defined in section 2 of the paper (k(x, z) = exp(-gamma ||x - z||^2)),
 * written out with explicit differences, so there is no cancellation from expanding the square.
 * X is n x d and Z is m x d, both row-major FP64; out is n x m row-major FP64.
 * Rows are split over OpenMP threads; each entry is summed in order t = 0..d-1.
 */
#include <math.h>
#include <stdint.h>

void oracle_rbf_block(const double* X, int64_t n, int64_t d, const double* Z, int64_t m, double gamma,
                      double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const double* x = X + i * d;
    for (int64_t k = 0; k < m; ++k) {
      const double* z = Z + k * d;
      double s = 0.0;
      for (int64_t t = 0; t < d; ++t) {
        double df = x[t] - z[t];
        s += df * df;
      }
      out[i * m + k] = exp(-gamma * s);
    }
  }
}
