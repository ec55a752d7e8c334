// C ABI of the SP-SVM library (declared in include/spsvm.h). Argument checks, status codes and the
// thread-local error text; the work itself is in trainer.cpp and the kernels.
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "trainer.h"

namespace {
thread_local std::string g_last_error;

spsvm_status fail(spsvm_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

template <typename F>
spsvm_status guarded(F&& body) {
  try {
    g_last_error.clear();
    body();
    return SPSVM_OK;
  } catch (const spsvm::Failure& e) {
    return fail((spsvm_status)e.status, e.what());
  } catch (const std::bad_alloc&) {
    return fail(SPSVM_E_OUT_OF_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(SPSVM_E_HIP, e.what());
  } catch (...) {
    return fail(SPSVM_E_HIP, "unknown failure");
  }
}

spsvm_options resolve(const spsvm_options* opt) {
  spsvm_options o;
  spsvm_options_default(&o);
  if (opt) {
    if (opt->struct_size != sizeof(spsvm_options))
      throw spsvm::Failure(SPSVM_E_INVALID_ARG, "spsvm_options.struct_size mismatch (use spsvm_options_default)");
    o = *opt;
  }
  if (o.kappa < 1 || o.kappa > 64) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "kappa must lie in [1, 64]");
  if (!(o.growth >= 0.0) || !std::isfinite(o.growth)) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "growth must be >= 0");
  if (o.chunk_cap < 1 || o.chunk_cap > 4096) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "chunk_cap must lie in [1, 4096]");
  if (!(o.newton_tol >= 0.0) || !(o.newton_ftol >= 0.0))
    throw spsvm::Failure(SPSVM_E_INVALID_ARG, "newton tolerances must be >= 0");
  if (o.newton_max_iter < 1) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "newton_max_iter must be >= 1");
  if (!(o.refactor_frac >= 0.0) || !std::isfinite(o.refactor_frac))
    throw spsvm::Failure(SPSVM_E_INVALID_ARG, "refactor_frac must be finite and >= 0");
  if (o.bias != 0 && o.bias != 1) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bias must be 0 or 1");
  if (!(o.eps_stop >= 0.0) || !std::isfinite(o.eps_stop))
    throw spsvm::Failure(SPSVM_E_INVALID_ARG, "eps_stop must be finite and >= 0");
  if (o.kxj_host != 0 && o.kxj_host != 1) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "kxj_host must be 0 or 1");
  if (o.precision != SPSVM_F64 && o.precision != SPSVM_F32 && o.precision != SPSVM_MIXED)
    throw spsvm::Failure(SPSVM_E_INVALID_ARG, "precision must be SPSVM_F64, SPSVM_F32 or SPSVM_MIXED");
  return o;
}

void check_problem(const void* X, spsvm_dtype xdt, const float* y, int64_t n, int64_t d, double C, double gamma,
                   int64_t J_max) {
  using spsvm::Failure;
  if (!X || !y) throw Failure(SPSVM_E_INVALID_ARG, "X and y must be device pointers");
  if (xdt != SPSVM_DT_F32 && xdt != SPSVM_DT_F64) throw Failure(SPSVM_E_INVALID_ARG, "unknown dtype");
  if (n < 1 || n > 0x7fffffffLL) throw Failure(SPSVM_E_INVALID_ARG, "n must lie in [1, 2^31 - 1]");
  if (d < 1) throw Failure(SPSVM_E_INVALID_ARG, "d must be >= 1");
  if (!(C > 0.0) || !std::isfinite(C)) throw Failure(SPSVM_E_INVALID_ARG, "C must be finite and > 0");
  if (!(gamma > 0.0) || !std::isfinite(gamma)) throw Failure(SPSVM_E_INVALID_ARG, "gamma must be finite and > 0");
  if (J_max < 1 || J_max > n || J_max > 65536) throw Failure(SPSVM_E_INVALID_ARG, "J_max must lie in [1, min(n, 65536)]");
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }
}  // namespace

extern "C" {

void spsvm_options_default(spsvm_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(spsvm_options);
  o->seed = 0;
  o->kappa = 59;
  o->growth = 0.25;
  o->chunk_cap = 256;
  o->newton_tol = 1e-10;
  o->newton_ftol = 1e-14;
  o->newton_max_iter = 50;
  o->precision = SPSVM_F32;
  o->log_level = 0;
  o->profile = 0;
  o->refactor_frac = 0.002;
  o->bias = 0;
  o->eps_stop = 0.0;
  o->kxj_host = 0;
}

spsvm_status spsvm_train_workspace_bytes(int64_t n, int64_t d, int64_t J_max, spsvm_dtype xdt,
                                         const spsvm_options* opt, size_t* bytes) {
  return guarded([&] {
    if (!bytes) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bytes must not be NULL");
    if (n < 1 || d < 1 || J_max < 1 || J_max > n) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bad sizes");
    if (xdt != SPSVM_DT_F32 && xdt != SPSVM_DT_F64) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "unknown dtype");
    *bytes = spsvm::make_plan(n, d, J_max, resolve(opt), true, xdt == SPSVM_DT_F64, false).bytes;
  });
}

spsvm_status spsvm_fixed_workspace_bytes(int64_t n, int64_t d, int64_t m, spsvm_dtype xdt, const spsvm_options* opt,
                                         size_t* bytes) {
  return guarded([&] {
    if (!bytes) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bytes must not be NULL");
    if (n < 1 || d < 1 || m < 1 || m > n) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bad sizes");
    if (xdt != SPSVM_DT_F32 && xdt != SPSVM_DT_F64) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "unknown dtype");
    *bytes = spsvm::make_plan(n, d, m, resolve(opt), false, xdt == SPSVM_DT_F64, false).bytes;
  });
}

spsvm_status spsvm_train(const void* X, spsvm_dtype xdt, const float* y, int64_t n, int64_t d, double C, double gamma,
                         int64_t J_max, const spsvm_options* opt, void* workspace, size_t ws_bytes, void* stream,
                         spsvm_model** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!out) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "out must not be NULL");
    const spsvm_options o = resolve(opt);
    check_problem(X, xdt, y, n, d, C, gamma, J_max);
    *out = spsvm::run_train(X, xdt == SPSVM_DT_F64, y, n, d, C, gamma, J_max, o, workspace, ws_bytes,
                            as_stream(stream), nullptr);
  });
}

spsvm_status spsvm_train_fixed_basis(const void* X, spsvm_dtype xdt, const float* y, int64_t n, int64_t d, double C,
                                     double gamma, const int64_t* J, int64_t m, const spsvm_options* opt,
                                     void* workspace, size_t ws_bytes, void* stream, spsvm_model** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!out) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "out must not be NULL");
    if (!J) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "J must be a host array");
    const spsvm_options o = resolve(opt);
    check_problem(X, xdt, y, n, d, C, gamma, m);
    *out = spsvm::run_train(X, xdt == SPSVM_DT_F64, y, n, d, C, gamma, m, o, workspace, ws_bytes, as_stream(stream), J);
  });
}

spsvm_status spsvm_batch_workspace_bytes(int64_t n, int64_t d, int64_t P, int64_t m, spsvm_dtype xdt,
                                         const spsvm_options* opt, size_t* bytes) {
  return guarded([&] {
    if (!bytes) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bytes must not be NULL");
    if (n < 1 || d < 1 || m < 1 || m > n || P < 1) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bad sizes");
    if (xdt != SPSVM_DT_F32 && xdt != SPSVM_DT_F64) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "unknown dtype");
    *bytes = spsvm::make_plan(n, d, m, resolve(opt), false, xdt == SPSVM_DT_F64, false, true, P).bytes;
  });
}

spsvm_status spsvm_train_batch(const void* X, spsvm_dtype xdt, int64_t n, int64_t d, int64_t P, const float* Y,
                               const double* C, const double* gamma, const int64_t* J, int64_t m,
                               const spsvm_options* opt, void* workspace, size_t ws_bytes, void* stream,
                               spsvm_model** out) {
  if (out && P > 0)
    for (int64_t p = 0; p < P; ++p) out[p] = nullptr;
  return guarded([&] {
    using spsvm::Failure;
    if (!out || !C || !gamma || !J) throw Failure(SPSVM_E_INVALID_ARG, "out, C, gamma and J must be host arrays");
    if (P < 1 || P > (1 << 20)) throw Failure(SPSVM_E_INVALID_ARG, "P must lie in [1, 2^20]");
    const spsvm_options o = resolve(opt);
    if (o.kxj_host) throw Failure(SPSVM_E_INVALID_ARG, "kxj_host does not apply to batches");
    for (int64_t p = 0; p < P; ++p) check_problem(X, xdt, Y, n, d, C[p], gamma[p], m);
    spsvm::run_train_batch(X, xdt == SPSVM_DT_F64, n, d, P, Y, C, gamma, J, m, o, workspace, ws_bytes,
                           as_stream(stream), out);
  });
}

spsvm_status spsvm_train_shared_workspace_bytes(int64_t n, int64_t d, int64_t P, const double* gamma, int64_t J_max,
                                                spsvm_dtype xdt, const spsvm_options* opt, size_t* bytes) {
  return guarded([&] {
    if (!bytes || !gamma) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bytes and gamma must not be NULL");
    if (n < 1 || d < 1 || J_max < 1 || J_max > n || P < 1 || P > (1 << 20))
      throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bad sizes");
    if (xdt != SPSVM_DT_F32 && xdt != SPSVM_DT_F64) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "unknown dtype");
    *bytes = spsvm::make_plan(n, d, J_max, resolve(opt), true, xdt == SPSVM_DT_F64, false, true, P, false,
                              spsvm::distinct_gammas(gamma, P))
                 .bytes;
  });
}

spsvm_status spsvm_train_shared(const void* X, spsvm_dtype xdt, int64_t n, int64_t d, int64_t P, const float* Y,
                                const double* C, const double* gamma, int64_t J_max, const spsvm_options* opt,
                                void* workspace, size_t ws_bytes, void* stream, spsvm_model** out) {
  if (out && P > 0 && P <= (1 << 20))
    for (int64_t p = 0; p < P; ++p) out[p] = nullptr;
  return guarded([&] {
    using spsvm::Failure;
    if (!out || !C || !gamma) throw Failure(SPSVM_E_INVALID_ARG, "out, C and gamma must be host arrays");
    if (P < 1 || P > (1 << 20)) throw Failure(SPSVM_E_INVALID_ARG, "P must lie in [1, 2^20]");
    const spsvm_options o = resolve(opt);
    if (o.bias || o.eps_stop > 0.0 || o.kxj_host)
      throw Failure(SPSVM_E_INVALID_ARG, "the shared basis takes neither the offset, the stopping rule nor kxj_host");
    for (int64_t p = 0; p < P; ++p) check_problem(X, xdt, Y, n, d, C[p], gamma[p], J_max);
    spsvm::run_train_shared(X, xdt == SPSVM_DT_F64, n, d, P, Y, C, gamma, J_max, o, workspace, ws_bytes,
                            as_stream(stream), out);
  });
}

spsvm_status spsvm_train_csr_workspace_bytes(int64_t n, int64_t d, int64_t J_max, const spsvm_options* opt,
                                             size_t* bytes) {
  return guarded([&] {
    if (!bytes) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bytes must not be NULL");
    if (n < 1 || d < 1 || J_max < 1 || J_max > n) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bad sizes");
    *bytes = spsvm::make_plan(n, d, J_max, resolve(opt), true, false, true, false, 1, true).bytes;
  });
}

spsvm_status spsvm_train_csr(const int64_t* indptr, const int32_t* indices, const float* values, int64_t n,
                             int64_t d, const float* y, double C, double gamma, int64_t J_max,
                             const spsvm_options* opt, void* workspace, size_t ws_bytes, void* stream,
                             spsvm_model** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    using spsvm::Failure;
    if (!out) throw Failure(SPSVM_E_INVALID_ARG, "out must not be NULL");
    if (!indptr || !indices || !values) throw Failure(SPSVM_E_INVALID_ARG, "indptr, indices and values must be device pointers");
    const spsvm_options o = resolve(opt);
    check_problem(values, SPSVM_DT_F32, y, n, d, C, gamma, J_max);
    if (d > 0x7fffffffLL) throw Failure(SPSVM_E_INVALID_ARG, "d must fit int32 feature indices");
    int64_t nnz = 0;
    SPSVM_HIP(hipMemcpy(&nnz, indptr + n, sizeof(int64_t), hipMemcpyDeviceToHost));
    if (nnz < 0) throw Failure(SPSVM_E_INVALID_ARG, "indptr[n] must be >= 0");
    spsvm::CsrX X;
    X.indptr = indptr;
    X.indices = indices;
    X.values = values;
    X.nnz = nnz;
    *out = spsvm::run_train_csr(X, y, n, d, C, gamma, J_max, o, workspace, ws_bytes, as_stream(stream));
  });
}

spsvm_status spsvm_predict_csr(const spsvm_model* md, const int64_t* indptr, const int32_t* indices,
                               const float* values, int64_t n_t, double* out, void* stream) {
  return guarded([&] {
    using spsvm::Failure;
    if (!md) throw Failure(SPSVM_E_INVALID_ARG, "model must not be NULL");
    if (n_t < 0) throw Failure(SPSVM_E_INVALID_ARG, "n_t must be >= 0");
    if (n_t == 0) return;
    if (!indptr || !indices || !values || !out) throw Failure(SPSVM_E_INVALID_ARG, "CSR arrays and out must be device pointers");
    spsvm::CsrX X;
    X.indptr = indptr;
    X.indices = indices;
    X.values = values;
    spsvm::run_predict_csr(md, X, n_t, out, as_stream(stream));
  });
}

spsvm_status spsvm_ovo_workspace_bytes(int64_t pair_rows, int64_t d, int64_t J_max, spsvm_dtype xdt,
                                       const spsvm_options* opt, size_t* bytes) {
  return guarded([&] {
    if (!bytes) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bytes must not be NULL");
    if (pair_rows < 2 || d < 1 || J_max < 1) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bad sizes");
    if (xdt != SPSVM_DT_F32 && xdt != SPSVM_DT_F64) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "unknown dtype");
    *bytes = spsvm::ovo_workspace_bytes(pair_rows, d, std::min(J_max, pair_rows), resolve(opt), xdt == SPSVM_DT_F64);
  });
}

spsvm_status spsvm_train_ovo(const void* X, spsvm_dtype xdt, const int32_t* classes, int64_t n, int64_t d, int32_t K,
                             double C, double gamma, int64_t J_max, const spsvm_options* opt, void* workspace,
                             size_t ws_bytes, void* stream, spsvm_model** out) {
  if (out && K >= 2 && K <= 4096)
    for (int64_t p = 0; p < (int64_t)K * (K - 1) / 2; ++p) out[p] = nullptr;
  return guarded([&] {
    using spsvm::Failure;
    if (!out) throw Failure(SPSVM_E_INVALID_ARG, "out must be a host array");
    if (!classes) throw Failure(SPSVM_E_INVALID_ARG, "classes must be a device pointer");
    if (K < 2 || K > 4096) throw Failure(SPSVM_E_INVALID_ARG, "K must lie in [2, 4096]");
    const spsvm_options o = resolve(opt);
    if (!X) throw Failure(SPSVM_E_INVALID_ARG, "X must be a device pointer");
    if (xdt != SPSVM_DT_F32 && xdt != SPSVM_DT_F64) throw Failure(SPSVM_E_INVALID_ARG, "unknown dtype");
    if (n < 2 || n > 0x7fffffffLL) throw Failure(SPSVM_E_INVALID_ARG, "n must lie in [2, 2^31 - 1]");
    if (d < 1) throw Failure(SPSVM_E_INVALID_ARG, "d must be >= 1");
    if (!(C > 0.0) || !std::isfinite(C)) throw Failure(SPSVM_E_INVALID_ARG, "C must be finite and > 0");
    if (!(gamma > 0.0) || !std::isfinite(gamma)) throw Failure(SPSVM_E_INVALID_ARG, "gamma must be finite and > 0");
    if (J_max < 1 || J_max > 65536) throw Failure(SPSVM_E_INVALID_ARG, "J_max must lie in [1, 65536]");
    spsvm::run_train_ovo(X, xdt == SPSVM_DT_F64, classes, n, d, K, C, gamma, J_max, o, workspace, ws_bytes,
                         as_stream(stream), out);
  });
}

spsvm_status spsvm_predict_ovo_workspace_bytes(int64_t n_t, int32_t K, size_t* bytes) {
  return guarded([&] {
    if (!bytes || n_t < 0 || K < 2) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bad arguments");
    *bytes = spsvm::ovo_predict_workspace_bytes(n_t, K);
  });
}

spsvm_status spsvm_predict_ovo(const spsvm_model* const* models, int32_t K, const void* Xt, spsvm_dtype xdt,
                               int64_t n_t, int32_t* classes, void* workspace, size_t ws_bytes, void* stream) {
  return guarded([&] {
    using spsvm::Failure;
    if (!models || K < 2 || K > 4096) throw Failure(SPSVM_E_INVALID_ARG, "models must hold K (K - 1) / 2 models, K >= 2");
    if (n_t < 0) throw Failure(SPSVM_E_INVALID_ARG, "n_t must be >= 0");
    if (n_t == 0) return;
    if (!Xt || !classes) throw Failure(SPSVM_E_INVALID_ARG, "Xt and classes must be device pointers");
    if (xdt != SPSVM_DT_F32 && xdt != SPSVM_DT_F64) throw Failure(SPSVM_E_INVALID_ARG, "unknown dtype");
    spsvm::run_predict_ovo(models, K, Xt, xdt == SPSVM_DT_F64, n_t, classes, workspace, ws_bytes, as_stream(stream));
  });
}

spsvm_status spsvm_model_get(const spsvm_model* md, int64_t* m, int64_t* J_idx, double* beta, double* objective) {
  return guarded([&] {
    if (!md) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "model must not be NULL");
    if (m) *m = md->m;
    if (J_idx && md->m) std::memcpy(J_idx, md->J.data(), md->m * sizeof(int64_t));
    if (beta && md->m) std::memcpy(beta, md->beta.data(), md->m * sizeof(double));
    if (objective) *objective = md->objective;
  });
}

spsvm_status spsvm_model_bias(const spsvm_model* md, double* b) {
  return guarded([&] {
    if (!md || !b) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "model and b must not be NULL");
    *b = md->bias;
  });
}

spsvm_status spsvm_model_stats(const spsvm_model* md, spsvm_stats* stats) {
  return guarded([&] {
    if (!md || !stats) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "model and stats must not be NULL");
    *stats = md->stats;
  });
}

spsvm_status spsvm_predict(const spsvm_model* md, const void* Xt, spsvm_dtype xdt, int64_t n_t, double* out,
                           void* stream) {
  return guarded([&] {
    if (!md) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "model must not be NULL");
    if (n_t < 0) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "n_t must be >= 0");
    if (n_t == 0) return;
    if (!Xt || !out) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "Xt and out must be device pointers");
    if (xdt != SPSVM_DT_F32 && xdt != SPSVM_DT_F64) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "unknown dtype");
    spsvm::run_predict(md, Xt, xdt == SPSVM_DT_F64, n_t, out, as_stream(stream));
  });
}

void spsvm_model_free(spsvm_model* md) { delete md; }

const char* spsvm_status_string(spsvm_status s) {
  switch (s) {
    case SPSVM_OK: return "ok";
    case SPSVM_E_INVALID_ARG: return "invalid argument";
    case SPSVM_E_OUT_OF_MEMORY: return "out of memory";
    case SPSVM_E_HIP: return "HIP runtime error";
    case SPSVM_E_NOT_PD: return "Newton matrix not positive definite";
    case SPSVM_E_NO_CONVERGENCE: return "no convergence";
    case SPSVM_E_WORKSPACE: return "workspace missing, misaligned or too small";
  }
  return "unknown status";
}

const char* spsvm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ------------------------------------------------------------------------------------------ components
#include "../../include/spsvm_components.h"
#include "launch.h"

extern "C" {

}  // extern "C"

static size_t rbf_ws(int64_t n, int64_t d, bool xd) {
  const int64_t xe = xd ? 8 : 4, ld = spsvm::round_up(d, 16 / xe);
  const size_t split = (size_t)spsvm::round_up(n * spsvm::split_ld(d) * 2, 256);  // one BF16 copy
  return (size_t)spsvm::round_up(n * 8, 256) + (size_t)spsvm::round_up(n * ld * xe, 256) + 2 * split + 256;
}

template <typename TX, typename TK>
static void rbf_typed(const TX* X, int64_t n, int64_t d, const int32_t* idx, int64_t ncols, double gamma, TK* out,
                      int64_t ldo, char* ws, hipStream_t st, bool split = false) {
  TK* nrm = (TK*)ws;
  const int64_t ld = spsvm::padded_ld<TX>(d);
  const TX* A = X;
  if (ld != d || ((uintptr_t)X & 15u)) {
    TX* Xp = (TX*)(ws + spsvm::round_up(n * 8, 256));
    spsvm::launch_pad_rows<TX>(X, n, d, Xp, ld, st);
    A = Xp;
  }
  spsvm::launch_row_norms<TX, TK>(X, n, d, d, nrm, st);
  if constexpr (std::is_same<TK, float>::value) {
    if (split) {
      const int64_t ldb = spsvm::split_ld(d);
      unsigned short* hi = (unsigned short*)(ws + spsvm::round_up(n * 8, 256) +
                                             spsvm::round_up(n * spsvm::padded_ld<TX>(d) * (int64_t)sizeof(TX), 256));
      unsigned short* lo = hi + spsvm::round_up(n * ldb * 2, 256) / 2;
      // rows whose values are all BF16 numbers have zero lo parts: single-pass products give the same values
      int32_t* flags = (int32_t*)(lo + spsvm::round_up(n * ldb * 2, 256) / 2);
      SPSVM_HIP(hipMemsetAsync(flags, 0, 16, st));
      spsvm::launch_check_inputs<TX>(X, n * d, nullptr, n, flags, st);
      int32_t f[4];
      SPSVM_HIP(hipMemcpyAsync(f, flags, 16, hipMemcpyDeviceToHost, st));
      SPSVM_HIP(hipStreamSynchronize(st));
      if (f[2] == 0) lo = nullptr;
      spsvm::launch_split_bf16<TX>(X, n, d, d, hi, lo, ldb, st);
      spsvm::launch_kblock_bf16(hi, lo, ldb, n, nrm, idx, (int)ncols, out, ldo, gamma, st);
      return;
    }
  }
  spsvm::launch_kblock<TX, TK>(A, ld, n, d, nrm, idx, (int)ncols, out, ldo, gamma, st);
}

extern "C" {

spsvm_status spsvm_rbf_block(const void* X, spsvm_dtype xdt, int64_t n, int64_t d, const int32_t* idx, int64_t ncols,
                             spsvm_precision precision, double gamma, void* out, int64_t ldo, void* workspace,
                             size_t ws_bytes, void* stream) {
  return guarded([&] {
    using spsvm::Failure;
    if (!X || !idx || !out) throw Failure(SPSVM_E_INVALID_ARG, "X, idx and out must be device pointers");
    if (n < 0 || d < 1 || ncols < 0 || ncols > 0x7fffffff || ldo < ncols)
      throw Failure(SPSVM_E_INVALID_ARG, "bad sizes");
    if (!(gamma > 0.0) || !std::isfinite(gamma)) throw Failure(SPSVM_E_INVALID_ARG, "gamma must be finite and > 0");
    if (precision != SPSVM_F64 && precision != SPSVM_F32 && precision != SPSVM_MIXED)
      throw Failure(SPSVM_E_INVALID_ARG, "bad precision");
    if (xdt != SPSVM_DT_F32 && xdt != SPSVM_DT_F64) throw Failure(SPSVM_E_INVALID_ARG, "unknown dtype");
    const bool xd = xdt == SPSVM_DT_F64;
    if (!workspace || ((uintptr_t)workspace & 255u) || ws_bytes < rbf_ws(n, d, xd))
      throw Failure(SPSVM_E_WORKSPACE, "workspace must be 256-byte aligned with >= spsvm_rbf_block_workspace_bytes");
    hipStream_t st = as_stream(stream);
    char* w = (char*)workspace;
    if (precision == SPSVM_F64) {
      if (xd)
        rbf_typed<double, double>((const double*)X, n, d, idx, ncols, gamma, (double*)out, ldo, w, st);
      else
        rbf_typed<float, double>((const float*)X, n, d, idx, ncols, gamma, (double*)out, ldo, w, st);
    } else {
      const bool split = precision == SPSVM_MIXED;
      if (xd)
        rbf_typed<double, float>((const double*)X, n, d, idx, ncols, gamma, (float*)out, ldo, w, st, split);
      else
        rbf_typed<float, float>((const float*)X, n, d, idx, ncols, gamma, (float*)out, ldo, w, st, split);
    }
    SPSVM_HIP(hipStreamSynchronize(st));
  });
}

spsvm_status spsvm_rbf_block_workspace_bytes(int64_t n, int64_t d, spsvm_dtype xdt, size_t* bytes) {
  return guarded([&] {
    if (!bytes || n < 0 || d < 1 || (xdt != SPSVM_DT_F32 && xdt != SPSVM_DT_F64))
      throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bad arguments");
    *bytes = rbf_ws(n, d, xdt == SPSVM_DT_F64);
  });
}

static size_t solve_ws(int64_t m) {
  return (size_t)spsvm::round_up((int64_t)spsvm::ceil_div(m, spsvm::kCholNB) * spsvm::kCholNB * spsvm::kCholNB * 8, 256) +
         (size_t)spsvm::round_up(m * 8, 256) + 256;
}

spsvm_status spsvm_newton_solve_workspace_bytes(int64_t m, size_t* bytes) {
  return guarded([&] {
    if (!bytes || m < 1) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "m must be >= 1 and bytes not NULL");
    *bytes = solve_ws(m);
  });
}

spsvm_status spsvm_newton_solve(double* H, int64_t ldh, int64_t m, const double* g, double* x, void* workspace,
                                size_t ws_bytes, void* stream) {
  return guarded([&] {
    using spsvm::Failure;
    if (!H || !g || !x) throw Failure(SPSVM_E_INVALID_ARG, "H, g and x must be device pointers");
    if (m < 1 || m > 65536 || ldh < m) throw Failure(SPSVM_E_INVALID_ARG, "bad sizes");
    if (!workspace || ((uintptr_t)workspace & 255u) || ws_bytes < solve_ws(m))
      throw Failure(SPSVM_E_WORKSPACE, "workspace missing, misaligned or too small");
    hipStream_t st = as_stream(stream);
    char* w = (char*)workspace;
    double* Linv = (double*)w;
    w += spsvm::round_up((int64_t)spsvm::ceil_div(m, spsvm::kCholNB) * spsvm::kCholNB * spsvm::kCholNB * 8, 256);
    double* z = (double*)w;
    w += spsvm::round_up(m * 8, 256);
    spsvm::NewtonScalars* sc = (spsvm::NewtonScalars*)w;
    SPSVM_HIP(hipMemsetAsync(sc, 0, sizeof(spsvm::NewtonScalars), st));
    spsvm::launch_cholesky(H, ldh, (int)m, Linv, sc, st);
    spsvm::launch_chol_solve(H, ldh, (int)m, Linv, g, x, z, st);
    int32_t fl = 0;
    SPSVM_HIP(hipMemcpyAsync(&fl, &sc->fail, 4, hipMemcpyDeviceToHost, st));
    SPSVM_HIP(hipStreamSynchronize(st));
    if (fl) throw Failure(SPSVM_E_NOT_PD, "Cholesky met a non-positive or non-finite pivot");
  });
}

// Scoring workspace: slot states, per-workgroup partial records of a pass, the candidate table, o at the
// candidate rows, zero hashes (no candidate is blocked) and the scalars.
static int64_t score_nblk_max(int64_t n) { return std::min<int64_t>(spsvm::ceil_div(n, 128), 4096); }
static size_t score_ws(int64_t n) {
  using spsvm::kCandSlots;
  return (size_t)spsvm::round_up((int64_t)spsvm::kCandStateBytes, 256) +
         (size_t)spsvm::round_up(score_nblk_max(n) * kCandSlots * 4 * 8, 256) + 4 * 256 * 2 +
         (size_t)spsvm::round_up((int64_t)sizeof(spsvm::NewtonScalars), 256);
}

spsvm_status spsvm_score_workspace_bytes(int64_t n, size_t* bytes) {
  return guarded([&] {
    if (!bytes || n < 1) throw spsvm::Failure(SPSVM_E_INVALID_ARG, "n must be >= 1 and bytes not NULL");
    *bytes = score_ws(n);
  });
}

spsvm_status spsvm_score_candidates(const double* o, const float* y, int64_t n, const void* Kc, spsvm_dtype kdt,
                                    int64_t ldc, const double* oc, int32_t ncand, double C, double* s_out,
                                    double* score_out, int32_t* status_out, int32_t* passes_out, int32_t* winner,
                                    void* workspace, size_t ws_bytes, void* stream) {
  return guarded([&] {
    using namespace spsvm;
    if (!o || !y || !Kc) throw Failure(SPSVM_E_INVALID_ARG, "o, y and Kc must be device pointers");
    if (!oc || !s_out || !score_out || !winner) throw Failure(SPSVM_E_INVALID_ARG, "oc, s_out, score_out and winner must be host arrays");
    if (n < 1 || n > 0x7fffffffLL || ldc < n || ncand < 1 || ncand > kCandSlots) throw Failure(SPSVM_E_INVALID_ARG, "bad sizes");
    if (kdt != SPSVM_DT_F32 && kdt != SPSVM_DT_F64) throw Failure(SPSVM_E_INVALID_ARG, "unknown dtype");
    if (!(C > 0.0) || !std::isfinite(C)) throw Failure(SPSVM_E_INVALID_ARG, "C must be finite and > 0");
    if (!workspace || ((uintptr_t)workspace & 255u) || ws_bytes < score_ws(n))
      throw Failure(SPSVM_E_WORKSPACE, "workspace must be 256-byte aligned with >= spsvm_score_workspace_bytes");
    const int nblk = score_blocks(n);
    if (nblk > score_nblk_max(n)) throw Failure(SPSVM_E_WORKSPACE, "more scoring workgroups than the workspace holds");
    hipStream_t st = as_stream(stream);
    char* w = (char*)workspace;
    CandState* cs = (CandState*)w;
    w += round_up((int64_t)kCandStateBytes, 256);
    double* partial = (double*)w;
    w += round_up(score_nblk_max(n) * kCandSlots * 4 * 8, 256);
    int32_t* cand = (int32_t*)w;
    double* ocd = (double*)(w + 256);
    uint64_t* hash = (uint64_t*)(w + 768);
    uint64_t* stage_hash = (uint64_t*)(w + 1280);
    int32_t* flags = (int32_t*)(w + 1792);  // input checks (3 words)
    NewtonScalars* sc = (NewtonScalars*)(w + 2048);
    {  // labels exactly +1 or -1 (the passes take y_i o_i as o_i with its sign flipped where y_i = -1)
      SPSVM_HIP(hipMemsetAsync(flags, 0, 16, st));
      launch_check_inputs<float>(nullptr, 0, y, n, flags, st);
      int32_t f[4] = {0, 0, 0, 0};
      SPSVM_HIP(hipMemcpyAsync(f, flags, 16, hipMemcpyDeviceToHost, st));
      SPSVM_HIP(hipStreamSynchronize(st));
      if (f[1]) throw Failure(SPSVM_E_INVALID_ARG, "labels must be exactly +1 or -1");
    }
    std::vector<int32_t> ch(kCandSlots, -1);
    std::vector<double> oh(kCandSlots, 0.0);
    std::vector<uint64_t> zh(kCandSlots, 0);
    for (int c = 0; c < ncand; ++c) {
      ch[c] = c;
      oh[c] = oc[c];
    }
    SPSVM_HIP(hipMemcpyAsync(cand, ch.data(), kCandSlots * 4, hipMemcpyHostToDevice, st));
    SPSVM_HIP(hipMemcpyAsync(ocd, oh.data(), kCandSlots * 8, hipMemcpyHostToDevice, st));
    SPSVM_HIP(hipMemcpyAsync(hash, zh.data(), kCandSlots * 8, hipMemcpyHostToDevice, st));
    launch_score_init(cand, ocd, hash, stage_hash, 0, cs, sc, nullptr, st);
    const double lam = 1.0 / C;
    std::vector<CandState> host(kCandSlots);
    for (int pass = 0; pass < 64;) {
      for (int r = 0; r < 4; ++r, ++pass) {
        if (kdt == SPSVM_DT_F64)
          launch_score_pass<double>((const double*)Kc, ldc, y, o, n, cs, partial, nblk, st);
        else
          launch_score_pass<float>((const float*)Kc, ldc, y, o, n, cs, partial, nblk, st);
        launch_score_update(cs, partial, nblk, lam, nullptr, st);
      }
      SPSVM_HIP(hipMemcpyAsync(host.data(), cs, kCandSlots * sizeof(CandState), hipMemcpyDeviceToHost, st));
      SPSVM_HIP(hipStreamSynchronize(st));
      bool open = false;
      for (int c = 0; c < ncand; ++c) open |= host[c].status == 0;
      if (!open) break;
    }
    *winner = -1;
    double best = -HUGE_VAL;
    for (int c = 0; c < ncand; ++c) {
      const CandState& s = host[c];
      s_out[c] = s.s;
      score_out[c] = s.status == 1 ? s.score : -HUGE_VAL;
      if (status_out) status_out[c] = s.status;
      if (passes_out) passes_out[c] = s.passes;
      if (s.status == 1 && (*winner < 0 || s.score > best)) {
        best = s.score;
        *winner = c;
      }
    }
  });
}

spsvm_status spsvm_newton_solve_noalloc(double* H, int64_t ldh, int64_t m, const double* g, double* x, void* stream) {
  return guarded([&] {
    using spsvm::Failure;
    if (!H || !g || !x) throw Failure(SPSVM_E_INVALID_ARG, "H, g and x must be device pointers");
    if (m < 1 || m > spsvm::newton_solve_noalloc_max())
      throw Failure(SPSVM_E_INVALID_ARG, "m = " + std::to_string(m) + " is outside [1, " +
                                             std::to_string(spsvm::newton_solve_noalloc_max()) +
                                             "] (the static scratch of the allocation-free solve)");
    if (ldh < m) throw Failure(SPSVM_E_INVALID_ARG, "ldh must be >= m");
    spsvm::newton_solve_noalloc(H, ldh, (int)m, g, x, as_stream(stream));
  });
}

spsvm_status spsvm_candidate_draw(uint64_t seed, int64_t t, int64_t n, int32_t kappa, int32_t* out) {
  return guarded([&] {
    if (!out || n < 1 || n > 0x7fffffffLL || kappa < 1 || kappa > 64 || t < 0)
      throw spsvm::Failure(SPSVM_E_INVALID_ARG, "bad arguments");
    std::vector<uint64_t> hashes((size_t)n);
    for (int64_t i = 0; i < n; ++i) hashes[i] = (uint64_t)i;  // all distinct, none blocked
    spsvm::draw_step(seed, t, n, kappa, hashes, {}, out);
  });
}

}  // extern "C"
