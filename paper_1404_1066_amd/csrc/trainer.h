// Host-side orchestration of SP-SVM training (stage loop, selection steps, Newton loop).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/spsvm.h"
#include "common.h"

struct spsvm_model {
  int64_t m = 0, d = 0, ldz = 0;  // ldz: row stride of the basis copy XJ
  int tk_double = 0;  // kernel values / basis copy in FP64 (else FP32)
  double C = 1.0, gamma = 1.0, objective = 0.0;
  double bias = 0.0;  // offset b of Eq. 4 (0 unless trained with it)
  std::vector<int64_t> J;
  std::vector<double> beta;
  void* XJ = nullptr;      // device, m x d, element type FP64 or FP32 (tk_double)
  void* XJnorm = nullptr;  // device, m
  double* beta_dev = nullptr;
  spsvm_stats stats{};
  ~spsvm_model();
};

namespace spsvm {

// SplitMix64 candidate draws for addition step t (same definition as the published generator:
// state advanced by 0x9E3779B97F4A7C15, output finalised with shifts 30/27/31).
void draw_step(uint64_t seed, int64_t t, int64_t n, int kappa, const std::vector<uint64_t>& row_hash,
               const std::vector<uint64_t>& blocked_sorted, int32_t* out64);
int64_t stage_size(int64_t J, int64_t J_max, double growth, int64_t cap);

// Offsets of one problem's Newton state inside its slot region of the workspace.
struct SlotPlan {
  size_t o, delta, act0, act1, I, cblk_cnt, cblk_sum, cblk_flips, beta, dvec, g, z, H, Hf, Linv, syrk_part,
      grad_part, ls_part, vJ, wJ, F_in, F_out, fcnt_in, fcnt_out;
  size_t bytes;
};

// Problems whose Newton solves run in lockstep in a batch (one slot each).
constexpr int kBatchSlots = 64;

struct Plan {
  int64_t n = 0, d = 0, J_max = 0, ldk = 0, ldh = 0, ldx = 0, ldj = 0;
  bool pad_x = false;  // X is copied with a padded row stride (rows on 16-byte boundaries)
  bool tk_double = false;
  bool batch = false;
  int off = 0;  // 1 when the offset b is a Newton coordinate: column 0 of K_XJ is all ones, row / column 0 of K_JJ
                // zero, coefficient 0 is b, and basis vector k sits at position k + 1 of every coefficient array
  size_t bytes = 0;
  // offsets into the workspace (shared by all slots)
  size_t xnorm, hash, KXJ, Kc, J, J32, cand_state, sel, ls, scalars, score_part, cand_table, cand_cols, stage_hash,
      m_dev, flags, XJ64, xjnorm, KJJ, iota, incomplete, Xp, D, DJJ, G, Xhi, Xlo, Zc;
  bool csr = false;  // CSR rows: the candidate rows are made dense in Zc (kCandSlots x d FP32) for each block
  bool kxj_host = false;  // K_XJ lives in pinned host memory (not in the workspace; KXJ offset unused)
  int64_t ldb = 0;  // row stride of the split-BF16 copies (MIXED)
  // per-problem regions: slot q starts at slots_at + q * slot.bytes; ls and scalars hold one entry per slot
  SlotPlan slot;
  size_t slots_at = 0;
  int slots = 1;
  // one basis shared by a batch (shared_gammas > 0): per distinct gamma g >= 1 its K_XJ, K_JJ and candidate block
  // (gamma 0 uses KXJ, KJJ and Kc above), per problem its outputs o, coefficients and scoring slot states
  int shared_gammas = 0;
  int64_t problems = 1;
  size_t sh_K = 0, sh_KJJ = 0, sh_Kc = 0, sh_o = 0, sh_beta = 0, sh_cst = 0;
  size_t sh_K_stride = 0, sh_KJJ_stride = 0, sh_Kc_stride = 0, sh_o_stride = 0, sh_beta_stride = 0, sh_cst_stride = 0;
};

Plan make_plan(int64_t n, int64_t d, int64_t J_max, const spsvm_options& opt, bool with_selection,
               bool x_double, bool x_aligned, bool batch = false, int64_t problems = 1, bool csr = false,
               int shared_gammas = 0);

// Feature matrix in compressed sparse rows (device arrays; FP32 values, features increasing within a row).
struct CsrX {
  const int64_t* indptr = nullptr;  // n + 1
  const int32_t* indices = nullptr;
  const float* values = nullptr;
  int64_t nnz = 0;
};
// Greedy training (F32 kernel values) on CSR rows.
spsvm_model* run_train_csr(const CsrX& X, const float* y, int64_t n, int64_t d, double C, double gamma,
                           int64_t J_max, const spsvm_options& opt, void* ws, size_t ws_bytes, hipStream_t stream);
void run_predict_csr(const spsvm_model* model, const CsrX& Xt, int64_t n_t, double* out, hipStream_t stream);

// Runs training; returns a new model (caller owns) or throws Failure.
spsvm_model* run_train(const void* X, bool x_double, const float* y, int64_t n, int64_t d, double C, double gamma,
                       int64_t J_max, const spsvm_options& opt, void* ws, size_t ws_bytes, hipStream_t stream,
                       const int64_t* J_fixed /*nullptr = greedy selection*/);

// P Newton re-optimisations on one shared basis J (m rows): problem p has labels Y + p n, C[p], gamma[p].
// out receives P models.
void run_train_batch(const void* X, bool x_double, int64_t n, int64_t d, int64_t P, const float* Y, const double* C,
                     const double* gamma, const int64_t* J, int64_t m, const spsvm_options& opt, void* ws,
                     size_t ws_bytes, hipStream_t stream, spsvm_model** out);

// Greedy growth of one basis (up to J_max rows) shared by P problems (labels Y + p n, C[p], gamma[p]), each
// re-optimised after every stage; out receives P models on the same basis.
void run_train_shared(const void* X, bool x_double, int64_t n, int64_t d, int64_t P, const float* Y, const double* C,
                      const double* gamma, int64_t J_max, const spsvm_options& opt, void* ws, size_t ws_bytes,
                      hipStream_t stream, spsvm_model** out);
// Distinct values among gamma[0 .. P), in order of first appearance.
int distinct_gammas(const double* gamma, int64_t P);

void run_predict(const spsvm_model* model, const void* Xt, bool x_double, int64_t n_t, double* out,
                 hipStream_t stream);

// One-vs-one: K (K - 1) / 2 greedy trainings, one per class pair on its rows (gathered into the workspace).
size_t ovo_workspace_bytes(int64_t pair_rows, int64_t d, int64_t J_max, const spsvm_options& opt, bool x_double);
void run_train_ovo(const void* X, bool x_double, const int32_t* classes, int64_t n, int64_t d, int K, double C,
                   double gamma, int64_t J_max, const spsvm_options& opt, void* ws, size_t ws_bytes, hipStream_t st,
                   spsvm_model** out);
size_t ovo_predict_workspace_bytes(int64_t n_t, int K);
void run_predict_ovo(const spsvm_model* const* models, int K, const void* Xt, bool x_double, int64_t n_t,
                     int32_t* classes, void* ws, size_t ws_bytes, hipStream_t st);

}  // namespace spsvm
