// Shared definitions for the SP-SVM HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace spsvm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex2 __attribute__((ext_vector_type(2)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Error raised by host code inside the library; the C ABI turns it into a status code.
struct Failure : std::runtime_error {
  int status;
  Failure(int st, const std::string& msg) : std::runtime_error(msg), status(st) {}
};

#define SPSVM_HIP(expr)                                                                                 \
  do {                                                                                                  \
    hipError_t _e = (expr);                                                                             \
    if (_e != hipSuccess)                                                                               \
      throw ::spsvm::Failure(3 /*SPSVM_E_HIP*/, std::string(#expr) + " failed: " + hipGetErrorString(_e) + \
                                                    " (" + __FILE__ + ":" + std::to_string(__LINE__) + ")"); \
  } while (0)

// Checks the last launch (launch-configuration errors surface here, not at execution).
#define SPSVM_LAUNCHED() SPSVM_HIP(hipGetLastError())

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }
__device__ __forceinline__ int64_t ceil_div_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ----------------------------------------------------------------------------------------- device helpers
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ int wave_sum_int(int v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block-wide sum of a double (fixed order: waves reduce by xor-butterfly, then wave 0 sums the waves in
// index order). Every thread receives the result. scratch: at least blockDim.x / 64 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) scratch[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += scratch[i];
  __syncthreads();
  return t;
}

__device__ __forceinline__ int block_sum_int(int v, int* scratch) {
  v = wave_sum_int(v);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) scratch[w] = v;
  __syncthreads();
  int t = 0;
  for (int i = 0; i < nw; ++i) t += scratch[i];
  __syncthreads();
  return t;
}

// a_i = 1 - y_i o_i with explicit rounding (no contraction), so every kernel draws the same violator set.
__device__ __forceinline__ double margin_gap(float y, double o) { return __dadd_rn(1.0, -__dmul_rn((double)y, o)); }

// exp(-g * d2) where g2 = g * log2(e) was folded in on the host: FP32 uses the hardware 2^x instruction as is
// (no rescaling of arguments below -126, so values under 2^-126 may come out as zero).
__device__ __forceinline__ float rbf_from_d2(float d2, float g2) {
  return __builtin_amdgcn_exp2f(-g2 * fmaxf(d2, 0.0f));
}
__device__ __forceinline__ double rbf_from_d2(double d2, double g) { return exp(-g * fmax(d2, 0.0)); }

}  // namespace spsvm
