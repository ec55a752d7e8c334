// Sparse (CSR) rows: the kernel block, row norms, row hashes, densified basis rows and prediction for feature
// matrices stored as compressed sparse rows, for data like KDDCup99 whose dense form is mostly zeros (section 5
// notes that the dense GPU implementation could not hold it). Row i has the values values[indptr[i] ..
// indptr[i + 1]) at the features indices[...], strictly increasing within a row; FP32 values.
#include "common.h"
#include "launch.h"

namespace spsvm {

// |x_i|^2 per row (FP64 sum of the squared FP32 values, rounded to TK), one wave per row.
template <typename TK>
__global__ __launch_bounds__(256) void k_csr_row_norms(const int64_t* __restrict__ indptr,
                                                       const float* __restrict__ values, int64_t n,
                                                       TK* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= n) return;
  double s = 0.0;
  for (int64_t k = indptr[row] + lane; k < indptr[row + 1]; k += kWave) {
    const double v = (double)(TK)values[k];
    s += v * v;
  }
  s = wave_sum(s);
  if (lane == 0) out[row] = (TK)s;
}

template <typename TK>
void launch_csr_row_norms(const int64_t* indptr, const float* values, int64_t n, TK* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_csr_row_norms<TK>), dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, indptr, values, n, out);
  SPSVM_LAUNCHED();
}
template void launch_csr_row_norms<float>(const int64_t*, const float*, int64_t, float*, hipStream_t);
template void launch_csr_row_norms<double>(const int64_t*, const float*, int64_t, double*, hipStream_t);

__device__ __forceinline__ uint64_t csr_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// 64-bit hash of a row's nonzero values and their features (an explicit zero value adds nothing, so rows that
// compare equal hash equal), mixed with d.
__global__ __launch_bounds__(256) void k_csr_row_hash(const int64_t* __restrict__ indptr,
                                                      const int32_t* __restrict__ indices,
                                                      const float* __restrict__ values, int64_t n, int64_t d,
                                                      uint64_t* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= n) return;
  unsigned long long h = 0;
  for (int64_t k = indptr[row] + lane; k < indptr[row + 1]; k += kWave) {
    const float v = values[k] + 0.0f;
    if (v != 0.0f)
      h += csr_mix64((uint64_t)__float_as_uint(v) ^ ((uint64_t)(indices[k] + 1) * 0x9E3779B97F4A7C15ull));
  }
  for (int off = 32; off > 0; off >>= 1) h += __shfl_xor(h, off, kWave);
  if (lane == 0) out[row] = csr_mix64(h ^ (uint64_t)d);
}

void launch_csr_row_hash(const int64_t* indptr, const int32_t* indices, const float* values, int64_t n, int64_t d,
                         uint64_t* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_csr_row_hash, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, indptr, indices, values, n, d,
                     out);
  SPSVM_LAUNCHED();
}

// flags[0] |= a feature index outside [0, d) or not increasing within its row.
__global__ __launch_bounds__(256) void k_csr_check(const int64_t* __restrict__ indptr,
                                                   const int32_t* __restrict__ indices, int64_t n, int64_t d,
                                                   int32_t* __restrict__ flags) {
  int bad = 0;
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n; row += (int64_t)gridDim.x * blockDim.x) {
    int64_t prev = -1;
    for (int64_t k = indptr[row]; k < indptr[row + 1]; ++k) {
      const int64_t t = indices[k];
      bad |= t <= prev || t >= d;
      prev = t;
    }
  }
  if (bad) atomicOr(flags, 1);
}

void launch_csr_check(const int64_t* indptr, const int32_t* indices, int64_t n, int64_t d, int32_t* flags,
                      hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_csr_check, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 2048)), dim3(256), 0, st, indptr,
                     indices, n, d, flags);
  SPSVM_LAUNCHED();
}

// Dense copies of rows idx[0 .. m) (out: m x ldo, zero outside the stored features; a negative index gives a
// zero row), one workgroup per row: zero fill, barrier, scatter.
template <typename TI, typename TK>
__global__ __launch_bounds__(256) void k_csr_gather(const int64_t* __restrict__ indptr,
                                                    const int32_t* __restrict__ indices,
                                                    const float* __restrict__ values, const TI* __restrict__ idx,
                                                    int64_t m, TK* __restrict__ out, int64_t ldo) {
  for (int64_t r = blockIdx.x; r < m; r += gridDim.x) {
    TK* __restrict__ dst = out + r * ldo;
    for (int64_t t = threadIdx.x; t < ldo; t += blockDim.x) dst[t] = (TK)0;
    __syncthreads();
    const int64_t src = (int64_t)idx[r];
    if (src >= 0)
      for (int64_t k = indptr[src] + threadIdx.x; k < indptr[src + 1]; k += blockDim.x) dst[indices[k]] = (TK)values[k];
    __syncthreads();
  }
}

template <typename TI, typename TK>
void launch_csr_gather(const int64_t* indptr, const int32_t* indices, const float* values, const TI* idx, int64_t m,
                       TK* out, int64_t ldo, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL((k_csr_gather<TI, TK>), dim3((unsigned)std::min<int64_t>(m, 8192)), dim3(256), 0, st, indptr,
                     indices, values, idx, m, out, ldo);
  SPSVM_LAUNCHED();
}
template void launch_csr_gather<int32_t, float>(const int64_t*, const int32_t*, const float*, const int32_t*, int64_t,
                                                float*, int64_t, hipStream_t);
template void launch_csr_gather<int64_t, float>(const int64_t*, const int32_t*, const float*, const int64_t*, int64_t,
                                                float*, int64_t, hipStream_t);
template void launch_csr_gather<int64_t, double>(const int64_t*, const int32_t*, const float*, const int64_t*,
                                                 int64_t, double*, int64_t, hipStream_t);

// Kernel block of sparse rows against up to 64 dense columns Z (ncols x ldz FP32, the candidate or basis rows made
// dense): one lane per row carries the 64 dot products x_i . z_c in FP32, walking its row's nonzeros against Z
// staged in LDS as [feature][column] over feature chunks of kCsrChunk; then d2 = |x_i|^2 + |z_c|^2 - 2 x_i . z_c
// and K = exp(-gamma d2) (the dense blocks' epilogue arithmetic). Column norms: xnorm[cidx[c]] when cidx is given
// (training rows; a negative index marks an empty slot, whose column is left untouched), else znorm[c].
//  mode 0: column-major out[c * ldo + i] (lanes write consecutive rows of a column);
//  mode 1: prediction, out_i += sum_c beta[c] K_ic in FP64 (out is FP64, added to).
constexpr int kCsrChunk = 128;  // features per LDS stage: 128 x 64 FP32 = 32 KB
__global__ __launch_bounds__(256) void k_csr_kblock(const int64_t* __restrict__ indptr,
                                                    const int32_t* __restrict__ indices,
                                                    const float* __restrict__ values, int64_t n, int64_t d,
                                                    const float* __restrict__ xnorm, const float* __restrict__ Z,
                                                    int64_t ldz, const float* __restrict__ znorm,
                                                    const int32_t* __restrict__ cidx, int ncols,
                                                    void* __restrict__ out, int64_t ldo, double gamma, int mode,
                                                    const double* __restrict__ beta) {
  __shared__ float zs[kCsrChunk][kCandSlots];
  __shared__ float zn[kCandSlots];
  __shared__ int zok[kCandSlots];
  if (threadIdx.x < kCandSlots) {
    const int c = threadIdx.x;
    const int64_t src = c < ncols ? (cidx ? (int64_t)cidx[c] : c) : -1;
    zok[c] = src >= 0;
    zn[c] = src >= 0 ? (cidx ? xnorm[src] : znorm[c]) : 0.0f;
  }
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool has = row < n;
  float acc[kCandSlots];
#pragma unroll
  for (int c = 0; c < kCandSlots; ++c) acc[c] = 0.0f;
  int64_t k = has ? indptr[row] : 0;
  const int64_t kend = has ? indptr[row + 1] : 0;
  for (int64_t t0 = 0; t0 < d; t0 += kCsrChunk) {
    __syncthreads();
    for (int e = threadIdx.x; e < kCsrChunk * kCandSlots; e += blockDim.x) {  // zs[t][c] = Z[c][t0 + t]
      const int c = e / kCsrChunk, t = e % kCsrChunk;
      zs[t][c] = (c < ncols && t0 + t < d) ? Z[(int64_t)c * ldz + t0 + t] : 0.0f;
    }
    __syncthreads();
    for (; k < kend; ++k) {  // this row's nonzeros in the chunk (features increase along the row)
      const int t = indices[k] - (int)t0;
      if (t >= kCsrChunk) break;
      const float v = values[k];
      const floatx4* zr = reinterpret_cast<const floatx4*>(&zs[t][0]);
#pragma unroll
      for (int q = 0; q < kCandSlots / 4; ++q) {
        const floatx4 z = zr[q];
        acc[4 * q] = __builtin_fmaf(v, z[0], acc[4 * q]);
        acc[4 * q + 1] = __builtin_fmaf(v, z[1], acc[4 * q + 1]);
        acc[4 * q + 2] = __builtin_fmaf(v, z[2], acc[4 * q + 2]);
        acc[4 * q + 3] = __builtin_fmaf(v, z[3], acc[4 * q + 3]);
      }
    }
  }
  if (!has) return;
  const float g2 = (float)(gamma * 1.4426950408889634), xn = xnorm[row];
  if (mode == 0) {
    float* o = (float*)out;
#pragma unroll
    for (int c = 0; c < kCandSlots; ++c)
      if (zok[c]) o[(int64_t)c * ldo + row] = rbf_from_d2(xn + zn[c] - 2.0f * acc[c], g2);
  } else {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kCandSlots; ++c)
      if (zok[c]) s += beta[c] * (double)rbf_from_d2(xn + zn[c] - 2.0f * acc[c], g2);
    ((double*)out)[row] += s;
  }
}

void launch_csr_kblock(const int64_t* indptr, const int32_t* indices, const float* values, int64_t n, int64_t d,
                       const float* xnorm, const float* Z, int64_t ldz, const float* znorm, const int32_t* cidx,
                       int ncols, void* out, int64_t ldo, double gamma, int mode, const double* beta, hipStream_t st) {
  if (n <= 0 || ncols <= 0) return;
  if (ncols > kCandSlots) throw Failure(1, "sparse kernel block: at most 64 columns per launch");
  hipLaunchKernelGGL(k_csr_kblock, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, indptr, indices, values, n, d,
                     xnorm, Z, ldz, znorm, cidx, ncols, out, ldo, gamma, mode, beta);
  SPSVM_LAUNCHED();
}

__global__ void k_add_scalar(double* out, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] += v;
}

void launch_add_scalar(double* out, int64_t n, double v, hipStream_t st) {
  if (n <= 0 || v == 0.0) return;
  hipLaunchKernelGGL(k_add_scalar, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 4096)), dim3(256), 0, st, out,
                     n, v);
  SPSVM_LAUNCHED();
}

}  // namespace spsvm
