// Kernel-block engine: row norms, row hashes, and the RBF block
//   out[i, c] = exp(-gamma * max(0, |x_i|^2 + |z_c|^2 - 2 x_i . z_c))
// as an MFMA GEMM (x_i . z_c) with the exp fused into the epilogue (RBF kernel of section 2; the block
// K(X, X_J) and the candidate columns of section 4, "Sparse primal optimization"). A predict variant
// multiplies by beta and reduces over the basis in the epilogue, so the n_t x m block is never stored.
#include "common.h"
#include "launch.h"

namespace spsvm {

// ------------------------------------------------------------------------------------------ row norms
// One wave per row; squares summed in FP64 from the values the GEMM sees (cast to TK first).
template <typename TX, typename TK>
__global__ __launch_bounds__(256) void k_row_norms(const TX* __restrict__ X, int64_t n, int64_t d,
                                                   TK* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= n) return;
  const TX* x = X + row * d;
  double s = 0.0;
  for (int64_t t = lane; t < d; t += kWave) {
    const double v = (double)(TK)x[t];
    s += v * v;
  }
  s = wave_sum(s);
  if (lane == 0) out[row] = (TK)s;
}

template <typename TX, typename TK>
void launch_row_norms(const TX* X, int64_t n, int64_t d, TK* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_row_norms<TX, TK>), dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, X, n, d, out);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------------------------------ row hashes
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t value_bits(float v) { return (uint64_t)__float_as_uint(v + 0.0f); }
__device__ __forceinline__ uint64_t value_bits(double v) { return (uint64_t)__double_as_longlong(v + 0.0); }

// 64-bit hash of a row's values: sum over t of mix64(bits(x_t) ^ salt(t)), then mixed with d. Adding
// +0.0 maps -0.0 to +0.0, so rows that compare equal hash equal.
template <typename TX>
__global__ __launch_bounds__(256) void k_row_hash(const TX* __restrict__ X, int64_t n, int64_t d,
                                                  uint64_t* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= n) return;
  const TX* x = X + row * d;
  unsigned long long h = 0;
  for (int64_t t = lane; t < d; t += kWave)
    h += mix64(value_bits(x[t]) ^ ((uint64_t)(t + 1) * 0x9E3779B97F4A7C15ull));
  for (int off = 32; off > 0; off >>= 1) h += __shfl_xor(h, off, kWave);
  if (lane == 0) out[row] = mix64(h ^ (uint64_t)d);
}

template <typename TX>
void launch_row_hash(const TX* X, int64_t n, int64_t d, uint64_t* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_row_hash<TX>), dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, X, n, d, out);
  SPSVM_LAUNCHED();
}

// ---------------------------------------------------------------------------------------- MFMA wrappers
// 16x16x4 MFMA, one A and one B value per lane: lane l holds A[l % 16][k = l / 16] and B[k = l / 16][l % 16].
// Output register r of lane l holds D[row(l, r)][l % 16]; the row map differs between f32 and f64
// (measured on gfx950).
template <typename TK>
struct Mfma;
template <>
struct Mfma<float> {
  using acc_t = floatx4;
  using vec4 = floatx4;
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) * 4 + r; }
};
template <>
struct Mfma<double> {
  using acc_t = doublex4;
  using vec4 = doublex4;
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <typename TK>
__device__ __forceinline__ TK gamma_scale(double g);
template <>
__device__ __forceinline__ float gamma_scale<float>(double g) { return (float)(g * 1.4426950408889634); }
template <>
__device__ __forceinline__ double gamma_scale<double>(double g) { return g; }

// ------------------------------------------------------------------------------------ kernel-block GEMM
// Tile: 128 rows of A x 64 rows of B per workgroup (4 waves, each 32 x 64 = 2 x 4 MFMA tiles), K loop over
// the feature dimension in chunks of 32 staged through LDS with rows contiguous along k. Inside a chunk,
// lane group g = l / 16 takes k = 4g..4g+3 over four MFMA steps, so each operand fetch is one 4-wide LDS
// read; A and B use the same k assignment, so the sum runs over every k exactly once.
constexpr int KB_BM = 128, KB_BN = 64, KB_BK = 32, KB_PAD = 4, KB_LD = KB_BK + KB_PAD;

template <typename TA, typename TB, typename TK>
struct KTile {
  using M = Mfma<TK>;
  typename M::acc_t acc[2][4];

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = typename M::acc_t{0, 0, 0, 0};
  }

  // acc += A[r0 .. r0+128) . B[rows of this column tile]^T over all d features. The next chunk's global
  // loads are issued into registers before the current chunk's MFMAs, so they overlap.
  __device__ __forceinline__ void run(const TA* __restrict__ A, int64_t nA, int64_t r0, const TB* __restrict__ B,
                                      const int32_t* __restrict__ bidx, int64_t c0, int ncols, int64_t d,
                                      TK (*As)[KB_LD], TK (*Bs)[KB_LD]) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, i16 = lane & 15;
    const int kk_a = tid & 31;  // every element this thread stages sits in column kk_a of the chunk
    int64_t brow[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = (tid + e * 256) >> 5;
      const int64_t col = c0 + c;
      brow[e] = col < ncols ? (bidx ? (int64_t)bidx[col] : col) : -1;
    }
    const TA* arow[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int64_t row = r0 + ((tid + e * 256) >> 5);
      arow[e] = row < nA ? A + row * d : nullptr;
    }
    TK ra[16], rb[8];
    auto fetch = [&](int64_t k0) {
      const bool kin = k0 + kk_a < d;
#pragma unroll
      for (int e = 0; e < 16; ++e) ra[e] = (arow[e] && kin) ? (TK)arow[e][k0 + kk_a] : (TK)0;
#pragma unroll
      for (int e = 0; e < 8; ++e) rb[e] = (brow[e] >= 0 && kin) ? (TK)B[brow[e] * d + k0 + kk_a] : (TK)0;
    };
    fetch(0);
    for (int64_t k0 = 0; k0 < d; k0 += KB_BK) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 16; ++e) As[(tid + e * 256) >> 5][kk_a] = ra[e];
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[(tid + e * 256) >> 5][kk_a] = rb[e];
      __syncthreads();
      if (k0 + KB_BK < d) fetch(k0 + KB_BK);
#pragma unroll
      for (int kk = 0; kk < KB_BK; kk += 16) {
        typename M::vec4 av[2], bv[4];
#pragma unroll
        for (int i = 0; i < 2; ++i) av[i] = *(const typename M::vec4*)&As[w * 32 + i * 16 + i16][kk + 4 * g];
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = *(const typename M::vec4*)&Bs[j * 16 + i16][kk + 4 * g];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = M::step(av[i][s], bv[j][s], acc[i][j]);
      }
    }
  }
};

// STORE: out[row * ldo + c] for the column tile blockIdx.y.
template <typename TX, typename TK>
__global__ __launch_bounds__(256) void k_kblock_store(const TX* __restrict__ X, int64_t n, int64_t d,
                                                      const TK* __restrict__ xnorm, const int32_t* __restrict__ cidx,
                                                      int ncols, TK* __restrict__ out, int64_t ldo, double gamma) {
  using M = Mfma<TK>;
  __shared__ __attribute__((aligned(32))) TK As[KB_BM][KB_LD];
  __shared__ __attribute__((aligned(32))) TK Bs[KB_BN][KB_LD];
  const int64_t r0 = (int64_t)blockIdx.x * KB_BM, c0 = (int64_t)blockIdx.y * KB_BN;
  KTile<TX, TX, TK> t;
  t.zero();
  t.run(X, n, r0, X, cidx, c0, ncols, d, As, Bs);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const TK gs = gamma_scale<TK>(gamma);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = c0 + j * 16 + (lane & 15);
    if (col >= ncols) continue;
    const int64_t zi = cidx ? (int64_t)cidx[col] : col;
    if (zi < 0) continue;  // empty candidate slot
    const TK zn = xnorm[zi];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + w * 32 + i * 16 + M::row(lane, r);
        if (row < n) {
          const TK d2 = xnorm[row] + zn - (TK)2 * t.acc[i][j][r];
          out[row * ldo + col] = rbf_from_d2(d2, gs);
        }
      }
  }
}

template <typename TX, typename TK>
void launch_kblock(const TX* X, int64_t n, int64_t d, const TK* xnorm, const int32_t* cidx, int ncols, TK* out,
                   int64_t ldo, double gamma, hipStream_t st) {
  if (n <= 0 || ncols <= 0) return;
  dim3 grid((unsigned)ceil_div(n, KB_BM), (unsigned)ceil_div(ncols, KB_BN));
  hipLaunchKernelGGL((k_kblock_store<TX, TK>), grid, dim3(256), 0, st, X, n, d, xnorm, cidx, ncols, out, ldo, gamma);
  SPSVM_LAUNCHED();
}

// PREDICT: out[row] = sum_c beta[c] exp(-gamma d2(row, c)) over all m basis rows Z (m x d, type TK),
// with FP64 accumulation; row norms of Xt are computed in the kernel.
template <typename TX, typename TK>
__global__ __launch_bounds__(256) void k_kblock_predict(const TX* __restrict__ Xt, int64_t n, int64_t d,
                                                        const TK* __restrict__ Z, const TK* __restrict__ znorm, int m,
                                                        const double* __restrict__ beta, double* __restrict__ out,
                                                        double gamma) {
  using M = Mfma<TK>;
  __shared__ __attribute__((aligned(32))) TK As[KB_BM][KB_LD];
  __shared__ __attribute__((aligned(32))) TK Bs[KB_BN][KB_LD];
  __shared__ TK xn[KB_BM];
  const int64_t r0 = (int64_t)blockIdx.x * KB_BM;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int rr = 0; rr < 32; ++rr) {
    const int64_t row = r0 + w * 32 + rr;
    double s = 0.0;
    if (row < n)
      for (int64_t k = lane; k < d; k += 64) {
        const double v = (double)(TK)Xt[row * d + k];
        s += v * v;
      }
    s = wave_sum(s);
    if (lane == 0) xn[w * 32 + rr] = (TK)s;
  }
  __syncthreads();
  const TK gs = gamma_scale<TK>(gamma);
  double racc[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
  for (int64_t c0 = 0; c0 < m; c0 += KB_BN) {
    KTile<TX, TK, TK> t;
    t.zero();
    t.run(Xt, n, r0, Z, nullptr, c0, m, d, As, Bs);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = c0 + j * 16 + (lane & 15);
      if (col >= m) continue;
      const TK zn = znorm[col];
      const double b = beta[col];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int lr = w * 32 + i * 16 + M::row(lane, r);
          const TK d2 = xn[lr] + zn - (TK)2 * t.acc[i][j][r];
          racc[i][r] += b * (double)rbf_from_d2(d2, gs);
        }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = racc[i][r];
      for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, kWave);
      const int64_t row = r0 + w * 32 + i * 16 + M::row(lane, r);
      if ((lane & 15) == 0 && row < n) out[row] = v;
    }
}

template <typename TX, typename TK>
void launch_predict(const TX* Xt, int64_t n, int64_t d, const TK* Z, const TK* znorm, int m, const double* beta,
                    double* out, double gamma, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_kblock_predict<TX, TK>), dim3((unsigned)ceil_div(n, KB_BM)), dim3(256), 0, st, Xt, n, d, Z,
                     znorm, m, beta, out, gamma);
  SPSVM_LAUNCHED();
}

// ---------------------------------------------------------------------------------- gather rows X_J
template <typename TX, typename TK>
__global__ void k_gather_rows(const TX* __restrict__ X, int64_t d, const int64_t* __restrict__ idx, int64_t m,
                              TK* __restrict__ out) {
  const int64_t k = blockIdx.y;
  const int64_t src = idx[k];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < d; t += (int64_t)gridDim.x * blockDim.x)
    out[k * d + t] = (TK)X[src * d + t];
}

template <typename TX, typename TK>
void launch_gather_rows(const TX* X, int64_t d, const int64_t* idx, int64_t m, TK* out, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL((k_gather_rows<TX, TK>), dim3((unsigned)std::min<int64_t>(ceil_div(d, 256), 64), (unsigned)m),
                     dim3(256), 0, st, X, d, idx, m, out);
  SPSVM_LAUNCHED();
}

__global__ void k_iota(int32_t* out, int64_t m) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x)
    out[k] = (int32_t)k;
}

void launch_iota(int32_t* out, int64_t m, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_iota, dim3((unsigned)std::min<int64_t>(ceil_div(m, 256), 256)), dim3(256), 0, st, out, m);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------------------------- input checks
// flags[0] |= some X value is NaN or infinite; flags[1] |= some label is not exactly +1 or -1.
template <typename TX>
__global__ __launch_bounds__(256) void k_check_inputs(const TX* __restrict__ X, int64_t total, const float* __restrict__ y,
                                                      int64_t n, int32_t* __restrict__ flags) {
  int bad_x = 0, bad_y = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const double v = (double)X[i];
    bad_x |= !(v - v == 0.0);
  }
  if (y)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
      bad_y |= !(y[i] == 1.0f || y[i] == -1.0f);
  if (__any(bad_x) && (threadIdx.x & 63) == 0) atomicOr(&flags[0], 1);
  if (__any(bad_y) && (threadIdx.x & 63) == 0) atomicOr(&flags[1], 1);
}

template <typename TX>
void launch_check_inputs(const TX* X, int64_t total, const float* y, int64_t n, int32_t* flags, hipStream_t st) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(std::max(total, n), 256), 4096));
  hipLaunchKernelGGL((k_check_inputs<TX>), dim3((unsigned)blocks), dim3(256), 0, st, X, total, y, n, flags);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------------------------ instantiations
#define SPSVM_INST(TX, TK)                                                                                    \
  template void launch_row_norms<TX, TK>(const TX*, int64_t, int64_t, TK*, hipStream_t);                      \
  template void launch_kblock<TX, TK>(const TX*, int64_t, int64_t, const TK*, const int32_t*, int, TK*, int64_t, \
                                      double, hipStream_t);                                                   \
  template void launch_predict<TX, TK>(const TX*, int64_t, int64_t, const TK*, const TK*, int, const double*,   \
                                       double*, double, hipStream_t);                                         \
  template void launch_gather_rows<TX, TK>(const TX*, int64_t, const int64_t*, int64_t, TK*, hipStream_t);
SPSVM_INST(float, float)
SPSVM_INST(float, double)
SPSVM_INST(double, float)
SPSVM_INST(double, double)
#undef SPSVM_INST
template void launch_row_hash<float>(const float*, int64_t, int64_t, uint64_t*, hipStream_t);
template void launch_row_hash<double>(const double*, int64_t, int64_t, uint64_t*, hipStream_t);
template void launch_check_inputs<float>(const float*, int64_t, const float*, int64_t, int32_t*, hipStream_t);
template void launch_check_inputs<double>(const double*, int64_t, const float*, int64_t, int32_t*, hipStream_t);

}  // namespace spsvm
