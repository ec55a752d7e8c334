// Kernel-block engine: row norms, row hashes, and the RBF block
//   out[i, c] = exp(-gamma * max(0, |x_i|^2 + |z_c|^2 - 2 x_i . z_c))
// as an MFMA GEMM (x_i . z_c) with the exp fused into the epilogue (RBF kernel of section 2; the block
// K(X, X_J) and the candidate columns of section 4, "Sparse primal optimization"). A predict variant
// multiplies by beta and reduces over the basis in the epilogue, so the n_t x m block is never stored.
#include <type_traits>
#include <cstdlib>
#include <string>
#include <mutex>
#include <map>
#include <fstream>

#include "common.h"
#include "launch.h"

namespace spsvm {

// ------------------------------------------------------------------------------------------ row norms
// One wave per row; squares summed in FP64 from the values the GEMM sees (cast to TK first).
template <typename TX, typename TK>
__global__ __launch_bounds__(256) void k_row_norms(const TX* __restrict__ X, int64_t n, int64_t d, int64_t ldx,
                                                   TK* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= n) return;
  const TX* x = X + row * ldx;
  double s = 0.0;
  for (int64_t t = lane; t < d; t += kWave) {
    const double v = (double)(TK)x[t];
    s += v * v;
  }
  s = wave_sum(s);
  if (lane == 0) out[row] = (TK)s;
}

template <typename TX, typename TK>
void launch_row_norms(const TX* X, int64_t n, int64_t d, int64_t ldx, TK* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_row_norms<TX, TK>), dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, X, n, d, ldx, out);
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

// XCD-aware tile order. Workgroups are dealt to the 8 XCDs round robin (workgroup L runs on XCD L % 8), each
// XCD with its own L2. The launch is one-dimensional over ceil(R / 8) * 8 * C workgroups for R row tiles and C
// column tiles; workgroup L takes row tile 8 ((L / 8) / C) + L % 8 and column tile (L / 8) % C, so the C
// column tiles of a row tile run back to back on one XCD and read its rows of X from that XCD's L2.
constexpr int kXcds = 8;
struct TileOf {
  int64_t r, c;
};
__device__ __forceinline__ TileOf xcd_tile(int64_t ctiles) {
  const int64_t L = blockIdx.x, q = L / kXcds;
  return TileOf{(q / ctiles) * kXcds + L % kXcds, q % ctiles};
}
inline unsigned xcd_grid(int64_t rtiles, int64_t ctiles) {
  return (unsigned)(round_up(rtiles, kXcds) * ctiles);
}

// Operand rows are read with 16-byte vector loads: every row of A and B starts at a multiple of lda / ldb
// elements with lda, ldb multiples of 16 / sizeof(element) (the caller pads the feature matrix when needed),
// and elements past d in a row are ignored.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = floatx4;
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  using type = double __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};

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
  __device__ __forceinline__ void run(const TA* __restrict__ A, int64_t lda, int64_t nA, int64_t r0,
                                      const TB* __restrict__ B, int64_t ldb, const int32_t* __restrict__ bidx,
                                      int64_t c0, int ncols, int64_t d, TK (*As)[KB_LD], TK (*Bs)[KB_LD]) {
    constexpr int VA = Vec16<TA>::n, VB = Vec16<TB>::n;
    constexpr int NA = KB_BM * KB_BK / VA / 256, NB = KB_BN * KB_BK / VB / 256;  // vector loads per thread
    constexpr int PA = KB_BK / VA, PB = KB_BK / VB;                              // vectors per row chunk
    using VTA = typename Vec16<TA>::type;
    using VTB = typename Vec16<TB>::type;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, i16 = lane & 15;
    const int ka = (tid % PA) * VA, kb = (tid % PB) * VB;  // first k of this thread's vectors in a chunk
    const TA* arow[NA];
    const TB* brow[NB];
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int64_t row = r0 + (tid + e * 256) / PA;
      arow[e] = row < nA ? A + row * lda : nullptr;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int64_t col = c0 + (tid + e * 256) / PB;
      const int64_t src = col < ncols ? (bidx ? (int64_t)bidx[col] : col) : -1;
      brow[e] = src >= 0 ? B + src * ldb : nullptr;
    }
    VTA ra[NA];
    VTB rb[NB];
    auto fetch = [&](int64_t k0) {
#pragma unroll
      for (int e = 0; e < NA; ++e) ra[e] = (arow[e] && k0 + ka < d) ? *(const VTA*)(arow[e] + k0 + ka) : VTA{};
#pragma unroll
      for (int e = 0; e < NB; ++e) rb[e] = (brow[e] && k0 + kb < d) ? *(const VTB*)(brow[e] + k0 + kb) : VTB{};
    };
    fetch(0);
    for (int64_t k0 = 0; k0 < d; k0 += KB_BK) {
      __syncthreads();
      // whole vectors: a row's elements past d are zero (the rows are padded with zeros, or d is a multiple of
      // the vector width), and vectors that start past d were fetched as zeros
#pragma unroll
      for (int e = 0; e < NA; ++e) {
        const int r = (tid + e * 256) / PA;
        if constexpr (std::is_same<TA, TK>::value) {
          *(VTA*)&As[r][ka] = ra[e];
        } else {
#pragma unroll
          for (int v = 0; v < VA; ++v) As[r][ka + v] = (TK)ra[e][v];
        }
      }
#pragma unroll
      for (int e = 0; e < NB; ++e) {
        const int r = (tid + e * 256) / PB;
        if constexpr (std::is_same<TB, TK>::value) {
          *(VTB*)&Bs[r][kb] = rb[e];
        } else {
#pragma unroll
          for (int v = 0; v < VB; ++v) Bs[r][kb + v] = (TK)rb[e][v];
        }
      }
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

// Fused first scoring pass (see Score0): lane-local sums over this lane's 8 rows of each of its 4 columns,
// then over the four lane groups (xor shuffles) and the four waves (LDS, in wave order).
struct Score0Acc {
  double P[4] = {0, 0, 0, 0}, Q[4] = {0, 0, 0, 0};
  __device__ __forceinline__ void add(int j, double a, float yv, double kv) {
    if (a > 0.0) {
      const double b = (double)yv * kv;
      P[j] += a * b;
      Q[j] += b * b;
    }
  }
  // partial records for every column of the block (64 columns): waves w * wpr .. w * wpr + wpr - 1 (each
  // covering 128 / wpr rows) form record rec0 + w; records at or past nrec are not written. Records are kept
  // slot-major (all nrec records of a column together), so the per-slot reduction reads them contiguously.
  __device__ __forceinline__ void finish(double* __restrict__ partial, int64_t rec0, int64_t nrec, int wpr,
                                         double (*red)[64][2]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      P[j] += __shfl_xor(P[j], 16, kWave);
      Q[j] += __shfl_xor(Q[j], 16, kWave);
      P[j] += __shfl_xor(P[j], 32, kWave);
      Q[j] += __shfl_xor(Q[j], 32, kWave);
      if (lane < 16) {
        red[w][j * 16 + lane][0] = P[j];
        red[w][j * 16 + lane][1] = Q[j];
      }
    }
    __syncthreads();
    const int grp = threadIdx.x >> 6, c = threadIdx.x & 63;
    if (grp < 4 / wpr && rec0 + grp < nrec) {
      double p = 0.0, q = 0.0;
      for (int v = 0; v < wpr; ++v) {
        p += red[grp * wpr + v][c][0];
        q += red[grp * wpr + v][c][1];
      }
      double* out = partial + ((int64_t)c * nrec + rec0 + grp) * 4;  // slot-major: [slot][record][4]
      out[0] = p;
      out[1] = q;
      out[2] = 0.0;
      out[3] = 0.0;
    }
  }
};

// Column-major store of a BM-row x NC-column FP32 tile (NC = NT / 4 for NT threads) through LDS, tr[column][row]
// (rows padded by 4 floats, so the 16-byte accesses of 8 lanes cover all 32 banks). After a barrier that ends
// the k loop's use of the LDS operand tiles (which tr may alias), each wave puts its 4-row pieces at their place
// (row, column). flush() then gives the eight consecutive lanes of group cb = t / 8 the whole of columns cb and
// cb + NC / 2: lane t % 8 holds rows 32 q + 4 (t % 8) .. + 3 of both, and each store instruction writes
// 128-byte runs (32 rows) of eight columns, so whole lines. Columns past ncols and empty candidate slots are
// skipped.
// Fused first scoring pass (see Score0; the tile's columns 0 .. 63 when it holds the first 64 columns): rows()
// puts a_i and y_i of the tile's rows in LDS (a_i = 0 past n) before that barrier; the lanes of a group sum
// a_i b_i and b_i^2 over their rows of each such column, one record per 128 rows, then over the group (xor
// shuffles); records at or past nrec are not written, empty columns get zero records.
template <int BM, int NT = 256>
struct ColStage {
  static_assert(BM % 128 == 0 && BM <= NT, "whole fused records, one row per thread in rows()");
  static constexpr int NC = NT / 4, HC = NC / 2;  // staged columns; column offset of a group's second column
  float (*tr)[BM + 4];
  double* ga;  // [BM] in LDS
  float* gy;   // [BM] in LDS
  __device__ __forceinline__ void rows(const Score0& s0, int64_t r0, int64_t n) const {
    if (threadIdx.x < BM) {
      const int64_t row = r0 + threadIdx.x, rc = row < n ? row : n - 1;
      const float yv = s0.y[rc];
      ga[threadIdx.x] = row < n ? margin_gap(yv, s0.o[rc]) : 0.0;
      gy[threadIdx.x] = yv;
    }
  }
  __device__ __forceinline__ void put(int col, int row, const floatx4& v) const { *(floatx4*)&tr[col][row] = v; }
  __device__ __forceinline__ void flush(float* __restrict__ out, int64_t ldo, int64_t n, int64_t r0, int64_t c0,
                                        int ncols, const int32_t* __restrict__ cidx, const Score0& s0, bool fused,
                                        int64_t rec0, int64_t nrec) const {
    constexpr int NQ = BM / 32, NR = BM / 128;  // row quads per lane, fused records per column
    const int sub = threadIdx.x & 7, cb = threadIdx.x >> 3;
    bool ok[2];  // loads first: a load issued after a store waits for it
    int64_t dcol[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t col = c0 + cb + HC * h;
      ok[h] = col < ncols && (!cidx || cidx[col] >= 0);
      dcol[h] = s0.dst && col < ncols ? (int64_t)s0.dst[col] : col;
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const bool f = fused && HC * h < 64;  // slots 0 .. 63 only (uniform)
      double P[NR], Q[NR];
#pragma unroll
      for (int e = 0; e < NR; ++e) P[e] = Q[e] = 0.0;
      float* ocol = out + dcol[h] * ldo;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int rr = 32 * q + 4 * sub;
        const floatx4 x = *(const floatx4*)&tr[cb + HC * h][rr];
        if (!ok[h]) continue;
        if (f) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double av = ga[rr + r];
            if (av > 0.0) {
              const double bv = (double)gy[rr + r] * (double)x[r];
              P[q / 4] += av * bv;
              Q[q / 4] += bv * bv;
            }
          }
        }
        const int64_t row = r0 + rr;
        if (row + 3 < n) {
          *(floatx4*)(ocol + row) = x;
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (row + r < n) ocol[row + r] = x[r];
        }
      }
      if (f) {
#pragma unroll
        for (int e = 0; e < NR; ++e)
#pragma unroll
          for (int m = 1; m < 8; m <<= 1) {
            P[e] += __shfl_xor(P[e], m, kWave);
            Q[e] += __shfl_xor(Q[e], m, kWave);
          }
        if (sub == 0) {
#pragma unroll
          for (int e = 0; e < NR; ++e) {
            if (rec0 + e >= nrec) continue;
            double* rec = s0.partial + ((int64_t)(cb + HC * h) * nrec + rec0 + e) * 4;  // [slot][record][4]
            rec[0] = P[e];
            rec[1] = Q[e];
            rec[2] = 0.0;
            rec[3] = 0.0;
          }
        }
      }
    }
  }
};

// Waves per SIMD the FP32 block is compiled for: four (at most 128 registers) keeps four workgroups of the
// launch on each CU; the other type combinations take what their registers allow.
template <typename TX, typename TK>
constexpr int kStoreWaves = (std::is_same<TX, float>::value && std::is_same<TK, float>::value) ? 4 : 1;

// STORE: out[row * ldo + c] for the tile of xcd_tile().
// gamma > 0: out = exp(-gamma d2); gamma == 0: out = d2 (the squared distance itself, clamped at 0).
template <typename TX, typename TK>
__global__ __launch_bounds__(256, (kStoreWaves<TX, TK>)) void k_kblock_store(const TX* __restrict__ X, int64_t ldx, int64_t n, int64_t d,
                                                      const TK* __restrict__ xnorm, const int32_t* __restrict__ cidx,
                                                      int ncols, TK* __restrict__ out, int64_t ldo, double gamma,
                                                      const Score0 s0, int cm) {
  using M = Mfma<TK>;
  // operand tiles during the k loop; afterwards (column-major out) the tile's values as [column][row]
  constexpr int kOps = (KB_BM + KB_BN) * KB_LD * (int)sizeof(TK), kTr = KB_BN * (KB_BM + 4) * 4;
  __shared__ __attribute__((aligned(32))) char smem[kOps > kTr ? kOps : kTr];
  TK(*As)[KB_LD] = reinterpret_cast<TK(*)[KB_LD]>(smem);
  TK(*Bs)[KB_LD] = reinterpret_cast<TK(*)[KB_LD]>(smem + KB_BM * KB_LD * sizeof(TK));
  const TileOf tile = xcd_tile(ceil_div_dev(ncols, KB_BN));
  const int64_t r0 = tile.r * KB_BM, c0 = tile.c * KB_BN;
  if (r0 >= n) return;  // padding of the row-tile count to a multiple of 8
  KTile<TX, TX, TK> t;
  t.zero();
  t.run(X, ldx, n, r0, X, ldx, cidx, c0, ncols, d, As, Bs);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const TK gs = gamma_scale<TK>(gamma);
  const bool fused = s0.partial != nullptr && tile.c == 0;  // the first 64 columns only
  // FP32 values: column-major out and the fused pass go through LDS (ColStage); FP64: both from registers
  constexpr bool kStaged = std::is_same<TK, float>::value;
  const bool rfused = !kStaged && fused;
  double ga[2][4];  // a_i of this lane's rows (fused pass from registers)
  float gy[2][4];
  if (rfused) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + w * 32 + i * 16 + M::row(lane, r);
        const int64_t rc = row < n ? row : n - 1;  // clamped: unconditional loads, no branches between them
        const float yv = s0.y[rc];
        const double ov = s0.o[rc];
        gy[i][r] = row < n ? yv : 0.0f;
        ga[i][r] = row < n ? margin_gap(yv, ov) : 0.0;
      }
  }
  // every norm this lane needs, loaded before the first store (a load issued after a store waits for it)
  TK xr[2][4], zn[4];
  bool zok[4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + w * 32 + i * 16 + M::row(lane, r);
      xr[i][r] = xnorm[row < n ? row : n - 1];  // rows past n are computed but never used
    }
  int64_t zis[4], zdst[4];  // source rows and output columns of this lane's columns: index loads first, then norms
  if (cidx) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = c0 + j * 16 + (lane & 15);
      zis[j] = cidx[col < ncols ? col : ncols - 1];
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) zis[j] = c0 + j * 16 + (lane & 15);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = c0 + j * 16 + (lane & 15);
    zdst[j] = s0.dst ? (int64_t)s0.dst[col < ncols ? col : ncols - 1] : col;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = c0 + j * 16 + (lane & 15);
    const int64_t zi = col < ncols ? zis[j] : -1;
    zok[j] = zi >= 0;  // false: past the block or an empty candidate slot
    zn[j] = xnorm[zok[j] ? zi : 0];
  }
  Score0Acc sa;
  __shared__ double sga[kStaged ? KB_BM : 1];
  __shared__ float sgy[kStaged ? KB_BM : 1];
  const ColStage<KB_BM> stage{reinterpret_cast<float(*)[KB_BM + 4]>(smem), sga, sgy};
  if (kStaged && cm) {
    if (fused) stage.rows(s0, r0, n);
    __syncthreads();  // the operand tiles are free for the staging
  }
  // Per 16-row group i: all values, then their stores (every load was issued above, so no store waits on one).
  // The uniform choices (exp or plain distance, fused pass or not) are taken once, outside the element loops;
  // rows past n have a_i = 0 and add nothing to the fused sums.
  auto group = [&](int i, auto rbf_tag, auto fused_tag) {
    constexpr bool RBF = decltype(rbf_tag)::value, FUSED = decltype(fused_tag)::value;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (!zok[j]) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const TK d2 = xr[i][r] + zn[j] - (TK)2 * t.acc[i][j][r];
        const TK kv = RBF ? rbf_from_d2(d2, gs) : (d2 > (TK)0 ? d2 : (TK)0);
        t.acc[i][j][r] = kv;
        if (FUSED) sa.add(j, ga[i][r], gy[i][r], (double)kv);
      }
    }
    if (cm) {
      if constexpr (!std::is_same<TK, float>::value) {  // FP64: direct column-major stores
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (!zok[j]) continue;
          TK* ocol = out + zdst[j] * ldo;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t row = r0 + w * 32 + i * 16 + M::row(lane, r);
            if (row < n) ocol[row] = t.acc[i][j][r];
          }
        }
      } else {  // FP32: staged through LDS, each column then written in whole 128-byte runs
#pragma unroll
        for (int j = 0; j < 4; ++j) stage.put(j * 16 + (lane & 15), w * 32 + i * 16 + M::row(lane, 0), t.acc[i][j]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + w * 32 + i * 16 + M::row(lane, r);
        if (row >= n) continue;
        TK* orow = out + row * ldo + c0 + (lane & 15);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (zok[j]) orow[j * 16] = t.acc[i][j][r];
      }
    }
  };
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (gamma > 0.0) {
      if (rfused)
        group(i, std::true_type{}, std::true_type{});
      else
        group(i, std::true_type{}, std::false_type{});
    } else {
      if (rfused)
        group(i, std::false_type{}, std::true_type{});
      else
        group(i, std::false_type{}, std::false_type{});
    }
  }
  if constexpr (kStaged) {
    if (cm) stage.flush(out, ldo, n, r0, c0, ncols, cidx, s0, fused, tile.r, ceil_div_dev(n, kKblockRows));
  }
  if (rfused) {
    __shared__ double red[4][64][2];
    sa.finish(s0.partial, tile.r, ceil_div_dev(n, kKblockRows), 4, red);
  }
}

// MFMA flops a launch_kblock call issues: whole 128 x 64 tiles, k in chunks of 32.
double kblock_issued_flops(int64_t n, int64_t d, int64_t ncols) {
  if (n <= 0 || ncols <= 0) return 0.0;
  return 2.0 * (double)round_up(n, KB_BM) * (double)round_up(ncols, KB_BN) * (double)round_up(d, KB_BK);
}

template <typename TX, typename TK>
void launch_kblock(const TX* X, int64_t ldx, int64_t n, int64_t d, const TK* xnorm, const int32_t* cidx, int ncols,
                   TK* out, int64_t ldo, double gamma, hipStream_t st, const Score0& s0, bool colmajor) {
  if (n <= 0 || ncols <= 0) return;
  if (ldx % Vec16<TX>::n != 0 || ((uintptr_t)X & 15u))
    throw Failure(1, "kernel block: rows must start on 16-byte boundaries");
  const dim3 grid(xcd_grid(ceil_div(n, KB_BM), ceil_div(ncols, KB_BN)));
  if (colmajor && (ldo % 4 != 0 || ((uintptr_t)out & 15u)))
    throw Failure(1, "kernel block: column-major out needs 16-byte aligned columns");
  if ((s0.partial || s0.dst) && !colmajor)
    throw Failure(1, "kernel block: the fused scoring pass and output columns need column-major out");
  hipLaunchKernelGGL((k_kblock_store<TX, TK>), grid, dim3(256), 0, st, X, ldx, n, d, xnorm, cidx, ncols, out, ldo,
                     gamma, s0, colmajor ? 1 : 0);
  SPSVM_LAUNCHED();
}

// ---------------------------------------------------------------------- split-BF16 kernel block (MIXED)
// Every operand value is split as x = hi + lo with hi = bf16(x) and lo = bf16(x - hi) (round to nearest
// even), and x . z is taken as hi.hi' + hi.lo' + lo.hi' on the BF16 MFMA (16x16x32, FP32 accumulation); the
// dropped lo.lo' term is below 2^-16 |x||z|. Lane l of a 16x16x32 MFMA supplies A[l % 16][8 (l / 16) .. +7]
// and B[8 (l / 16) .. +7][l % 16] (measured on gfx950); the output layout is that of the FP32 16x16 MFMA.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne_bits(float x) {
  const unsigned int b = __float_as_uint(x);
  return (unsigned short)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_bits_to_float(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

constexpr int SB_BK = 32, SB_LD = SB_BK + 8;  // bf16 elements per LDS row (16-byte aligned rows)

// The split copies: hi and lo, n x ldb each (ldb = d rounded up to 32, zero padded), computed once per run.
int64_t split_ld(int64_t d) { return round_up(d, SB_BK); }

template <typename TX>
__global__ __launch_bounds__(256) void k_split_bf16(const TX* __restrict__ X, int64_t n, int64_t d, int64_t ldx,
                                                    unsigned short* __restrict__ hi, unsigned short* __restrict__ lo,
                                                    int64_t ldb) {
  const int64_t total = n * ldb;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / ldb, k = e - i * ldb;
    const double v = k < d ? (double)X[i * ldx + k] : 0.0;
    const unsigned short h = bf16_rne_bits((float)v);
    hi[e] = h;
    if (lo) lo[e] = bf16_rne_bits((float)(v - (double)bf16_bits_to_float(h)));
  }
}

template <typename TX>
void launch_split_bf16(const TX* X, int64_t n, int64_t d, int64_t ldx, unsigned short* hi, unsigned short* lo,
                       int64_t ldb, hipStream_t st) {
  if (n <= 0) return;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n * ldb, 256), 65536));
  hipLaunchKernelGGL((k_split_bf16<TX>), dim3((unsigned)blocks), dim3(256), 0, st, X, n, d, ldx, hi, lo, ldb);
  SPSVM_LAUNCHED();
}

// Split-BF16 block from the split copies: tiles of 128 rows x 64 columns, 4 waves of 32 x 64, the k loop in
// chunks of 32 staged through LDS by 16-byte copies (no conversion in the loop); the next chunk is loaded
// into registers while the current one is multiplied. SPLIT = false: every value is exactly a BF16 number,
// so lo = 0 and the correction products are exact zeros; only hi.hi' is issued (the same result bit for bit).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool SPLIT, int RTW>
__global__ __launch_bounds__(256, RTW == 4 ? 2 : 3) void k_kblock_bf16(const unsigned short* __restrict__ hi,
                                                     const unsigned short* __restrict__ lo, int64_t ldb, int64_t n,
                                                     const float* __restrict__ xnorm,
                                                     const int32_t* __restrict__ cidx, int ncols,
                                                     float* __restrict__ out, int64_t ldo, double gamma,
                                                     const Score0 s0, int cm) {
  constexpr int BM = 64 * RTW;  // rows per workgroup: 4 waves of RTW 16-row tiles
  // operand tiles during the k loop; afterwards (column-major out) the tile's values as [column][row]
  constexpr int kA = BM * SB_LD * 2, kB = KB_BN * SB_LD * 2, kOps = SPLIT ? 2 * (kA + kB) : kA + kB,
                kTr = KB_BN * (BM + 4) * 4;
  __shared__ __attribute__((aligned(16))) char smem[kOps > kTr ? kOps : kTr];
  typedef unsigned short Row[SB_LD];
  Row* Ah = reinterpret_cast<Row*>(smem);
  Row* Bh = reinterpret_cast<Row*>(smem + kA);
  Row* Al = reinterpret_cast<Row*>(smem + kA + kB);             // SPLIT only
  Row* Bl = reinterpret_cast<Row*>(smem + (SPLIT ? 2 * kA : kA) + kB);  // SPLIT only
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, i16 = lane & 15;
  const TileOf tile = xcd_tile(ceil_div_dev(ncols, KB_BN));
  const int64_t r0 = tile.r * BM, c0 = tile.c * KB_BN;
  if (r0 >= n) return;  // padding of the row-tile count to a multiple of 8
  const int part = tid & 3;  // which 8 of the chunk's 32 k this thread stages
  int64_t aoff[RTW], boff;
#pragma unroll
  for (int q = 0; q < RTW; ++q) {
    const int64_t row = r0 + ((tid + 256 * q) >> 2);
    aoff[q] = row < n ? row * ldb + 8 * part : -1;
  }
  {
    const int64_t col = c0 + (tid >> 2);
    const int64_t src = col < ncols ? (cidx ? (int64_t)cidx[col] : col) : -1;
    boff = src >= 0 ? src * ldb + 8 * part : -1;
  }
  floatx4 acc[RTW][4];
#pragma unroll
  for (int i = 0; i < RTW; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0, 0, 0, 0};
  u32x4 rah[RTW], ral[RTW], rbh, rbl;
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < RTW; ++q) {
      rah[q] = aoff[q] >= 0 ? *(const u32x4*)(hi + aoff[q] + k0) : u32x4{0, 0, 0, 0};
      if (SPLIT) ral[q] = aoff[q] >= 0 ? *(const u32x4*)(lo + aoff[q] + k0) : u32x4{0, 0, 0, 0};
    }
    rbh = boff >= 0 ? *(const u32x4*)(hi + boff + k0) : u32x4{0, 0, 0, 0};
    if (SPLIT) rbl = boff >= 0 ? *(const u32x4*)(lo + boff + k0) : u32x4{0, 0, 0, 0};
  };
  fetch(0);
  for (int64_t k0 = 0; k0 < ldb; k0 += SB_BK) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RTW; ++q) {
      const int r = (tid + 256 * q) >> 2;
      *(u32x4*)&Ah[r][8 * part] = rah[q];
      if (SPLIT) *(u32x4*)&Al[r][8 * part] = ral[q];
    }
    *(u32x4*)&Bh[tid >> 2][8 * part] = rbh;
    if (SPLIT) *(u32x4*)&Bl[tid >> 2][8 * part] = rbl;
    __syncthreads();
    if (k0 + SB_BK < ldb) fetch(k0 + SB_BK);
    bf16x8 ah[RTW], al[RTW], bh[4], bl[4];
#pragma unroll
    for (int i = 0; i < RTW; ++i) {
      ah[i] = *(const bf16x8*)&Ah[w * 16 * RTW + i * 16 + i16][8 * g];
      if (SPLIT) al[i] = *(const bf16x8*)&Al[w * 16 * RTW + i * 16 + i16][8 * g];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bh[j] = *(const bf16x8*)&Bh[j * 16 + i16][8 * g];
      if (SPLIT) bl[j] = *(const bf16x8*)&Bl[j * 16 + i16][8 * g];
    }
#pragma unroll
    for (int i = 0; i < RTW; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (SPLIT) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        }
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
  }
  const float gs = (float)(gamma * 1.4426950408889634);
  const bool fused = s0.partial != nullptr && tile.c == 0;  // the first 64 columns only (column-major out)
  // every norm this lane needs, loaded before the first store (a load issued after a store waits for it)
  float xr[RTW][4], zn[4];
  bool zok[4];
#pragma unroll
  for (int i = 0; i < RTW; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + w * 16 * RTW + i * 16 + (lane >> 4) * 4 + r;
      xr[i][r] = xnorm[row < n ? row : n - 1];  // rows past n are computed but never used
    }
  int64_t zis[4];  // source rows of this lane's columns: all index loads first, then all norm loads
  if (cidx) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = c0 + j * 16 + i16;
      zis[j] = cidx[col < ncols ? col : ncols - 1];
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) zis[j] = c0 + j * 16 + i16;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = c0 + j * 16 + i16;
    const int64_t zi = col < ncols ? zis[j] : -1;
    zok[j] = zi >= 0;
    zn[j] = xnorm[zok[j] ? zi : 0];
  }
  __shared__ double sga[BM];
  __shared__ float sgy[BM];
  const ColStage<BM> stage{reinterpret_cast<float(*)[BM + 4]>(smem), sga, sgy};
  if (cm) {
    if (fused) stage.rows(s0, r0, n);
    __syncthreads();  // the operand tiles are free for the staging
  }
  // Per 16-row group i: all values, then their stores (every load was issued above, so no store waits on one).
#pragma unroll
  for (int i = 0; i < RTW; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (!zok[j]) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float d2 = xr[i][r] + zn[j] - 2.0f * acc[i][j][r];
        const float kv = gamma > 0.0 ? rbf_from_d2(d2, gs) : fmaxf(d2, 0.0f);
        acc[i][j][r] = kv;
      }
    }
    if (cm) {  // column-major: staged through LDS, each column then written in whole 128-byte runs
#pragma unroll
      for (int j = 0; j < 4; ++j) stage.put(j * 16 + i16, w * 16 * RTW + i * 16 + g * 4, acc[i][j]);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + w * 16 * RTW + i * 16 + (lane >> 4) * 4 + r;
        if (row >= n) continue;
        float* orow = out + row * ldo + c0 + i16;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (zok[j]) orow[j * 16] = acc[i][j][r];
      }
    }
  }
  if (cm)
    stage.flush(out, ldo, n, r0, c0, ncols, cidx, s0, fused, tile.r * (BM / kKblockRows), ceil_div_dev(n, kKblockRows));
}

// Split-BF16 block in 256 x 256 tiles for blocks with many columns (grouped candidate steps, a whole basis):
// 8 waves in a 4 x 2 grid, each 64 rows x 128 columns (4 x 8 MFMA tiles). Every A fragment read from LDS feeds
// 8 tiles and every B fragment 4, and each staged byte feeds twice the products of a 256 x 64 tile; two waves
// share each SIMD. With WGC = 1 the tile is 256 x 128 (4 waves, one wave column, 68 KiB of LDS with single-pass
// products), so two workgroups share each CU and one can multiply while the other waits at a barrier or writes
// its epilogue. Two LDS stages of one k chunk each: chunk t is multiplied from one stage while chunk t + 1 goes
// from registers into the other and chunk t + 2 is loaded from memory into registers, so each chunk costs one
// barrier and a load has a whole chunk of products to arrive in. The chunk is BK = 32 wide with the split
// correction (three products per pair of fragments) and 64 wide for single-pass products, whose chunk of 32 would
// leave too few products per chunk to cover the loads. The single-pass 64-wide form orders its instructions
// explicitly (scheduling groups): each B fragment is read one group of 4 MFMAs ahead of its use, the second k step's
// fragments during the first step's last groups, and the next chunk's LDS stores and global loads (branch-free,
// out-of-range parts zeroed at the store) go between the two k steps (4% faster on the dense workload, same bits).
// The k chunks run over ldb (a multiple of 32) in order;
// a last half chunk of 32 (ldb not a multiple of 64) loads zeros for its missing half and skips its products.
// 16-byte LDS accesses are served 8 lanes at a time over 32 four-byte banks: the 16-byte part p of row r is kept
// at position p ^ ((r >> 1) & 3) in 64-byte rows (BK = 32) and p ^ (r & 7) in 128-byte rows (BK = 64), which
// makes both the staging writes and the fragment reads (8 rows at one part) conflict-free. Within a 32-wide k step
// the order of the three products and the epilogue are those of k_kblock_bf16, so both give the same bits.
template <bool SPLIT, int BK, int WGC>
__global__ __launch_bounds__(256 * WGC) __attribute__((amdgpu_waves_per_eu(2))) void k_kblock_bf16_wide(
    const unsigned short* __restrict__ hi, const unsigned short* __restrict__ lo, int64_t ldb, int64_t n,
    const float* __restrict__ xnorm, const int32_t* __restrict__ cidx, int ncols, float* __restrict__ out,
    int64_t ldo, double gamma, const Score0 s0, int cm) {
  // single-pass 64-wide chunks: branch-free loads, fragments read one group of MFMAs ahead, and the next chunk
  // staged between the two k steps (chunk64 below)
  constexpr bool OPT = !SPLIT && BK == 64;
  constexpr int NT = 256 * WGC;               // 4 x WGC waves, each 64 rows x 128 columns
  constexpr int BM = 256, BN = 128 * WGC;
  constexpr int PARTS = BK / 8;               // 16-byte parts per staged row
  constexpr int NQA = BM * PARTS / NT, NQB = BN * PARTS / NT;  // 16-byte vectors per thread per chunk
  constexpr int NC = NT / 4;                  // columns the epilogue stages through LDS at a time
  // two stages of the operand chunks during the k loop; afterwards (column-major out) NC columns of the tile at a
  // time as [column][row]
  typedef unsigned short StageA[BM][BK];
  typedef unsigned short StageB[BN][BK];
  static_assert(BK == 32 || BK == 64, "32- or 64-wide k chunks");
  static_assert(WGC == 1 || WGC == 2, "one or two wave columns");
  constexpr int kOps = (SPLIT ? 4 : 2) * (int)(sizeof(StageA) + sizeof(StageB)), kTr = NC * (BM + 4) * 4;
  __shared__ __attribute__((aligned(16))) char smem[kOps > kTr ? kOps : kTr];
  StageA* Ah = reinterpret_cast<StageA*>(smem);
  StageB* Bh = reinterpret_cast<StageB*>(smem + 2 * sizeof(StageA));
  StageA* Al = reinterpret_cast<StageA*>(smem + 2 * (sizeof(StageA) + sizeof(StageB)));  // SPLIT only
  StageB* Bl = reinterpret_cast<StageB*>(smem + 4 * sizeof(StageA) + 2 * sizeof(StageB));  // SPLIT only
  auto phys = [](int row, int p) { return BK == 32 ? p ^ ((row >> 1) & 3) : p ^ (row & 7); };
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w & 3, wc = w >> 2, g = lane >> 4,
            i16 = lane & 15;
  const TileOf tile = xcd_tile(ceil_div_dev(ncols, BN));
  const int64_t r0 = tile.r * BM, c0 = tile.c * BN;
  if (r0 >= n) return;  // padding of the row-tile count to a multiple of 8
  const int part = tid % PARTS;  // which 8 of the chunk's BK values of k this thread stages
  int64_t aoff[NQA], boff[NQB];
#pragma unroll
  for (int q = 0; q < NQA; ++q) {
    const int64_t row = r0 + (tid + NT * q) / PARTS;
    aoff[q] = row < n ? row * ldb + 8 * part : -1;
  }
#pragma unroll
  for (int q = 0; q < NQB; ++q) {
    const int64_t col = c0 + (tid + NT * q) / PARTS;
    const int64_t src = col < ncols ? (cidx ? (int64_t)cidx[col] : col) : -1;
    boff[q] = src >= 0 ? src * ldb + 8 * part : -1;
  }
  floatx4 acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = floatx4{0, 0, 0, 0};
  u32x4 rah[NQA], ral[NQA], rbh[NQB], rbl[NQB];
  auto fetch = [&](int64_t k0) {
    const bool in = k0 + 8 * part < ldb;  // a last half chunk reads zeros past ldb
    if (OPT) {  // no branches: every lane loads from a valid address; what lies outside is zeroed at the store
      const int64_t kq = in ? k0 : 0;
#pragma unroll
      for (int q = 0; q < NQA; ++q) rah[q] = *(const u32x4*)(hi + (aoff[q] >= 0 ? aoff[q] : 8 * part) + kq);
#pragma unroll
      for (int q = 0; q < NQB; ++q) rbh[q] = *(const u32x4*)(hi + (boff[q] >= 0 ? boff[q] : 8 * part) + kq);
      return;
    }
#pragma unroll
    for (int q = 0; q < NQA; ++q) {
      rah[q] = in && aoff[q] >= 0 ? *(const u32x4*)(hi + aoff[q] + k0) : u32x4{0, 0, 0, 0};
      if (SPLIT) ral[q] = in && aoff[q] >= 0 ? *(const u32x4*)(lo + aoff[q] + k0) : u32x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int q = 0; q < NQB; ++q) {
      rbh[q] = in && boff[q] >= 0 ? *(const u32x4*)(hi + boff[q] + k0) : u32x4{0, 0, 0, 0};
      if (SPLIT) rbl[q] = in && boff[q] >= 0 ? *(const u32x4*)(lo + boff[q] + k0) : u32x4{0, 0, 0, 0};
    }
  };
  auto store = [&](int b, int64_t k0) {  // k0: the chunk the registers hold (the masks of a branch-free fetch)
    if (OPT) {
      const bool in = k0 + 8 * part < ldb;
#pragma unroll
      for (int q = 0; q < NQA; ++q) {
        const int rr = (tid + NT * q) / PARTS, pp = 8 * phys(rr, part);
        *(u32x4*)&Ah[b][rr][pp] = in && aoff[q] >= 0 ? rah[q] : u32x4{0, 0, 0, 0};
      }
#pragma unroll
      for (int q = 0; q < NQB; ++q) {
        const int rr = (tid + NT * q) / PARTS, pp = 8 * phys(rr, part);
        *(u32x4*)&Bh[b][rr][pp] = in && boff[q] >= 0 ? rbh[q] : u32x4{0, 0, 0, 0};
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < NQA; ++q) {
      const int rr = (tid + NT * q) / PARTS, pp = 8 * phys(rr, part);
      *(u32x4*)&Ah[b][rr][pp] = rah[q];
      if (SPLIT) *(u32x4*)&Al[b][rr][pp] = ral[q];
    }
#pragma unroll
    for (int q = 0; q < NQB; ++q) {
      const int rr = (tid + NT * q) / PARTS, pp = 8 * phys(rr, part);
      *(u32x4*)&Bh[b][rr][pp] = rbh[q];
      if (SPLIT) *(u32x4*)&Bl[b][rr][pp] = rbl[q];
    }
  };
  auto compute_step = [&](int b, int kk) {  // one 32-wide k step of the chunk in stage b
    {
      bf16x8 ah[4], al[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int ra = wr * 64 + i * 16 + i16, pa = 8 * phys(ra, 4 * kk + g);
        ah[i] = *(const bf16x8*)&Ah[b][ra][pa];
        if (SPLIT) al[i] = *(const bf16x8*)&Al[b][ra][pa];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int rb = wc * 128 + j * 16 + i16, pb = 8 * phys(rb, 4 * kk + g);
        const bf16x8 bh = *(const bf16x8*)&Bh[b][rb][pb];
        bf16x8 bl;
        if (SPLIT) bl = *(const bf16x8*)&Bl[b][rb][pb];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (SPLIT) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
          }
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
        }
      }
    }
  };
  auto compute = [&](int b, int ksteps) {
#pragma unroll
    for (int kk = 0; kk < BK / 32; ++kk) {
      if (kk >= ksteps) break;  // uniform: the missing half of a last half chunk
      compute_step(b, kk);
    }
  };
  // Single-pass 64-wide chunk (OPT): the fragments of each group of 4 MFMAs are read one group ahead, and the second
  // k step's A fragments and first B fragment during the first step's last groups; `between` (the next chunk's
  // stores and loads) runs between the two steps. Products and their order are those of compute().
  auto afrag = [&](int b, int kk, int i) {
    const int ra = wr * 64 + i * 16 + i16, pa = 8 * phys(ra, 4 * kk + g);
    return *(const bf16x8*)&Ah[b][ra][pa];
  };
  auto bfrag2 = [&](int b, int kk, int j) {
    const int rb = wc * 128 + j * 16 + i16, pb = 8 * phys(rb, 4 * kk + g);
    return *(const bf16x8*)&Bh[b][rb][pb];
  };
  auto chunk64 = [&](int b, bool two, auto&& between) {
    bf16x8 a0[4], a1[4], bcur, b1;
#pragma unroll
    for (int i = 0; i < 4; ++i) a0[i] = afrag(b, 0, i);
    bcur = bfrag2(b, 0, 0);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      bf16x8 bnext = bcur;
      if (j < 7) bnext = bfrag2(b, 0, j + 1);
      // read whether or not the second step runs (a last half chunk's second half holds zeros): no branch
      if (j >= 4) a1[j - 4] = afrag(b, 1, j - 4);
      if (j == 7) b1 = bfrag2(b, 1, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0[i], bcur, acc[i][j], 0, 0, 0);
      bcur = bnext;
    }
    __builtin_amdgcn_sched_group_barrier(0x100, 5, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
    }
#pragma unroll
    for (int j = 4; j < 7; ++j) {
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
    between();
    if (!two) return;
    bcur = b1;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      bf16x8 bnext = bcur;
      if (j < 7) bnext = bfrag2(b, 1, j + 1);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[i], bcur, acc[i][j], 0, 0, 0);
      bcur = bnext;
    }
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
  };
  const int nk32 = (int)(ldb / 32);               // 32-wide k steps
  const int nk = (nk32 * 32 + BK - 1) / BK;        // chunks
  auto steps_of = [&](int t) { return nk32 - t * (BK / 32) < BK / 32 ? nk32 - t * (BK / 32) : BK / 32; };
  fetch(0);
  store(0, 0);
  if (nk > 1) fetch(BK);
  __syncthreads();
  for (int t = 0; t < nk; ++t) {
    if constexpr (OPT) {
      // the next chunk's stores and the loads of the one after go between the two 32-wide k steps, so the
      // MFMAs of the second step cover them and only the barrier separates two chunks' products
      chunk64(t & 1, steps_of(t) > 1, [&] {
        if (t + 1 < nk) {
          store((t + 1) & 1, (int64_t)(t + 1) * BK);
          if (t + 2 < nk) fetch((int64_t)(t + 2) * BK);
        }
      });
    } else {
      compute(t & 1, steps_of(t));
      // the other stage was last read for chunk t - 1, which every wave finished before the previous barrier
      if (t + 1 < nk) {
        store((t + 1) & 1, (int64_t)(t + 1) * BK);
        if (t + 2 < nk) fetch((int64_t)(t + 2) * BK);
      }
    }
    __syncthreads();
  }
  const float gs = (float)(gamma * 1.4426950408889634);
  // the fused first scoring pass covers the block's first 64 columns (column-major out)
  const bool fused = s0.partial != nullptr && tile.c == 0;
  // every norm this lane needs, loaded before the first store (a load issued after a store waits for it)
  float xr[4][4], zn[8];
  bool zok[8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + wr * 64 + i * 16 + g * 4 + r;
      xr[i][r] = xnorm[row < n ? row : n - 1];  // rows past n are computed but never used
    }
  int64_t zis[8];  // source rows of this lane's columns: all index loads first, then all norm loads
  if (cidx) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t col = c0 + wc * 128 + j * 16 + i16;
      zis[j] = cidx[col < ncols ? col : ncols - 1];
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) zis[j] = c0 + wc * 128 + j * 16 + i16;
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t col = c0 + wc * 128 + j * 16 + i16;
    const int64_t zi = col < ncols ? zis[j] : -1;
    zok[j] = zi >= 0;
    zn[j] = xnorm[zok[j] ? zi : 0];
  }
  // Per 16-row group i: all values, then (row-major out) their stores; every load was issued above.
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (!zok[j]) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float d2 = xr[i][r] + zn[j] - 2.0f * acc[i][j][r];
        acc[i][j][r] = gamma > 0.0 ? rbf_from_d2(d2, gs) : fmaxf(d2, 0.0f);
      }
    }
    if (!cm) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + wr * 64 + i * 16 + g * 4 + r;
        if (row >= n) continue;
        float* orow = out + row * ldo + c0 + wc * 128 + i16;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (zok[j]) orow[j * 16] = acc[i][j][r];
      }
    }
  }
  if (cm) {  // through LDS, NC columns at a time (128: one wave column; 64: half of the single wave column)
    __shared__ double sga[BM];
    __shared__ float sgy[BM];
    const ColStage<BM, NT> stage{reinterpret_cast<float(*)[BM + 4]>(smem), sga, sgy};
    if (fused) stage.rows(s0, r0, n);
#pragma unroll
    for (int h = 0; h < BN / NC; ++h) {
      __syncthreads();  // h = 0: the operand stages are dead; then: the previous columns have been read back
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int col = wc * 128 + j * 16;  // this fragment's first column in the tile
        if (col >= h * NC && col < (h + 1) * NC)
#pragma unroll
          for (int i = 0; i < 4; ++i) stage.put(col - h * NC + i16, wr * 64 + i * 16 + g * 4, acc[i][j]);
      }
      stage.flush(out, ldo, n, r0, c0 + NC * h, ncols, cidx, s0, fused && h == 0, tile.r * (BM / kKblockRows),
                  ceil_div_dev(n, kKblockRows));
    }
  }
}

// Tiles of 256 rows (each wave 64 x 64: more MFMAs per LDS fragment) once the matrix has enough of them to
// fill the chip and rows are long enough for the k loop to dominate; 128 rows otherwise.
constexpr int64_t kWideRows = 65536;
// 256 x 256 tiles from this many columns on (and enough tiles to fill the chip)
constexpr int64_t kWideCols = 192;

// ---------------------------------------------------------------------- variants and their autotuner
// The split-BF16 / single-pass block has five kernel variants, all of which give the same bits (the same k
// chunks of 32 in the same order per output, the same epilogue arithmetic and fused records): 128 x 64 and
// 256 x 64 tiles of k_kblock_bf16, the 256 x 256 tiles of k_kblock_bf16_wide with 32- or 64-wide k chunks in
// LDS (the split instance always uses 32), and its 256 x 128 tiles (single pass only). Without tuning the choice
// is fixed by the shape; with the environment variable SPSVM_AUTOTUNE=1 every variant is timed with HIP events on
// the caller's stream the first time a shape class is met (one warm and two timed launches each, writing the same
// output), and the fastest is kept. Shape classes: split or single pass, column-major or not, fused first pass or
// not, n rounded up to a power of two, ldb, and the column count. With SPSVM_TUNE_CACHE=<file> the choices are
// read from and appended to that JSON file. SPSVM_KBLOCK_VARIANT=<name> forces one variant wherever it applies
// (for tests and measurements; it takes precedence over the cache and the timing).
enum KbVariant { kVRows128 = 0, kVRows256 = 1, kVWide = 2, kVWideK32 = 3, kVWideHalf = 4 };
constexpr int kVariants = 5;
static const char* const kVariantName[] = {"rows128", "rows256", "wide", "wide_k32", "wide_half"};
static bool single_pass_only(int v) { return v == kVWideK32 || v == kVWideHalf; }

static int heuristic_variant(int64_t n, int64_t ldb, int64_t ncols) {
  if (ncols >= kWideCols && ceil_div(n, 256) * ceil_div(ncols, 256) >= 256) return kVWide;
  return n >= kWideRows && ldb >= 256 ? kVRows256 : kVRows128;  // short rows: 128-row tiles keep more waves resident
}

static void launch_variant(int v, const unsigned short* hi, const unsigned short* lo, int64_t ldb, int64_t n,
                           const float* xnorm, const int32_t* cidx, int ncols, float* out, int64_t ldo, double gamma,
                           hipStream_t st, const Score0& s0, int cm) {
  if (v == kVWideHalf && !lo) {  // 256 x 128 tiles, 4 waves: two workgroups share a CU (single pass only: the
                                 // split form's operand stages would not leave LDS for a second workgroup)
    const dim3 grid(xcd_grid(ceil_div(n, 256), ceil_div(ncols, 128)));
    hipLaunchKernelGGL((k_kblock_bf16_wide<false, 32, 1>), grid, dim3(256), 0, st, hi, lo, ldb, n, xnorm, cidx, ncols,
                       out, ldo, gamma, s0, cm);
  } else if (v == kVWide || v == kVWideK32) {
    const dim3 grid(xcd_grid(ceil_div(n, 256), ceil_div(ncols, 256)));
    if (lo)
      hipLaunchKernelGGL((k_kblock_bf16_wide<true, 32, 2>), grid, dim3(512), 0, st, hi, lo, ldb, n, xnorm, cidx,
                         ncols, out, ldo, gamma, s0, cm);
    else if (v == kVWide)
      hipLaunchKernelGGL((k_kblock_bf16_wide<false, 64, 2>), grid, dim3(512), 0, st, hi, lo, ldb, n, xnorm, cidx,
                         ncols, out, ldo, gamma, s0, cm);
    else
      hipLaunchKernelGGL((k_kblock_bf16_wide<false, 32, 2>), grid, dim3(512), 0, st, hi, lo, ldb, n, xnorm, cidx,
                         ncols, out, ldo, gamma, s0, cm);
  } else {
    const bool rows256 = v == kVRows256;
    const dim3 grid(xcd_grid(ceil_div(n, rows256 ? 256 : 128), ceil_div(ncols, KB_BN)));
    if (rows256) {
      if (lo)
        hipLaunchKernelGGL((k_kblock_bf16<true, 4>), grid, dim3(256), 0, st, hi, lo, ldb, n, xnorm, cidx, ncols, out,
                           ldo, gamma, s0, cm);
      else
        hipLaunchKernelGGL((k_kblock_bf16<false, 4>), grid, dim3(256), 0, st, hi, lo, ldb, n, xnorm, cidx, ncols, out,
                           ldo, gamma, s0, cm);
    } else {
      if (lo)
        hipLaunchKernelGGL((k_kblock_bf16<true, 2>), grid, dim3(256), 0, st, hi, lo, ldb, n, xnorm, cidx, ncols, out,
                           ldo, gamma, s0, cm);
      else
        hipLaunchKernelGGL((k_kblock_bf16<false, 2>), grid, dim3(256), 0, st, hi, lo, ldb, n, xnorm, cidx, ncols, out,
                           ldo, gamma, s0, cm);
    }
  }
  SPSVM_LAUNCHED();
}

namespace {
struct Tuner {
  std::mutex mu;
  bool init = false, tune = false;
  std::string path;
  std::map<std::string, int> choice;
  int force = -1;

  static std::string key(bool split, int cm, bool fused, int64_t n, int64_t ldb, int64_t ncols) {
    int lg = 0;
    while ((int64_t(1) << lg) < n) ++lg;
    return "split=" + std::to_string(split ? 1 : 0) + " cm=" + std::to_string(cm) + " fused=" +
           std::to_string(fused ? 1 : 0) + " n<=2^" + std::to_string(lg) + " ldb=" + std::to_string(ldb) +
           " ncols=" + std::to_string(ncols);
  }
  void setup() {  // mu held
    if (init) return;
    init = true;
    const char* t = std::getenv("SPSVM_AUTOTUNE");
    tune = t && t[0] == '1';
    const char* fv = std::getenv("SPSVM_KBLOCK_VARIANT");
    for (int i = 0; fv && i < kVariants; ++i)
      if (std::string(fv) == kVariantName[i]) force = i;
    const char* f = std::getenv("SPSVM_TUNE_CACHE");
    if (!f || !f[0]) return;
    path = f;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {  // one entry per line: {"key": "...", "variant": "...", ...}
      const size_t k0 = line.find("\"key\": \""), v0 = line.find("\"variant\": \"");
      if (k0 == std::string::npos || v0 == std::string::npos) continue;
      const size_t k1 = line.find('"', k0 + 8), v1 = line.find('"', v0 + 12);
      if (k1 == std::string::npos || v1 == std::string::npos) continue;
      const std::string k = line.substr(k0 + 8, k1 - k0 - 8), v = line.substr(v0 + 12, v1 - v0 - 12);
      const bool split = k.compare(0, 8, "split=1 ") == 0;
      for (int i = 0; i < kVariants; ++i)  // a split shape takes no single-pass-only form
        if (v == kVariantName[i] && !(split && single_pass_only(i))) choice[k] = i;
    }
  }
  int forced(bool split) const {  // mu held; the forced variant if it applies to this instance, else -1
    return force >= 0 && !(split && single_pass_only(force)) ? force : -1;
  }
  void save(const std::string& k, int v, const float* us) {  // mu held
    if (path.empty()) return;
    std::ofstream o(path, std::ios::app);
    o << "{\"key\": \"" << k << "\", \"variant\": \"" << kVariantName[v] << "\", \"us\": {";
    for (int i = 0; i < kVariants; ++i) o << (i ? ", " : "") << "\"" << kVariantName[i] << "\": " << us[i];
    o << "}}\n";
  }
};
Tuner g_tuner;
}  // namespace

// The variant a call of this shape uses (a tuned choice when there is one, else the shape heuristic).
static int chosen_variant(bool split, int cm, bool fused, int64_t n, int64_t ldb, int64_t ncols) {
  std::lock_guard<std::mutex> lock(g_tuner.mu);
  g_tuner.setup();
  if (g_tuner.forced(split) >= 0) return g_tuner.force;
  const auto it = g_tuner.choice.find(Tuner::key(split, cm, fused, n, ldb, ncols));
  return it != g_tuner.choice.end() ? it->second : heuristic_variant(n, ldb, ncols);
}

int kblock_bf16_variant(int64_t n, int64_t ldb, int64_t ncols, bool split, bool candidates) {
  return chosen_variant(split, candidates ? 1 : 0, candidates, n, ldb, ncols);
}

// MFMA flops a launch_kblock_bf16 call issues: whole tiles of the variant it uses, k over ldb, three products per
// multiply-add with the split correction (one without).
double kblock_bf16_issued_flops(int64_t n, int64_t ldb, int64_t ncols, bool split, bool candidates) {
  if (n <= 0 || ncols <= 0) return 0.0;
  // candidate blocks are column-major with the fused first pass; basis blocks row-major without it
  const int v = chosen_variant(split, candidates ? 1 : 0, candidates, n, ldb, ncols);
  const int64_t bm = v == kVRows128 ? 128 : 256, bn = v == kVWideHalf ? 128 : (v >= kVWide ? 256 : KB_BN);
  return 2.0 * (double)round_up(n, bm) * (double)round_up(ncols, bn) * (double)ldb * (split ? 3.0 : 1.0);
}

void launch_kblock_bf16(const unsigned short* hi, const unsigned short* lo, int64_t ldb, int64_t n,
                        const float* xnorm, const int32_t* cidx, int ncols, float* out, int64_t ldo, double gamma,
                        hipStream_t st, const Score0& s0, bool colmajor) {
  if (n <= 0 || ncols <= 0) return;
  if (colmajor && (ldo % 4 != 0 || ((uintptr_t)out & 15u)))
    throw Failure(1, "kernel block: column-major out needs 16-byte aligned columns");
  if ((s0.partial || s0.dst) && !colmajor)
    throw Failure(1, "kernel block: the fused scoring pass and output columns need column-major out");
  const int cm = colmajor ? 1 : 0;
  if (ldb % SB_BK != 0 || ((uintptr_t)hi & 15u) || ((uintptr_t)lo & 15u))
    throw Failure(1, "kernel block: split copies must be 16-byte aligned with ldb a multiple of 32");
  const bool split = lo != nullptr, fused = s0.partial != nullptr;
  int v;
  {
    std::lock_guard<std::mutex> lock(g_tuner.mu);
    g_tuner.setup();
    const std::string k = Tuner::key(split, cm, fused, n, ldb, ncols);
    const auto it = g_tuner.choice.find(k);
    if (g_tuner.forced(split) >= 0) {
      v = g_tuner.force;
    } else if (it != g_tuner.choice.end()) {
      v = it->second;
    } else if (!g_tuner.tune) {
      v = heuristic_variant(n, ldb, ncols);
    } else {  // time every variant once on this shape (each writes the same output)
      float us[kVariants] = {-1.f, -1.f, -1.f, -1.f, -1.f};
      hipEvent_t a, b;
      SPSVM_HIP(hipEventCreate(&a));
      SPSVM_HIP(hipEventCreate(&b));
      v = heuristic_variant(n, ldb, ncols);
      float best = 0.f;
      for (int c = 0; c < kVariants; ++c) {
        if (split && single_pass_only(c)) continue;  // single-pass forms only
        launch_variant(c, hi, lo, ldb, n, xnorm, cidx, ncols, out, ldo, gamma, st, s0, cm);
        SPSVM_HIP(hipEventRecord(a, st));
        for (int r = 0; r < 2; ++r) launch_variant(c, hi, lo, ldb, n, xnorm, cidx, ncols, out, ldo, gamma, st, s0, cm);
        SPSVM_HIP(hipEventRecord(b, st));
        SPSVM_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        SPSVM_HIP(hipEventElapsedTime(&ms, a, b));
        us[c] = 500.f * ms;
        if (best == 0.f || us[c] < best) {
          best = us[c];
          v = c;
        }
      }
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      g_tuner.choice[k] = v;
      g_tuner.save(k, v, us);
      return;  // the output is written (every variant wrote it)
    }
  }
  launch_variant(v, hi, lo, ldb, n, xnorm, cidx, ncols, out, ldo, gamma, st, s0, cm);
}

// PREDICT: out[row] = sum_c beta[c] exp(-gamma d2(row, c)) over all m basis rows Z (m x d, type TK),
// with FP64 accumulation; row norms of Xt are computed in the kernel.
template <typename TX, typename TK>
__global__ __launch_bounds__(256) void k_kblock_predict(const TX* __restrict__ Xt, int64_t ldxt, int64_t n, int64_t d,
                                                        const TK* __restrict__ Z, int64_t ldz,
                                                        const TK* __restrict__ znorm, int m,
                                                        const double* __restrict__ beta, double* __restrict__ out,
                                                        double gamma, double bias) {
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
        const double v = (double)(TK)Xt[row * ldxt + k];
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
    t.run(Xt, ldxt, n, r0, Z, ldz, nullptr, c0, m, d, As, Bs);
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
      if ((lane & 15) == 0 && row < n) out[row] = v + bias;
    }
}

template <typename TX, typename TK>
void launch_predict(const TX* Xt, int64_t ldxt, int64_t n, int64_t d, const TK* Z, int64_t ldz, const TK* znorm, int m,
                    const double* beta, double* out, double gamma, double bias, hipStream_t st) {
  if (n <= 0) return;
  if (ldxt % Vec16<TX>::n != 0 || ((uintptr_t)Xt & 15u) || ldz % Vec16<TK>::n != 0 || ((uintptr_t)Z & 15u))
    throw Failure(1, "predict: rows must start on 16-byte boundaries");
  hipLaunchKernelGGL((k_kblock_predict<TX, TK>), dim3((unsigned)ceil_div(n, KB_BM)), dim3(256), 0, st, Xt, ldxt, n, d,
                     Z, ldz, znorm, m, beta, out, gamma, bias);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------------------- K = exp(-gamma D)
// Applies the RBF map to a block of squared distances (rows of ncols values, leading dimension ld), with the
// same arithmetic as the fused epilogue of the kernel-block GEMM.
template <typename TK>
__global__ __launch_bounds__(256) void k_rbf_from_dist(const TK* __restrict__ D, int64_t rows, int ncols, int64_t ld,
                                                       TK* __restrict__ K, double gamma) {
  const TK gs = gamma_scale<TK>(gamma);
  const int64_t total = rows * ncols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ncols, c = e - r * ncols;
    K[r * ld + c] = rbf_from_d2(D[r * ld + c], gs);
  }
}

template <typename TK>
void launch_rbf_from_dist(const TK* D, int64_t rows, int ncols, int64_t ld, TK* K, double gamma, hipStream_t st) {
  if (rows <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL((k_rbf_from_dist<TK>), dim3((unsigned)std::min<int64_t>(ceil_div(rows * ncols, 256), 65536)),
                     dim3(256), 0, st, D, rows, ncols, ld, K, gamma);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------------------------- padded copies
// out (n x ldo) = X (n x d) with zero padding, so that every row starts on a 16-byte boundary.
template <typename TX>
__global__ void k_pad_rows(const TX* __restrict__ X, int64_t n, int64_t d, TX* __restrict__ out, int64_t ldo) {
  const int64_t total = n * ldo;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ldo, c = e - r * ldo;
    out[e] = c < d ? X[r * d + c] : (TX)0;
  }
}

template <typename TX>
void launch_pad_rows(const TX* X, int64_t n, int64_t d, TX* out, int64_t ldo, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_pad_rows<TX>), dim3((unsigned)std::min<int64_t>(ceil_div(n * ldo, 256), 65536)), dim3(256), 0,
                     st, X, n, d, out, ldo);
  SPSVM_LAUNCHED();
}

// ---------------------------------------------------------------------------------- gather rows X_J
// out[k, :] = X[idx[k], :] converted to TK, rows of out with stride ldo (the padding is zeroed).
template <typename TX, typename TK>
__global__ void k_gather_rows(const TX* __restrict__ X, int64_t d, const int64_t* __restrict__ idx, int64_t m,
                              TK* __restrict__ out, int64_t ldo) {
  const int64_t k = blockIdx.y;
  const int64_t src = idx[k];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ldo; t += (int64_t)gridDim.x * blockDim.x)
    out[k * ldo + t] = t < d ? (TK)X[src * d + t] : (TK)0;
}

template <typename TX, typename TK>
void launch_gather_rows(const TX* X, int64_t d, const int64_t* idx, int64_t m, TK* out, int64_t ldo, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL((k_gather_rows<TX, TK>), dim3((unsigned)std::min<int64_t>(ceil_div(ldo, 256), 64), (unsigned)m),
                     dim3(256), 0, st, X, d, idx, m, out, ldo);
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

// K[i * ld + col] = v for every row i (the all-ones column of the offset b).
template <typename TK>
__global__ void k_fill_column(TK* K, int64_t rows, int64_t ld, int64_t col, TK v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x)
    K[i * ld + col] = v;
}

template <typename TK>
void launch_fill_column(TK* K, int64_t rows, int64_t ld, int64_t col, double v, hipStream_t st) {
  if (rows <= 0) return;
  hipLaunchKernelGGL((k_fill_column<TK>), dim3((unsigned)std::min<int64_t>(ceil_div(rows, 256), 4096)), dim3(256), 0,
                     st, K, rows, ld, col, (TK)v);
  SPSVM_LAUNCHED();
}
template void launch_fill_column<float>(float*, int64_t, int64_t, int64_t, double, hipStream_t);
template void launch_fill_column<double>(double*, int64_t, int64_t, int64_t, double, hipStream_t);

// ------------------------------------------------------------------------------------- input checks
// flags[0] |= some X value is NaN or infinite; flags[1] |= some label is not exactly +1 or -1;
// flags[2] |= some X value is not exactly a BF16 number (then the split-BF16 lo parts are not all zero).
template <typename TX>
__global__ __launch_bounds__(256) void k_check_inputs(const TX* __restrict__ X, int64_t total, const float* __restrict__ y,
                                                      int64_t n, int32_t* __restrict__ flags) {
  int bad_x = 0, bad_y = 0, inexact = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const double v = (double)X[i];
    bad_x |= !(v - v == 0.0);
    inexact |= (double)bf16_bits_to_float(bf16_rne_bits((float)v)) != v;
  }
  if (y)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
      bad_y |= !(y[i] == 1.0f || y[i] == -1.0f);
  if (__any(bad_x) && (threadIdx.x & 63) == 0) atomicOr(&flags[0], 1);
  if (__any(bad_y) && (threadIdx.x & 63) == 0) atomicOr(&flags[1], 1);
  if (__any(inexact) && (threadIdx.x & 63) == 0) atomicOr(&flags[2], 1);
}

template <typename TX>
void launch_check_inputs(const TX* X, int64_t total, const float* y, int64_t n, int32_t* flags, hipStream_t st) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(std::max(total, n), 256), 4096));
  hipLaunchKernelGGL((k_check_inputs<TX>), dim3((unsigned)blocks), dim3(256), 0, st, X, total, y, n, flags);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------------------------ instantiations
#define SPSVM_INST(TX, TK)                                                                                    \
  template void launch_row_norms<TX, TK>(const TX*, int64_t, int64_t, int64_t, TK*, hipStream_t);             \
  template void launch_kblock<TX, TK>(const TX*, int64_t, int64_t, int64_t, const TK*, const int32_t*, int, TK*, \
                                      int64_t, double, hipStream_t, const Score0&, bool);                                    \
  template void launch_predict<TX, TK>(const TX*, int64_t, int64_t, int64_t, const TK*, int64_t, const TK*, int,  \
                                       const double*, double*, double, double, hipStream_t);                          \
  template void launch_gather_rows<TX, TK>(const TX*, int64_t, const int64_t*, int64_t, TK*, int64_t, hipStream_t);
SPSVM_INST(float, float)
SPSVM_INST(float, double)
SPSVM_INST(double, float)
SPSVM_INST(double, double)
#undef SPSVM_INST
template void launch_row_hash<float>(const float*, int64_t, int64_t, uint64_t*, hipStream_t);
template void launch_row_hash<double>(const double*, int64_t, int64_t, uint64_t*, hipStream_t);
template void launch_split_bf16<float>(const float*, int64_t, int64_t, int64_t, unsigned short*, unsigned short*,
                                       int64_t, hipStream_t);
template void launch_split_bf16<double>(const double*, int64_t, int64_t, int64_t, unsigned short*, unsigned short*,
                                        int64_t, hipStream_t);
template void launch_rbf_from_dist<float>(const float*, int64_t, int, int64_t, float*, double, hipStream_t);
template void launch_rbf_from_dist<double>(const double*, int64_t, int, int64_t, double*, double, hipStream_t);
template void launch_pad_rows<float>(const float*, int64_t, int64_t, float*, int64_t, hipStream_t);
template void launch_pad_rows<double>(const double*, int64_t, int64_t, double*, int64_t, hipStream_t);
template void launch_check_inputs<float>(const float*, int64_t, const float*, int64_t, int32_t*, hipStream_t);
template void launch_check_inputs<double>(const double*, int64_t, const float*, int64_t, int32_t*, hipStream_t);

}  // namespace spsvm
