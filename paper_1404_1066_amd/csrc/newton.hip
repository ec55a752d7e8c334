// Newton re-optimisation of Eq. 4 on a fixed basis J (section 4, "Sparse primal optimization"; Newton's
// method on the squared-hinge primal of section 4, "Primal optimization"):
//   f(beta) = lambda/2 beta^T K_JJ beta + 1/2 sum_i max(0, a_i)^2,  a_i = 1 - y_i o_i,  o = K_XJ beta,
//   grad f  = lambda K_JJ beta + K_I^T (o_I - y_I),     H = lambda K_JJ + K_I^T K_I,   I = {i : a_i > 0}.
// K_JJ is kept as its own FP64 matrix (computed from the basis rows), so the regulariser stays positive
// definite whatever precision the n x |J| block K_XJ is stored in.
// Kernels: GEMV o = K_XJ x (one wave per 4 rows), violator compaction (wave ballot + block prefix sums),
// gradient (GEMV^T over the compacted rows), the SYRK of H over the compacted rows with MFMA, and the
// exact line search along d (bracketed semismooth Newton on the piecewise-linear derivative).
// All reductions run in a fixed order, so results are bitwise reproducible.
#include "common.h"
#include "launch.h"

namespace spsvm {

// ------------------------------------------------------------------------------------------------ GEMV
// Each wave takes 4 consecutive rows; lane l reads the 4 values j = 4 l + 256 u .. + 3 of every row (one 16-byte
// load per row for FP32, 32 bytes for FP64) and the matching 4 values of x once for all 4 rows, two chunks in flight.
// Row rows start on 16-byte (FP32) / 32-byte (FP64) boundaries: ld is a multiple of 4 and K, x are aligned. A
// lane's products are added in column order, then the wave's 64 partial sums by xor butterfly.
template <typename TK>
struct Vec4Of;
template <>
struct Vec4Of<float> {
  typedef floatx4 T;
};
template <>
struct Vec4Of<double> {
  typedef doublex4 T;
};

constexpr int kGemvRows = 4;  // rows per wave

template <typename TK>
__global__ __launch_bounds__(256) void k_gemv(const TK* __restrict__ K, int64_t ldk, int64_t n, int m,
                                              const double* __restrict__ x, double* __restrict__ out) {
  typedef typename Vec4Of<TK>::T V;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + threadIdx.x / kWave) * kGemvRows;
  if (r0 >= n) return;
  const TK* rp[kGemvRows];
#pragma unroll
  for (int r = 0; r < kGemvRows; ++r) rp[r] = K + (r0 + r < n ? r0 + r : r0) * ldk;
  double s[kGemvRows] = {0.0, 0.0, 0.0, 0.0};
  const int m4 = m & ~3;
  auto add = [&](const doublex4& xv, const V* kv) {
#pragma unroll
    for (int r = 0; r < kGemvRows; ++r)
#pragma unroll
      for (int e = 0; e < 4; ++e) s[r] += (double)kv[r][e] * xv[e];
  };
  int j = 4 * lane;
  for (; j + 4 * kWave < m4; j += 8 * kWave) {  // two chunks of 256 columns: all loads first
    const doublex4 x0 = *(const doublex4*)(x + j), x1 = *(const doublex4*)(x + j + 4 * kWave);
    V k0[kGemvRows], k1[kGemvRows];
#pragma unroll
    for (int r = 0; r < kGemvRows; ++r) {
      k0[r] = *(const V*)(rp[r] + j);
      k1[r] = *(const V*)(rp[r] + j + 4 * kWave);
    }
    add(x0, k0);
    add(x1, k1);
  }
  for (; j < m4; j += 4 * kWave) {
    const doublex4 x0 = *(const doublex4*)(x + j);
    V k0[kGemvRows];
#pragma unroll
    for (int r = 0; r < kGemvRows; ++r) k0[r] = *(const V*)(rp[r] + j);
    add(x0, k0);
  }
  if (lane < m - m4) {  // the last m % 4 columns, one per lane
    const int c = m4 + lane;
#pragma unroll
    for (int r = 0; r < kGemvRows; ++r) s[r] += (double)rp[r][c] * x[c];
  }
#pragma unroll
  for (int r = 0; r < kGemvRows; ++r) {
    const double t = wave_sum(s[r]);
    if (lane == 0 && r0 + r < n) out[r0 + r] = t;
  }
}

template <typename TK>
void launch_gemv(const TK* K, int64_t ldk, int64_t n, int m, const double* x, double* out, hipStream_t s) {
  if (n <= 0) return;
  if (ldk % 4 != 0 || ((uintptr_t)K & (4 * sizeof(TK) - 1)) || ((uintptr_t)x & 31u))
    throw Failure(1, "GEMV: rows and x must be aligned to 4 values");
  hipLaunchKernelGGL((k_gemv<TK>), dim3((unsigned)ceil_div(n, 4 * kGemvRows)), dim3(256), 0, s, K, ldk, n, m, x, out);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------------------------------ compaction
constexpr int kCompactRows = 1024;  // rows per block: 4 chunks of 256 (about 100 workgroups at n = 100000)


// Grid y = slot of the batch.
__global__ __launch_bounds__(256) void k_compact_count(const CompactBatch bt, int64_t n) {
  const int q = blockIdx.y;
  const double* __restrict__ o = bt.o[q];
  const float* __restrict__ y = bt.y[q];
  const uint8_t* __restrict__ act_ref = bt.act_ref[q];
  int32_t* __restrict__ cnt = bt.cnt[q];
  double* __restrict__ bsum = bt.bsum[q];
  int32_t* __restrict__ bflips = bt.bflips[q];
  __shared__ double rd[4];
  __shared__ int ri[4];
  const int64_t lo = (int64_t)blockIdx.x * kCompactRows;
  constexpr int NJ = kCompactRows / 256;
  int c = 0, fl = 0;
  double s = 0.0;
  double av[NJ];  // every row's loads first (the rows of a block are few, so latency decides), then in order
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t i = lo + j * 256 + threadIdx.x;
    av[j] = i < n ? margin_gap(y[i], o[i]) : 0.0;
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t i = lo + j * 256 + threadIdx.x;
    if (i < n) {
      const double a = av[j];
      const int v = a > 0.0;
      c += v;
      if (v) s += a * a;
      if (act_ref) fl += (v != (int)act_ref[i]);
    }
  }
  c = block_sum_int(c, ri);
  fl = block_sum_int(fl, ri);
  s = block_sum(s, rd);
  if (threadIdx.x == 0) {
    cnt[blockIdx.x] = c;
    bsum[blockIdx.x] = s;
    bflips[blockIdx.x] = fl;
  }
}

// Grid y = slot of the batch.
__global__ __launch_bounds__(256) void k_compact_write(const CompactBatch bt, int64_t n, int nblk) {
  const int q = blockIdx.y;
  const double* __restrict__ o = bt.o[q];
  const float* __restrict__ y = bt.y[q];
  const int32_t* __restrict__ cnt = bt.cnt[q];
  const double* __restrict__ bsum = bt.bsum[q];
  const int32_t* __restrict__ bflips = bt.bflips[q];
  uint8_t* __restrict__ act_out = bt.act_out[q];
  int32_t* __restrict__ I = bt.I[q];
  NewtonScalars* sc = bt.sc[q];
  __shared__ int ri[4];
  __shared__ int wc[4];
  int part = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += 256) part += cnt[b];
  int offset = block_sum_int(part, ri);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t lo = (int64_t)blockIdx.x * kCompactRows;
  constexpr int NJ = kCompactRows / 256;
  bool vr[NJ];  // every row classified first (all loads in flight), then the ranks chunk by chunk
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t i = lo + j * 256 + threadIdx.x;
    vr[j] = i < n && margin_gap(y[i], o[i]) > 0.0;
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t i = lo + j * 256 + threadIdx.x;
    const int v = vr[j] ? 1 : 0;
    if (i < n) act_out[i] = (uint8_t)v;
    const unsigned long long mask = __ballot(v);
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wc[w] = __popcll(mask);
    __syncthreads();
    int base = offset;
    for (int q = 0; q < w; ++q) base += wc[q];
    if (v) I[base + rank] = (int32_t)i;
    offset += wc[0] + wc[1] + wc[2] + wc[3];
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int tot = 0, fl = 0;
    double s = 0.0;
#pragma unroll 8
    for (int b = 0; b < nblk; ++b) {  // in order; several blocks' values in flight
      tot += cnt[b];
      fl += bflips[b];
      s += bsum[b];
    }
    sc->n_sv = tot;
    sc->flips = fl;
    sc->sum_a2 = s;
  }
}

int compact_blocks(int64_t n) { return (int)std::max<int64_t>(1, ceil_div(n, kCompactRows)); }
int ls_blocks(int64_t n) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, ceil_div(n, 128))); }

void launch_compact_batch(const CompactBatch& b, int64_t n, hipStream_t s) {
  if (b.count <= 0) return;
  if (b.count > kMaxBatch) throw Failure(1, "compaction batch: too many slots");
  const int nblk = compact_blocks(n);
  hipLaunchKernelGGL(k_compact_count, dim3(nblk, b.count), dim3(256), 0, s, b, n);
  SPSVM_LAUNCHED();
  hipLaunchKernelGGL(k_compact_write, dim3(nblk, b.count), dim3(256), 0, s, b, n, nblk);
  SPSVM_LAUNCHED();
}

// Training errors for the stopping rule: rows with y_i o_i <= 0, summed per workgroup, then one integer atomic per
// workgroup (integer sums do not depend on their order) into a count the launcher clears first.
__global__ __launch_bounds__(256) void k_count_errors(const double* __restrict__ o, const float* __restrict__ y,
                                                      int64_t n, int32_t* __restrict__ out) {
  __shared__ int ri[4];
  int c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c += ((double)y[i] * o[i] <= 0.0) ? 1 : 0;
  c = block_sum_int(c, ri);
  if (threadIdx.x == 0 && c) atomicAdd(out, c);
}

void launch_count_errors(const double* o, const float* y, int64_t n, NewtonScalars* sc, hipStream_t s) {
  SPSVM_HIP(hipMemsetAsync(&sc->n_err, 0, sizeof(int32_t), s));
  hipLaunchKernelGGL(k_count_errors, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 1024), 1024))),
                     dim3(256), 0, s, o, y, n, &sc->n_err);
  SPSVM_LAUNCHED();
}

void launch_compact(const double* o, const float* y, int64_t n, const uint8_t* act_ref, uint8_t* act_out, int32_t* I,
                    int32_t* blk_count, double* blk_sum, int32_t* blk_flips, NewtonScalars* sc, hipStream_t s) {
  CompactBatch b{};
  b.o[0] = o;
  b.y[0] = y;
  b.act_ref[0] = act_ref;
  b.act_out[0] = act_out;
  b.I[0] = I;
  b.cnt[0] = blk_count;
  b.bsum[0] = blk_sum;
  b.bflips[0] = blk_flips;
  b.sc[0] = sc;
  b.count = 1;
  launch_compact_batch(b, n, s);
}

// -------------------------------------------------------------------------------------------- gradient
// Lane value l of v (l uniform across the wave): v_readlane, no LDS traffic.
__device__ __forceinline__ int lane_int(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double lane_double(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Partial sums of K_I^T (o_I - y_I) over a chunk of violator rows, one column per thread. The rows' indices and
// coefficients o_i - y_i are loaded 64 at a time, one row per lane, and handed to the wave with v_readlane, so the
// only per-row load is the 256 bytes of the wave's columns; eight rows' loads are in flight, summed in row order.
template <typename TK>
__global__ __launch_bounds__(256) void k_grad_partial(const TK* __restrict__ K, int64_t ldk, int m,
                                                      const int32_t* __restrict__ I,
                                                      const NewtonScalars* __restrict__ sc,
                                                      const double* __restrict__ o, const float* __restrict__ y,
                                                      double* __restrict__ partial) {
  // |I| as the compaction left it on the device (no host read-back between compaction and gradient); the
  // gridDim.y chunks split it evenly
  const int n_sv = sc->n_sv;
  const int rows_per_chunk = n_sv > (int)gridDim.y ? (n_sv + (int)gridDim.y - 1) / (int)gridDim.y : 1;
  const int lane = threadIdx.x & (kWave - 1);
  const int k = blockIdx.x * 256 + threadIdx.x;
  const int lo = blockIdx.y * rows_per_chunk;
  const int hi = lo + rows_per_chunk < n_sv ? lo + rows_per_chunk : n_sv;
  if (blockIdx.x * 256 + (threadIdx.x & ~(kWave - 1)) >= m) return;  // whole wave past the last column
  const int kc = k < m ? k : m - 1;  // lanes past the last column load a valid column and store nothing
  double acc = 0.0;
  for (int r = lo; r < hi; r += kWave) {
    const int rr = r + lane;
    const int iv = rr < hi ? I[rr] : 0;
    const double cv = rr < hi ? o[iv] - (double)y[iv] : 0.0;
    const int cnt = hi - r < kWave ? hi - r : kWave;
    int u = 0;
    for (; u + 8 <= cnt; u += 8) {
      TK kv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) kv[e] = K[(int64_t)lane_int(iv, u + e) * ldk + kc];
#pragma unroll
      for (int e = 0; e < 8; ++e) acc += (double)kv[e] * lane_double(cv, u + e);
    }
    for (; u < cnt; ++u) acc += (double)K[(int64_t)lane_int(iv, u) * ldk + kc] * lane_double(cv, u);
  }
  if (k < m) partial[(int64_t)blockIdx.y * m + k] = acc;
}

// g = lambda v + sum of the chunk partials, with v = K_JJ beta. Each workgroup owns 64 columns; lane group j
// (of 16) sums chunks j, j + 16, ... and thread k adds the 16 group sums in order. Per-workgroup partial sums
// of |g|^2 and beta . v go to blk (2 doubles per workgroup).
__global__ __launch_bounds__(1024) void k_grad_reduce(int m, const double* __restrict__ partial, int nchunk,
                                                      const double* __restrict__ v, const double* __restrict__ beta,
                                                      double lam, double* __restrict__ g, double* __restrict__ blk) {
  __shared__ double red[16][64];
  __shared__ double rd[2];
  const int c = threadIdx.x & 63, j = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + c;
  double a = 0.0;
  if (k < m) {
#pragma unroll 8
    for (int q = j; q < nchunk; q += 16) a += partial[(int64_t)q * m + k];  // in order; loads issued ahead
  }
  red[j][c] = a;
  __syncthreads();
  if (threadIdx.x < 64) {
    double gn = 0.0, bo = 0.0;
    if (k < m) {
      double s = 0.0;
      for (int q = 0; q < 16; ++q) s += red[q][c];
      s += lam * v[k];
      g[k] = s;
      gn = s * s;
      bo = beta[k] * v[k];
    }
    gn = wave_sum(gn);
    bo = wave_sum(bo);
    if (threadIdx.x == 0) {
      blk[2 * blockIdx.x] = gn;
      blk[2 * blockIdx.x + 1] = bo;
    }
  }
}

__global__ __launch_bounds__(64) void k_grad_norms(int nblk, const double* __restrict__ blk, NewtonScalars* sc) {
  double gn = 0.0, bo = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) {
    gn += blk[2 * b];
    bo += blk[2 * b + 1];
  }
  gn = wave_sum(gn);
  bo = wave_sum(bo);
  if (threadIdx.x == 0) {
    sc->gnorm2 = gn;
    sc->beta_oJ = bo;
  }
}

// Chunks of violator rows for the gradient partials; nchunk * m + 2 * ceil(m / 64) <= 1024 * 256 doubles
// (the partial buffer) for every m <= 65536.
int gradient_chunks(int m, int n_sv) {
  const int colblocks = (int)ceil_div(std::max(m, 1), 256);
  int c = std::max(1, 1024 / colblocks - 1);
  c = std::min<int>(c, (int)std::max<int64_t>(1, ceil_div(n_sv, 64)));
  return c;
}

template <typename TK>
void launch_gradient(const TK* K, int64_t ldk, int m, const int32_t* I, const double* o, const float* y,
                     const double* v, const double* beta, double lam, double* partial, int nchunk, double* g,
                     NewtonScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL((k_grad_partial<TK>), dim3((unsigned)ceil_div(m, 256), nchunk), dim3(256), 0, s, K, ldk, m, I,
                     sc, o, y, partial);
  SPSVM_LAUNCHED();
  const int nb = (int)ceil_div(m, 64);
  double* blk = partial + (int64_t)nchunk * m;  // the partial buffer holds 1024 * 256 doubles; see gradient_chunks
  hipLaunchKernelGGL(k_grad_reduce, dim3(nb), dim3(1024), 0, s, m, partial, nchunk, v, beta, lam, g, blk);
  SPSVM_LAUNCHED();
  hipLaunchKernelGGL(k_grad_norms, dim3(1), dim3(64), 0, s, nb, blk, sc);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------------------------------------ SYRK
// Partial H tiles over a range of violator rows: P[split][tile] = sum_{r in split} K[I_r, T_r]^T K[I_r, T_c]
// for the lower tiles (T_r >= T_c) of 128 x 128. Each workgroup has 4 waves (2 x 2), each owning a 64 x 64
// block (4 x 4 MFMA blocks); the strictly upper block of a diagonal tile is never read and its wave exits.
// Operands go straight from global memory into MFMA registers, no LDS and no barriers: in an MFMA step lane
// (g, i) supplies gathered row g of the step and the four consecutive columns 4i..4i+3 of its 64-column
// stripe (one 16-byte load), so MFMA block i holds the columns congruent to i mod 4 and the output is
// permuted back when written. The next 16 rows are loaded while the current 16 are multiplied. The products
// run on FP64 MFMA: a product of two FP32 values is exact in FP64, so the Gram part of H is accumulated to
// FP64 accuracy and stays positive semi-definite even for nearly dependent basis columns.
constexpr int SY_T = 128;

__device__ __forceinline__ void tile_of(int t, int& tr, int& tc) {
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  tr = r;
  tc = t - r * (r + 1) / 2;
}

// Four consecutive values of a row, cnt of them valid (cnt = 4: one vector load; the rest are zero).
__device__ __forceinline__ void load4(const float* p, int cnt, float (&v)[4]) {
  if (cnt >= 4) {
    const floatx4 t = *reinterpret_cast<const floatx4*>(p);
    v[0] = t[0], v[1] = t[1], v[2] = t[2], v[3] = t[3];
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = e < cnt ? p[e] : 0.0f;
  }
}
__device__ __forceinline__ void load4(const double* p, int cnt, double (&v)[4]) {
  if (cnt >= 4) {
    const doublex2 a = *reinterpret_cast<const doublex2*>(p), b = *reinterpret_cast<const doublex2*>(p + 2);
    v[0] = a[0], v[1] = a[1], v[2] = b[0], v[3] = b[1];
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = e < cnt ? p[e] : 0.0;
  }
}

// K: n x ldk row-major with ldk a multiple of 4 (16-byte aligned rows for FP32). Grid: x = tile, y = split,
// z = slot; workgroups beyond a slot's tile range or split count exit at once.
template <typename TK>
__global__ __launch_bounds__(256) void k_syrk(const SyrkBatch<TK> b, int64_t ldk, int m) {
  const int q = blockIdx.z;
  const int ntiles = b.tile_hi[q] - b.tile_lo[q], nsplit = b.nsplit[q], n_sv = b.n_rows[q];
  if ((int)blockIdx.x >= ntiles || (int)blockIdx.y >= nsplit) return;
  const TK* __restrict__ K = b.K[q];
  const int32_t* __restrict__ I = b.rows[q];
  double* __restrict__ partial = b.partial[q];
  const int rows_per_split = n_sv > nsplit ? (n_sv + nsplit - 1) / nsplit : 1;
  int tr, tc;
  tile_of(b.tile_lo[q] + blockIdx.x, tr, tc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, i16 = lane & 15;
  const int wr = w >> 1, wc = w & 1;
  if (tr == tc && wr < wc) return;  // wave-uniform
  const bool same = tr == tc && wr == wc;
  const int lo = blockIdx.y * rows_per_split;
  const int hi = lo + rows_per_split < n_sv ? lo + rows_per_split : n_sv;
  const int ca = tr * SY_T + wr * 64 + 4 * i16, cb = tc * SY_T + wc * 64 + 4 * i16;
  const int cnt_a = min(max(m - ca, 0), 4), cnt_b = min(max(m - cb, 0), 4);
  doublex4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = doublex4{0, 0, 0, 0};
  // Software pipeline: the row indices of chunk c + 2 and the values of chunk c + 1 are in flight while
  // chunk c is multiplied, so no load waits on a just-loaded index.
  int32_t ix[4];
  TK xa[4][4], xb[4][4];
  auto fetch_idx = [&](int r0) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int r = r0 + 4 * s + g;
      ix[s] = r < hi ? I[r] : -1;
    }
  };
  auto fetch_val = [&]() {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const TK* row = K + (int64_t)(ix[s] < 0 ? 0 : ix[s]) * ldk;
      load4(row + ca, ix[s] < 0 ? 0 : cnt_a, xa[s]);
      if (!same) load4(row + cb, ix[s] < 0 ? 0 : cnt_b, xb[s]);
    }
  };
  if (lo < hi) {
    fetch_idx(lo);
    fetch_val();
    fetch_idx(lo + 16);
  }
  for (int r0 = lo; r0 < hi; r0 += 16) {
    TK va[4][4], vb[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        va[s][e] = xa[s][e];
        vb[s][e] = same ? xa[s][e] : xb[s][e];
      }
    if (r0 + 16 < hi) {
      fetch_val();
      fetch_idx(r0 + 32);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double av[4], bv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        av[e] = (double)va[s][e];
        bv[e] = (double)vb[s][e];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
  }
  // FP64 MFMA output: acc[i][j][r] is row g + 4r of block (i, j), column i16, i.e. tile entry
  // (wr*64 + 4*(g + 4r) + i, wc*64 + 4*i16 + j).
  double* out = partial + ((int64_t)blockIdx.y * ntiles + blockIdx.x) * (SY_T * SY_T);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double* o = out + (wr * 64 + 4 * (g + 4 * r) + i) * SY_T + wc * 64 + 4 * i16;
      *reinterpret_cast<doublex2*>(o) = doublex2{acc[i][0][r], acc[i][1][r]};
      *reinterpret_cast<doublex2*>(o + 2) = doublex2{acc[i][2][r], acc[i][3][r]};
    }
}

int syrk_tiles(int m) {
  const int t = (int)ceil_div(m, SY_T);
  return t * (t + 1) / 2;
}

// Row splits per tile. Two workgroups fit on a CU (the accumulators take 128 AGPRs), so a launch runs in
// rounds of 512 workgroups; the split count minimises rounds x (rows per split + start-up) plus the cost of
// reducing the split partials, with at most kSyrkMaxPartials partial tiles and at least 64 rows per split.
constexpr int kSyrkSlots = 512, kSyrkMaxPartials = 8192;

static int syrk_max_splits(int nt) { return std::max(1, std::min(256, kSyrkMaxPartials / std::max(nt, 1))); }

int syrk_splits(int nt, int n_sv) {
  const int smax = std::min<int>(syrk_max_splits(nt), (int)std::max<int64_t>(1, ceil_div(n_sv, 64)));
  int best = 1;
  double best_cost = 0.0;
  for (int s = 1; s <= smax; ++s) {
    const double rounds = (double)ceil_div((int64_t)nt * s, kSyrkSlots);
    const double cost = rounds * ((double)ceil_div(n_sv, s) + 32.0) + 0.1 * s * nt;
    if (s == 1 || cost < best_cost) best = s, best_cost = cost;
  }
  return best;
}

// In a batch the other problems fill the chip, so a problem's rows are split at most in two, and only when it
// has few tiles. The choice depends on the problem alone, so a problem's result does not depend on which
// other problems share its batch.
int syrk_splits_batch(int nt, int n_sv) { return (nt < 128 && n_sv >= 128) ? kSyrkBatchSplits : 1; }

size_t syrk_partial_doubles_batch(int m_max) {
  return (size_t)kSyrkBatchSplits * syrk_tiles(std::max(m_max, 1)) * SY_T * SY_T;
}

size_t syrk_partial_doubles(int m_max) {
  size_t best = 0;
  for (int t = 1; t <= ceil_div(std::max(m_max, 1), SY_T); ++t) {
    const int nt = t * (t + 1) / 2;
    best = std::max(best, (size_t)syrk_max_splits(nt) * nt * SY_T * SY_T);
  }
  return best;
}

int syrk_tile_rows(int m) { return (int)ceil_div(m, SY_T); }
int syrk_tile_size() { return SY_T; }

template <typename TK>
void launch_syrk_batch(const SyrkBatch<TK>& b, int64_t ldk, int m, hipStream_t s) {
  int nt = 0, ns = 0;
  for (int q = 0; q < b.count; ++q) {
    if (b.nsplit[q] < 1 || b.tile_lo[q] < 0 || b.tile_hi[q] > syrk_tiles(m) || b.n_rows[q] < 0)
      throw Failure(1, "SYRK batch: invalid slot descriptor");
    nt = std::max(nt, b.tile_hi[q] - b.tile_lo[q]);
    ns = std::max(ns, b.nsplit[q]);
  }
  if (b.count <= 0 || b.count > kMaxBatch || nt <= 0) return;
  hipLaunchKernelGGL((k_syrk<TK>), dim3(nt, ns, b.count), dim3(256), 0, s, b, ldk, m);
  SPSVM_LAUNCHED();
}

template <typename TK>
void launch_syrk(const TK* K, int64_t ldk, int m, const int32_t* I, int n_rows, int tile_lo, int tile_hi, int nsplit,
                 double* partial, hipStream_t s) {
  SyrkBatch<TK> b{};
  b.K[0] = K;
  b.rows[0] = I;
  b.partial[0] = partial;
  b.n_rows[0] = n_rows;
  b.nsplit[0] = nsplit;
  b.tile_lo[0] = tile_lo;
  b.tile_hi[0] = tile_hi;
  b.count = 1;
  launch_syrk_batch(b, ldk, m, s);
}

// For the tiles tile_lo.. of the lower triangle: mode 0 sets H = lambda K_JJ + sum of the split partials,
// mode +1 adds the partial sums to H, mode -1 subtracts them (rows that joined or left the violator set).
// K_JJ is the FP64 kernel matrix of the basis rows (row-major, leading dimension ldh).
__global__ __launch_bounds__(256) void k_syrk_reduce(const ReduceBatch b, int m, int64_t ldh) {
  const int q = blockIdx.z;
  const int ntiles = b.tile_hi[q] - b.tile_lo[q], nsplit = b.nsplit[q], mode = b.mode[q];
  if ((int)blockIdx.x >= ntiles) return;
  int tr, tc;
  tile_of(b.tile_lo[q] + blockIdx.x, tr, tc);
  const int idx = blockIdx.y * 256 + threadIdx.x, r = idx / SY_T, c = idx % SY_T;
  const int gr = tr * SY_T + r, gc = tc * SY_T + c;
  if (gr >= m || gc >= m || gc > gr) return;
  const double* __restrict__ partial = b.partial[q];
  double s = 0.0;
#pragma unroll 8
  for (int p = 0; p < nsplit; ++p) s += partial[((int64_t)p * ntiles + blockIdx.x) * (SY_T * SY_T) + idx];  // in order
  double* h = b.H[q] + (int64_t)gr * ldh + gc;
  if (mode == 0)
    *h = b.lam[q] * b.KJJ[q][(int64_t)gr * ldh + gc] + s;
  else if (mode > 0)
    *h += s;
  else
    *h -= s;
}

void launch_syrk_reduce_batch(const ReduceBatch& b, int m, int64_t ldh, hipStream_t s) {
  int nt = 0;
  for (int q = 0; q < b.count; ++q) {
    if (b.nsplit[q] < 1 || b.tile_lo[q] < 0 || b.tile_hi[q] > syrk_tiles(m))
      throw Failure(1, "SYRK reduce batch: invalid slot descriptor");
    nt = std::max(nt, b.tile_hi[q] - b.tile_lo[q]);
  }
  if (b.count <= 0 || b.count > kMaxBatch || nt <= 0) return;
  hipLaunchKernelGGL(k_syrk_reduce, dim3(nt, SY_T * SY_T / 256, b.count), dim3(256), 0, s, b, m, ldh);
  SPSVM_LAUNCHED();
}

void launch_syrk_reduce(const double* KJJ, int m, double lam, const double* partial, int nsplit, int tile_lo,
                        int tile_hi, int mode, double* H, int64_t ldh, hipStream_t s) {
  ReduceBatch b{};
  b.KJJ[0] = KJJ;
  b.partial[0] = partial;
  b.H[0] = H;
  b.lam[0] = lam;
  b.nsplit[0] = nsplit;
  b.tile_lo[0] = tile_lo;
  b.tile_hi[0] = tile_hi;
  b.mode[0] = mode;
  b.count = 1;
  launch_syrk_reduce_batch(b, m, ldh, s);
}

__global__ __launch_bounds__(256) void k_scaled_sum_lower(double* __restrict__ H, const double* __restrict__ KJJ,
                                                          const double* __restrict__ G, double lam, int m,
                                                          int64_t ldh) {
  const int r = blockIdx.y;
  for (int c = blockIdx.x * 256 + threadIdx.x; c <= r && c < m; c += gridDim.x * 256) {
    const int64_t e = (int64_t)r * ldh + c;
    H[e] = lam * KJJ[e] + G[e];
  }
}

void launch_scaled_sum_lower(double* H, const double* KJJ, const double* G, double lam, int m, int64_t ldh,
                             hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_scaled_sum_lower, dim3((unsigned)ceil_div(m, 256), (unsigned)m), dim3(256), 0, s, H, KJJ, G,
                     lam, m, ldh);
  SPSVM_LAUNCHED();
}

__global__ void k_add_diag(double* __restrict__ H, int64_t ldh, int m, double v) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < m; k += gridDim.x * blockDim.x) H[(int64_t)k * ldh + k] += v;
}

void launch_add_diag(double* H, int64_t ldh, int m, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_add_diag, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(m, 256), 64))),
                     dim3(256), 0, s, H, ldh, m, v);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------------------------- batched GEMV
// One wave per RT x 16 rows of K (RT 16-row MFMA tiles) and NCB x 16 vectors. In an MFMA step lane (g, i)
// supplies K[row i][k] and x_{slot i}[k] for k = k0 + 4g + t (t = 0..3 over four steps), so one 16-byte load per
// row feeds four steps; acc[i][j][r] ends as out_{slot 16j + i16}[row 16i + g + 4r]. The next 16 k are loaded
// while the current ones are multiplied.
template <typename TK, int RT, int NCB>
__global__ __launch_bounds__(64) void k_gemv_batch(const TK* __restrict__ K, int64_t ldk, int64_t n, int m,
                                                   const GemvBatch b) {
  const int lane = threadIdx.x, g = lane >> 4, i16 = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.x * (RT * 16);
  const TK* krow[RT];
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    const int64_t row = r0 + i * 16 + i16;
    krow[i] = row < n ? K + row * ldk : nullptr;
  }
  const double* xs[NCB];
#pragma unroll
  for (int j = 0; j < NCB; ++j) {
    const int q = j * 16 + i16;
    xs[j] = q < b.count ? b.x[q] : nullptr;
  }
  doublex4 acc[RT][NCB];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < NCB; ++j) acc[i][j] = doublex4{0, 0, 0, 0};
  TK kv[RT][4];
  double xv[NCB][4];
  auto fetch = [&](int k0) {
    const int kb = k0 + 4 * g;
    const int cnt = min(max(m - kb, 0), 4);
#pragma unroll
    for (int i = 0; i < RT; ++i) load4(krow[i] ? krow[i] + kb : K, krow[i] ? cnt : 0, kv[i]);
#pragma unroll
    for (int j = 0; j < NCB; ++j) load4(xs[j] ? xs[j] + kb : b.x[0], xs[j] ? cnt : 0, xv[j]);
  };
  fetch(0);
  for (int k0 = 0; k0 < m; k0 += 16) {
    double a[RT][4], c[NCB][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int i = 0; i < RT; ++i) a[i][t] = (double)kv[i][t];
#pragma unroll
      for (int j = 0; j < NCB; ++j) c[j][t] = xv[j][t];
    }
    if (k0 + 16 < m) fetch(k0 + 16);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < NCB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][t], c[j][t], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < NCB; ++j) {
    const int q = j * 16 + i16;
    if (q >= b.count) continue;
    double* out = b.out[q];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + i * 16 + g + 4 * r;
        if (row < n) out[row] = acc[i][j][r];
      }
  }
}

template <typename TK>
void launch_gemv_batch(const TK* K, int64_t ldk, int64_t n, int m, const GemvBatch& b, hipStream_t s) {
  if (n <= 0 || b.count <= 0) return;
  if (b.count > kMaxBatch || (ldk & 3) || ((uintptr_t)K & 15u)) throw Failure(1, "GEMV batch: bad arguments");
  for (int q = 0; q < b.count; ++q)
    if ((uintptr_t)b.x[q] & 31u) throw Failure(1, "GEMV batch: vectors must be 32-byte aligned");
  // 32-row waves fill the chip for tall blocks; 16-row waves for short ones (K_JJ)
  if (n >= 16384) {
    const dim3 grid((unsigned)ceil_div(n, 32));
    if (b.count <= 16)
      hipLaunchKernelGGL((k_gemv_batch<TK, 2, 1>), grid, dim3(64), 0, s, K, ldk, n, m, b);
    else if (b.count <= 32)
      hipLaunchKernelGGL((k_gemv_batch<TK, 2, 2>), grid, dim3(64), 0, s, K, ldk, n, m, b);
    else
      hipLaunchKernelGGL((k_gemv_batch<TK, 2, 3>), grid, dim3(64), 0, s, K, ldk, n, m, b);
  } else {
    const dim3 grid((unsigned)ceil_div(n, 16));
    if (b.count <= 16)
      hipLaunchKernelGGL((k_gemv_batch<TK, 1, 1>), grid, dim3(64), 0, s, K, ldk, n, m, b);
    else if (b.count <= 32)
      hipLaunchKernelGGL((k_gemv_batch<TK, 1, 2>), grid, dim3(64), 0, s, K, ldk, n, m, b);
    else
      hipLaunchKernelGGL((k_gemv_batch<TK, 1, 3>), grid, dim3(64), 0, s, K, ldk, n, m, b);
  }
  SPSVM_LAUNCHED();
}

// --------------------------------------------------------------------------------- batched gradient
// Dense K^T r for NCB x 16 slots: one wave per 64 columns of K and chunk of rows. In an MFMA step lane (g, i)
// supplies K[row][16 jt + i] and r_{slot i}[row] for row = i0 + 4g + t (t = 0..3 over four steps), with
// r = o - y on violators and 0 elsewhere; acc[jt][c][r] ends as the partial of column 16 jt + g + 4r for slot
// 16 c + i.
template <typename TK, int NCB>
__global__ __launch_bounds__(64) void k_grad_batch(const TK* __restrict__ K, int64_t ldk, int64_t n, int m,
                                                   int64_t rows_per_chunk, const GradBatch b) {
  const int lane = threadIdx.x, g = lane >> 4, i16 = lane & 15;
  const int j0 = blockIdx.x * 64;
  const int64_t lo = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t hi = lo + rows_per_chunk < n ? lo + rows_per_chunk : n;
  const double* os[NCB];
  const float* ys[NCB];
#pragma unroll
  for (int c = 0; c < NCB; ++c) {
    const int q = c * 16 + i16;
    os[c] = q < b.count ? b.o[q] : nullptr;
    ys[c] = q < b.count ? b.y[q] : nullptr;
  }
  doublex4 acc[4][NCB];
#pragma unroll
  for (int jt = 0; jt < 4; ++jt)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[jt][c] = doublex4{0, 0, 0, 0};
  // operands of 16 rows: K values and o, y of this lane group's four rows; the next block is loaded while the
  // current one is multiplied
  TK kx[4][4];
  double ox[NCB][4];
  float yx[NCB][4];
  auto fetch = [&](int64_t i0) {
    const int64_t ib = i0 + 4 * g;
    const int64_t cnt = hi - ib;
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
      load4(os[c] && cnt > 0 ? os[c] + ib : b.o[0], os[c] ? (int)min<int64_t>(max<int64_t>(cnt, 0), 4) : 0, ox[c]);
#pragma unroll
      for (int t = 0; t < 4; ++t) yx[c][t] = (os[c] && t < cnt) ? ys[c][ib + t] : 0.0f;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const TK* krow = K + (ib + t < hi ? ib + t : lo) * ldk;
#pragma unroll
      for (int jt = 0; jt < 4; ++jt) {
        const int col = j0 + jt * 16 + i16;
        kx[t][jt] = (t < cnt && col < m) ? krow[col] : (TK)0;
      }
    }
  };
  if (lo < hi) fetch(lo);
  for (int64_t i0 = lo; i0 < hi; i0 += 16) {
    const int64_t cnt = hi - (i0 + 4 * g);
    double rv[NCB][4], kv[4][4];
#pragma unroll
    for (int c = 0; c < NCB; ++c)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool in = os[c] && t < cnt;
        rv[c][t] = (in && margin_gap(yx[c][t], ox[c][t]) > 0.0) ? ox[c][t] - (double)yx[c][t] : 0.0;
      }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int jt = 0; jt < 4; ++jt) kv[t][jt] = (double)kx[t][jt];
    if (i0 + 16 < hi) fetch(i0 + 16);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int jt = 0; jt < 4; ++jt)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
          acc[jt][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(kv[t][jt], rv[c][t], acc[jt][c], 0, 0, 0);
  }
#pragma unroll
  for (int c = 0; c < NCB; ++c) {
    const int q = c * 16 + i16;
    if (q >= b.count) continue;
    double* part = b.partial[q] + (int64_t)blockIdx.y * m;
#pragma unroll
    for (int jt = 0; jt < 4; ++jt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = j0 + jt * 16 + g + 4 * r;
        if (j < m) part[j] = acc[jt][c][r];
      }
  }
}

// Row chunks of the dense gradient: at least 512 rows each, and the partials fit the gradient buffer
// (nchunk * m + 2 * ceil(m / 64) <= 1024 * 256 doubles).
int gradient_chunks_dense(int64_t n, int m) {
  const int64_t room = (1024 * 256 - 2 * ceil_div(std::max(m, 1), 64)) / std::max(m, 1);
  return (int)std::max<int64_t>(1, std::min<int64_t>(room, ceil_div(n, 512)));
}

// Per slot: g = lambda v + sum of the chunk partials, then |g|^2 and beta . v (grid z = slot).
__global__ __launch_bounds__(1024) void k_grad_reduce_batch(int m, int nchunk, const GradBatch b) {
  const int q = blockIdx.z;
  __shared__ double red[16][64];
  const int c = threadIdx.x & 63, j = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + c;
  const double* partial = b.partial[q];
  double a = 0.0;
  if (k < m)
#pragma unroll 8
    for (int p = j; p < nchunk; p += 16) a += partial[(int64_t)p * m + k];  // in order; loads issued ahead
  red[j][c] = a;
  __syncthreads();
  if (threadIdx.x < 64) {
    double gn = 0.0, bo = 0.0;
    if (k < m) {
      double s = 0.0;
      for (int p = 0; p < 16; ++p) s += red[p][c];
      s += b.lam[q] * b.v[q][k];
      b.g[q][k] = s;
      gn = s * s;
      bo = b.beta[q][k] * b.v[q][k];
    }
    gn = wave_sum(gn);
    bo = wave_sum(bo);
    if (threadIdx.x == 0) {
      double* blk = b.partial[q] + (int64_t)nchunk * m;
      blk[2 * blockIdx.x] = gn;
      blk[2 * blockIdx.x + 1] = bo;
    }
  }
}

__global__ __launch_bounds__(64) void k_grad_norms_batch(int m, int nchunk, int nblk, const GradBatch b) {
  const int q = blockIdx.z;
  const double* blk = b.partial[q] + (int64_t)nchunk * m;
  double gn = 0.0, bo = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 64) {
    gn += blk[2 * i];
    bo += blk[2 * i + 1];
  }
  gn = wave_sum(gn);
  bo = wave_sum(bo);
  if (threadIdx.x == 0) {
    b.sc[q]->gnorm2 = gn;
    b.sc[q]->beta_oJ = bo;
  }
}

template <typename TK>
void launch_gradient_batch(const TK* K, int64_t ldk, int64_t n, int m, const GradBatch& b, hipStream_t s) {
  if (b.count <= 0 || m <= 0) return;
  if (b.count > kMaxBatch) throw Failure(1, "gradient batch: too many slots");
  for (int q = 0; q < b.count; ++q)
    if ((uintptr_t)b.o[q] & 31u) throw Failure(1, "gradient batch: o must be 32-byte aligned");
  const int nchunk = gradient_chunks_dense(n, m);
  // chunks start on multiples of 16 rows, so each lane group's four o values are one aligned vector load
  const int64_t rows = round_up(ceil_div(std::max<int64_t>(n, 1), nchunk), 16);
  const dim3 grid((unsigned)ceil_div(m, 64), (unsigned)nchunk);
  if (n > 0) {
    if (b.count <= 16)
      hipLaunchKernelGGL((k_grad_batch<TK, 1>), grid, dim3(64), 0, s, K, ldk, n, m, rows, b);
    else if (b.count <= 32)
      hipLaunchKernelGGL((k_grad_batch<TK, 2>), grid, dim3(64), 0, s, K, ldk, n, m, rows, b);
    else
      hipLaunchKernelGGL((k_grad_batch<TK, 3>), grid, dim3(64), 0, s, K, ldk, n, m, rows, b);
    SPSVM_LAUNCHED();
  }
  const int nb = (int)ceil_div(m, 64);
  hipLaunchKernelGGL(k_grad_reduce_batch, dim3(nb, 1, b.count), dim3(1024), 0, s, m, n > 0 ? nchunk : 0, b);
  SPSVM_LAUNCHED();
  hipLaunchKernelGGL(k_grad_norms_batch, dim3(1, 1, b.count), dim3(64), 0, s, m, n > 0 ? nchunk : 0, nb, b);
  SPSVM_LAUNCHED();
}

// --------------------------------------------------------------------------------------- flipped rows
// Lists of rows whose violator status differs between act_new and act_old: joined (new 1, old 0) and left
// (new 0, old 1), each in ascending order. Same block scheme as the violator compaction.
// Grid y = slot of the batch.
__global__ __launch_bounds__(256) void k_flip_count(const FlipBatch bt, int64_t n) {
  const int q = blockIdx.y;
  const uint8_t* __restrict__ act_new = bt.act_new[q];
  const uint8_t* __restrict__ act_old = bt.act_old[q];
  int32_t* __restrict__ cnt_in = bt.cnt_in[q];
  int32_t* __restrict__ cnt_out = bt.cnt_out[q];
  __shared__ int ri[4];
  const int64_t lo = (int64_t)blockIdx.x * kCompactRows;
  int a = 0, b = 0;
  for (int j = 0; j < kCompactRows / 256; ++j) {
    const int64_t i = lo + j * 256 + threadIdx.x;
    if (i < n) {
      a += act_new[i] && !act_old[i];
      b += !act_new[i] && act_old[i];
    }
  }
  a = block_sum_int(a, ri);
  b = block_sum_int(b, ri);
  if (threadIdx.x == 0) {
    cnt_in[blockIdx.x] = a;
    cnt_out[blockIdx.x] = b;
  }
}

// Grid y = slot of the batch.
__global__ __launch_bounds__(256) void k_flip_write(const FlipBatch bt, int64_t n, int nblk) {
  const int q = blockIdx.y;
  const uint8_t* __restrict__ act_new = bt.act_new[q];
  const uint8_t* __restrict__ act_old = bt.act_old[q];
  const int32_t* __restrict__ cnt_in = bt.cnt_in[q];
  const int32_t* __restrict__ cnt_out = bt.cnt_out[q];
  int32_t* __restrict__ F_in = bt.F_in[q];
  int32_t* __restrict__ F_out = bt.F_out[q];
  NewtonScalars* sc = bt.sc[q];
  __shared__ int ri[4];
  __shared__ int wc[2][4];
  int pa = 0, pb = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += 256) {
    pa += cnt_in[b];
    pb += cnt_out[b];
  }
  int off_in = block_sum_int(pa, ri), off_out = block_sum_int(pb, ri);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t lo = (int64_t)blockIdx.x * kCompactRows;
  for (int j = 0; j < kCompactRows / 256; ++j) {
    const int64_t i = lo + j * 256 + threadIdx.x;
    int vi = 0, vo = 0;
    if (i < n) {
      vi = act_new[i] && !act_old[i];
      vo = !act_new[i] && act_old[i];
    }
    const unsigned long long mi = __ballot(vi), mo = __ballot(vo);
    const unsigned long long below = (1ull << lane) - 1ull;
    if (lane == 0) {
      wc[0][w] = __popcll(mi);
      wc[1][w] = __popcll(mo);
    }
    __syncthreads();
    int bi = off_in, bo = off_out;
    for (int q = 0; q < w; ++q) {
      bi += wc[0][q];
      bo += wc[1][q];
    }
    if (vi) F_in[bi + __popcll(mi & below)] = (int32_t)i;
    if (vo) F_out[bo + __popcll(mo & below)] = (int32_t)i;
    off_in += wc[0][0] + wc[0][1] + wc[0][2] + wc[0][3];
    off_out += wc[1][0] + wc[1][1] + wc[1][2] + wc[1][3];
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int a = 0, b = 0;
    for (int q = 0; q < nblk; ++q) {
      a += cnt_in[q];
      b += cnt_out[q];
    }
    sc->n_in = a;
    sc->n_out = b;
  }
}

void launch_flip_lists_batch(const FlipBatch& b, int64_t n, hipStream_t s) {
  if (b.count <= 0) return;
  if (b.count > kMaxBatch) throw Failure(1, "flip-list batch: too many slots");
  const int nblk = compact_blocks(n);
  hipLaunchKernelGGL(k_flip_count, dim3(nblk, b.count), dim3(256), 0, s, b, n);
  SPSVM_LAUNCHED();
  hipLaunchKernelGGL(k_flip_write, dim3(nblk, b.count), dim3(256), 0, s, b, n, nblk);
  SPSVM_LAUNCHED();
}

__global__ __launch_bounds__(256) void k_trace(const double* __restrict__ H, int64_t ldh, int m, NewtonScalars* sc) {
  __shared__ double rd[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < m; k += 256) s += H[(int64_t)k * ldh + k];
  s = block_sum(s, rd);
  if (threadIdx.x == 0) sc->trace = s;
}

void launch_trace(const double* H, int64_t ldh, int m, NewtonScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, s, H, ldh, m, sc);
  SPSVM_LAUNCHED();
}

// ---------------------------------------------------------------------------------------- line search
// phi(t) = f(beta + t d) = const + lambda (t c1 + t^2 c2 / 2) + 1/2 sum max(0, a_i - t b_i)^2,
// a_i = 1 - y_i o_i, b_i = y_i delta_i, delta = K_XJ d, c1 = beta^T K_JJ d, c2 = d^T K_JJ d (from w = K_JJ d).
// Grid x = slot of the batch.
__global__ __launch_bounds__(256) void k_c1c2(const LsBatch bt, int m) {
  const int q = blockIdx.x;
  const double* __restrict__ beta = bt.beta[q];
  const double* __restrict__ dvec = bt.dvec[q];
  const double* __restrict__ w = bt.w[q];
  LineState* ls = bt.ls[q];
  __shared__ double rd[4];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < m; k += 256) {
    a += beta[k] * w[k];
    b += dvec[k] * w[k];
  }
  a = block_sum(a, rd);
  b = block_sum(b, rd);
  if (threadIdx.x == 0) {
    LineState s;
    s.c1 = a;
    s.c2 = b;
    s.t = 1.0;
    s.t_prev = 0.0;
    s.lo = 0.0;
    s.hi = __builtin_huge_val();
    s.dec = 0.0;
    s.status = 0;
    s.newton = 0;
    s.passes = 0;
    s.pad = 0;
    *ls = s;
  }
}

void launch_c1c2_batch(const LsBatch& b, int m, hipStream_t s) {
  if (b.count <= 0) return;
  if (b.count > kMaxBatch) throw Failure(1, "line-search batch: too many slots");
  hipLaunchKernelGGL(k_c1c2, dim3(b.count), dim3(256), 0, s, b, m);
  SPSVM_LAUNCHED();
}

// Pass 0 evaluates t = 0 and t = 1 (slots A and B); later passes evaluate t (slot B) with flips against t_prev.
// Partial record per block: {P_A, Q_A, P_B, Q_B, V_B, flips}.
// Grid y = slot of the batch.
__global__ __launch_bounds__(256) void k_ls_pass(const LsBatch bt, int64_t n, int64_t rows_per_blk) {
  const int q = blockIdx.y;
  const double* __restrict__ o = bt.o[q];
  const double* __restrict__ delta = bt.delta[q];
  const float* __restrict__ y = bt.y[q];
  const LineState* __restrict__ ls = bt.ls[q];
  double* __restrict__ partial = bt.partial[q];
  __shared__ double rd[4];
  if (ls->status != 0) return;
  const bool first = ls->passes == 0;
  const double t = ls->t, tp = ls->t_prev;
  const int64_t lo = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t hi = lo + rows_per_blk < n ? lo + rows_per_blk : n;
  double pa = 0.0, qa = 0.0, pb = 0.0, qb = 0.0, vb = 0.0;
  int fl = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const double yi = (double)y[i];
    const double a = 1.0 - yi * o[i];
    const double b = yi * delta[i];
    const double ep = a - tp * b, e = a - t * b;
    if (first && ep > 0.0) {
      pa += a * b;
      qa += b * b;
    }
    if (e > 0.0) {
      pb += a * b;
      qb += b * b;
    }
    const double u = fmax(a, 0.0), w = fmax(e, 0.0);
    vb += (w - u) * (w + u);
    fl += ((e > 0.0) != (ep > 0.0)) ? 1 : 0;
  }
  double v[6] = {pa, qa, pb, qb, vb, (double)fl};
  for (int k = 0; k < 6; ++k) {
    const double r = block_sum(v[k], rd);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * 6 + k] = r;
  }
}

// Grid x = slot of the batch.
__global__ __launch_bounds__(256) void k_ls_update(const LsBatch bt, int nblk) {
  const int q = blockIdx.x;
  LineState* ls = bt.ls[q];
  const double* __restrict__ partial = bt.partial[q];
  const double lam = bt.lam[q];
  __shared__ double red[6][256];
  if (ls->status != 0) return;
  {
    double a[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll 4
    for (int b = threadIdx.x; b < nblk; b += 256)
      for (int k = 0; k < 6; ++k) a[k] += partial[(int64_t)b * 6 + k];
    for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = a[k];
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {  // fixed-order tree
    if (threadIdx.x < w)
      for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  LineState s = *ls;
  double v[6];
  for (int k = 0; k < 6; ++k) v[k] = red[k][0];
  const double P = v[2], Q = v[3], V = v[4], F = v[5];
  const double lc1 = lam * s.c1, lc2 = lam * s.c2;
  bool done = false;
  if (s.passes == 0) {
    const double P0 = v[0], Q0 = v[1];
    s.passes = 1;
    const double g0 = lc1 - P0;
    if (g0 >= 0.0) {  // no descent along d
      s.t = 0.0;
      s.dec = 0.0;
      s.status = 1;
      *ls = s;
      return;
    }
    if (F == 0.0) {  // active set constant on [0, 1]: phi' is one linear piece there
      const double r = (P0 - lc1) / (lc2 + Q0);
      if (r >= 0.0 && r <= 1.0) {
        s.t = r;
        s.dec = -(r * lc1 + 0.5 * r * r * lc2) + r * P0 - 0.5 * r * r * Q0;
        s.status = 1;
        *ls = s;
        return;
      }
    }
    const double g1 = lc1 + lc2 - (P - Q);
    if (g1 < 0.0)
      s.lo = 1.0;
    else
      s.hi = 1.0;
    const double r1 = (P - lc1) / (lc2 + Q);
    const double r0 = (P0 - lc1) / (lc2 + Q0);
    if (r1 > s.lo && r1 < s.hi) {
      s.t_prev = 1.0;
      s.t = r1;
      s.newton = 1;
    } else if (r0 > s.lo && r0 < s.hi) {
      s.t_prev = 0.0;
      s.t = r0;
      s.newton = 1;
    } else {
      s.t_prev = 1.0;
      s.newton = 0;
      s.t = s.hi < __builtin_huge_val() ? 0.5 * (s.lo + s.hi) : s.lo + fmax(1.0, s.lo);
    }
    *ls = s;
    return;
  }
  s.passes += 1;
  const double g = lc1 + s.t * lc2 - (P - s.t * Q);
  done = (s.newton && F == 0.0) || g == 0.0;
  if (!done) {
    if (g < 0.0)
      s.lo = s.t;
    else
      s.hi = s.t;
    const double r = (P - lc1) / (lc2 + Q);
    double nx;
    int nw;
    if (r > s.lo && r < s.hi) {
      nx = r;
      nw = 1;
    } else {
      nw = 0;
      nx = s.hi < __builtin_huge_val() ? 0.5 * (s.lo + s.hi) : s.lo + fmax(1.0, s.lo);
    }
    if (nx > s.lo && nx < s.hi && s.passes < 64) {
      s.t_prev = s.t;
      s.t = nx;
      s.newton = nw;
    } else {
      done = true;
    }
  }
  if (done) {
    s.status = 1;
    s.dec = -(s.t * lc1 + 0.5 * s.t * s.t * lc2) - 0.5 * V;
  }
  *ls = s;
}

void launch_ls_round_batch(const LsBatch& b, int64_t n, int nblk, hipStream_t s) {
  if (b.count <= 0) return;
  if (b.count > kMaxBatch) throw Failure(1, "line-search batch: too many slots");
  const int64_t rows = ceil_div(n, nblk);
  hipLaunchKernelGGL(k_ls_pass, dim3(nblk, b.count), dim3(256), 0, s, b, n, rows);
  SPSVM_LAUNCHED();
  hipLaunchKernelGGL(k_ls_update, dim3(b.count), dim3(256), 0, s, b, nblk);
  SPSVM_LAUNCHED();
}

// Grid y = slot of the batch.
__global__ __launch_bounds__(256) void k_apply_step(const LsBatch bt, int m, int64_t n) {
  const int q = blockIdx.y;
  double* __restrict__ beta = bt.beta[q];
  const double* __restrict__ dvec = bt.dvec[q];
  double* __restrict__ o = bt.o[q];
  const double* __restrict__ delta = bt.delta[q];
  const double t = bt.ls[q]->t;
  if (t == 0.0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) o[i] += t * delta[i];
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += stride) beta[k] += t * dvec[k];
}

void launch_apply_step_batch(const LsBatch& b, int m, int64_t n, hipStream_t s) {
  if (b.count <= 0) return;
  if (b.count > kMaxBatch) throw Failure(1, "line-search batch: too many slots");
  const int64_t blocks = std::min<int64_t>(ceil_div(std::max<int64_t>(n, m), 256), 2048);
  hipLaunchKernelGGL(k_apply_step, dim3((unsigned)blocks, b.count), dim3(256), 0, s, b, m, n);
  SPSVM_LAUNCHED();
}

__global__ void k_scale(double* v, int m, double a) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < m; k += gridDim.x * blockDim.x) v[k] *= a;
}
void launch_scale(double* v, int m, double a, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(m, 256), 64))),
                     dim3(256), 0, s, v, m, a);
  SPSVM_LAUNCHED();
}

// ------------------------------------------------------------------------------------ instantiations
template void launch_gemv<float>(const float*, int64_t, int64_t, int, const double*, double*, hipStream_t);
template void launch_gemv<double>(const double*, int64_t, int64_t, int, const double*, double*, hipStream_t);
template void launch_gradient<float>(const float*, int64_t, int, const int32_t*, const double*, const float*,
                                     const double*, const double*, double, double*, int, double*, NewtonScalars*,
                                     hipStream_t);
template void launch_gradient<double>(const double*, int64_t, int, const int32_t*, const double*, const float*,
                                      const double*, const double*, double, double*, int, double*, NewtonScalars*,
                                      hipStream_t);
template void launch_gradient_batch<float>(const float*, int64_t, int64_t, int, const GradBatch&, hipStream_t);
template void launch_gradient_batch<double>(const double*, int64_t, int64_t, int, const GradBatch&, hipStream_t);
template void launch_gemv_batch<float>(const float*, int64_t, int64_t, int, const GemvBatch&, hipStream_t);
template void launch_gemv_batch<double>(const double*, int64_t, int64_t, int, const GemvBatch&, hipStream_t);
template void launch_syrk_batch<float>(const SyrkBatch<float>&, int64_t, int, hipStream_t);
template void launch_syrk_batch<double>(const SyrkBatch<double>&, int64_t, int, hipStream_t);
template void launch_syrk<float>(const float*, int64_t, int, const int32_t*, int, int, int, int, double*, hipStream_t);
template void launch_syrk<double>(const double*, int64_t, int, const int32_t*, int, int, int, int, double*,
                                  hipStream_t);

}  // namespace spsvm
