// One-vs-one multiclass (section 5 trains MNIST8M with one classifier per pair of classes, each on the rows of its
// two classes): gathering a pair's rows, and the pairwise votes of prediction.
#include "common.h"
#include "launch.h"

namespace spsvm {

// out[r] = X[rows[r]] for r < m (rows of d values, dense), one wave per row.
template <typename TX>
__global__ __launch_bounds__(256) void k_gather_pair(const TX* __restrict__ X, int64_t d,
                                                     const int64_t* __restrict__ rows, int64_t m,
                                                     TX* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / 64; r < m; r += (int64_t)gridDim.x * 4) {
    const TX* __restrict__ src = X + rows[r] * d;
    TX* __restrict__ dst = out + r * d;
    for (int64_t t = lane; t < d; t += 64) dst[t] = src[t];
  }
}

template <typename TX>
void launch_gather_pair(const TX* X, int64_t d, const int64_t* rows, int64_t m, TX* out, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL((k_gather_pair<TX>), dim3((unsigned)std::min<int64_t>(ceil_div(m, 4), 8192)), dim3(256), 0, st,
                     X, d, rows, m, out);
  SPSVM_LAUNCHED();
}
template void launch_gather_pair<float>(const float*, int64_t, const int64_t*, int64_t, float*, hipStream_t);
template void launch_gather_pair<double>(const double*, int64_t, const int64_t*, int64_t, double*, hipStream_t);

// votes[i * K + (dec[i] > 0 ? a : b)] += 1: a positive decision of pair (a, b) is a vote for a, any other for b.
__global__ __launch_bounds__(256) void k_ovo_vote(const double* __restrict__ dec, int64_t n, int a, int b, int K,
                                                  int32_t* __restrict__ votes) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    votes[i * K + (dec[i] > 0.0 ? a : b)] += 1;
}

// classes[i] = the class with the most votes, the lowest one on ties.
__global__ __launch_bounds__(256) void k_ovo_argmax(const int32_t* __restrict__ votes, int64_t n, int K,
                                                    int32_t* __restrict__ classes) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int best = 0, bv = votes[i * K];
    for (int c = 1; c < K; ++c) {
      const int v = votes[i * K + c];
      if (v > bv) {
        bv = v;
        best = c;
      }
    }
    classes[i] = best;
  }
}

void launch_ovo_vote(const double* dec, int64_t n, int a, int b, int K, int32_t* votes, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_ovo_vote, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 4096)), dim3(256), 0, st, dec, n,
                     a, b, K, votes);
  SPSVM_LAUNCHED();
}

void launch_ovo_argmax(const int32_t* votes, int64_t n, int K, int32_t* classes, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_ovo_argmax, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 4096)), dim3(256), 0, st,
                     votes, n, K, classes);
  SPSVM_LAUNCHED();
}

}  // namespace spsvm
