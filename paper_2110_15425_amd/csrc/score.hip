// score.hip -- grid score and best allocation.
//
// A control node evaluates every allocation and keeps the best one; when
// several allocations tie it picks one at random (Distill, Sec. 2.1 and the
// fixed-size reservoir sampling of Sec. 3.3).  Here the pick is
// order-independent: each tied setting s gets the priority word
// Philox(seed; 0, s, ~0, ~0).w0 and the tie with the smallest (priority, s)
// wins -- a uniform choice among ties, like reservoir sampling, without any
// dependence on the order in which threads visit the grid.
//
// score[s] = reward * (correct[s] / trials) - cost * sum_k c_k^2, evaluated
// in this order in double with no fused multiply-add, so every setting's
// score is bit-reproducible.
#include "prep_score.hpp"

namespace cm {
namespace {

constexpr int kScoreBlock = 1024;

// One workgroup per sweep of the batch.
__global__ __launch_bounds__(kScoreBlock) void score_kernel(ScoreBatch batch) {
  __shared__ double red_d[kScoreBlock / 64];
  __shared__ unsigned long long red_k[kScoreBlock / 64];
  __shared__ unsigned long long red_c[kScoreBlock / 64];
  score_sweep<kScoreBlock / 64>(batch.a[blockIdx.x], red_d, red_k, red_c);
}

}  // namespace

hipError_t launch_score(const ScoreBatch& b, hipStream_t st) {
  if (b.n > kMaxBatch) return hipErrorInvalidValue;
  if (!b.n) return hipSuccess;
  hipLaunchKernelGGL(score_kernel, dim3(b.n), dim3(kScoreBlock), 0, st, b);
  return hipGetLastError();
}

}  // namespace cm
