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
#include "internal.hpp"
#include "rng.hpp"

namespace cm {
namespace {

constexpr int kScoreBlock = 1024;

// One workgroup per sweep of the batch.
__global__ __launch_bounds__(kScoreBlock) void score_kernel(ScoreBatch batch) {
  const ScoreArgs& a = batch.a[blockIdx.x];
  __shared__ double red_d[kScoreBlock / 64];
  __shared__ unsigned long long red_k[kScoreBlock / 64];
  __shared__ unsigned long long red_c[kScoreBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;

  double mx = -INFINITY;
  for (uint64_t s = threadIdx.x; s < a.n_settings; s += blockDim.x) {
    const double q = (double)a.stats[s * CM_NSTAT + CM_ST_CORRECT] / (double)a.trials;
    double pen = 0.0;
    for (uint32_t k = 0; k < a.n_signals; ++k) {
      const double c = a.grid[s * a.n_signals + k];
      pen = pen + c * c;
    }
    const double sc = a.reward * q - a.cost * pen;
    a.score[s] = sc;
    mx = sc > mx ? sc : mx;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double v = __shfl_xor(mx, o, 64);
    mx = v > mx ? v : mx;
  }
  if (lane == 0) red_d[wave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red_d[0];
    for (int w = 1; w < nw; ++w) m = red_d[w] > m ? red_d[w] : m;
    red_d[0] = m;
  }
  __syncthreads();
  const double best = red_d[0];
  if (!a.best) return;

  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  unsigned long long key = ~0ull, cnt = 0;
  for (uint64_t s = threadIdx.x; s < a.n_settings; s += blockDim.x) {
    if (a.score[s] != best) continue;
    ++cnt;
    const Words w = philox(0u, (uint32_t)s, kStreamTie, kStreamTie, k0, k1);
    const unsigned long long kk = ((unsigned long long)w.w0 << 32) | (uint32_t)s;
    key = kk < key ? kk : key;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long v = __shfl_xor(key, o, 64);
    key = v < key ? v : key;
    cnt += __shfl_xor(cnt, o, 64);
  }
  __syncthreads();
  if (lane == 0) {
    red_k[wave] = key;
    red_c[wave] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long k = red_k[0], c = red_c[0];
    for (int w = 1; w < nw; ++w) {
      k = red_k[w] < k ? red_k[w] : k;
      c += red_c[w];
    }
    a.best[0] = (int64_t)(k & 0xFFFFFFFFull);
    a.best[1] = (int64_t)c;
  }
}

}  // namespace

hipError_t launch_score(const ScoreBatch& b, hipStream_t st) {
  if (b.n > kMaxBatch) return hipErrorInvalidValue;
  if (!b.n) return hipSuccess;
  hipLaunchKernelGGL(score_kernel, dim3(b.n), dim3(kScoreBlock), 0, st, b);
  return hipGetLastError();
}

}  // namespace cm
