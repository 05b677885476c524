// prep_score.hpp -- the per-index work of a sweep's preparation and the
// per-sweep score, as device routines shared by their own kernels and by the
// device work queue's persistent kernel (each compilation unit gets its own
// copy of the same code, so both paths compute the same bits).
#pragma once

#include "internal.hpp"
#include "rng.hpp"

namespace cm {
namespace {

__device__ __forceinline__ double logistic(double v) { return 1.0 / (1.0 + exp(-v)); }

// Correct response to stimulus `stim`: the argmax of the relevant pathway (A)
// alone at unit control, lowest index on ties.
__device__ void write_correct(const DriveArgs& a, int stim) {
  const double* WA = a.weights;
  const double* OA = a.weights + 24;
  const int ia = stim / 3;
  double sc[2];
  for (int j = 0; j < 2; ++j) {
    double acc = 0.0;
    for (int k = 0; k < 4; ++k) acc = acc + OA[j * 4 + k] * logistic(a.gain * (WA[k * 3 + ia] + a.bias));
    sc[j] = acc;
  }
  a.correct[stim] = sc[1] > sc[0] ? 1 : 0;
}

// Drive of both accumulators for entry i = 9 * setting + stimulus.
__device__ void write_drive(const DriveArgs& a, uint64_t i) {
  const double* WA = a.weights;
  const double* WB = a.weights + 12;
  const double* OA = a.weights + 24;
  const double* OB = a.weights + 32;
  const uint64_t s = i / 9u;
  const int stim = (int)(i - s * 9u), ia = stim / 3, ib = stim % 3;
  double cA, cB;
  if (a.levels) {  // closed loop: allocation s of the level grid
    const uint32_t L = a.levels, i = (uint32_t)(s / L), k = (uint32_t)(s % L);
    cA = L == 1 ? a.amax : (a.amax * (double)i) / (double)(L - 1);
    cB = L == 1 ? a.amax : (a.amax * (double)k) / (double)(L - 1);
    if (stim == 0) a.norm2[s] = cA * cA + cB * cB;  // the allocation's squared norm, once
  } else {
    cA = a.n_signals ? a.grid[s * a.n_signals] : 1.0;
    cB = a.n_signals ? a.grid[s * a.n_signals + 1] : 1.0;
  }
  double hA[4], hB[4];
  for (int k = 0; k < 4; ++k) {
    hA[k] = logistic((cA * a.gain) * (WA[k * 3 + ia] + a.bias));
    hB[k] = logistic((cB * a.gain) * (WB[k * 3 + ib] + a.bias));
  }
  for (int j = 0; j < 2; ++j) {
    double sA = 0.0, sB = 0.0;
    for (int k = 0; k < 4; ++k) sA = sA + OA[j * 4 + k] * hA[k];
    for (int k = 0; k < 4; ++k) sB = sB + OB[j * 4 + k] * hB[k];
    a.drive[i * 2u + j] = (sA + sB) + a.offset;
  }
}

// Index j of a preparation item's range [hist | stats | extra | tables]:
// zero words first, then one index per correct-table entry (the DDM's one
// entry, the conflict network's nine) and one per (setting, stimulus) drive.
__device__ __forceinline__ void prep_index(const PrepItem& p, uint64_t j) {
  if (j < p.n_hist) {
    p.hist[j] = 0ull;
    return;
  }
  j -= p.n_hist;
  if (j < p.n_stats) {
    p.stats[j] = 0ull;
    return;
  }
  j -= p.n_stats;
  if (j < p.n_extra) {
    p.extra[j] = 0ull;
    return;
  }
  j -= p.n_extra;
  if (p.kind == CM_DDM) {
    p.d.correct[0] = 1;  // the upper boundary is the correct response
  } else if (j < 9) {  // conflict network and its closed loop
    write_correct(p.d, (int)j);
  } else {
    write_drive(p.d, j - 9);
  }
}

// score[s] = reward * (correct[s] / trials) - cost * sum_k c_k^2 in this
// order in double with no fused multiply-add, and the best setting: ties
// broken by the smallest (Philox(seed; 0, s, ~0, ~0).w0, s), so the result
// does not depend on the order in which threads visit the grid or on how
// many there are.  The whole workgroup (NW wavefronts) calls it; red_* are
// LDS arrays of NW entries.
template <int NW>
__device__ __forceinline__ void score_sweep(const ScoreArgs& a, double* red_d, unsigned long long* red_k,
                                            unsigned long long* red_c) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = NW;

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
}  // namespace cm
