// prep.hip -- per-sweep preparation, all sweeps of a launch in one kernel:
// output zero-fill, the correct-response table and the conflict network's
// feed-forward drive.
//
// The drive of each accumulator depends only on (setting, stimulus), not on
// the step, so it is evaluated once per pair instead of once per step: the
// loop-invariant motion across model nodes that the Distill paper credits to
// model-wide optimisation (Sec. 3.5).  The network is two one-hot 3-unit
// inputs -> two 4-unit logistic hidden layers whose gain the pathway's
// control signal multiplies -> [2x4] projections summed onto the two
// accumulators (logistic transfer and projections, Sec. 3.4.2).
#include <algorithm>

#include "internal.hpp"

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

// One thread per launch index.  An item's range is [hist | stats | extra | tables]:
// zero words first, then one index per correct-table entry (the DDM's one
// entry, the conflict network's nine) and one per (setting, stimulus) drive.
__global__ void prep_kernel(PrepBatch b) {
  const uint64_t total = b.it[b.n - 1].end;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t k = 0;
    while (i >= b.it[k].end) ++k;
    const PrepItem& p = b.it[k];
    uint64_t j = i - (k ? b.it[k - 1].end : 0);
    if (j < p.n_hist) {
      p.hist[j] = 0ull;
      continue;
    }
    j -= p.n_hist;
    if (j < p.n_stats) {
      p.stats[j] = 0ull;
      continue;
    }
    j -= p.n_stats;
    if (j < p.n_extra) {
      p.extra[j] = 0ull;
      continue;
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
}

}  // namespace

hipError_t launch_prep(const PrepBatch& b, hipStream_t st) {
  if (b.n < 1 || b.n > kMaxBatch) return hipErrorInvalidValue;
  const uint64_t total = b.it[b.n - 1].end;
  if (!total) return hipSuccess;
  const uint64_t g = std::min<uint64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(prep_kernel, dim3((uint32_t)g), dim3(256), 0, st, b);
  return hipGetLastError();
}

}  // namespace cm
