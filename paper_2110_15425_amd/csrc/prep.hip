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

#include "prep_score.hpp"

namespace cm {
namespace {

// One thread per launch index.  An item's range is [hist | stats | extra | tables].
__global__ void prep_kernel(PrepBatch b) {
  const uint64_t total = b.it[b.n - 1].end;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t k = 0;
    while (i >= b.it[k].end) ++k;
    prep_index(b.it[k], i - (k ? b.it[k - 1].end : 0));
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
