// prep.hip -- per-sweep preparation kernels: output zero-fill and the
// conflict network's feed-forward drive.
//
// The drive of each accumulator depends only on (setting, stimulus), not on
// the step, so it is evaluated once per pair instead of once per step: the
// loop-invariant motion across model nodes that the Distill paper credits to
// model-wide optimisation (Sec. 3.5).  The network is two one-hot 3-unit
// inputs -> two 4-unit logistic hidden layers whose gain the pathway's
// control signal multiplies -> [2x4] projections summed onto the two
// accumulators (logistic transfer and projections, Sec. 3.4.2).
#include "internal.hpp"

namespace cm {
namespace {

__global__ void zero_u64_kernel(uint64_t* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void fill_i32_kernel(int32_t* p, uint64_t n, int32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__device__ __forceinline__ double logistic(double v) { return 1.0 / (1.0 + exp(-v)); }

// One thread per (setting, stimulus); block 0 also writes the correct
// response per stimulus: the argmax of the relevant pathway (A) alone at
// unit control, lowest index on ties.
__global__ void drive_kernel(DriveArgs a) {
  const double* WA = a.weights;
  const double* WB = a.weights + 12;
  const double* OA = a.weights + 24;
  const double* OB = a.weights + 32;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x < 9) {
    const int ia = threadIdx.x / 3;
    double sc[2];
    for (int j = 0; j < 2; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 4; ++k) acc = acc + OA[j * 4 + k] * logistic(a.gain * (WA[k * 3 + ia] + a.bias));
      sc[j] = acc;
    }
    a.correct[threadIdx.x] = sc[1] > sc[0] ? 1 : 0;
  }
  if (i >= a.n_settings * 9u) return;
  const uint64_t s = i / 9u;
  const int stim = (int)(i - s * 9u), ia = stim / 3, ib = stim % 3;
  const double cA = a.n_signals ? a.grid[s * a.n_signals] : 1.0;
  const double cB = a.n_signals ? a.grid[s * a.n_signals + 1] : 1.0;
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

uint32_t grid_for(uint64_t n, uint32_t block) {
  uint64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65535) g = 65535;
  return (uint32_t)g;
}

}  // namespace

hipError_t launch_zero_u64(uint64_t* p, uint64_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(zero_u64_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, uint64_t n, int32_t v, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_drive(const DriveArgs& a, hipStream_t st) {
  const uint64_t n = a.n_settings * 9u;
  hipLaunchKernelGGL(drive_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace cm
