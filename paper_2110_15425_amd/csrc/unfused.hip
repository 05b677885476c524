// unfused.hip -- the same sweep executed node by node (ablation).
//
// The Distill paper contrasts compiling each model node separately, with the
// scheduler still switching between nodes, against compiling the whole model
// with its scheduler (Sec. 6.2: 3.4x vs 778x over CPython).  This file is the
// GPU analogue of the per-node design: every mechanism of a step is its own
// kernel -- random numbers, the accumulator update, the threshold test with
// compaction of the still-active runs -- with all run state in HBM between
// kernels and the host driving the step loop.  It computes exactly what the
// fused kernels compute (same operations in the same order, so identical
// results); only the execution structure differs.
#include "internal.hpp"
#include "lca_step.hpp"
#include "rng.hpp"

namespace cm {
namespace {

constexpr int kUfBlock = 256;

__device__ __forceinline__ bool near_th(double q, double th, double eps) {
  return fabs(q - th) < eps;
}

__device__ __forceinline__ void run_index(const UnfusedArgs& a, uint32_t r, uint32_t& s, uint32_t& t) {
  s = (uint32_t)(r / a.trials);
  t = (uint32_t)(r - (uint64_t)s * a.trials);
}

__global__ void uf_init_kernel(UnfusedArgs a) {
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.total_runs;
       r += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t s, t;
    run_index(a, (uint32_t)r, s, t);
    a.x[2 * r] = a.kind == CM_DDM ? a.start : 0.0;
    a.x[2 * r + 1] = 0.0;
    a.n[r] = 0;
    a.flag[r] = 0;
    a.choice[r] = -1;
    a.active[r] = (uint32_t)r;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.count[0] = (uint32_t)a.total_runs;
    a.count[1] = 0;
  }
}

// Node 1: random numbers of step n for every active run.
template <int PREC>
__global__ void uf_rng_kernel(UnfusedArgs a, uint32_t n, int cur) {
  const uint32_t cnt = a.count[cur];
  const uint32_t* act = a.active + (uint64_t)cur * a.total_runs;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
    const uint32_t r = act[i];
    uint32_t s, t;
    run_index(a, r, s, t);
    const uint32_t k = a.kind == CM_DDM ? (n - 1u) >> 1 : n - 1u;
    const Words w = philox(k, t, s, 0u, k0, k1);
    if (PREC == CM_FP64) {
      double z0, z1;
      normals64(w, z0, z1);
      if (a.kind == CM_DDM) {
        a.z[2 * (uint64_t)r] = ((n - 1u) & 1u) ? z1 : z0;
      } else {
        a.z[2 * (uint64_t)r] = z0;
        a.z[2 * (uint64_t)r + 1] = z1;
      }
    } else {
      float z0, z1;
      normals32(w, z0, z1);
      if (a.kind == CM_DDM) {
        a.z[2 * (uint64_t)r] = (double)(((n - 1u) & 1u) ? z1 : z0);
      } else {
        a.z[2 * (uint64_t)r] = (double)z0;
        a.z[2 * (uint64_t)r + 1] = (double)z1;
      }
    }
  }
}

// Node 2: the accumulator update.
template <int PREC>
__global__ void uf_update_kernel(UnfusedArgs a, int cur) {
  const uint32_t cnt = a.count[cur];
  const uint32_t* act = a.active + (uint64_t)cur * a.total_runs;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
    const uint32_t r = act[i];
    uint32_t s, t;
    run_index(a, r, s, t);
    double* x = a.x + 2 * (uint64_t)r;
    const double* z = a.z + 2 * (uint64_t)r;
    if (a.kind == CM_DDM) {
      const double drift = a.n_signals ? a.grid[(uint64_t)s * a.n_signals] : a.drift;
      const double as = drift * a.dt;
      if (PREC == CM_FP64) x[0] = (x[0] + as) + a.b * z[0];
      else x[0] = x[0] + (double)fmaf((float)a.b, (float)z[0], (float)as);
    } else {
      const uint32_t stim = t % 9u;
      const double* d = a.drive + ((uint64_t)s * 9u + stim) * 2u;
      double y0, y1;
      if (PREC == CM_FP64) {
        y0 = (x[0] + (((d[0] - a.leak * x[0]) - a.comp * x[1]) * a.dt)) + a.b * z[0];
        y1 = (x[1] + (((d[1] - a.leak * x[1]) - a.comp * x[0]) * a.dt)) + a.b * z[1];
      } else {
        const LcaF32 pf = lca_f32(a.leak, a.comp, a.dt, a.b);
        const float xf0 = (float)x[0], xf1 = (float)x[1];
        y0 = x[0] + (double)lca_inc_f32(pf, (float)(d[0] * a.dt), xf0, xf1, (float)z[0]);
        y1 = x[1] + (double)lca_inc_f32(pf, (float)(d[1] * a.dt), xf1, xf0, (float)z[1]);
      }
      if (a.nonneg) {
        if (y0 < 0.0) y0 = 0.0;
        if (y1 < 0.0) y1 = 0.0;
      }
      x[0] = y0;
      x[1] = y1;
    }
  }
}

// Node 3: threshold test and compaction of the runs that go on.
__global__ void uf_check_kernel(UnfusedArgs a, uint32_t n, int cur) {
  const uint32_t cnt = a.count[cur];
  const uint32_t* act = a.active + (uint64_t)cur * a.total_runs;
  uint32_t* nxt = a.active + (uint64_t)(1 - cur) * a.total_runs;
  const double th = a.thresh, eps = a.flag_eps;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
    const uint32_t r = act[i];
    const double* x = a.x + 2 * (uint64_t)r;
    bool done = false;
    int c = -1;
    bool fl = false;
    if (a.kind == CM_DDM) {
      fl = near_th(x[0], th, eps) || near_th(x[0], -th, eps);
      if (x[0] >= th) { c = 1; done = true; }
      else if (x[0] <= -th) { c = 0; done = true; }
    } else {
      fl = near_th(x[0], th, eps) || near_th(x[1], th, eps);
      const double mx = x[0] > x[1] ? x[0] : x[1];
      if (mx >= th) {
        c = x[1] > x[0] ? 1 : 0;
        if (fabs(x[0] - x[1]) < eps) fl = true;
        done = true;
      }
    }
    if (!done && n == a.max_steps) done = true;
    if (fl) a.flag[r] = 1;
    a.n[r] = n;
    if (done) a.choice[r] = (int8_t)c;
    else nxt[atomicAdd(&a.count[1 - cur], 1u)] = r;
  }
}

__global__ void uf_reset_kernel(uint32_t* count, int idx) { count[idx] = 0; }

// Reduction of the per-run outcomes into histograms and statistics.
__global__ void uf_reduce_kernel(UnfusedArgs a) {
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.total_runs;
       r += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t s, t;
    run_index(a, (uint32_t)r, s, t);
    const int c = a.choice[r];
    const uint32_t nn = a.n[r];
    uint64_t* st = a.stats + (uint64_t)s * CM_NSTAT;
    const int target = a.kind == CM_DDM ? 1 : a.correct[t % 9u];
    if (c >= 0) {
      const uint32_t bin = ((nn - 1u) * a.n_bins) / a.max_steps;
      atomicAdd((unsigned long long*)&a.hist[((uint64_t)s * 2u + c) * a.n_bins + bin], 1ull);
      atomicAdd((unsigned long long*)&st[CM_ST_DEC0 + c], 1ull);
      atomicAdd((unsigned long long*)&st[CM_ST_SUMN0 + c], (unsigned long long)nn);
      atomicAdd((unsigned long long*)&st[CM_ST_SUMSQ0 + c], (unsigned long long)nn * nn);
      if (c == target) atomicAdd((unsigned long long*)&st[CM_ST_CORRECT], 1ull);
    } else {
      atomicAdd((unsigned long long*)&st[CM_ST_UNDEC], 1ull);
    }
    if (a.flag[r]) atomicAdd((unsigned long long*)&st[CM_ST_FLAGGED], 1ull);
    if (a.run_choice) {
      a.run_choice[r] = (int8_t)c;
      a.run_step[r] = nn;
      a.run_flag[r] = a.flag[r];
      if (a.run_state) {
        const int width = a.kind == CM_DDM ? 1 : 2;
        for (int i = 0; i < width; ++i) a.run_state[r * width + i] = a.x[2 * r + i];
      }
    }
  }
}

uint32_t grid_of(uint64_t n) {
  uint64_t g = (n + kUfBlock - 1) / kUfBlock;
  return (uint32_t)(g < 1 ? 1 : (g > 65535 ? 65535 : g));
}

}  // namespace

hipError_t launch_uf_init(const UnfusedArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(uf_init_kernel, dim3(grid_of(a.total_runs)), dim3(kUfBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_uf_step(const UnfusedArgs& a, int precision, uint32_t n, int cur, uint64_t bound,
                          hipStream_t st) {
  const dim3 g(grid_of(bound)), b(kUfBlock);
  if (precision == CM_FP64) hipLaunchKernelGGL((uf_rng_kernel<CM_FP64>), g, b, 0, st, a, n, cur);
  else hipLaunchKernelGGL((uf_rng_kernel<CM_FP32_STEP>), g, b, 0, st, a, n, cur);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (precision == CM_FP64) hipLaunchKernelGGL((uf_update_kernel<CM_FP64>), g, b, 0, st, a, cur);
  else hipLaunchKernelGGL((uf_update_kernel<CM_FP32_STEP>), g, b, 0, st, a, cur);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(uf_check_kernel, g, b, 0, st, a, n, cur);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(uf_reset_kernel, dim3(1), dim3(1), 0, st, a.count, cur);
  return hipGetLastError();
}

hipError_t launch_uf_reduce(const UnfusedArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(uf_reduce_kernel, dim3(grid_of(a.total_runs)), dim3(kUfBlock), 0, st, a);
  return hipGetLastError();
}

}  // namespace cm
