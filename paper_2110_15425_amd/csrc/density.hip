// density.hip -- exact first-passage distribution of the discretised DDM.
//
// Instead of simulating thousands of runs, propagate the probability density
// of the walk's state: the Distill paper notes that a drift-diffusion model
// has an analytical solution and that recognising one saves thousands of
// model executions (Sec. 1, Sec. 4.4).  For the Euler-Maruyama walk
// x_n = x_{n-1} + a + b z_n with absorbing bounds +-theta, the survivor mass
// on M cells of (-theta, theta) evolves by a Gaussian transition kernel: the
// mass moving from cell i to cell j depends only on j - i (a convolution),
// and the mass absorbed at either bound from cell i is a Gaussian tail.  The
// first step leaves the exact start point; later steps leave cell centres
// (midpoint rule, error O(h^2)).  One workgroup per setting keeps the kernel
// row, the absorption tables and the mass vector in LDS for all steps.
#include "internal.hpp"

namespace cm {
namespace {

constexpr int kDensBlock = 256;

__device__ __forceinline__ double Phi(double x) { return 0.5 * erfc(-x * 0.70710678118654752440); }

__global__ __launch_bounds__(kDensBlock) void ddm_density_kernel(DensityArgs a) {
  extern __shared__ double sh[];
  __shared__ double red[2][kDensBlock / 64];
  const uint32_t M = a.cells, tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  double* f = sh;             // [2M - 1] (+4 zero pad), offset k = d - (M - 1)
  double* up = f + (2 * M + 3);
  double* lo = up + M;
  double* m0 = lo + M;
  double* m1 = m0 + M;
  const uint64_t s = blockIdx.x;
  const double drift = a.n_signals ? a.grid[s * a.n_signals] : a.drift;
  const double as = drift * a.dt, b = a.b, th = a.thresh, h = (2.0 * th) / (double)M;
  double* out_lo = a.out + (s * 2u) * a.max_steps;  // choice 0: lower bound
  double* out_up = out_lo + a.max_steps;             // choice 1: upper bound

  for (uint32_t d = tid; d < 2 * M + 3; d += nt) {
    const double k = (double)((int)d - (int)(M - 1));
    f[d] = d < 2 * M - 1 ? Phi(((k + 0.5) * h - as) / b) - Phi(((k - 0.5) * h - as) / b) : 0.0;
  }
  for (uint32_t i = tid; i < M; i += nt) {
    const double c = -th + ((double)i + 0.5) * h;
    up[i] = Phi(-((th - c) - as) / b);
    lo[i] = Phi(((-th - c) - as) / b);
    // first step from the start point, exact
    const double x0 = a.start;
    const double e0 = -th + (double)i * h, e1 = -th + (double)(i + 1) * h;
    m0[i] = Phi(((e1 - x0) - as) / b) - Phi(((e0 - x0) - as) / b);
  }
  if (tid == 0) {
    out_up[0] = Phi(-((th - a.start) - as) / b);
    out_lo[0] = Phi(((-th - a.start) - as) / b);
  }
  __syncthreads();

  double* cur = m0;
  double* nxt = m1;
  uint32_t n = 2;
  for (; n <= a.max_steps; ++n) {
    // absorbed at step n, and the survivor mass after it
    double pu = 0.0, pl = 0.0;
    for (uint32_t i = tid; i < M; i += nt) {
      pu = fma(cur[i], up[i], pu);
      pl = fma(cur[i], lo[i], pl);
    }
    for (int o = 32; o > 0; o >>= 1) {
      pu += __shfl_xor(pu, o, 64);
      pl += __shfl_xor(pl, o, 64);
    }
    if (lane == 0) {
      red[0][wave] = pu;
      red[1][wave] = pl;
    }
    // new mass: a 1-D convolution of the mass with the kernel row.  Each
    // thread produces 4 consecutive cells; the 4 kernel values it needs for
    // source cell i are a window sliding by one per i, so each LDS read of
    // the kernel row feeds 4 multiply-adds.
    for (uint32_t jb = 4u * tid; jb < M; jb += 4u * nt) {
      const double* fw = f + (M - 1) + jb;  // fw[q - i] = f[j - i + M - 1] for j = jb + q
      double w0 = fw[0], w1 = fw[1], w2 = fw[2], w3 = fw[3];
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      for (uint32_t i = 0; i < M; ++i) {
        const double c = cur[i];
        a0 = fma(c, w0, a0);
        a1 = fma(c, w1, a1);
        a2 = fma(c, w2, a2);
        a3 = fma(c, w3, a3);
        w3 = w2;
        w2 = w1;
        w1 = w0;
        w0 = (i + 1u < M) ? fw[-(int)(i + 1u)] : 0.0;
      }
      nxt[jb] = a0;
      if (jb + 1u < M) nxt[jb + 1u] = a1;
      if (jb + 2u < M) nxt[jb + 2u] = a2;
      if (jb + 3u < M) nxt[jb + 3u] = a3;
    }
    __syncthreads();
    if (tid == 0) {
      double su = 0.0, sl = 0.0;
      for (int w = 0; w < nw; ++w) {
        su += red[0][w];
        sl += red[1][w];
      }
      out_up[n - 1] = su;
      out_lo[n - 1] = sl;
    }
    // survivor mass: stop once it is negligible
    double sv = 0.0;
    for (uint32_t j = tid; j < M; j += nt) sv += nxt[j];
    for (int o = 32; o > 0; o >>= 1) sv += __shfl_xor(sv, o, 64);
    __syncthreads();
    if (lane == 0) red[0][wave] = sv;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < nw; ++w) tot += red[0][w];
    double* t = cur;
    cur = nxt;
    nxt = t;
    if (tot < a.tol) break;
    __syncthreads();
  }
  for (uint32_t k = n + 1 + tid; k <= a.max_steps; k += nt) {
    out_up[k - 1] = 0.0;
    out_lo[k - 1] = 0.0;
  }
}

}  // namespace

hipError_t launch_ddm_density(const DensityArgs& a, hipStream_t st) {
  const size_t lds = (size_t)(2 * a.cells + 3 + 4 * a.cells) * sizeof(double);
  hipLaunchKernelGGL(ddm_density_kernel, dim3((uint32_t)a.n_settings), dim3(kDensBlock), lds, st, a);
  return hipGetLastError();
}

}  // namespace cm
