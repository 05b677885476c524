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
// row and the mass vectors in LDS for all steps; up to eight groups of
// threads split the source cells of each step and add their partial sums.
#include "internal.hpp"

namespace cm {
namespace {

constexpr int kOut = 8;       // consecutive output cells per thread
constexpr int kFPad = 16;     // zero cells in front of the kernel row
constexpr int kMaxThreads = 1024;

__device__ __forceinline__ double Phi(double x) { return 0.5 * erfc(-x * 0.70710678118654752440); }

// A double from another lane: DPP patterns within 16-lane rows (swap pairs,
// swap pairs of pairs, mirror within 8, mirror within 16), lane shuffles
// across rows.  Round r joins the halves of aligned groups of 2^(r+1) lanes.
template <int R>
__device__ __forceinline__ double partner(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
  constexpr int ctrl = R == 0 ? 0xB1 : R == 1 ? 0x4E : R == 2 ? 0x141 : 0x140;
  if constexpr (R < 4) {
    lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, ctrl, 0xF, 0xF, false);
    hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi, ctrl, 0xF, 0xF, false);
  } else {
    lo = (uint32_t)__shfl_xor((int)lo, 1 << R, 64);
    hi = (uint32_t)__shfl_xor((int)hi, 1 << R, 64);
  }
  return __longlong_as_double((long long)((uint64_t)lo | ((uint64_t)hi << 32)));
}

// Sum over the wavefront, the same value in every lane (all lanes active).
__device__ __forceinline__ double wave_sum(double v) {
  v += partner<0>(v);
  v += partner<1>(v);
  v += partner<2>(v);
  v += partner<3>(v);
  v += partner<4>(v);
  v += partner<5>(v);
  return v;
}

// LDS position of kernel-row entry x (x >= -kFPad), u = x + kFPad: one pad
// slot after every 8 entries.  Threads own 8 consecutive output cells, so
// within a wavefront their reads of the row are 8 entries, i.e. 9 slots (18
// banks) apart: no two of them share a bank.  The 8 entries 8m..8m+7 sit
// contiguously at 9m..9m+7, which lets the source loop read them as a group.
__device__ __forceinline__ uint32_t fpos_u(uint32_t u) { return u + (u >> 3); }
__device__ __forceinline__ uint32_t fpos(int x) { return fpos_u((uint32_t)(x + kFPad)); }

// Logical and LDS sizes of the row: 2M - 1 entries after kFPad zeros, and up
// to 8 past them read by the windows of output cells beyond M.
__host__ __device__ inline uint32_t frow_entries(uint32_t M) { return ((2u * M + kFPad + 8u + 7u) / 8u) * 8u; }
__host__ __device__ inline uint32_t frow_slots(uint32_t M) { return frow_entries(M) / 8u * 9u; }
// Rows of the split groups' partial sums use the same padding (cell j at
// j + j/8), so that threads writing 8 consecutive cells do not collide.
__host__ __device__ inline uint32_t prow_slots(uint32_t M) { return (M + M / 8u + 2u) & ~1u; }

// Launch geometry, computed on the host: Q thread groups split the source
// cells of each step, each group has TPQ threads (a multiple of 64 covering
// the ceil(M/8) output blocks), block = Q * TPQ.
__global__ __launch_bounds__(kMaxThreads) void ddm_density_kernel(DensityArgs a) {
  extern __shared__ double sh[];
  __shared__ double red[2][kMaxThreads / 64];
  __shared__ double red_sv[kMaxThreads / 64];
  const uint32_t M = a.cells, tid = threadIdx.x, nt = blockDim.x;
  const uint32_t Q = a.splits, TPQ = nt / Q, q = tid / TPQ, blk = tid - q * TPQ;
  const uint32_t nb = (M + kOut - 1) / kOut;
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  const uint32_t fsize = frow_entries(M);
  double* f = sh;                   // kernel row at fpos, [frow_slots]
  double* m0 = f + frow_slots(M);   // mass vectors [M]
  double* m1 = m0 + M;
  double* part = m1 + M;     // partial sums of the Q splits, [Q][prow_slots]
  const uint32_t PM = prow_slots(M);
  double* upc = part + Q * PM;  // per cell: mass absorbed at the upper bound in one step
  double* loc = upc + M;        // and at the lower bound
  const uint64_t s = blockIdx.x;
  const double drift = a.n_signals ? a.grid[s * a.n_signals] : a.drift;
  const double as = drift * a.dt, b = a.b, th = a.thresh, h = (2.0 * th) / (double)M;
  double* out_lo = a.out + (s * 2u) * a.max_steps;  // choice 0: lower bound
  double* out_up = out_lo + a.max_steps;             // choice 1: upper bound

  // kernel row: entry x = d + (M - 1) is the mass moving d cells up
  for (uint32_t u = tid; u < fsize; u += nt) {
    const int x = (int)u - kFPad;
    double v = 0.0;
    if (x >= 0 && x < (int)(2 * M - 1)) {
      const double k = (double)(x - (int)(M - 1));
      v = Phi(((k + 0.5) * h - as) / b) - Phi(((k - 0.5) * h - as) / b);
    }
    f[fpos_u(u)] = v;
  }
  // absorption tables (in LDS, so that the registers hold the convolution's
  // window and sums)
  for (uint32_t i = tid; i < M; i += nt) {
    const double c = -th + ((double)i + 0.5) * h;
    upc[i] = Phi(-((th - c) - as) / b);
    loc[i] = Phi(((-th - c) - as) / b);
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

  // this thread's share of the convolution: output cells jb..jb+7 from the
  // source cells [i0, i1) of its group
  // Split boundaries after the first sit at sources i = M - 1 (mod 8): there
  // the incoming row entries of every output block start an aligned group,
  // so only the first split has a lead of single sources (and only the last
  // a tail of one).
  auto split_start = [&](uint32_t g) -> uint32_t {
    if (g == 0u) return 0u;
    if (g >= Q) return M;
    const uint32_t base = (g * M) / Q, r = (M - 1u) & 7u;
    return base < r ? 0u : base - ((base - r) & 7u);
  };
  const uint32_t jb = blk * kOut, i0 = split_start(q), i1 = split_start(q + 1u);
  const bool active = blk < nb;
  double* cur = m0;
  double* nxt = m1;
  uint32_t n = 2;
  for (; n <= a.max_steps; ++n) {
    // absorbed at step n
    double pu = 0.0, pl = 0.0;
    for (uint32_t i = tid; i < M; i += nt) {
      pu = fma(cur[i], upc[i], pu);
      pl = fma(cur[i], loc[i], pl);
    }
    pu = wave_sum(pu);
    pl = wave_sum(pl);
    if (lane == 0) {
      red[0][wave] = pu;
      red[1][wave] = pl;
    }
    // survivor mass: a 1-D convolution with the kernel row.  The 8 row
    // entries a thread needs for source cell i slide by one per i, so each
    // LDS read of the row feeds 8 multiply-adds; the source mass cur[i] is
    // the same for the whole wavefront (a broadcast read).
    double acc[kOut];
#pragma unroll
    for (int k = 0; k < kOut; ++k) acc[k] = 0.0;
    if (active) {
      const int x0 = (int)jb - (int)i0 + (int)(M - 1);  // row entry of (jb, i0)
      double w[kOut];
#pragma unroll
      for (int k = 0; k < kOut; ++k) w[k] = f[fpos(x0 + k)];
      // Source i brings in entry x0 - 1 - (i - i0) (>= -1: a zero pad entry
      // at the end).  Sources whose incoming entries fill an aligned group
      // 8m+7 .. 8m are taken 8 at a time: the group is read at once and the
      // window slides by register renaming.  u0 mod 8 is the same for every
      // thread of the split group, so the lead and tail lengths are uniform.
      const uint32_t u0 = (uint32_t)(x0 - 1 + kFPad);
      const uint32_t lead = min((((u0 & 7u) + 1u) & 7u), i1 - i0);
      auto one = [&](uint32_t i) {
        const double c = cur[i];
#pragma unroll
        for (int k = 0; k < kOut; ++k) acc[k] = fma(c, w[k], acc[k]);
#pragma unroll
        for (int k = kOut - 1; k > 0; --k) w[k] = w[k - 1];
        w[0] = f[fpos(x0 - (int)(i - i0) - 1)];
      };
      uint32_t i = i0;
      for (; i < i0 + lead; ++i) one(i);
      auto group = [&](uint32_t i) {
        const uint32_t ub = u0 - (i - i0);  // 8m + 7
        const double* g = f + fpos_u(ub - 7u);
        double nf[8], c8[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          nf[r] = g[r];
          c8[r] = cur[i + r];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
#pragma unroll
          for (int k = 0; k < kOut; ++k) acc[k] = fma(c8[t], w[k], acc[k]);
#pragma unroll
          for (int k = kOut - 1; k > 0; --k) w[k] = w[k - 1];
          w[0] = nf[7 - t];
        }
      };
      // two groups per iteration: the window then returns to its registers
      // every 16 sources rather than every 8 (fewer register moves)
      for (; i + 16u <= i1; i += 16u) {
        group(i);
        group(i + 8u);
      }
      if (i + 8u <= i1) {
        group(i);
        i += 8u;
      }
      for (; i < i1; ++i) one(i);
      double* pq = part + q * PM;
#pragma unroll
      for (int k = 0; k < kOut; ++k)
        if (jb + k < M) pq[fpos_u(jb + k)] = acc[k];
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
    // new mass of every cell: the splits' partial sums in split order, one
    // cell per thread; and the survivor mass, to stop once it is negligible
    double sv = 0.0;
    for (uint32_t j = tid; j < M; j += nt) {
      const uint32_t pj = fpos_u(j);
      double v = part[pj];
      for (uint32_t r = 1; r < Q; ++r) v += part[r * PM + pj];
      nxt[j] = v;
      sv += v;
    }
    sv = wave_sum(sv);
    if (lane == 0) red_sv[wave] = sv;
    // One barrier per step besides the one after the partial sums: the next
    // step's reads of the new mass and writes of partial sums and of red
    // come after it, and every read of this step's partial sums and red
    // comes before it.
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < nw; ++w) tot += red_sv[w];
    double* t = cur;
    cur = nxt;
    nxt = t;
    if (tot < a.tol) break;
  }
  for (uint32_t k = n + 1 + tid; k <= a.max_steps; k += nt) {
    out_up[k - 1] = 0.0;
    out_lo[k - 1] = 0.0;
  }
}

}  // namespace

// LDS: the kernel row (frow_slots), two mass vectors, the partial sums of
// the splits and the two absorption tables.
size_t density_lds_bytes(uint32_t cells, uint32_t splits) {
  return ((size_t)frow_slots(cells) + 4u * (size_t)cells + (size_t)splits * prow_slots(cells)) * sizeof(double);
}

uint32_t density_threads_per_split(uint32_t cells) {
  const uint32_t nb = (cells + kOut - 1) / kOut;
  return ((nb + 63) / 64) * 64;
}

hipError_t launch_ddm_density(const DensityArgs& a, hipStream_t st) {
  const uint32_t tpq = density_threads_per_split(a.cells);
  if (a.splits < 1 || a.splits * tpq > (uint32_t)kMaxThreads) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ddm_density_kernel, dim3((uint32_t)a.n_settings), dim3(a.splits * tpq),
                     density_lds_bytes(a.cells, a.splits), st, a);
  return hipGetLastError();
}

}  // namespace cm
