// density.hip -- exact first-passage distribution of the discretised DDM.
//
// Instead of simulating thousands of runs, propagate the probability density
// of the walk's state: the Distill paper notes that a drift-diffusion model
// has an analytical solution and that recognising one saves thousands of
// model executions (Sec. 1, Sec. 4.4).  For the Euler-Maruyama walk
// x_n = x_{n-1} + a + b z_n with absorbing bounds +-theta, the survivor mass
// on M cells of (-theta, theta) evolves by a Gaussian transition kernel: the
// mass moving from cell i to cell j depends only on j - i (a Toeplitz
// matrix T), and the mass absorbed at either bound from cell i is a Gaussian
// tail.  The first step leaves the exact start point; later steps leave cell
// centres (midpoint rule, error O(h^2)).
//
// One workgroup per setting keeps the kernel row and the mass vectors in LDS
// for all steps.  The product T m is a dense contraction on the FP64 matrix
// cores: with cells grouped in blocks of 16, block-diagonal d of T is one
// 16x16 matrix F_d (F_d[alpha][gamma] = f(16 d + alpha - gamma)), so
//   y_block(a) = sum_d F_d m_block(a - d),
// i.e. for every d a 16x16 by 16 x (blocks) product.  Each 16x16x4 product
// takes its F_d fragment straight from the kernel row in LDS and its mass
// fragment from the (zero-padded) mass vector.  Block-diagonals whose
// entries are all below 2^-60 (the Gaussian's far tails, at most 2^-60 of a
// row's mass each) are skipped, as are blocks whose mass columns lie outside
// the grid.  Wavefront (tile t, group g) accumulates the output columns
// 16 t .. 16 t + 15 over its share (the g-th of G contiguous ranges) of the
// block-diagonals; the groups' partial sums are added in group order
// through LDS.
#include "internal.hpp"

namespace cm {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxThreads = 1024;
constexpr int kBS = 17;  // LDS slots per 16-cell block of a mass vector (one pad)
constexpr int kWin = 16; // steps whose sums are reduced together

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

// Sum over the 16-lane row, the same value in every lane of the row.
__device__ __forceinline__ double row_sum(double v) {
  v += partner<0>(v);
  v += partner<1>(v);
  v += partner<2>(v);
  v += partner<3>(v);
  return v;
}

__device__ __forceinline__ int floor_div16(int v) { return v >= 0 ? v / 16 : -((15 - v) / 16); }
__device__ __forceinline__ int ceil_div16(int v) { return -floor_div16(-v); }

}  // namespace

// Launch geometry of M cells: NB blocks of 16 cells, NT output tiles of 16
// blocks, G wavefronts per tile (W = NT G, 6 to 12; measured on MI355X at
// 1000 cells, four tiles: with every fragment read from LDS, 2 per tile 5 %
// faster than 4 and 1 per tile 25 % slower; with the kernel fragments of
// the first diagonals in registers, 3 per tile (12 diagonals each) 2 %
// faster than 2 (24 each) and 4 (6 each)), the
// kernel row's offset
// FOFF (entry of displacement 0) and width FW, and CB blocks per mass vector
// (NB zero blocks on either side of the 16 NT output blocks).
struct DensityGeo {
  uint32_t M, NB, NT, G, W, FOFF, FW, CB;
};
__host__ __device__ inline DensityGeo density_geo(uint32_t M) {
  DensityGeo g;
  g.M = M;
  g.NB = (M + 15u) / 16u;
  g.NT = (g.NB + 15u) / 16u;
  g.G = g.NT == 4u ? 3u : 8u / g.NT > 2u ? 8u / g.NT : 2u;
  g.W = g.NT * g.G;
  g.FOFF = 16u * g.NB + 16u;
  g.FW = 2u * g.FOFF + 1u;
  g.CB = 16u * g.NT + 2u * g.NB;
  return g;
}

namespace {

// MAXT: workgroup size bound; REGD: diagonals per wavefront whose kernel
// fragments stay in registers (at two wavefronts per SIMD a wavefront's 256
// registers hold 24 diagonals' fragments beside the rest, at three 12;
// measured on MI355X at 1000 cells: 6 % faster than reading them from LDS
// every step.
// One wavefront per tile with 48 diagonals in registers and the accumulator
// as the new mass -- no partial sums, one barrier per step -- was 8 % slower
// than reading everything from LDS, with one accumulation chain or two).
template <int MAXT, int REGD>
__global__ __launch_bounds__(MAXT) void ddm_density_kernel(DensityArgs a) {
  extern __shared__ double sh[];
  __shared__ double red[3][kMaxThreads / 64];
  __shared__ double wsum[3][kWin];
  __shared__ int band[2];
  const DensityGeo geo = density_geo(a.cells);
  const uint32_t M = geo.M, NB = geo.NB, NT = geo.NT, G = geo.G;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const int lane = (int)(tid & 63u), wave = (int)(tid >> 6), nw = (int)(nt >> 6);
  double* f = sh;                       // kernel row: f[FOFF + delta], [FW]
  double* m0 = f + geo.FW;              // mass vectors, block c at (c + NB) * kBS
  double* m1 = m0 + geo.CB * kBS;
  double* part = m1 + geo.CB * kBS;     // partial sums [G][NT][4][64]
  // per step of a window: the 16-lane rows' sums of the new mass, and of the
  // mass the next step absorbs at either bound, [kWin][3][rows]
  double* ring = part + G * NT * 256u;
  const uint64_t s = blockIdx.x;
  const double drift = a.n_signals ? a.grid[s * a.n_signals] : a.drift;
  const double as = drift * a.dt, b = a.b, th = a.thresh, h = (2.0 * th) / (double)M;
  double* out_lo = a.out + (s * 2u) * a.max_steps;  // choice 0: lower bound
  double* out_up = out_lo + a.max_steps;             // choice 1: upper bound

  if (tid == 0) {
    band[0] = 0x7FFFFFFF;
    band[1] = -0x7FFFFFFF;
  }
  for (uint32_t i = tid; i < 2u * geo.CB * kBS; i += nt) m0[i] = 0.0;
  __syncthreads();
  // kernel row: entry delta is the mass moving delta cells up; the band of
  // displacements whose entries reach 2^-60
  for (uint32_t x = tid; x < geo.FW; x += nt) {
    const int d = (int)x - (int)geo.FOFF;
    double v = 0.0;
    if (d > -(int)M && d < (int)M) {
      const double k = (double)d;
      v = Phi(((k + 0.5) * h - as) / b) - Phi(((k - 0.5) * h - as) / b);
    }
    f[x] = v;
    if (v >= 0x1p-60) {
      atomicMin(&band[0], d);
      atomicMax(&band[1], d);
    }
  }
  // This thread's output slots: slot t is register r of lane l of tile tt's
  // accumulator, cell 16 (16 tt + l % 16) + 4 r + l / 16 (the 16x16x4 FP64
  // accumulator holds row 4 r + l / 16, column l % 16).  Their absorption
  // tables stay in registers; the first step's mass comes from the start
  // point exactly.
  constexpr int kSlots = 2;
  double upc[kSlots], loc[kSlots];
  uint32_t pos[kSlots];
  bool real[kSlots];
  double pu = 0.0, pl = 0.0;
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    const uint32_t t = tid + (uint32_t)k * nt;
    const uint32_t tt = t >> 8, r = (t >> 6) & 3u, l = t & 63u;
    const uint32_t blk = 16u * tt + (l & 15u), j = 16u * blk + 4u * r + (l >> 4);
    real[k] = t < 256u * NT && j < M;
    pos[k] = (blk + NB) * kBS + 4u * r + (l >> 4);
    upc[k] = loc[k] = 0.0;
    if (real[k]) {
      const double c = -th + ((double)j + 0.5) * h;
      upc[k] = Phi(-((th - c) - as) / b);
      loc[k] = Phi(((-th - c) - as) / b);
      const double e0 = -th + (double)j * h, e1 = -th + (double)(j + 1) * h;
      const double v = Phi(((e1 - a.start) - as) / b) - Phi(((e0 - a.start) - as) / b);
      m0[pos[k]] = v;
      pu = fma(v, upc[k], pu);
      pl = fma(v, loc[k], pl);
    }
  }
  pu = wave_sum(pu);
  pl = wave_sum(pl);
  if (lane == 0) {
    red[1][wave] = pu;
    red[2][wave] = pl;
  }
  __syncthreads();
  if (tid == 0) {
    out_up[0] = Phi(-((th - a.start) - as) / b);
    out_lo[0] = Phi(((-th - a.start) - as) / b);
    if (a.max_steps >= 2u) {
      double su = 0.0, sl = 0.0;
      for (int w = 0; w < nw; ++w) {
        su += red[1][w];
        sl += red[2][w];
      }
      out_up[1] = su;
      out_lo[1] = sl;
    }
  }
  // Block-diagonals holding an entry of the band (diagonal d covers
  // displacements 16 d - 15 .. 16 d + 15) whose mass blocks a - d, for the
  // columns a of this wavefront's tile, reach the grid: a contiguous range,
  // split into G contiguous shares, one per group.  All wave-uniform.
  // (the lowest d with 16 d + 15 >= band[0], the highest with 16 d - 15 <= band[1])
  const int dlo = ceil_div16(band[0] - 15), dhi = floor_div16(band[1] + 15);
  const uint32_t wv = __builtin_amdgcn_readfirstlane((uint32_t)wave);
  const uint32_t tile = wv / G, grp = wv - tile * G;
  const int nbi = (int)NB, c0 = 16 * (int)tile;
  const int dA = max(dlo, c0 - nbi + 1), dB = min(dhi, min(c0 + 15, nbi - 1));
  const int nd = dB >= dA ? dB - dA + 1 : 0;
  const int dS = dA + (nd * (int)grp) / (int)G, dE = dA + (nd * ((int)grp + 1)) / (int)G;
  const int l16 = lane & 15, l4 = lane >> 4;
  // The kernel row does not change from step to step: the F_d fragments of
  // this wavefront's first REGD diagonals stay in registers, so each step
  // reads only their mass fragments from LDS.
  const double* fa = f + (int)geo.FOFF + l16 - l4;
  double Ar[REGD > 0 ? REGD : 1][4];
#pragma unroll
  for (int i = 0; i < REGD; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) Ar[i][q] = dS + i < dE ? fa[16 * (dS + i) - 4 * q] : 0.0;
  double* cur = m0;
  double* nxt = m1;
  uint32_t n = 2;
  for (; n <= a.max_steps; ++n) {
    // (A) this wavefront's share of T m on the matrix cores; the fragments
    // of the next diagonal are read while the current products run
    f64x4 C = {0.0, 0.0, 0.0, 0.0};
    if (tile < NT) {
      const double* mb = cur + (c0 + l16 + nbi) * kBS + l4;
      double A[4], B[4];
      if (dS < dE) {
#pragma unroll
        for (int q = 0; q < 4; ++q) B[q] = mb[4 * q - dS * kBS];
      }
      // two mass-fragment buffers in turn, so that the next diagonal's
      // fragments are read while this diagonal's products run
      double B1[4];
#pragma unroll
      for (int i = 0; i < REGD; ++i) {
        const int d = dS + i;
        if (d < dE) {
          double* cu = (i & 1) ? B1 : B;
          double* nx = (i & 1) ? B : B1;
          const int dn = d + 1 < dE ? d + 1 : d;
#pragma unroll
          for (int q = 0; q < 4; ++q) nx[q] = mb[4 * q - dn * kBS];
#pragma unroll
          for (int q = 0; q < 4; ++q) C = __builtin_amdgcn_mfma_f64_16x16x4f64(Ar[i][q], cu[q], C, 0, 0, 0);
        }
      }
      if (REGD & 1) {  // the last register diagonal left the next fragments in B1
#pragma unroll
        for (int q = 0; q < 4; ++q) B[q] = B1[q];
      }
      const int dR = dS + REGD;  // the rest, fragments of both operands from LDS
      if (dR < dE) {
#pragma unroll
        for (int q = 0; q < 4; ++q) A[q] = fa[16 * dR - 4 * q];
      }
      for (int d = dR; d < dE; ++d) {
        double An[4], Bn[4];
        const int dn = d + 1 < dE ? d + 1 : d;  // the last diagonal re-reads its own
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          An[q] = fa[16 * dn - 4 * q];
          Bn[q] = mb[4 * q - dn * kBS];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) C = __builtin_amdgcn_mfma_f64_16x16x4f64(A[q], B[q], C, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          A[q] = An[q];
          B[q] = Bn[q];
        }
      }
      double* pw = part + ((grp * NT + tile) * 4u) * 64u + (uint32_t)lane;
#pragma unroll
      for (int r = 0; r < 4; ++r) pw[r * 64] = C[r];
    }
    __syncthreads();
    // (B) the new mass: the groups' partial sums in group order; its total
    // and the mass it will lose at either bound in the next step
    double sv = 0.0;
    pu = 0.0;
    pl = 0.0;
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
      const uint32_t t = tid + (uint32_t)k * nt;
      if (t < 256u * NT) {
        const double* pr = part + t;  // [grp][tile][r][l] with (tile, r, l) = t
        double v = pr[0];
        for (uint32_t g = 1; g < G; ++g) v += pr[g * NT * 256u];
        if (!real[k]) v = 0.0;
        nxt[pos[k]] = v;
        sv += v;
        pu = fma(v, upc[k], pu);
        pl = fma(v, loc[k], pl);
      }
    }
    // 16-lane row sums into the window's ring; whole sums once a window is
    // full (the stop test and the absorbed masses need no per-step barrier
    // of their own)
    const uint32_t rows = nt >> 4, k = (n - 2u) % kWin;
    sv = row_sum(sv);
    pu = row_sum(pu);
    pl = row_sum(pl);
    if ((lane & 15) == 0) {
      double* rw = ring + (k * 3u) * rows + (tid >> 4);
      rw[0] = sv;
      rw[rows] = pu;
      rw[2u * rows] = pl;
    }
    // Reads of this step's partial sums and writes of the new mass come
    // before this barrier; the next step's products read the new mass and
    // overwrite the partial sums after it.
    __syncthreads();
    double* t = cur;
    cur = nxt;
    nxt = t;
    if (k == kWin - 1u || n == a.max_steps) {
      // window steps n0 .. n: whole sums in row order, one per thread
      const uint32_t cnt = k + 1u, n0 = n - k;
      if (tid < 3u * cnt) {
        const uint32_t q = tid / cnt, kk = tid - q * cnt;
        const double* rw = ring + (kk * 3u + q) * rows;
        double v = 0.0;
        for (uint32_t r = 0; r < rows; ++r) v += rw[r];
        wsum[q][kk] = v;
      }
      __syncthreads();
      // the first step of the window whose survivor mass is below tol
      uint32_t stop = cnt;
      for (uint32_t kk = 0; kk < cnt; ++kk)
        if (wsum[0][kk] < a.tol) {
          stop = kk;
          break;
        }
      // absorbed at step m + 1, for the window's steps m before the stop
      if (tid < stop) {
        const uint32_t m = n0 + tid;
        if (m < a.max_steps) {
          out_up[m] = wsum[1][tid];
          out_lo[m] = wsum[2][tid];
        }
      }
      if (stop < cnt) {
        n = n0 + stop;
        break;
      }
    }
  }
  if (n > a.max_steps) n = a.max_steps + 1u;
  // after a stop at step n, steps n + 1 .. N absorb nothing
  for (uint32_t k = n + tid; k < a.max_steps; k += nt) {
    out_up[k] = 0.0;
    out_lo[k] = 0.0;
  }
}

}  // namespace

// LDS: the kernel row, two zero-padded mass vectors, the partial sums and
// the window's row sums.
size_t density_lds_bytes(uint32_t cells) {
  const DensityGeo g = density_geo(cells);
  return ((size_t)g.FW + 2u * (size_t)g.CB * kBS + (size_t)g.G * g.NT * 256u +
          (size_t)kWin * 3u * (g.W * 64u / 16u)) * sizeof(double);
}

hipError_t launch_ddm_density(const DensityArgs& a, hipStream_t st) {
  const DensityGeo g = density_geo(a.cells);
  if (a.cells < 16u || g.W * 64u > (uint32_t)kMaxThreads || 2u * g.W * 64u < 256u * g.NT)
    return hipErrorInvalidValue;
  if (g.NT == 4u)
    hipLaunchKernelGGL((ddm_density_kernel<768, 12>), dim3((uint32_t)a.n_settings), dim3(g.W * 64u),
                       density_lds_bytes(a.cells), st, a);
  else if (g.W <= 8u)
    hipLaunchKernelGGL((ddm_density_kernel<512, 24>), dim3((uint32_t)a.n_settings), dim3(g.W * 64u),
                       density_lds_bytes(a.cells), st, a);
  else
    hipLaunchKernelGGL((ddm_density_kernel<kMaxThreads, 0>), dim3((uint32_t)a.n_settings), dim3(g.W * 64u),
                       density_lds_bytes(a.cells), st, a);
  return hipGetLastError();
}

}  // namespace cm
