// rnn.hip -- the recurrent logistic rate network on matrix cores.
//
// Each run steps n logistic rate units coupled by a weight-matrix
// projection (the logistic transfer and projections of Distill, Sec. 3.4.2;
// the simultaneous update reads the previous step's outputs, the
// current/previous output buffers of Sec. 3.3):
//   r = logistic(x);  p = W r;
//   x <- x + dt (-x + p + g u) + b xi;      y <- y + dt R (r - 1/2)
// until max(y) >= theta or the step cap.  u is the run's fixed input drive,
// xi fresh noise per unit and step, y a two-unit readout.
//
// Many runs share W, so the projection of 16 runs is one 16-column matrix
// product per step.  A workgroup of four wavefronts owns 16 run slots; wave
// w owns a quarter of the units of all 16 runs.  In the 16x16 MFMA output
// layout lane j + 16 g holds units 16b + 4g + q (q = 0..3) of run j, so each
// lane updates its own units, evaluates their logistic and publishes them
// through LDS in blocks of 16 units; the bf16 product reads them back as the
// B operand of 16x16x32 MFMAs (two published quads per lane and K block).
//
// bf16 path: each wave keeps its quarter of W (bf16, matrix-core fragment
// order) in registers for the whole kernel; r goes through LDS as bf16 B
// fragments.  FP64 path: W's fp64 fragments stream from L2 (512 KB does not
// fit on chip) and r goes through LDS in fp64.
//
// Run slots are refilled as runs end: the workgroup's runs are
// r = wg + G k, k = 0, 1, ..., handed to slots in order of slot index as
// they free up.  Every wave evaluates the slot decisions identically from
// the same LDS partial sums, so the assignment needs no atomics.
#include <algorithm>

#include "internal.hpp"
#include "rng.hpp"

namespace cm {
namespace {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kRnnBlock = 256;

__device__ __forceinline__ bool near_th(double q, double th, double eps) {
  return fabs(q - th) < eps;
}

__device__ __forceinline__ float logistic_f(float x) {
  // 1 / (1 + e^-x) with the hardware exp2 and reciprocal
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.44269504f * x));
}

// Finished-run bookkeeping shared by both precisions (one lane per run).
__device__ __forceinline__ void record_run(const RnnArgs& a, uint32_t s, uint32_t t, uint32_t n,
                                           int choice, bool flag, double y0, double y1) {
  uint64_t* st = a.stats + (uint64_t)s * CM_NSTAT;
  const unsigned long long nn = n;
  if (choice >= 0) {
    const uint32_t bin = ((n - 1u) * a.n_bins) / a.max_steps;
    atomicAdd((unsigned long long*)&a.hist[((uint64_t)s * 2u + choice) * a.n_bins + bin], 1ull);
    atomicAdd((unsigned long long*)&st[CM_ST_DEC0 + choice], 1ull);
    atomicAdd((unsigned long long*)&st[CM_ST_SUMN0 + choice], nn);
    atomicAdd((unsigned long long*)&st[CM_ST_SUMSQ0 + choice], nn * nn);
  } else {
    atomicAdd((unsigned long long*)&st[CM_ST_UNDEC], 1ull);
  }
  if (flag) atomicAdd((unsigned long long*)&st[CM_ST_FLAGGED], 1ull);
  if (a.run_choice) {
    const uint64_t idx = (uint64_t)s * a.trials + t;
    a.run_choice[idx] = (int8_t)choice;
    a.run_step[idx] = n;
    a.run_flag[idx] = flag ? 1 : 0;
    if (a.run_state) {
      a.run_state[idx * (2u + a.n_units)] = y0;
      a.run_state[idx * (2u + a.n_units) + 1] = y1;
    }
  }
}

// Per-slot control state, identical in every lane of a slot (and every wave).
struct Slot {
  uint64_t run;
  uint32_t s, t, n;
  bool active, flag;
  double y0, y1;
  float acc0, acc1;  // readout sum of R (r - 1/2) for the next y update
};

__device__ __forceinline__ void slot_begin(const RnnArgs& a, Slot& S, uint64_t run) {
  S.run = run;
  S.active = run < a.total_runs;
  const uint64_t r = S.active ? run : 0;
  S.s = (uint32_t)(r / a.trials);
  S.t = (uint32_t)(r - (uint64_t)S.s * a.trials);
  S.n = 0;
  S.flag = false;
  S.y0 = 0.0;
  S.y1 = 0.0;
  S.acc0 = 0.0f;  // r = logistic(0) = 1/2 exactly, so R (r - 1/2) = 0
  S.acc1 = 0.0f;
}

// Decision after the readout update; returns true when the run ends.
__device__ __forceinline__ bool slot_decide(const RnnArgs& a, Slot& S, int& choice) {
  const double th = a.thresh, eps = a.flag_eps;
  if (near_th(S.y0, th, eps) || near_th(S.y1, th, eps)) S.flag = true;
  const double mx = S.y0 > S.y1 ? S.y0 : S.y1;
  if (mx >= th) {
    choice = S.y1 > S.y0 ? 1 : 0;
    if (fabs(S.y0 - S.y1) < eps) S.flag = true;
    return true;
  }
  choice = -1;
  return S.n == a.max_steps;
}

// ---------------------------------------------------------------------------
// bf16 projection, fp32 steps, fp64 accumulators.
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(kRnnBlock, 2) void rnn_bf16_kernel(RnnArgs a) {
  constexpr int NBW = NB / 4;  // output blocks per wave
  constexpr int NU = NB * 16;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, j = l & 15, g = l >> 4;
  __shared__ bf16x4 rt[NB][64];  // r of the 16 slots: [16-unit block][lane j + 16 g] = 4 units
  __shared__ float ypart[4][2][16];
  __shared__ float Rs[2][NU];

  // this wave's quarter of W as A fragments: block b = w NBW + bw, K block kb
  // of 32 units
  constexpr int NK = NB / 2;
  bf16x8 A[NBW][NK];
  const bf16x8* wf = (const bf16x8*)a.wfrag;
#pragma unroll
  for (int bw = 0; bw < NBW; ++bw)
#pragma unroll
    for (int kb = 0; kb < NK; ++kb) A[bw][kb] = wf[((w * NBW + bw) * NK + kb) * 64 + l];
  // B operand of K block kb: units 32 kb + 8 g + 0..7 of run j, i.e. the
  // quads published by lanes j + 16 (2 (g & 1)) and j + 16 (2 (g & 1) + 1)
  // for 16-unit block 2 kb + g / 2
  const int bh = g >> 1, bl = j + 32 * (g & 1);
  for (int i = tid; i < 2 * NU; i += kRnnBlock) Rs[i / NU][i % NU] = (float)a.R[i];

  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const float dtf = (float)a.dt, bf = (float)a.b;
  const uint64_t G = gridDim.x, wg = blockIdx.x;

  double x[NBW][4];
  float gu[NBW][4];
  Slot S;
  uint32_t knext = 16;  // next run ordinal of this workgroup

  // Initialise a run in this lane's units: x = 0, drive g u, r = 1/2.
  auto begin_units = [&]() {
    const float gf = (float)(a.n_signals ? a.grid[(uint64_t)S.s * a.n_signals] : a.gain);
#pragma unroll
    for (int bw = 0; bw < NBW; ++bw) {
      const int b = w * NBW + bw;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t m = (uint32_t)(8 * b + 2 * g + h);  // unit pair (2m, 2m+1)
        const Words wd = philox(m, S.t, S.s, kStreamDrive, k0, k1);
        float u0, u1;
        normals32(wd, u0, u1);
        gu[bw][2 * h] = gf * u0;
        gu[bw][2 * h + 1] = gf * u1;
        x[bw][2 * h] = 0.0;
        x[bw][2 * h + 1] = 0.0;
      }
      rt[b][l] = bf16x4{(__bf16)0.5f, (__bf16)0.5f, (__bf16)0.5f, (__bf16)0.5f};
    }
  };

  slot_begin(a, S, wg + G * (uint64_t)j);
  begin_units();
  __syncthreads();

  for (;;) {
    // every lane of every wave sees the same slot states
    if (!__any(S.active)) break;

    // (1) projection p = W r for this wave's output blocks and all 16 slots
    f32x4 P[NBW];
#pragma unroll
    for (int bw = 0; bw < NBW; ++bw) P[bw] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < NK; ++kb) {
      const bf16x4 lo = rt[2 * kb + bh][bl], hi = rt[2 * kb + bh][bl + 16];
      const bf16x8 B = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
#pragma unroll
      for (int bw = 0; bw < NBW; ++bw)
        P[bw] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[bw][kb], B, P[bw], 0, 0, 0);
    }
    __syncthreads();  // all reads of rt done

    // (2) unit update, new rates, readout partial sums
    S.n += 1;
    float ya = 0.0f, yb = 0.0f;
#pragma unroll
    for (int bw = 0; bw < NBW; ++bw) {
      const int b = w * NBW + bw;
      float r4[4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t m = (uint32_t)(8 * b + 2 * g + h);
        const Words wd = philox(S.n - 1u, S.t, S.s, m, k0, k1);
        float xi[2];
        normals32(wd, xi[0], xi[1]);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int q = 2 * h + e;
          const float xf = (float)x[bw][q];
          const float inc = fmaf(dtf, (P[bw][q] - xf) + gu[bw][q], bf * xi[e]);
          x[bw][q] = x[bw][q] + (double)inc;
          r4[q] = logistic_f((float)x[bw][q]);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int u = 16 * b + 4 * g + q;
        ya = fmaf(Rs[0][u], r4[q] - 0.5f, ya);
        yb = fmaf(Rs[1][u], r4[q] - 0.5f, yb);
      }
      rt[b][l] = bf16x4{(__bf16)r4[0], (__bf16)r4[1], (__bf16)r4[2], (__bf16)r4[3]};
    }
    ya += __shfl_xor(ya, 16, 64);
    yb += __shfl_xor(yb, 16, 64);
    ya += __shfl_xor(ya, 32, 64);
    yb += __shfl_xor(yb, 32, 64);
    if (g == 0) {
      ypart[w][0][j] = ya;
      ypart[w][1][j] = yb;
    }
    __syncthreads();

    // (3) readout update and decision, replicated in every lane of the slot
    S.y0 = S.y0 + (double)(dtf * S.acc0);
    S.y1 = S.y1 + (double)(dtf * S.acc1);
    S.acc0 = ((ypart[0][0][j] + ypart[1][0][j]) + ypart[2][0][j]) + ypart[3][0][j];
    S.acc1 = ((ypart[0][1][j] + ypart[1][1][j]) + ypart[2][1][j]) + ypart[3][1][j];
    int choice = -1;
    const bool done = S.active && slot_decide(a, S, choice);
    const uint64_t mask = __ballot(done) & 0xFFFFull;  // one bit per slot (lanes 0..15)
    if (mask) {  // uniform across the workgroup
      if (done) {
        if (w == 0 && g == 0) record_run(a, S.s, S.t, S.n, choice, S.flag, S.y0, S.y1);
        if (a.run_state) {
          const uint64_t idx = (uint64_t)S.s * a.trials + S.t;
#pragma unroll
          for (int bw = 0; bw < NBW; ++bw)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              a.run_state[idx * (2u + a.n_units) + 2u + 16u * (w * NBW + bw) + 4u * g + q] = x[bw][q];
        }
        const uint32_t rank = __builtin_popcountll(mask & ((1ull << j) - 1ull));
        slot_begin(a, S, wg + G * (uint64_t)(knext + rank));
        begin_units();
      }
      knext += (uint32_t)__builtin_popcountll(mask);
      __syncthreads();  // refilled slots' rt entries visible to the next projection
    }
  }
}

// ---------------------------------------------------------------------------
// fp64 throughout.  K blocks are (b, q): units 16 b + 4 k + q, k = 0..3, which
// is the B layout of the 16x16x4 fp64 MFMA (lane j + 16 k supplies row k).
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(kRnnBlock, 2) void rnn_f64_kernel(RnnArgs a) {
  constexpr int NBW = NB / 4;
  constexpr int NU = NB * 16;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, j = l & 15, g = l >> 4;
  __shared__ double rt[NB * 4][64];  // [K block (b, q)][lane]
  __shared__ double ypart[4][2][16];
  __shared__ double Rs[2][NU];
  for (int i = tid; i < 2 * NU; i += kRnnBlock) Rs[i / NU][i % NU] = a.R[i];

  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const uint64_t G = gridDim.x, wg = blockIdx.x;
  const double* wf = (const double*)a.wfrag;

  double x[NBW][4], gu[NBW][4];
  Slot S;
  double acc0 = 0.0, acc1 = 0.0;  // fp64 readout sums (S.acc* unused here)
  uint32_t knext = 16;

  auto begin_units = [&]() {
    const double gd = a.n_signals ? a.grid[(uint64_t)S.s * a.n_signals] : a.gain;
#pragma unroll
    for (int bw = 0; bw < NBW; ++bw) {
      const int b = w * NBW + bw;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t m = (uint32_t)(8 * b + 2 * g + h);
        const Words wd = philox(m, S.t, S.s, kStreamDrive, k0, k1);
        double u0, u1;
        normals64(wd, u0, u1);
        gu[bw][2 * h] = gd * u0;
        gu[bw][2 * h + 1] = gd * u1;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        x[bw][q] = 0.0;
        rt[4 * b + q][l] = 0.5;
      }
    }
    acc0 = 0.0;
    acc1 = 0.0;
  };

  slot_begin(a, S, wg + G * (uint64_t)j);
  begin_units();
  __syncthreads();

  for (;;) {
    if (!__any(S.active)) break;

    f64x4 P[NBW];
#pragma unroll
    for (int bw = 0; bw < NBW; ++bw) P[bw] = f64x4{0.0, 0.0, 0.0, 0.0};
    // W's fragments come from L2: each is loaded PF K blocks ahead of its
    // product, so that the loads' latency overlaps the products in between
    // (one load then its product back to back waits out the whole latency).
    constexpr int K = NB * 4, PF = 4;
    const double* wbase = wf + (uint64_t)(w * NBW) * K * 64 + l;  // + (bw K + kb) 64
    double Af[PF][NBW];
#pragma unroll
    for (int f = 0; f < PF; ++f)
#pragma unroll
      for (int bw = 0; bw < NBW; ++bw) Af[f][bw] = wbase[((uint64_t)bw * K + f) * 64];
#pragma unroll 1
    for (int kb0 = 0; kb0 < K; kb0 += PF) {
#pragma unroll
      for (int f = 0; f < PF; ++f) {
        const int kb = kb0 + f;
        const double B = rt[kb][l];
        double cur[NBW];
#pragma unroll
        for (int bw = 0; bw < NBW; ++bw) cur[bw] = Af[f][bw];
        // (the last PF blocks reload their own fragments: no branch in the loop)
        const int kn = kb + PF < K ? kb + PF : kb;
#pragma unroll
        for (int bw = 0; bw < NBW; ++bw) Af[f][bw] = wbase[((uint64_t)bw * K + kn) * 64];
#pragma unroll
        for (int bw = 0; bw < NBW; ++bw)
          P[bw] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[bw], B, P[bw], 0, 0, 0);
      }
    }
    __syncthreads();

    S.n += 1;
    double ya = 0.0, yb = 0.0;
#pragma unroll
    for (int bw = 0; bw < NBW; ++bw) {
      const int b = w * NBW + bw;
      double r4[4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t m = (uint32_t)(8 * b + 2 * g + h);
        const Words wd = philox(S.n - 1u, S.t, S.s, m, k0, k1);
        double xi[2];
        normals64(wd, xi[0], xi[1]);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int q = 2 * h + e;
          x[bw][q] = (x[bw][q] + a.dt * ((P[bw][q] - x[bw][q]) + gu[bw][q])) + a.b * xi[e];
          r4[q] = 1.0 / (1.0 + exp(-x[bw][q]));
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int u = 16 * b + 4 * g + q;
        ya = fma(Rs[0][u], r4[q] - 0.5, ya);
        yb = fma(Rs[1][u], r4[q] - 0.5, yb);
        rt[4 * b + q][l] = r4[q];
      }
    }
    ya += __shfl_xor(ya, 16, 64);
    yb += __shfl_xor(yb, 16, 64);
    ya += __shfl_xor(ya, 32, 64);
    yb += __shfl_xor(yb, 32, 64);
    if (g == 0) {
      ypart[w][0][j] = ya;
      ypart[w][1][j] = yb;
    }
    __syncthreads();

    S.y0 = S.y0 + a.dt * acc0;
    S.y1 = S.y1 + a.dt * acc1;
    acc0 = ((ypart[0][0][j] + ypart[1][0][j]) + ypart[2][0][j]) + ypart[3][0][j];
    acc1 = ((ypart[0][1][j] + ypart[1][1][j]) + ypart[2][1][j]) + ypart[3][1][j];
    int choice = -1;
    const bool done = S.active && slot_decide(a, S, choice);
    const uint64_t mask = __ballot(done) & 0xFFFFull;
    if (mask) {
      if (done) {
        if (w == 0 && g == 0) record_run(a, S.s, S.t, S.n, choice, S.flag, S.y0, S.y1);
        if (a.run_state) {
          const uint64_t idx = (uint64_t)S.s * a.trials + S.t;
#pragma unroll
          for (int bw = 0; bw < NBW; ++bw)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              a.run_state[idx * (2u + a.n_units) + 2u + 16u * (w * NBW + bw) + 4u * g + q] = x[bw][q];
        }
        const uint32_t rank = __builtin_popcountll(mask & ((1ull << j) - 1ull));
        slot_begin(a, S, wg + G * (uint64_t)(knext + rank));
        begin_units();
      }
      knext += (uint32_t)__builtin_popcountll(mask);
      __syncthreads();
    }
  }
}

// W (fp64 row-major n x n) -> matrix-core fragment order.
//  bf16: fragment (b, kb) for 16x16x32 MFMAs, lane l = i + 16 k8 holds
//        W[16b + i][32kb + 8k8 + 0..7].
//  fp64: fragment (b, kb4 = 4 bb + q), lane l = i + 16 k holds
//        W[16b + 4 (i % 4) + i / 4][16bb + 4k + q].
__global__ void rnn_prep_kernel(const double* W, uint32_t n, void* out, int bf16) {
  const uint32_t NB = n / 16;
  const uint64_t total = (uint64_t)n * n;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x) {
    if (bf16) {
      // e enumerates (b, kb, lane, item)
      const uint32_t item = e & 7u, lane = (e >> 3) & 63u, NK = NB / 2u;
      const uint64_t frag = e >> 9;
      const uint32_t kb = (uint32_t)(frag % NK), b = (uint32_t)(frag / NK);
      const uint32_t i = lane & 15u, k8 = lane >> 4;
      const double v = W[(uint64_t)(16u * b + i) * n + 32u * kb + 8u * k8 + item];
      ((__bf16*)out)[e] = (__bf16)(float)v;
    } else {
      // e enumerates (b, kb4, lane).  The fp64 16x16x4 accumulator holds row
      // 4 reg + lane/16 in register reg of a lane, so row position i of block
      // b stands for unit 16 b + 4 (i % 4) + i / 4: each lane then holds four
      // consecutive units (16 b + 4 g + reg), as in the bf16 layout.
      const uint32_t lane = e & 63u;
      const uint64_t frag = e >> 6;
      const uint32_t kb4 = (uint32_t)(frag % (4u * NB)), b = (uint32_t)(frag / (4u * NB));
      const uint32_t bb = kb4 >> 2, q = kb4 & 3u, i = lane & 15u, k = lane >> 4;
      const uint32_t row = 16u * b + 4u * (i & 3u) + (i >> 2);
      ((double*)out)[e] = W[(uint64_t)row * n + 16u * bb + 4u * k + q];
    }
  }
}

template <int NB>
hipError_t launch_nb(int precision, const RnnArgs& a, uint32_t groups, hipStream_t st) {
  if (precision == CM_FP64)
    hipLaunchKernelGGL((rnn_f64_kernel<NB>), dim3(groups), dim3(kRnnBlock), 0, st, a);
  else
    hipLaunchKernelGGL((rnn_bf16_kernel<NB>), dim3(groups), dim3(kRnnBlock), 0, st, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rnn_prep(const double* W, uint32_t n, void* out, bool bf16, hipStream_t st) {
  const uint64_t total = (uint64_t)n * n;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(rnn_prep_kernel, dim3(grid), dim3(256), 0, st, W, n, out, bf16 ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_rnn(int precision, const RnnArgs& a, uint32_t groups, hipStream_t st) {
  switch (a.n_units) {
    case 64: return launch_nb<4>(precision, a, groups, st);
    case 128: return launch_nb<8>(precision, a, groups, st);
    case 192: return launch_nb<12>(precision, a, groups, st);
    case 256: return launch_nb<16>(precision, a, groups, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cm
