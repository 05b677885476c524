// loop.hip -- closed-loop control of the conflict network.
//
// Before every step of a run, the control node searches the L x L grid of
// allocations (c_A, c_B): each allocation is scored by M sampled one-step
// look-aheads of the leaky competing accumulator (each with its own random
// stream) as cost * |c|^2 minus the mean gain in evidence x_c - x_w for the
// correct response, and the lowest score wins (exact ties: the smallest
// Philox priority, a random pick).  The step then runs with the chosen
// allocation on the run's own stream, and the state carries to the next
// search: the control loop nested inside each time step of the Distill
// paper's predator-prey model (Sec. 2.1), with its allocations and samples
// evaluated in parallel (Sec. 3.6).
//
// Mapping: a team of P lanes (P = 1, 4, 16 or 64, the power of two that
// covers the L^2 allocations, capped at a wavefront) owns one run at a time;
// a search so wide that every lane of a workgroup still has four or more
// allocations, over too few runs to fill the GPU with wavefront teams, takes
// the whole workgroup (P = 256).  Lane i of the team evaluates allocations
// i, i + P, ... with all their samples (four at a time when it has several,
// so that independent random-number chains overlap).  A wavefront team finds
// the best score by one minimum over the wavefront, the winner by a ballot of
// the lanes at it (exact ties, rare, by the smallest (priority, allocation)),
// and the second-best score by a second minimum; smaller teams use a
// butterfly of (score, second score, allocation) cross-lane moves (DPP within
// 16-lane rows, shuffles across them), and P = 256 adds a fold of the four
// wavefronts' results through LDS.  Every lane of the team then applies the
// chosen step to its own copy of the state (identical arithmetic, identical
// bits), so the team never broadcasts and its control flow stays uniform; a
// wavefront team draws the normals of its run's own steps 64 at a time, one
// step per lane, and reads each step's from its lane.  Teams take runs in a
// fixed stride, and a finished run
// is counted straight into global memory by the team's first lane: a run
// costs L^2 M look-ahead steps per step, so the atomics are negligible.  The
// allocation drive table [L^2][9][2] and the allocations' squared norms
// c_A^2 + c_B^2 [L^2] are computed once per sweep by the preparation kernel.
#include <type_traits>

#include "internal.hpp"
#include "lca_step.hpp"
#include "rng.hpp"

namespace cm {
namespace {

constexpr int kLoopBlock = 256;
constexpr int kLoopChains = 4;  // allocations a lane of a wide search evaluates together
constexpr uint32_t kStreamLook = 0x80000000u;  // | (allocation * M + sample)

// Philox4x32-10 on the counter (k, t, s, c3) with many stream words c3 at one
// step k of one run (the closed loop's look-ahead samples): the work that
// depends only on (k, t, s) -- round 1 but for c3's xor, round 2's product
// with the constant c0, round 3's product with the constant c2 -- is done
// once per step.  The words equal philox(k, t, s, c3, k0, k1) bit for bit.

struct StreamKey {
  uint32_t e2;  // round 1: hi(M0 k) ^ k1, xored with c3
  uint32_t b1;  // round 2: lo(M1 s) ^ (k0 + W0), xored with hi(M1 c2)
  uint32_t g1;  // round 3: hi(M1 c2'') ^ (k0 + 2 W0), xored with round 2's lo(M1 c2)
  uint32_t l1;  // round 3: lo(M1 c2''), the new c1
  uint32_t d3;  // round 3: lo(M0 c0') ^ (k1 + 2 W1), xored with hi(M0 c0'')
};

__device__ __forceinline__ StreamKey stream_key(uint32_t k, uint32_t t, uint32_t s, uint32_t k0,
                                                uint32_t k1) {
  const uint64_t p0 = (uint64_t)kPhiloxM0 * k, p1 = (uint64_t)kPhiloxM1 * s;
  const uint32_t c0 = (uint32_t)(p1 >> 32) ^ t ^ k0;  // round 1's c0, c1 and c3
  const uint32_t c1 = (uint32_t)p1, c3 = (uint32_t)p0;
  const uint64_t q0 = (uint64_t)kPhiloxM0 * c0;  // round 2's c2 and c3
  const uint32_t c2b = (uint32_t)(q0 >> 32) ^ c3 ^ (k1 + kPhiloxW1);
  const uint64_t u1 = (uint64_t)kPhiloxM1 * c2b;
  StreamKey r;
  r.e2 = (uint32_t)(p0 >> 32) ^ k1;
  r.b1 = c1 ^ (k0 + kPhiloxW0);
  r.g1 = (uint32_t)(u1 >> 32) ^ (k0 + 2u * kPhiloxW0);
  r.l1 = (uint32_t)u1;
  r.d3 = (uint32_t)q0 ^ (k1 + 2u * kPhiloxW1);
  return r;
}

__device__ __forceinline__ Words philox_stream(const StreamKey& r, uint32_t c3, uint32_t k0,
                                               uint32_t k1) {
  const uint64_t q1 = (uint64_t)kPhiloxM1 * (r.e2 ^ c3);  // round 2, lane part
  const uint64_t u0 = (uint64_t)kPhiloxM0 * ((uint32_t)(q1 >> 32) ^ r.b1);  // round 3
  uint32_t c0 = (uint32_t)q1 ^ r.g1, c1 = r.l1;
  uint32_t c2 = (uint32_t)(u0 >> 32) ^ r.d3, c3n = (uint32_t)u0;
#pragma unroll
  for (uint32_t round = 3; round < 10; ++round) {
    const uint64_t v0 = (uint64_t)kPhiloxM0 * c0, v1 = (uint64_t)kPhiloxM1 * c2;
    const uint32_t m0 = xor3((uint32_t)(v1 >> 32), c1, k0 + round * kPhiloxW0);
    const uint32_t m2 = xor3((uint32_t)(v0 >> 32), c3n, k1 + round * kPhiloxW1);
    c1 = (uint32_t)v1;
    c3n = (uint32_t)v0;
    c0 = m0;
    c2 = m2;
  }
  return Words{c0, c1, c2, c3n};
}
constexpr uint32_t kStreamPick = 0xC0000000u;  // | allocation
constexpr uint32_t kNone = 0xFFFFFFFFu;

// One LCA step in the model's precision from its normals (z0, z1 in FP64;
// zf0, zf1 in FP32 steps, with idt_i = float(I_i dt)): the arithmetic of the
// open-loop LCA kernel, so that a one-allocation loop reproduces it bit for
// bit.
template <int PREC>
__device__ __forceinline__ void lca_update(const LoopArgs& a, double x0, double x1, double in0,
                                           double in1, float idt0, float idt1, double z0, double z1,
                                           float zf0, float zf1, double& y0, double& y1) {
  if (PREC == CM_FP64) {
    y0 = (x0 + (((in0 - a.leak * x0) - a.comp * x1) * a.dt)) + a.b * z0;
    y1 = (x1 + (((in1 - a.leak * x1) - a.comp * x0) * a.dt)) + a.b * z1;
  } else {
    const LcaF32 pf = lca_f32(a.leak, a.comp, a.dt, a.b);
    const float xf0 = (float)x0, xf1 = (float)x1;
    y0 = x0 + (double)lca_inc_f32(pf, idt0, xf0, xf1, zf0);
    y1 = x1 + (double)lca_inc_f32(pf, idt1, xf1, xf0, zf1);
  }
  if (a.nonneg) {
    if (y0 < 0.0) y0 = 0.0;
    if (y1 < 0.0) y1 = 0.0;
  }
}

// The same step from a random block.
template <int PREC>
__device__ __forceinline__ void lca_step(const LoopArgs& a, double x0, double x1, double in0,
                                         double in1, float idt0, float idt1, const Words& w,
                                         double& y0, double& y1) {
  double z0 = 0.0, z1 = 0.0;
  float zf0 = 0.0f, zf1 = 0.0f;
  if (PREC == CM_FP64) normals64(w, z0, z1);
  else normals32(w, zf0, zf1);
  lca_update<PREC>(a, x0, x1, in0, in1, idt0, idt1, z0, z1, zf0, zf1, y0, y1);
}

// Tie rule among allocations with equal scores: the smaller (Philox priority,
// allocation) wins.  kNone stands for "no allocation yet".
__device__ __forceinline__ bool tie_wins(uint32_t j, uint32_t bj, uint32_t k, uint32_t t, uint32_t s,
                                         uint32_t k0, uint32_t k1) {
  if (j == bj || j == kNone) return false;
  if (bj == kNone) return true;
  const uint32_t pj = philox(k, t, s, kStreamPick | j, k0, k1).w0;
  const uint32_t pb = philox(k, t, s, kStreamPick | bj, k0, k1).w0;
  return pj < pb || (pj == pb && j < bj);
}

// The partner's value in round r of a team's reduction; each round joins the
// two halves of aligned lane groups of 2^(r+1).  Rounds 0-3 stay within a
// 16-lane row and use DPP moves (swap pairs, swap pairs of pairs, mirror
// within 8, mirror within 16: no LDS round trip); rounds 4 and 5 cross rows
// by lane shuffles.  The reduction's combine is commutative and associative,
// so any pairing that joins the two halves of each group gives the same
// result in every lane.
template <int R>
__device__ __forceinline__ uint32_t partner(uint32_t v) {
  if constexpr (R == 0) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
  else if constexpr (R == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
  else if constexpr (R == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);
  else if constexpr (R == 3) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);
  else return (uint32_t)__shfl_xor((int)v, 1 << R, 64);
}

template <int R>
__device__ __forceinline__ double partner(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t lo = partner<R>((uint32_t)u), hi = partner<R>((uint32_t)(u >> 32));
  return __longlong_as_double((long long)(lo | (hi << 32)));
}

// Lane src's value (src wave-uniform).
__device__ __forceinline__ double read_lane(double v, int src) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
  return __longlong_as_double((long long)((uint64_t)lo | ((uint64_t)hi << 32)));
}

// The two halves of the wavefront's 16-lane row pairs (R = 4: rows 0|1 and
// 2|3) or of its 32-lane halves (R = 5), lane by lane: gfx950's row swaps
// between two copies of a register (the odd rows, or the upper half, of one
// copy trade places with the even rows, or the lower half, of the other)
// leave one half's values in one result and the other's in the other, in
// every lane of the pair (which is which does not matter to a minimum).
template <int R>
__device__ __forceinline__ void halves(uint32_t v, uint32_t& a, uint32_t& b) {
  if constexpr (R == 4) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    a = r[0];
    b = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    a = r[0];
    b = r[1];
  }
}
template <int R>
__device__ __forceinline__ double halves_min(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  uint32_t la, lb, ha, hb;
  halves<R>((uint32_t)u, la, lb);
  halves<R>((uint32_t)(u >> 32), ha, hb);
  return fmin(__longlong_as_double((long long)((uint64_t)la | ((uint64_t)ha << 32))),
              __longlong_as_double((long long)((uint64_t)lb | ((uint64_t)hb << 32))));
}
template <int R>
__device__ __forceinline__ uint64_t halves_min(uint64_t v) {
  uint32_t la, lb, ha, hb;
  halves<R>((uint32_t)v, la, lb);
  halves<R>((uint32_t)(v >> 32), ha, hb);
  const uint64_t a = (uint64_t)la | ((uint64_t)ha << 32), b = (uint64_t)lb | ((uint64_t)hb << 32);
  return a < b ? a : b;
}

// Minimum over the wavefront, the same value in every lane (all lanes
// active; NaN loses to any number, as the scan's comparisons ignore it):
// rounds 0-3 within rows by DPP, then the row pairs and the two halves by
// row swaps (no LDS round trip).
__device__ __forceinline__ double wave_min(double v) {
  v = fmin(v, partner<0>(v));
  v = fmin(v, partner<1>(v));
  v = fmin(v, partner<2>(v));
  v = fmin(v, partner<3>(v));
  v = halves_min<4>(v);
  return halves_min<5>(v);
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  auto step = [&](auto round) {
    constexpr int R = decltype(round)::value;
    const uint64_t o = (uint64_t)partner<R>((uint32_t)v) | ((uint64_t)partner<R>((uint32_t)(v >> 32)) << 32);
    v = o < v ? o : v;
  };
  step(std::integral_constant<int, 0>{});
  step(std::integral_constant<int, 1>{});
  step(std::integral_constant<int, 2>{});
  step(std::integral_constant<int, 3>{});
  v = halves_min<4>(v);
  return halves_min<5>(v);
}

template <int PREC, int P, int U>
__global__ __launch_bounds__(kLoopBlock) void loop_kernel(LoopArgs a) {
  // P = kLoopBlock: the whole workgroup is one team; its four wavefronts
  // fold their results through LDS, double-buffered by the parity of a fold
  // count that runs on across runs (consecutive folds use different buffers,
  // so one barrier per fold suffices).  Every thread of the workgroup
  // follows the same run and takes the same decisions, so the barrier is
  // reached uniformly.
  __shared__ double fold_v[2][kLoopBlock / 64], fold_s[2][kLoopBlock / 64];
  __shared__ uint32_t fold_j[2][kLoopBlock / 64];
  uint32_t folds = 0;
  const uint32_t j0 = P > 64 ? threadIdx.x : (threadIdx.x & 63u) % (uint32_t)P;
  const uint32_t teams_per_block = kLoopBlock / P;
  const uint64_t n_teams = (uint64_t)gridDim.x * teams_per_block;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const uint32_t T = (uint32_t)a.trials, J = a.J, M = a.M, N = a.max_steps;
  const double th = a.thresh, eps = a.flag_eps;
  // a wavefront-or-wider team's run index is the same in every lane
  const uint32_t team = P >= 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / P) : threadIdx.x / P;
  const uint32_t lane = threadIdx.x & 63u;
  for (uint64_t run = (uint64_t)blockIdx.x * teams_per_block + team; run < a.total_runs;
       run += n_teams) {
    const uint32_t s = (uint32_t)(run / T), t = (uint32_t)(run - (uint64_t)s * T);
    const uint32_t stim = t % 9u;
    const int c = a.correct[stim];
    const double kappa = a.n_signals ? a.grid[s] : a.cost;
    // the mean over M samples: a power of two divides exactly as a product
    // with its reciprocal, which saves a division per allocation and step
    const bool pow2 = (M & (M - 1u)) == 0u;
    const double inv_m = 1.0 / (double)M;
    double x0 = 0.0, x1 = 0.0;
    bool flag = false;
    int choice = -1;
    // P = 64: the run's own normals for steps 64 b .. 64 b + 63, lane i
    // holding step 64 b + i's (drawn when step 64 b comes up, read back by
    // lane each step: one block per wavefront and 64 steps)
    double ez0 = 0.0, ez1 = 0.0;
    float ef0 = 0.0f, ef1 = 0.0f;
    uint32_t n = 1;
    for (; n <= N; ++n) {
      const uint32_t k = n - 1u;
      if constexpr (P == 64) {
        if ((k & 63u) == 0u) {
          const Words w = philox(k + lane, t, s, 0u, k0, k1);
          if (PREC == CM_FP64) normals64(w, ez0, ez1);
          else normals32(w, ef0, ef1);
        }
      }
      const double dx = c ? x1 - x0 : x0 - x1;  // x_c - x_w
      // the look-ahead blocks of this step differ only in their stream word
      const StreamKey sk = stream_key(k, t, s, k0, k1);
      double bv = INFINITY, sv = INFINITY;
      uint32_t bj = kNone;
      // A lane's allocations j0, j0 + P, ... are evaluated U at a time, so
      // that U independent random-number chains are in flight (a wide search
      // otherwise waits on one chain's latency); they are compared in
      // allocation order, as one at a time would.  Slots past J repeat
      // allocation j and are discarded.
      for (uint32_t j = j0; j < J; j += U * P) {
        double gs[U], i0[U], i1[U];
        float f0[U], f1[U];
        uint32_t ju[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
          ju[u] = j + u * P < J ? j + u * P : j;
          const double* d = a.drive + ((uint64_t)ju[u] * 9u + stim) * 2u;
          i0[u] = d[0];
          i1[u] = d[1];
          if constexpr (P == 64) {  // rounded once per allocation and step
            f0[u] = (float)(i0[u] * a.dt);
            f1[u] = (float)(i1[u] * a.dt);
          }
          gs[u] = 0.0;
        }
        for (uint32_t m = 0; m < M; ++m) {
#pragma unroll
          for (uint32_t u = 0; u < U; ++u) {
            const Words w = philox_stream(sk, kStreamLook | (ju[u] * M + m), k0, k1);
            double y0, y1;
            if constexpr (P == 64)
              lca_step<PREC>(a, x0, x1, i0[u], i1[u], f0[u], f1[u], w, y0, y1);
            else
              lca_step<PREC>(a, x0, x1, i0[u], i1[u], (float)(i0[u] * a.dt), (float)(i1[u] * a.dt), w,
                             y0, y1);
            gs[u] = gs[u] + ((c ? y1 - y0 : y0 - y1) - dx);
          }
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
          if (j + u * P >= J) break;
          const uint32_t jj = ju[u];
          double mean;
          if (pow2) {
            mean = gs[u] * inv_m;
          } else {
            // a branch of its own: the division is not evaluated beside the
            // product when M is a power of two
            asm volatile("" ::: "memory");
            mean = gs[u] / (double)M;
          }
          const double V = kappa * a.norm2[jj] - mean;
          if (V < bv) {
            sv = bv;
            bv = V;
            bj = jj;
          } else if (V == bv) {
            sv = V;
            if (tie_wins(jj, bj, k, t, s, k0, k1)) bj = jj;
          } else if (V < sv) {
            sv = V;
          }
        }
      }
      bool near_pick = false;
      if constexpr (P == 64) {
        // The best score over the wavefront; an exact tie anywhere (several
        // lanes at it, or a lane holding two allocations at it) goes to the
        // smallest (priority, allocation), else the one lane at it holds the
        // winner.  The second-lowest score is the winner's own second or
        // another lane's best; exact ties leave none above the best.
        const double gb = wave_min(bv);
        const bool at = bv == gb;
        const uint64_t tied = __builtin_amdgcn_ballot_w64(at);
        const bool tie = __popcll(tied) > 1 || __builtin_amdgcn_ballot_w64(sv == gb) != 0;
        uint32_t pick;
        if (__builtin_expect(!tie, 1)) {
          pick = (uint32_t)__builtin_amdgcn_readlane((int)bj, (int)__builtin_ctzll(tied));
        } else {
          uint64_t key = ~0ull;
          if (at && bj != kNone)
            key = ((uint64_t)philox(k, t, s, kStreamPick | bj, k0, k1).w0 << 32) | bj;
          pick = (uint32_t)wave_min_u64(key);
        }
        const double second = wave_min(at ? sv : bv);
        near_pick = !tie && second > gb && second - gb < eps;
        bv = gb;
        bj = pick;
      }
      auto join = [&](auto round) {
        constexpr int R = decltype(round)::value;
        if constexpr (P != 64 && (1 << R) < (P < 64 ? P : 64)) {
          const double ov = partner<R>(bv), os = partner<R>(sv);
          const uint32_t oj = partner<R>(bj);
          const double ns = fmin(fmin(sv, os), fmax(bv, ov));
          if (ov < bv || (ov == bv && tie_wins(oj, bj, k, t, s, k0, k1))) {
            bv = ov;
            bj = oj;
          }
          sv = ns;
        }
      };
      join(std::integral_constant<int, 0>{});
      join(std::integral_constant<int, 1>{});
      join(std::integral_constant<int, 2>{});
      join(std::integral_constant<int, 3>{});
      join(std::integral_constant<int, 4>{});
      join(std::integral_constant<int, 5>{});
      if constexpr (P > 64) {
        const uint32_t wv = threadIdx.x >> 6, par = folds++ & 1u;
        if ((threadIdx.x & 63u) == 0) {
          fold_v[par][wv] = bv;
          fold_s[par][wv] = sv;
          fold_j[par][wv] = bj;
        }
        __syncthreads();
        bv = fold_v[par][0];
        sv = fold_s[par][0];
        bj = fold_j[par][0];
#pragma unroll
        for (uint32_t v = 1; v < kLoopBlock / 64; ++v) {
          const double ov = fold_v[par][v], os = fold_s[par][v];
          const uint32_t oj = fold_j[par][v];
          const double ns = fmin(fmin(sv, os), fmax(bv, ov));
          if (ov < bv || (ov == bv && tie_wins(oj, bj, k, t, s, k0, k1))) {
            bv = ov;
            bj = oj;
          }
          sv = ns;
        }
      }
      if (P == 64 ? near_pick : (sv > bv && sv - bv < eps)) flag = true;
      // the step itself, with the chosen allocation, on the run's own stream
      // (allocation 0 if no score compared as a number)
      const double* d = a.drive + ((uint64_t)(bj == kNone ? 0u : bj) * 9u + stim) * 2u;
      const double e0 = d[0], e1 = d[1];
      const float g0 = (float)(e0 * a.dt), g1 = (float)(e1 * a.dt);
      double y0, y1;
      if constexpr (P == 64) {
        const int src = (int)(k & 63u);
        double z0 = 0.0, z1 = 0.0;
        float zf0 = 0.0f, zf1 = 0.0f;
        if (PREC == CM_FP64) {
          z0 = read_lane(ez0, src);
          z1 = read_lane(ez1, src);
        } else {
          zf0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ef0), src));
          zf1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ef1), src));
        }
        lca_update<PREC>(a, x0, x1, e0, e1, g0, g1, z0, z1, zf0, zf1, y0, y1);
      } else {
        lca_step<PREC>(a, x0, x1, e0, e1, g0, g1, philox(k, t, s, 0u, k0, k1), y0, y1);
      }
      x0 = y0;
      x1 = y1;
      if (fabs(x0 - th) < eps || fabs(x1 - th) < eps) flag = true;
      const double mx = x0 > x1 ? x0 : x1;
      if (mx >= th) {
        choice = x1 > x0 ? 1 : 0;
        if (fabs(x0 - x1) < eps) flag = true;
        break;
      }
    }
    if (j0 == 0) {
      const uint32_t steps = choice >= 0 ? n : N;
      uint64_t* st = a.stats + (uint64_t)s * CM_NSTAT;
      if (choice >= 0) {
        const uint32_t bin = udiv_magic((steps - 1u) * a.n_bins, a.steps_magic);
        atomicAdd((unsigned long long*)&a.hist[((uint64_t)s * 2u + choice) * a.n_bins + bin], 1ull);
        atomicAdd((unsigned long long*)&st[CM_ST_DEC0 + choice], 1ull);
        atomicAdd((unsigned long long*)&st[CM_ST_SUMN0 + choice], (unsigned long long)steps);
        atomicAdd((unsigned long long*)&st[CM_ST_SUMSQ0 + choice],
                  (unsigned long long)steps * (unsigned long long)steps);
        if (choice == c) atomicAdd((unsigned long long*)&st[CM_ST_CORRECT], 1ull);
      } else {
        atomicAdd((unsigned long long*)&st[CM_ST_UNDEC], 1ull);
      }
      if (flag) atomicAdd((unsigned long long*)&st[CM_ST_FLAGGED], 1ull);
      if (a.run_choice) {
        a.run_choice[run] = (int8_t)choice;
        a.run_step[run] = steps;
        a.run_flag[run] = flag ? 1 : 0;
        if (a.run_state) {
          a.run_state[run * 2u] = x0;
          a.run_state[run * 2u + 1u] = x1;
        }
      }
    }
  }
}

template <int PREC>
hipError_t launch_prec(const LoopArgs& a, uint32_t team, uint32_t blocks, hipStream_t st) {
  if (team == kLoopBlock)
    hipLaunchKernelGGL((loop_kernel<PREC, kLoopBlock, kLoopChains>), dim3(blocks), dim3(kLoopBlock), 0,
                       st, a);
  else if (a.J == 1)
    hipLaunchKernelGGL((loop_kernel<PREC, 1, 1>), dim3(blocks), dim3(kLoopBlock), 0, st, a);
  else if (a.J <= 4)
    hipLaunchKernelGGL((loop_kernel<PREC, 4, 1>), dim3(blocks), dim3(kLoopBlock), 0, st, a);
  else if (a.J <= 16)
    hipLaunchKernelGGL((loop_kernel<PREC, 16, 1>), dim3(blocks), dim3(kLoopBlock), 0, st, a);
  else if (a.J < 4u * 64u)  // fewer than four allocations per lane
    hipLaunchKernelGGL((loop_kernel<PREC, 64, 1>), dim3(blocks), dim3(kLoopBlock), 0, st, a);
  else
    hipLaunchKernelGGL((loop_kernel<PREC, 64, kLoopChains>), dim3(blocks), dim3(kLoopBlock), 0, st, a);
  return hipGetLastError();
}

}  // namespace

// Lanes per run: the power of two covering the allocations, up to a
// wavefront; a whole workgroup when every lane of it still has four or more
// allocations and one-wavefront teams would leave the GPU short of
// wavefronts (fewer than 8 per SIMD).
uint32_t loop_team_lanes(uint32_t J, uint64_t runs, uint32_t cus) {
  if (J >= 4u * kLoopBlock && runs < 32ull * cus) return kLoopBlock;
  return J == 1 ? 1u : J <= 4 ? 4u : J <= 16 ? 16u : 64u;
}

// team: kLoopBlock, or the wavefront-or-smaller team loop_team_lanes gives
// for a.J (any other value is rejected).
hipError_t launch_loop(int precision, const LoopArgs& a, uint32_t team, uint32_t blocks, hipStream_t st) {
  if (blocks < 1 || (team != kLoopBlock && team != loop_team_lanes(a.J, ~0ull, 0u)))
    return hipErrorInvalidValue;
  return precision == CM_FP64 ? launch_prec<CM_FP64>(a, team, blocks, st)
                              : launch_prec<CM_FP32_STEP>(a, team, blocks, st);
}

}  // namespace cm
