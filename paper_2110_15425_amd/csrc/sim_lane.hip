// sim_lane.hip -- one wavefront lane per run: the drift-diffusion model and the
// conflict network's leaky competing accumulator.
//
// Each run is an evaluation of the model's trial loop (Distill, Sec. 2.2):
// the mechanisms are stepped until a threshold is crossed or the step cap is
// reached.  Runs are independent (Sec. 3.6), so every lane owns one run with
// its whole state in registers; read-only parameters arrive as kernel
// arguments (the RO/RW split of Sec. 3.3) and the loop-invariant
// feed-forward drive of the conflict network is precomputed once per
// (setting, stimulus) by a separate kernel (the cross-node loop-invariant
// code motion of Sec. 3.5).
//
// Scheduling: a workgroup owns a contiguous chunk of runs (setting-major).
// Lanes claim runs from an LDS counter; a lane whose run ended takes the next
// one at the following refill point, so waves stay dense while run lengths
// vary by orders of magnitude.  Once the chunk's queue is empty the
// workgroup drains: it repeatedly packs its unfinished runs into the first
// wavefronts so that the others stop issuing.  Finished runs are counted into an LDS
// histogram covering the few settings the chunk spans and flushed with one
// global 64-bit atomic per nonzero bin when the chunk is done.  All
// reductions are integer additions: results do not depend on the schedule.
#include <type_traits>

#include "internal.hpp"
#include "prep_score.hpp"
#include "lca_step.hpp"
#include "rng.hpp"

namespace cm {
namespace {

constexpr int kBlock = 256;
constexpr int kScanBlockMax = 512;  // the scan kernel runs 256 or 512 threads per workgroup
constexpr int kDrainSteps = 16;  // steps between packings once a chunk's queue is empty

struct Lane {
  uint32_t s, t;   // setting, trial
  uint32_t n;      // executed steps
  int32_t target;  // correct response for this trial's stimulus (-1: none)
  int choice;      // -1 undecided
  bool flag;
  uint32_t next_sample;  // time-course variant: next sample step
  uint32_t sample_k;     // time-course variant: index of that sample
};

// A lane's bookkeeping as it is staged through LDS while a workgroup drains
// (whole words only, so that the copy moves no padding bytes).
struct LaneWords {
  uint32_t s, t, n;
  int32_t target, choice;
  uint32_t flag;
};

// Time-course sums.  A sample adds the count and the fixed-point values
// q(v) = round-half-even(v 2^32) (clamped to +-2^62) of x0, x1, x0^2, x1^2
// and comp (x0 x1), with two's-complement 64-bit sums: integer additions, so
// the totals do not depend on the order in which runs arrive.
__device__ __forceinline__ uint64_t tc_quant(double v) {
  const double lim = 4611686018427387904.0;  // 2^62
  double t = __builtin_rint(v * 4294967296.0);
  t = t > lim ? lim : t;
  t = t < -lim ? -lim : t;
  return (uint64_t)(int64_t)t;
}

// q(v) for |v| < 2^19, the same value in three instructions: v 2^32 is exact
// and below 2^51 in magnitude, so adding 1.5 2^52 lands in [2^52, 2^53],
// where the spacing is 1 and the one rounding of the sum is the
// round-half-even of v 2^32 (1.5 2^52 is even); the integer then sits in the
// low bits of the sum's encoding.
__device__ __forceinline__ uint64_t tc_quant_small(double v) {
  const double shift = 6755399441055744.0;  // 1.5 2^52, encoded 0x4338000000000000
  return (uint64_t)__double_as_longlong(__builtin_fma(v, 4294967296.0, shift)) -
         0x4338000000000000ull;
}

__device__ __forceinline__ void tc_add(unsigned long long* w, double x0, double x1, double comp) {
  const double v[5] = {x0, x1, x0 * x0, x1 * x1, comp * (x0 * x1)};
  const double small = 524288.0;  // 2^19
  bool fits = true;
  for (int i = 0; i < 5; ++i) fits &= fabs(v[i]) < small;
  uint64_t q[5];
  // the wavefront's sampling lanes take one form together
  if (__builtin_expect(__builtin_amdgcn_ballot_w64(!fits) == 0, 1)) {
    for (int i = 0; i < 5; ++i) q[i] = tc_quant_small(v[i]);
  } else {
    for (int i = 0; i < 5; ++i) q[i] = tc_quant(v[i]);
  }
  atomicAdd(&w[0], 1ull);
  for (int i = 0; i < 5; ++i) atomicAdd(&w[1 + i], (unsigned long long)q[i]);
}

// Per-step hooks of the mechanisms.  NoSample compiles to nothing; Sample
// adds the state after step n when n is the lane's next sample step, into the
// workgroup's LDS window (the time-course block after the settings' records)
// or, in direct mode, into global memory.
struct NoSample {
  static constexpr bool kPerStep = false;
  __device__ __forceinline__ void operator()(Lane&, double, double) const {}
};

struct Sample {
  static constexpr bool kPerStep = true;
  unsigned long long* base;  // [window or n_settings][K][kTcWords]
  uint32_t s_lo, every, K;
  double comp;
  __device__ __forceinline__ void operator()(Lane& L, double x0, double x1) const {
    if (__builtin_expect(L.n == L.next_sample, 0)) {
      L.next_sample += every;
      const uint32_t k = L.sample_k++;
      tc_add(base + ((uint64_t)(L.s - s_lo) * K + k) * kTcWords, x0, x1, comp);
    }
  }
};

__device__ __forceinline__ bool near_th(double q, double th, double eps) {
  return fabs(q - th) < eps;
}


// Record one finished run: LDS window (or global atomics in direct mode) and
// optional per-run dumps.
__device__ __forceinline__ void record(const SimArgs& a, uint32_t* lds, uint32_t s_lo,
                                       const Lane& L, const double* state, int width) {
  const uint64_t n = L.n;
  const int c = L.choice;
  if (a.direct) {
    uint64_t* st = a.stats + (uint64_t)L.s * CM_NSTAT;
    if (c >= 0) {
      const uint32_t bin = udiv_magic((L.n - 1u) * a.n_bins, a.steps_magic);
      atomicAdd((unsigned long long*)&a.hist[((uint64_t)L.s * 2u + c) * a.n_bins + bin], 1ull);
      atomicAdd((unsigned long long*)&st[CM_ST_DEC0 + c], 1ull);
      atomicAdd((unsigned long long*)&st[CM_ST_SUMN0 + c], (unsigned long long)n);
      atomicAdd((unsigned long long*)&st[CM_ST_SUMSQ0 + c], (unsigned long long)(n * n));
      if (c == L.target) atomicAdd((unsigned long long*)&st[CM_ST_CORRECT], 1ull);
    } else {
      atomicAdd((unsigned long long*)&st[CM_ST_UNDEC], 1ull);
    }
    if (L.flag) atomicAdd((unsigned long long*)&st[CM_ST_FLAGGED], 1ull);
  } else {
    const uint32_t B = a.n_bins;
    uint32_t* rec = lds + (L.s - s_lo) * rec_words(B);
    uint32_t* cnt = rec + 2u * B;
    unsigned long long* sums = (unsigned long long*)(cnt + kCntWords);
    if (c >= 0) {
      const uint32_t bin = udiv_magic((L.n - 1u) * B, a.steps_magic);
      atomicAdd(&rec[c * B + bin], 1u);
      atomicAdd(&cnt[kCntDec0 + c], 1u);
      if (c == L.target) atomicAdd(&cnt[kCntCorrect], 1u);
      atomicAdd(&sums[c], (unsigned long long)n);
      atomicAdd(&sums[2 + c], (unsigned long long)(n * n));
    } else {
      atomicAdd(&cnt[kCntUndec], 1u);
    }
    if (L.flag) atomicAdd(&cnt[kCntFlagged], 1u);
  }
  if (a.run_choice) {
    const uint64_t idx = (uint64_t)L.s * a.trials + L.t;
    a.run_choice[idx] = (int8_t)c;
    a.run_step[idx] = L.n;
    a.run_flag[idx] = L.flag ? 1 : 0;
    if (a.run_state)
      for (int i = 0; i < width; ++i) a.run_state[idx * width + i] = state[i];
  }
}

// Flush the LDS window into the global histogram and statistics.
__device__ void flush(const SimArgs& a, const uint32_t* lds, uint32_t s_lo) {
  const uint32_t B = a.n_bins, per = 2u * B + CM_NSTAT, rw = rec_words(B);
  for (uint32_t i = threadIdx.x; i < a.window * per; i += blockDim.x) {
    const uint32_t w = i / per, j = i - w * per;
    const uint64_t sg = (uint64_t)s_lo + w;
    if (sg >= a.n_settings) continue;
    const uint32_t* rec = lds + w * rw;
    const uint32_t* cnt = rec + 2u * B;
    const unsigned long long* sums = (const unsigned long long*)(cnt + kCntWords);
    unsigned long long v;
    unsigned long long* dst;
    if (j < 2u * B) {
      v = rec[j];
      dst = (unsigned long long*)&a.hist[sg * 2u * B + j];
    } else {
      const uint32_t k = j - 2u * B;
      switch (k) {
        case CM_ST_DEC0: v = cnt[kCntDec0]; break;
        case CM_ST_DEC1: v = cnt[kCntDec1]; break;
        case CM_ST_UNDEC: v = cnt[kCntUndec]; break;
        case CM_ST_CORRECT: v = cnt[kCntCorrect]; break;
        case CM_ST_SUMN0: v = sums[0]; break;
        case CM_ST_SUMN1: v = sums[1]; break;
        case CM_ST_SUMSQ0: v = sums[2]; break;
        case CM_ST_SUMSQ1: v = sums[3]; break;
        default: v = cnt[kCntFlagged]; break;
      }
      dst = (unsigned long long*)&a.stats[sg * CM_NSTAT + k];
    }
    if (v) atomicAdd(dst, v);
  }
  if (a.tc) {
    const uint32_t per_tc = a.tc_k * kTcWords;
    const unsigned long long* src =
        (const unsigned long long*)(lds + a.window * rec_words(a.n_bins));
    for (uint32_t i = threadIdx.x; i < a.window * per_tc; i += blockDim.x) {
      const uint32_t w = i / per_tc;
      if ((uint64_t)s_lo + w >= a.n_settings) continue;
      const unsigned long long v = src[i];
      if (v) atomicAdd((unsigned long long*)&a.tc[(uint64_t)s_lo * per_tc + i], v);
    }
  }
}

// The largest count not above `want` that no active lane's `left` is below:
// the wave-uniform trip count of a step loop.  The per-lane minimum is taken
// only when some lane is within `want` (one lane read per such lane).
__device__ __forceinline__ uint32_t uniform_trips(uint32_t want, uint32_t left) {
  uint32_t t = want;
  uint64_t m = __builtin_amdgcn_ballot_w64(left < want);
  while (m) {
    const int l = __builtin_ctzll(m);
    t = min(t, (uint32_t)__builtin_amdgcn_readlane((int)left, l));
    m &= m - 1ull;
  }
  return t;
}

// The scalar multiple of M0 entering a block's first product, kept opaque so
// that the product stays one multiply-add instead of a per-lane running sum.
__device__ __forceinline__ uint64_t opaque_s(uint64_t v) {
  asm("" : "+s"(v));
  return v;
}

// ---------------------------------------------------------------------------
// Mechanisms.  Each model provides: begin(lane) -- set up a run; advance() --
// execute up to `steps` steps (a step pair per random block for the DDM),
// returning false once the run has ended; state() for dumps.
//
// The step loops count with a wave-uniform counter k: a run's step number is
// its steps before the call, n0, plus k, and enters the random numbers only
// through the first Philox product M0 (n0 + k) = M0 n0 + M0 k, whose second
// term is a scalar.  A run's own step count is therefore written only when
// it ends or the call returns.  When some lane is within `steps` of the cap
// the loop also stops each lane at its own cap (a rarely taken second form
// of the same loop).
// ---------------------------------------------------------------------------

// Drift-diffusion (Euler-Maruyama): x <- (x + a) + b z, bounds +-theta.
// Step n uses element (n-1) & 1 of block (n-1) >> 1.
template <int PREC>
struct DDM {
  double x, a_step;
  RunKey rk;
  static constexpr int kWidth = 1;

  __device__ __forceinline__ void begin(const SimArgs& A, Lane& L, uint32_t k0, uint32_t k1) {
    const double drift = A.n_signals ? A.grid[(uint64_t)L.s * A.n_signals] : A.drift;
    a_step = drift * A.dt;
    x = A.start;
    L.target = 1;  // the upper boundary is the correct response
    rk = run_key(L.t, L.s, k0, k1);
  }

  // One step from normal z (zf in FP32 steps); false once the run has ended
  // (L.n is then its decision step n).  guard = thresh - 2 eps: nearer the
  // origin no bound is within flag distance.
  template <class H>
  __device__ __forceinline__ bool one(const SimArgs& A, Lane& L, uint32_t n, double z, float zf,
                                      float af, double guard, const H& hook) {
    if (PREC == CM_FP64) x = (x + a_step) + A.b * z;
    else x = x + (double)fmaf(A.bf, zf, af);
    if constexpr (H::kPerStep) {
      L.n = n;
      hook(L, x, 0.0);
    }
    // one comparison per step; the exact tests run only within 2 eps of a
    // bound (the whole wavefront takes the branch when any lane is near; the
    // exact tests are false for the others)
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(fabs(x) >= guard) != 0, 0)) {
      const double th = A.thresh;
      if (near_th(x, th, A.flag_eps) || near_th(x, -th, A.flag_eps)) L.flag = true;
      if (x >= th) { L.choice = 1; L.n = n; return false; }
      if (x <= -th) { L.choice = 0; L.n = n; return false; }
    }
    return true;
  }

  // `pairs` step pairs (wave-uniform), every active lane having at least
  // that many whole pairs left before the cap.
  template <class H>
  __device__ __forceinline__ bool pairs_loop(const SimArgs& A, Lane& L, uint32_t k0, uint32_t k1,
                                             uint32_t pairs, const H& hook) {
    const float af = (float)a_step;
    const double guard = A.thresh - 2.0 * A.flag_eps;
    const uint32_t n0 = L.n, b0 = n0 >> 1;  // a running lane enters at an even step count
    uint64_t kM = 0;
    for (uint32_t p = 0; p < pairs; ++p) {
      const Words w = philox_run(b0, opaque_s(kM), rk, k0, k1);
      double z0 = 0, z1 = 0;
      float f0 = 0, f1 = 0;
      if (PREC == CM_FP64) normals64(w, z0, z1);
      else normals32(w, f0, f1);
      const uint32_t n = n0 + 2u * p;
      if (!one(A, L, n + 1u, z0, f0, af, guard, hook)) return false;
      if (!one(A, L, n + 2u, z1, f1, af, guard, hook)) return false;
      kM += kPhiloxM0;
    }
    L.n = n0 + 2u * pairs;
    return true;
  }

  // A running lane enters at an even step count (runs start at 0 and take
  // whole pairs until they end), so the pairs that end at or before the cap
  // need no cap test; an odd cap leaves one single step.
  template <class H>
  __device__ __forceinline__ bool advance(const SimArgs& A, Lane& L, uint32_t k0, uint32_t k1,
                                          int pairs, const H& hook) {
    const uint32_t t = uniform_trips((uint32_t)pairs, (A.max_steps - L.n) >> 1);
    if (!pairs_loop(A, L, k0, k1, t, hook)) return false;
    if (L.n + 1u == A.max_steps) {  // an odd cap's own step, first of a pair
      const Words w = philox_run(L.n >> 1, 0ull, rk, k0, k1);
      double z0 = 0, z1 = 0;
      float f0 = 0, f1 = 0;
      if (PREC == CM_FP64) normals64(w, z0, z1);
      else normals32(w, f0, f1);
      const uint32_t n = L.n + 1u;
      if (!one(A, L, n, z0, f0, (float)a_step, A.thresh - 2.0 * A.flag_eps, hook)) return false;
      L.n = n;
    }
    if (L.n == A.max_steps) {  // the cap, reached without a crossing
      L.choice = -1;
      return false;
    }
    return true;
  }

  __device__ __forceinline__ void state(double* out) const { out[0] = x; }

  // Ceiling measurement: the random numbers and updates of `steps` steps
  // (rounded up to pairs) with no tests, exits or bookkeeping.
  __device__ __forceinline__ void free_init(const SimArgs& A, const Lane& L, uint32_t k0, uint32_t k1) {
    a_step = A.drift * A.dt;
    x = A.start;
    rk = run_key(L.t, L.s, k0, k1);
  }
  __device__ __forceinline__ void free_steps(const SimArgs& A, Lane& L, uint32_t k0, uint32_t k1,
                                             uint32_t steps) {
    const float af = (float)a_step;
    const uint32_t b0 = L.n >> 1;
    uint64_t kM = 0;
    for (uint32_t p = 0; p < (steps + 1u) / 2u; ++p) {
      const Words w = philox_run(b0, opaque_s(kM), rk, k0, k1);
      kM += kPhiloxM0;
      if (PREC == CM_FP64) {
        double z0, z1;
        normals64(w, z0, z1);
        x = (x + a_step) + A.b * z0;
        x = (x + a_step) + A.b * z1;
      } else {
        float f0, f1;
        normals32(w, f0, f1);
        x = x + (double)fmaf(A.bf, f0, af);
        x = x + (double)fmaf(A.bf, f1, af);
      }
    }
    L.n += 2u * ((steps + 1u) / 2u);
  }
};

// Two-unit leaky competing accumulator with simultaneous update:
// x_i <- x_i + ((I_i - leak x_i - comp x_j) dt) + b z_i.  The run's drive:
// I_i in double (FP64), float(I_i dt) in FP32 steps.
struct LcaDrive64 {
  double in0, in1;
};
struct LcaDrive32 {
  float idt0, idt1;
};

template <int PREC>
struct LCA : std::conditional<PREC == CM_FP64, LcaDrive64, LcaDrive32>::type {
  double x0, x1;
  RunKey rk;
  static constexpr int kWidth = 2;

  __device__ __forceinline__ void begin(const SimArgs& A, Lane& L, uint32_t k0, uint32_t k1) {
    const uint32_t stim = L.t % 9u;
    const double* d = A.drive + ((uint64_t)L.s * 9u + stim) * 2u;
    if constexpr (PREC == CM_FP64) {
      this->in0 = d[0];
      this->in1 = d[1];
    } else {
      this->idt0 = (float)(d[0] * A.dt);
      this->idt1 = (float)(d[1] * A.dt);
    }
    x0 = 0.0;
    x1 = 0.0;
    L.target = A.correct[stim];
    rk = run_key(L.t, L.s, k0, k1);
  }

  // One step from the block w; false when the new state is near the
  // threshold (L.n is then n).  xf0, xf1: the float images of the state
  // (FP32 steps).
  template <class H>
  __device__ __forceinline__ bool one(const SimArgs& A, Lane& L, uint32_t n, const Words& w,
                                      float& xf0, float& xf1, const H& hook) {
    double y0, y1;
    if constexpr (PREC == CM_FP64) {
      double z0, z1;
      normals64(w, z0, z1);
      y0 = (x0 + (((this->in0 - A.leak * x0) - A.comp * x1) * A.dt)) + A.b * z0;
      y1 = (x1 + (((this->in1 - A.leak * x1) - A.comp * x0) * A.dt)) + A.b * z1;
    } else {
      float z0, z1;
      normals32(w, z0, z1);
      y0 = x0 + (double)lca_inc_f32(A.pf, this->idt0, xf0, xf1, z0);
      y1 = x1 + (double)lca_inc_f32(A.pf, this->idt1, xf1, xf0, z1);
    }
    if (A.nonneg) {
      if (y0 < 0.0) y0 = 0.0;
      if (y1 < 0.0) y1 = 0.0;
    }
    x0 = y0;
    x1 = y1;
    if constexpr (H::kPerStep) {
      L.n = n;
      hook(L, x0, x1);
    }
    // one cheap comparison per step: a lane whose new state is within 2 eps
    // of the threshold (or across it) leaves the loop at this step, and the
    // exact tests run once after the loop (advance).  FP32 steps compare the
    // float images of the new state (which the next step needs anyway) with
    // the float image of the guard: rounding is monotone, so x >= guard
    // implies float(x) >= float(guard).
    bool near;
    if constexpr (PREC == CM_FP64) {
      near = (x0 > x1 ? x0 : x1) >= A.thresh - 2.0 * A.flag_eps;
    } else {
      xf0 = (float)x0;
      xf1 = (float)x1;
      near = (xf0 >= A.guard_f) | (xf1 >= A.guard_f);
    }
    if (near) {
      L.n = n;
      return false;
    }
    return true;
  }

  // `steps` steps (wave-uniform), every active lane having at least that
  // many left before the cap.
  template <class H>
  __device__ __forceinline__ bool steps_loop(const SimArgs& A, Lane& L, uint32_t k0, uint32_t k1,
                                             uint32_t steps, const H& hook) {
    const uint32_t n0 = L.n;
    float xf0 = (float)x0, xf1 = (float)x1;
    uint64_t kM = 0;
    for (uint32_t k = 0; k < steps; ++k) {
      const Words w = philox_run(n0, opaque_s(kM), rk, k0, k1);
      if (!one(A, L, n0 + k + 1u, w, xf0, xf1, hook)) return false;
      kM += kPhiloxM0;
    }
    L.n = n0 + steps;
    return true;
  }

  template <class H>
  __device__ __forceinline__ bool advance(const SimArgs& A, Lane& L, uint32_t k0, uint32_t k1,
                                          int steps, const H& hook) {
    // the step cap bounds the trip count, so the body needs no cap test
    const uint32_t t = uniform_trips((uint32_t)steps, A.max_steps - L.n);
    if (!steps_loop(A, L, k0, k1, t, hook)) {
      // stopped near the threshold after step L.n: the exact tests
      const double th = A.thresh, eps = A.flag_eps;
      if (near_th(x0, th, eps) || near_th(x1, th, eps)) L.flag = true;
      const double mx = x0 > x1 ? x0 : x1;
      if (mx >= th) {
        L.choice = (x1 > x0) ? 1 : 0;
        if (fabs(x0 - x1) < eps) L.flag = true;
        return false;
      }
      // within 2 eps below the threshold: the run goes on from step L.n
    }
    if (L.n == A.max_steps) {  // the cap, reached without a crossing
      L.choice = -1;
      return false;
    }
    return true;
  }

  __device__ __forceinline__ void state(double* out) const {
    out[0] = x0;
    out[1] = x1;
  }

  // Ceiling measurement: the random numbers and updates of `steps` steps
  // with no tests, exits or bookkeeping (fixed drive).
  __device__ __forceinline__ void free_init(const SimArgs& A, const Lane& L, uint32_t k0, uint32_t k1) {
    if constexpr (PREC == CM_FP64) {
      this->in0 = 0.3;
      this->in1 = 0.2;
    } else {
      this->idt0 = (float)(0.3 * A.dt);
      this->idt1 = (float)(0.2 * A.dt);
    }
    x0 = 0.0;
    x1 = 0.0;
    rk = run_key(L.t, L.s, k0, k1);
  }
  __device__ __forceinline__ void free_steps(const SimArgs& A, Lane& L, uint32_t k0, uint32_t k1,
                                             uint32_t steps) {
    float xf0 = 0.0f, xf1 = 0.0f;
    const uint32_t n0 = L.n;
    uint64_t kM = 0;
    for (uint32_t k = 0; k < steps; ++k) {
      const Words w = philox_run(n0, opaque_s(kM), rk, k0, k1);
      kM += kPhiloxM0;
      if constexpr (PREC == CM_FP64) {
        double z0, z1;
        normals64(w, z0, z1);
        const double y0 = (x0 + (((this->in0 - A.leak * x0) - A.comp * x1) * A.dt)) + A.b * z0;
        const double y1 = (x1 + (((this->in1 - A.leak * x1) - A.comp * x0) * A.dt)) + A.b * z1;
        x0 = y0;
        x1 = y1;
      } else {
        float z0, z1;
        normals32(w, z0, z1);
        x0 = x0 + (double)lca_inc_f32(A.pf, this->idt0, xf0, xf1, z0);
        x1 = x1 + (double)lca_inc_f32(A.pf, this->idt1, xf1, xf0, z1);
        xf0 = (float)x0;
        xf1 = (float)x1;
      }
    }
    L.n = n0 + steps;
  }
};

// One launch covers up to kMaxBatch sweeps of the same kind and precision:
// workgroups [base[i], base[i+1]) belong to sweep i.
// TC: the time-course variant, which also samples the state every
// tc_every steps (one sweep per launch in practice; the LDS window then holds
// each setting's time-course block after all the settings' records, and the
// drain stage follows them).
//
// OCC: 0 leaves register allocation to the compiler; 4 or 8 caps the
// registers so that that many wavefronts fit on each SIMD (the register use
// versus occupancy trade-off of the paper's GPU study, Sec. 6.3; a cap below
// the kernel's natural use spills or recomputes values).
// One workgroup's chunk of a sweep: runs r0 .. r0 + chunk - 1 through the
// refill queue, the drain and the window flush.  lds: the dynamic LDS (the
// window, then the drain stage); next, drain_cnt: the workgroup's own
// counters.
template <class M, bool TC, int BLOCK>
__device__ __forceinline__ void lane_chunk(const SimArgs& a, uint64_t r0, uint32_t* lds, uint32_t& next,
                                           uint32_t* drain_cnt) {
  const uint64_t r1 = min(r0 + a.chunk, a.total_runs);
  const uint32_t len = (uint32_t)(r1 - r0);
  const uint32_t s_lo = (uint32_t)(r0 / a.trials);
  const uint32_t t_lo = (uint32_t)(r0 - (uint64_t)s_lo * a.trials);
  const uint32_t T = (uint32_t)a.trials;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);

  if (!a.direct) {
    const uint32_t words = a.window * (rec_words(a.n_bins) + (TC ? tc_words(a.tc_k) : 0u));
    for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) lds[i] = 0u;
  }
  if (threadIdx.x == 0) next = blockDim.x;
  __syncthreads();

  typename std::conditional<TC, Sample, NoSample>::type hook{};
  if constexpr (TC) {
    hook.every = a.tc_every;
    hook.K = a.tc_k;
    hook.comp = a.comp;
    hook.s_lo = a.direct ? 0u : s_lo;
    hook.base = a.direct ? (unsigned long long*)a.tc
                         : (unsigned long long*)(lds + a.window * rec_words(a.n_bins));
  }

  M m;
  Lane L;
  uint32_t off = threadIdx.x;
  bool have = off < len;
  auto setup = [&](uint32_t o) {
    const uint32_t local = t_lo + o;  // < 2^31 + chunk
    L.s = s_lo + udiv_magic(local, a.trials_magic);
    L.t = local - (L.s - s_lo) * T;
    L.n = 0;
    L.choice = -1;
    L.flag = false;
    L.next_sample = a.tc_every;
    L.sample_k = 0;
    m.begin(a, L, k0, k1);
  };
  if (have) setup(off);

  auto finish = [&]() {
    double st[M::kWidth];
    m.state(st);
    record(a, lds, s_lo, L, st, M::kWidth);
  };
  // Refill from the chunk's queue while it lasts.
  for (;;) {
    // one LDS word, the same for the whole wavefront
    if (__hip_atomic_load(&next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= len) break;
    bool running = have;
    if (running) running = m.advance(a, L, k0, k1, (int)a.steps_per_sync, hook);
    if (have && !running) {
      finish();
      off = atomicAdd(&next, 1u);
      have = off < len;
      if (have) setup(off);
    }
  }
  // Drain: every kDrainSteps steps the workgroup packs its unfinished runs
  // into the first wavefronts (through LDS); the wavefronts beyond the
  // packed list wait at the barriers without issuing vector work, which
  // leaves their issue slots to the other workgroups on the compute unit
  // instead of stepping a few live lanes each.
  M* stage_m = (M*)(lds + a.window * (rec_words(a.n_bins) + (TC ? tc_words(a.tc_k) : 0u)));
  LaneWords* stage_l = (LaneWords*)(stage_m + BLOCK);
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint64_t below = (1ull << lane) - 1ull;
  for (;;) {
    __syncthreads();  // the stage's previous contents are consumed
    const uint64_t act = __ballot(have);
    if (lane == 0) drain_cnt[w] = (uint32_t)__popcll(act);
    __syncthreads();
    uint32_t base = 0, total = 0;
    for (uint32_t v = 0; v < BLOCK / 64; ++v) {
      if (v < w) base += drain_cnt[v];
      total += drain_cnt[v];
    }
    if (have) {
      const uint32_t i = base + (uint32_t)__popcll(act & below);
      stage_m[i] = m;
      stage_l[i] = LaneWords{L.s, L.t, L.n, L.target, L.choice, L.flag ? 1u : 0u};
    }
    __syncthreads();
    if (total == 0) break;  // every run of the chunk is recorded
    const uint32_t i = w * 64u + lane;
    have = i < total;
    if (have) {
      m = stage_m[i];
      const LaneWords lw = stage_l[i];
      L.s = lw.s;
      L.t = lw.t;
      L.n = lw.n;
      L.target = lw.target;
      L.choice = lw.choice;
      L.flag = lw.flag != 0u;
      if constexpr (TC) {  // samples fall on multiples of tc_every
        L.sample_k = L.n / a.tc_every;
        L.next_sample = (L.sample_k + 1u) * a.tc_every;
      }
    }
    bool running = have;
    if (__any(running)) running = running && m.advance(a, L, k0, k1, kDrainSteps, hook);
    if (have && !running) {
      finish();
      have = false;
    }
  }
  if (!a.direct) flush(a, lds, s_lo);  // the last barrier follows every record
}

template <class M, bool TC, int OCC, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(OCC ? OCC : 1)))
void sim_lane_kernel(LaneBatch batch) {
  extern __shared__ unsigned long long lds_u64[];  // 8-byte aligned window
  __shared__ uint32_t next;
  __shared__ uint32_t drain_cnt[BLOCK / 64];
  uint32_t sw = 0;
  while (sw + 1 < batch.n && blockIdx.x >= batch.base[sw + 1]) ++sw;
  const SimArgs& a = batch.a[sw];
  lane_chunk<M, TC, BLOCK>(a, (uint64_t)(blockIdx.x - batch.base[sw]) * a.chunk, (uint32_t*)lds_u64, next,
                           drain_cnt);
}

// The persistent kernel of the device work queue.
//
// Claim: thread 0 reads the claim word (r, c) and the device's copy count.
// While request r is copied to the device and has items left (c below its
// count), one fetch-and-add takes the next item -- whichever request the
// word names by then, which is at most the newest copied one, so the item is
// run if it exists.  Once every item of r is claimed and r + 1 is copied, a
// compare-and-swap moves the word to (r + 1, 0); increments that raced past
// the count are dropped with it.  With nothing to claim, the one workgroup
// that takes the pull lock reads the host's count and copies newly published
// ring entries and their descriptors into device memory (batch by batch,
// moving the copy count forward), or passes on the host's stop flag.  A
// workgroup ends when the stop flag is set or when nothing came for
// idle_ticks of the real-time clock.  Waiting loops read with relaxed loads
// and take one acquire fence once their condition holds, so an idle
// workgroup does not keep invalidating the caches of the busy ones.
//
// A preparation piece zero-fills and writes its share of the request's
// outputs and tables, then counts itself done (release); a chunk first waits
// until every piece of its request is done -- a request's pieces are its
// first items, so they are running or finished -- and then runs as
// lane_chunk.  The workgroup that finishes a request's last chunk scores the
// sweep when it is scored and stores the request's ticket in its
// host-visible done word with a system-scope release.  Before each count or
// store that publishes work, every wavefront waits until its own stores and
// atomics are performed, the workgroup meets at a barrier, and thread 0
// publishes with one release: one L2 write-back per chunk, where a fence in
// every wavefront would write the L2 back once per wavefront.  A workgroup
// waits for a request's preparation (acquire) only on its first chunk of it.
template <class M>
__global__ __launch_bounds__(kBlock) void queue_kernel(QueueArgs q) {
  extern __shared__ unsigned long long lds_u64[];
  __shared__ uint32_t next;
  __shared__ uint32_t drain_cnt[kBlock / 64];
  __shared__ QueueDesc desc;
  __shared__ uint32_t claim[3];  // action, then (slot, item) or the pull's range [from, to)
  __shared__ QueueReq batch[kBlock];
  __shared__ double red_d[kBlock / 64];
  __shared__ unsigned long long red_k[kBlock / 64], red_c[kBlock / 64];
  constexpr uint32_t kItem = 0, kQuit = 1, kPull = 2;
  uint32_t seen_slot = ~0u;  // thread 0: the request whose preparation this workgroup last waited for
  uint64_t seen_target = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      uint32_t action = kQuit, w1 = 0, w2 = 0;
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      for (;;) {
        const unsigned long long w = __hip_atomic_load(q.word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t r = (uint32_t)(w >> 32), c = (uint32_t)w;
        const uint32_t dt = __hip_atomic_load(q.dev_tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (r < dt) {
          // An entry whose number is not r was replaced by a later request,
          // which the host publishes only once r is done: r has no items left.
          // A first look without a fence (an idle workgroup looks at the last,
          // exhausted request over and over); a fence and a second look
          // before acting on it.
          const QueueReq* e = q.dring + r % q.cap_ring;
          unsigned long long ni = __hip_atomic_load(&e->num_items, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          bool left = (uint32_t)(ni >> 32) == r && c < (uint32_t)ni;
          if (left || r + 1u < dt) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the copies made before dev_tail passed r
            ni = __hip_atomic_load(&e->num_items, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            left = (uint32_t)(ni >> 32) == r && c < (uint32_t)ni;
          }
          if (left) {
            const unsigned long long v = __hip_atomic_fetch_add(q.word, 1ull, __ATOMIC_ACQUIRE,
                                                                __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t r2 = (uint32_t)(v >> 32), c2 = (uint32_t)v;
            const QueueReq* e2 = q.dring + r2 % q.cap_ring;
            const unsigned long long ni2 = __hip_atomic_load(&e2->num_items, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((uint32_t)(ni2 >> 32) == r2 && c2 < (uint32_t)ni2) {  // a held item keeps r2's entry in place
              action = kItem;
              w1 = __hip_atomic_load(&e2->slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              w2 = c2;
              break;
            }
            continue;  // raced past the last item of r2
          }
          if (r + 1u < dt) {  // every item of r is claimed and r + 1 is on the device
            unsigned long long expect = w;
            __hip_atomic_compare_exchange_strong(q.word, &expect, (unsigned long long)(r + 1u) << 32,
                                                 __ATOMIC_RELEASE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            continue;
          }
        }
        if (__hip_atomic_load(q.pull_lock, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u &&
            atomicCAS(q.pull_lock, 0u, 1u) == 0u) {
          const uint32_t ht = __hip_atomic_load(q.tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          // a read-modify-write returns the latest copy count, with no fence
          const uint32_t d2 = __hip_atomic_fetch_add(q.dev_tail, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (ht != d2) {  // the lock is held until the copy is published
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // system scope: the host's ring and descriptors
            action = kPull;
            w1 = d2;
            w2 = ht;
            break;
          }
          if (__hip_atomic_load(q.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))
            __hip_atomic_store(q.dev_stop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          // nothing was written under the lock: a plain release of it (a
          // release fence here, in every idle workgroup's loop, would write
          // back the L2 under the busy workgroups again and again)
          __hip_atomic_store(q.pull_lock, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (__hip_atomic_load(q.dev_stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
            __builtin_amdgcn_s_memrealtime() - t0 > q.idle_ticks)
          break;  // kQuit
        __builtin_amdgcn_s_sleep(64);
      }
      claim[0] = action;
      claim[1] = w1;
      claim[2] = w2;
    }
    __syncthreads();
    const uint32_t action = claim[0];
    if (action == kQuit) return;  // the whole workgroup; it holds no lock
    if (action == kPull) {
      const uint32_t from = claim[1], to = claim[2];
      for (uint32_t base = from; base != to;) {  // counts wrap only past 2^32 requests, which the host refuses
        const uint32_t n = min(to - base, (uint32_t)kBlock);
        if (threadIdx.x < n) {
          const uint32_t at = (base + threadIdx.x) % q.cap_ring;
          QueueReq e;
          e.num_items = __hip_atomic_load(&q.ring[at].num_items, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          e.slot = __hip_atomic_load(&q.ring[at].slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          e.pad = 0;
          batch[threadIdx.x] = e;
          __hip_atomic_store(&q.dring[at].slot, e.slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&q.dring[at].num_items, e.num_items, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        for (uint32_t k = 0; k < n; ++k) {  // every entry starts a request: copy its descriptor
          const unsigned long long* src = (const unsigned long long*)&q.desc[batch[k].slot];
          unsigned long long* dst = (unsigned long long*)&q.ddesc[batch[k].slot];
          for (uint32_t i = threadIdx.x; i < sizeof(QueueDesc) / 8u; i += kBlock)
            dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        base += n;
        __builtin_amdgcn_s_waitcnt(0);  // this wave's copies are stored
        __syncthreads();                // and every wave's; batch[] is free
        if (threadIdx.x == 0) __hip_atomic_store(q.dev_tail, base, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (threadIdx.x == 0) __hip_atomic_store(q.pull_lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      continue;
    }
    const uint32_t slot = claim[1], item = claim[2];
    {
      const unsigned long long* src = (const unsigned long long*)&q.ddesc[slot];
      unsigned long long* dst = (unsigned long long*)&desc;
      for (uint32_t i = threadIdx.x; i < sizeof(QueueDesc) / 8u; i += kBlock)
        dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (item < desc.pieces) {
      const uint64_t j0 = (uint64_t)item * kQueuePrepSpan;
      const uint64_t j1 = min(j0 + kQueuePrepSpan, desc.prep.end);
      for (uint64_t j = j0 + threadIdx.x; j < j1; j += kBlock) prep_index(desc.prep, j);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0)
        __hip_atomic_fetch_add(&q.prep_done[slot], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      continue;
    }
    if (threadIdx.x == 0 && (slot != seen_slot || desc.prep_target != seen_target)) {
      while (__hip_atomic_load(&q.prep_done[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < desc.prep_target)
        __builtin_amdgcn_s_sleep(16);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      seen_slot = slot;  // this request's tables are visible to the workgroup from now on
      seen_target = desc.prep_target;
    }
    __syncthreads();
    lane_chunk<M, false, kBlock>(desc.a, (uint64_t)(item - desc.pieces) * desc.a.chunk, (uint32_t*)lds_u64,
                                 next, drain_cnt);
    __builtin_amdgcn_s_waitcnt(0);  // this wave's flushes are performed
    __syncthreads();                // and every wave's
    if (threadIdx.x == 0) {
      const uint64_t old = __hip_atomic_fetch_add(&q.chunk_done[slot], 1ull, __ATOMIC_RELEASE,
                                                  __HIP_MEMORY_SCOPE_AGENT);
      const bool last = old + 1ull == desc.chunk_target;
      if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every chunk's flushes
      claim[2] = last;
    }
    __syncthreads();
    if (claim[2]) {  // the request's last chunk
      if (desc.scored) score_sweep<kBlock / 64>(desc.score, red_d, red_k, red_c);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0)
        __hip_atomic_store(&q.done[slot], desc.ticket, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __syncthreads();  // claim[], desc and the LDS are free for the next item
  }
}

// Drift-diffusion with one wavefront per run.  Each lane draws one random
// block -- the normals of two consecutive steps -- so a wave advances its run
// 128 steps at a time.  The walk's state after any step is the start plus a
// prefix sum of independent increments a + b z, so the 128 states come from
// a wave-wide prefix scan (six shuffle rounds) and the first step that
// leaves (-theta, theta) from one ballot.  Work per run-step stays close to
// the lane-per-run kernel's (the random block and normals dominate both),
// while a run's latency drops by the scan width: the reference sweep of 10^4
// trials is only ~160 wavefronts of lane-per-run work, far too few to fill
// the GPU, so its time is the latency of its longest runs.  The scan sums the
// increments in a different order than the sequential update; the results
// differ by rounding only (far below the flag distance).
template <int PREC>
__global__ __launch_bounds__(kScanBlockMax) void ddm_scan_kernel(LaneBatch batch) {
  extern __shared__ unsigned long long lds_u64[];
  uint32_t* lds = (uint32_t*)lds_u64;
  uint32_t sw = 0;
  while (sw + 1 < batch.n && blockIdx.x >= batch.base[sw + 1]) ++sw;
  const SimArgs& a = batch.a[sw];
  const uint64_t r0 = (uint64_t)(blockIdx.x - batch.base[sw]) * a.chunk;
  const uint64_t r1 = min(r0 + a.chunk, a.total_runs);
  const uint32_t len = (uint32_t)(r1 - r0);
  const uint32_t s_lo = (uint32_t)(r0 / a.trials);
  const uint32_t t_lo = (uint32_t)(r0 - (uint64_t)s_lo * a.trials);
  const uint32_t T = (uint32_t)a.trials;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const int lane = threadIdx.x & 63;
  const uint32_t N = a.max_steps;
  const double th = a.thresh, eps = a.flag_eps;

  if (!a.direct)
    for (uint32_t i = threadIdx.x; i < a.window * rec_words(a.n_bins); i += blockDim.x) lds[i] = 0u;
  __syncthreads();

  // The wavefronts take the chunk's runs round-robin.  Every loop exit
  // depends only on wave-uniform values (scalar registers), so each loop is
  // left by the whole wavefront at once and needs no per-lane bookkeeping.
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t nwave = blockDim.x >> 6;
  for (uint32_t off = wave; off < len; off += nwave) {
    Lane L;
    const uint32_t local = t_lo + off;
    L.s = s_lo + udiv_magic(local, a.trials_magic);
    L.t = local - (L.s - s_lo) * T;
    L.target = 1;
    L.flag = false;
    L.choice = -1;
    L.n = N;
    const double drift = a.n_signals ? a.grid[(uint64_t)L.s * a.n_signals] : a.drift;
    const double as = drift * a.dt;
    const float af = (float)as, bf = a.bf;
    const RunKey rk = run_key(L.t, L.s, k0, k1);
    double xs = a.start;  // state before the block
    uint32_t n0 = 0;      // steps executed before the block
    for (;;) {
      const uint32_t s1 = n0 + 2u * (uint32_t)lane + 1u, s2 = s1 + 1u;  // this lane's steps
      // block (n0 / 2) + lane: the wave's common part enters as a scalar
      const Words w = philox_run((uint32_t)lane, (uint64_t)kPhiloxM0 * (n0 >> 1), rk, k0, k1);
      double d1, d2;
      if (PREC == CM_FP64) {
        double z0, z1;
        normals64(w, z0, z1);
        d1 = as + a.b * z0;
        d2 = as + a.b * z1;
      } else {
        float z0, z1;
        normals32(w, z0, z1);
        d1 = (double)fmaf(bf, z0, af);
        d2 = (double)fmaf(bf, z1, af);
      }
      double p = d1 + d2;  // inclusive prefix over lanes of the pair sums
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const double v = __shfl_up(p, o, 64);
        if (lane >= o) p = p + v;
      }
      double ex = __shfl_up(p, 1, 64);
      ex = lane ? ex : 0.0;
      const double x1 = (xs + ex) + d1, x2 = xs + p;
      const bool v1 = s1 <= N, v2 = s2 <= N;
      const bool c1 = v1 && (x1 >= th || x1 <= -th);
      const bool c2 = v2 && (x2 >= th || x2 <= -th);
      const uint64_t crossed = __ballot(c1 || c2);
      uint32_t dstep = 0xFFFFFFFFu;
      int lc = 0;
      if (crossed) {
        lc = (int)__builtin_ctzll(crossed);
        dstep = __builtin_amdgcn_readfirstlane((uint32_t)__shfl((int)(c1 ? s1 : s2), lc, 64));
      }
      const bool f1 = v1 && s1 <= dstep && (near_th(x1, th, eps) || near_th(x1, -th, eps));
      const bool f2 = v2 && s2 <= dstep && (near_th(x2, th, eps) || near_th(x2, -th, eps));
      if (__ballot(f1 || f2)) L.flag = true;
      if (crossed) {
        xs = __shfl(c1 ? x1 : x2, lc, 64);
        L.n = dstep;
        L.choice = xs >= th ? 1 : 0;
        break;
      }
      if (n0 + 128u >= N) {  // the cap falls in this block: undecided at step N
        const int ln = (int)((N - n0 - 1u) >> 1);
        xs = __shfl(((N - n0) & 1u) ? x1 : x2, ln, 64);
        L.n = N;
        L.choice = -1;
        break;
      }
      xs = __shfl(x2, 63, 64);
      n0 += 128u;
    }
    if (lane == 0) record(a, lds, s_lo, L, &xs, 1);
  }
  if (!a.direct) {
    __syncthreads();
    flush(a, lds, s_lo);
  }
}

// The lane kernels' step with everything else taken away: every lane runs
// `steps` steps of random numbers and updates from the start state and
// writes its final first unit (so the work cannot be optimised out).  The
// rate it reaches is the measured ceiling of the step's instruction mix.
template <class M>
__global__ __launch_bounds__(kBlock) void ceiling_kernel(SimArgs a, uint32_t steps, double* out) {
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Lane L{};
  L.s = 0;
  L.t = (uint32_t)g;
  L.n = 2u * ((uint32_t)g & 255u);  // lanes of a sweep are at different steps
  M m;
  m.free_init(a, L, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
  m.free_steps(a, L, (uint32_t)a.seed, (uint32_t)(a.seed >> 32), steps);
  double st[M::kWidth];
  m.state(st);
  out[g] = st[0];
}

template <class M, int BLOCK>
void launch_occ(const LaneBatch& b, uint32_t occ, size_t lds, hipStream_t st) {
  const dim3 grid(b.base[b.n]), block(BLOCK);
  if (occ == 4)
    hipLaunchKernelGGL((sim_lane_kernel<M, false, 4, BLOCK>), grid, block, lds, st, b);
  else if (occ == 8)
    hipLaunchKernelGGL((sim_lane_kernel<M, false, 8, BLOCK>), grid, block, lds, st, b);
  else
    hipLaunchKernelGGL((sim_lane_kernel<M, false, 0, BLOCK>), grid, block, lds, st, b);
}

template <class M>
hipError_t launch_model(const LaneBatch& b, bool tc, uint32_t occ, uint32_t block, size_t lds,
                        hipStream_t st) {
  if (tc)
    hipLaunchKernelGGL((sim_lane_kernel<M, true, 0, kBlock>), dim3(b.base[b.n]), dim3(kBlock), lds, st, b);
  else if (block == 512)
    launch_occ<M, 512>(b, occ, lds, st);
  else if (block == 1024)
    launch_occ<M, 1024>(b, occ, lds, st);
  else
    launch_occ<M, kBlock>(b, occ, lds, st);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sim_lane(int kind, int precision, uint32_t scan_block, bool tc, uint32_t occ,
                           uint32_t block, const LaneBatch& b, size_t lds_bytes, hipStream_t st) {
  if (b.n < 1 || b.n > kMaxBatch || (scan_block && tc) || (occ && occ != 4 && occ != 8) ||
      (block != 256 && block != 512 && block != 1024) || (tc && block != (uint32_t)kBlock))
    return hipErrorInvalidValue;
  if (scan_block) {
    if (kind != CM_DDM || (scan_block != 256u && scan_block != (uint32_t)kScanBlockMax))
      return hipErrorInvalidValue;
    if (precision == CM_FP64)
      hipLaunchKernelGGL((ddm_scan_kernel<CM_FP64>), dim3(b.base[b.n]), dim3(scan_block), lds_bytes, st, b);
    else
      hipLaunchKernelGGL((ddm_scan_kernel<CM_FP32_STEP>), dim3(b.base[b.n]), dim3(scan_block), lds_bytes, st, b);
    return hipGetLastError();
  }
  if (kind == CM_DDM)
    return precision == CM_FP64 ? launch_model<DDM<CM_FP64>>(b, tc, occ, block, lds_bytes, st)
                                : launch_model<DDM<CM_FP32_STEP>>(b, tc, occ, block, lds_bytes, st);
  return precision == CM_FP64 ? launch_model<LCA<CM_FP64>>(b, tc, occ, block, lds_bytes, st)
                              : launch_model<LCA<CM_FP32_STEP>>(b, tc, occ, block, lds_bytes, st);
}

hipError_t launch_queue(int kind, int precision, const QueueArgs& q, uint32_t groups, size_t lds_bytes,
                        hipStream_t st) {
  if (kind != CM_CONFLICT_LCA || groups < 1) return hipErrorInvalidValue;
  if (precision == CM_FP64)
    hipLaunchKernelGGL(queue_kernel<LCA<CM_FP64>>, dim3(groups), dim3(kBlock), lds_bytes, st, q);
  else
    hipLaunchKernelGGL(queue_kernel<LCA<CM_FP32_STEP>>, dim3(groups), dim3(kBlock), lds_bytes, st, q);
  return hipGetLastError();
}

size_t lane_stage_bytes(int kind, int precision, uint32_t block) {
  size_t m;
  if (kind == CM_DDM) m = precision == CM_FP64 ? sizeof(DDM<CM_FP64>) : sizeof(DDM<CM_FP32_STEP>);
  else m = precision == CM_FP64 ? sizeof(LCA<CM_FP64>) : sizeof(LCA<CM_FP32_STEP>);
  return (size_t)block * (m + sizeof(LaneWords));
}

hipError_t launch_ceiling(int kind, int precision, const SimArgs& a, uint32_t steps, uint64_t lanes,
                          double* out, hipStream_t st) {
  if (lanes % kBlock || lanes / kBlock > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((uint32_t)(lanes / kBlock)), block(kBlock);
  if (kind == CM_DDM) {
    if (precision == CM_FP64)
      hipLaunchKernelGGL((ceiling_kernel<DDM<CM_FP64>>), grid, block, 0, st, a, steps, out);
    else
      hipLaunchKernelGGL((ceiling_kernel<DDM<CM_FP32_STEP>>), grid, block, 0, st, a, steps, out);
  } else {
    if (precision == CM_FP64)
      hipLaunchKernelGGL((ceiling_kernel<LCA<CM_FP64>>), grid, block, 0, st, a, steps, out);
    else
      hipLaunchKernelGGL((ceiling_kernel<LCA<CM_FP32_STEP>>), grid, block, 0, st, a, steps, out);
  }
  return hipGetLastError();
}

}  // namespace cm
