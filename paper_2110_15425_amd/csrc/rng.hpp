// rng.hpp -- counter-based random numbers for the simulation kernels.
//
// Every evaluation draws from its own stream, so that any lane, in any
// order, reproduces the same numbers (the per-evaluation generator
// requirement of the Distill paper, Sec. 3.6).  Instead of a per-thread
// generator state saved and restored around each evaluation (which cost the
// paper's GPU code kilobytes of private memory per thread, Sec. 6.3), the
// stream is Philox4x32-10 (Salmon et al., SC'11) evaluated on a counter:
// key = seed, counter = (step block k, trial, setting, stream id).  No state
// lives in memory; a block costs ten rounds of two 32x32->64 multiplies.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cm {

constexpr uint32_t kStreamDrive = 0x40000000u;  // rate network input drive
constexpr uint32_t kStreamTie = 0xFFFFFFFFu;    // tie-break priorities

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

struct Words {
  uint32_t w0, w1, w2, w3;
};

// a ^ b ^ k in one VALU instruction: gfx950's three-input bitwise op with the
// truth table of a three-way exclusive or (0x96); k is wave-uniform.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

// k0, k1 must be wave-uniform (they are: the key is the sweep's seed).
__device__ __forceinline__ Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;  // one v_mad_u64_u32 each
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
  return Words{c0, c1, c2, c3};
}

// Philox4x32-10 on the counter (n, t, s, 0) of a run's own stream, with the
// work that depends only on the run -- trial t and setting s, not the step
// n -- done once per run.  Of round 1 only the product with n varies; round
// 2 multiplies the run's constant c0 (its product is a per-run constant) and
// leaves c3 = lo of that product, a per-run constant that round 3 xors in.
// The words equal philox(n, t, s, 0, k0, k1) bit for bit.

struct RunKey {
  uint32_t a;    // round 1: c0 = hi(M1 s) ^ t ^ k0
  uint32_t b2;   // round 2: lo(M1 s) ^ (k0 + W0), xored with hi(M1 c2)
  uint32_t c2;   // round 2: hi(M0 a) ^ (k1 + W1), xored with c3
  uint32_t d3;   // round 3: lo(M0 a) ^ (k1 + 2 W1), xored with hi(M0 c0)
};

__device__ __forceinline__ RunKey run_key(uint32_t t, uint32_t s, uint32_t k0, uint32_t k1) {
  const uint64_t p1 = (uint64_t)kPhiloxM1 * s;
  RunKey r;
  r.a = (uint32_t)(p1 >> 32) ^ t ^ k0;
  r.b2 = (uint32_t)p1 ^ (k0 + kPhiloxW0);
  const uint64_t pa = (uint64_t)kPhiloxM0 * r.a;
  r.c2 = (uint32_t)(pa >> 32) ^ (k1 + kPhiloxW1);
  r.d3 = (uint32_t)pa ^ (k1 + 2u * kPhiloxW1);
  return r;
}

// The block of counter n + k: M0 (n + k) = M0 n + kM with kM = M0 k
// (wave-uniform, supplied by the caller) is one multiply-add; n + k < 2^32.
__device__ __forceinline__ Words philox_run(uint32_t n, uint64_t kM, const RunKey& r, uint32_t k0,
                                            uint32_t k1) {
  // round 1: (a, lo(M1 s), hi(M0 n') ^ k1, lo(M0 n')) for n' = n + k
  const uint64_t p0 = (uint64_t)kPhiloxM0 * n + kM;
  const uint32_t x2 = (uint32_t)(p0 >> 32) ^ k1, x3 = (uint32_t)p0;
  // round 2: the product with a is per run (in c2 and d3)
  const uint64_t q1 = (uint64_t)kPhiloxM1 * x2;
  uint32_t c0 = (uint32_t)(q1 >> 32) ^ r.b2, c1 = (uint32_t)q1, c2 = x3 ^ r.c2;
  // round 3: its c3 input is the per-run lo(M0 a)
  const uint64_t u0 = (uint64_t)kPhiloxM0 * c0, u1 = (uint64_t)kPhiloxM1 * c2;
  c0 = xor3((uint32_t)(u1 >> 32), c1, k0 + 2u * kPhiloxW0);
  c1 = (uint32_t)u1;
  c2 = (uint32_t)(u0 >> 32) ^ r.d3;
  uint32_t c3 = (uint32_t)u0;
  // rounds 4..10
#pragma unroll
  for (uint32_t round = 3; round < 10; ++round) {
    const uint64_t v0 = (uint64_t)kPhiloxM0 * c0, v1 = (uint64_t)kPhiloxM1 * c2;
    const uint32_t m0 = xor3((uint32_t)(v1 >> 32), c1, k0 + round * kPhiloxW0);
    const uint32_t m2 = xor3((uint32_t)(v0 >> 32), c3, k1 + round * kPhiloxW1);
    c1 = (uint32_t)v1;
    c3 = (uint32_t)v0;
    c0 = m0;
    c2 = m2;
  }
  return Words{c0, c1, c2, c3};
}

// 53-bit uniform in (0, 1] from a word pair: ((hi:lo) >> 11) + 1, times 2^-53.
// Built from two exact int->double conversions (the value fits in 53 bits).
__device__ __forceinline__ double uniform53(uint32_t lo, uint32_t hi) {
  const uint32_t top = hi >> 11;                   // bits 52..32 of the 53-bit value
  const uint32_t bot = (hi << 21) | (lo >> 11);    // bits 31..0
  const double v = __dadd_rn(__dmul_rn((double)top, 4294967296.0), (double)bot);
  return __dmul_rn(__dadd_rn(v, 1.0), 0x1p-53);
}

// Two standard normals (Box-Muller) from one block, in double:
// rho = sqrt(-2 ln u_a), angle 2 pi u_b.  The angle is evaluated as
// sincospi(2 u_b): 2 u_b is exact, so the argument reduction is a trivial
// exact one instead of a general Payne-Hanek reduction, and the result is
// cos/sin of 2 pi u_b without the rounding of the product 2 pi u_b.
__device__ __forceinline__ void normals64(const Words& w, double& z0, double& z1) {
  const double ua = uniform53(w.w0, w.w1);
  const double ub = uniform53(w.w2, w.w3);
  const double rho = sqrt(__dmul_rn(-2.0, log(ua)));
  double s, c;
  sincospi(__dmul_rn(2.0, ub), &s, &c);
  z0 = __dmul_rn(rho, c);
  z1 = __dmul_rn(rho, s);
}

// Two standard normals in float from the top 24 bits of words 1 and 3, on
// the hardware transcendental units: v_log_f32 is log2, and v_sin_f32 /
// v_cos_f32 take their argument in revolutions, so the angle 2*pi*u needs no
// multiply.  rho = sqrt(-2 ln u) = sqrt(-2 ln2 * log2 u).
__device__ __forceinline__ void normals32(const Words& w, float& z0, float& z1) {
  // ((m >> 8) + 1) 2^-24 as one exact fused multiply-add: (m >> 8) < 2^24 is
  // exact in float and so is the result
  const float ua = fmaf((float)(w.w1 >> 8), 0x1p-24f, 0x1p-24f);
  const float ub = fmaf((float)(w.w3 >> 8), 0x1p-24f, 0x1p-24f);
  const float rho = __builtin_amdgcn_sqrtf(-1.38629436f * __builtin_amdgcn_logf(ua));
  z0 = rho * __builtin_amdgcn_cosf(ub);
  z1 = rho * __builtin_amdgcn_sinf(ub);
}

}  // namespace cm
