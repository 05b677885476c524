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
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;  // one v_mad_u64_u32 each
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
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
