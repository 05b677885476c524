// lca_step.hpp -- the two-unit leaky competing accumulator's step in the
// FP32-steps mode, shared by every kernel that steps it (fused, closed-loop,
// node-by-node), so that they agree bit for bit.
//
// x_i <- x_i + ((I_i - leak x_i - comp x_j) dt) + b z_i, with the increment in
// float: the products leak dt, comp dt and I_i dt are rounded to float once,
// and each unit's increment is then three fused multiply-adds,
// inc_i = b z_i + (I_i dt - leak dt x_i - comp dt x_j), added to the double
// accumulator.
#pragma once

#include <hip/hip_runtime.h>

namespace cm {

struct LcaF32 {
  float ldt, cdt, b;
};

__host__ __device__ inline LcaF32 lca_f32(double leak, double comp, double dt, double b) {
  return LcaF32{(float)(leak * dt), (float)(comp * dt), (float)b};
}

// idt = float(I_i dt); xi, xj = float images of the unit and its competitor.
__device__ __forceinline__ float lca_inc_f32(const LcaF32& p, float idt, float xi, float xj, float z) {
  return fmaf(p.b, z, fmaf(-p.cdt, xj, fmaf(-p.ldt, xi, idt)));
}

}  // namespace cm
