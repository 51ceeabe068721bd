// The Heisenberg Metropolis move of the sweep kernels (Sec. 4): a proposal
// uniform on the sphere from two uniforms and the float32 acceptance test.
// Both sweep kernels use these functions, so they agree bit for bit.
//
// The trigonometric and exponential functions are the hardware ones:
// v_sin_f32 / v_cos_f32 take their argument in revolutions (sin(2 pi x)),
// which is the proposal's angle 2 pi u1 without a multiplication or range
// reduction; v_exp_f32 is 2^x; v_sqrt_f32 is the square root.  Their errors
// are a few float32 ulps, far below the 1e-5 per-component agreement with
// a float64 computation of the same move.
#pragma once
#include <hip/hip_runtime.h>

namespace smc {

__device__ __forceinline__ float3 heis_proposal(float u0, float u1) {
    const float z = 2.0f * u0 - 1.0f;
    const float rho = __builtin_amdgcn_sqrtf(1.0f - z * z);
    const float sn = __builtin_amdgcn_sinf(u1), cs = __builtin_amdgcn_cosf(u1);
    return make_float3(rho * cs, rho * sn, z);
}

// exp(-beta dE) as 2^(-beta dE log2 e).
__device__ __forceinline__ float heis_boltzmann(float beta, float dE) {
    return __builtin_amdgcn_exp2f(-beta * dE * 1.4426950408889634f);
}

// s / |s|: the renormalisation of a spin (after every 16th sweep).  The
// separate renormalisation kernel and the one-pass sweep, which applies it
// as it stores the sweep's last plane, share this function.
__device__ __forceinline__ float3 heis_unit(float x, float y, float z) {
    const float n = sqrtf(__builtin_fmaf(x, x, __builtin_fmaf(y, y, z * z)));
    return make_float3(x / n, y / n, z / n);
}

}  // namespace smc
