// act.h -- node activation functions of the forward kernels (device code).
//
// The activations of the node encoding (codes in program.h) are built on
// the hardware's base-2 exponential and reciprocal instead of the general
// library routines, which cost several times more instructions.  Each is
// accurate to a few units in the last place of fp32 in absolute terms for
// results of magnitude <= 1 (tanh, sigmoid, sin, gaussian) -- far inside
// the 1e-5 absolute parity tolerance against the double-precision oracle:
//
//   sigmoid(z) = 1 / (1 + 2^(-z log2 e))
//   tanh(z)    = 1 - 2 / (1 + 2^(2 z log2 e))         (exact limits +-1 at +-inf)
//   gaussian(z)= 2^(-(z z) log2 e)
//   sin(z)     : Cody-Waite reduction by pi/2 (two-constant split with fma),
//                then the Taylor polynomials of sin / cos on [-pi/4, pi/4]
//                (degree 9 and 10) selected by quadrant
//   relu(z)    = z unless z <= 0 (so NaN propagates), abs and identity exact.
#pragma once

#include <hip/hip_runtime.h>

#include "program.h"

namespace neat {

__device__ __forceinline__ float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float act_sigmoid(float z) {
    return rcp_hw(1.0f + exp2_hw(z * -1.4426950216293335f));
}

__device__ __forceinline__ float act_tanh(float z) {
    const float t = exp2_hw(z * 2.885390043258667f);
    return fmaf(-2.0f, rcp_hw(1.0f + t), 1.0f);
}

__device__ __forceinline__ float act_gauss(float z) {
    return exp2_hw((z * z) * -1.4426950216293335f);
}

__device__ __forceinline__ float act_relu(float z) { return !(z <= 0.0f) ? z : 0.0f; }

__device__ __forceinline__ float act_sin(float z) {
    // k = nearest integer to z / (pi/2); r = z - k pi/2 with pi/2 = P1 + P2
    const float kf = __builtin_rintf(z * 0.6366197466850281f);
    float r = fmaf(kf, -1.5707963705062866f, z);
    r = fmaf(kf, 4.371138828673793e-08f, r);
    const int q = (int)kf;
    const float r2 = r * r;
    // sin r = r + r^3 (-1/6 + r^2 (1/120 + r^2 (-1/5040 + r^2 / 362880)))
    float ps = fmaf(r2, 2.7557318844628753e-06f, -0.00019841270113829523f);
    ps = fmaf(r2, ps, 0.008333333767950535f);
    ps = fmaf(r2, ps, -0.1666666716337204f);
    const float s = fmaf(r * r2, ps, r);
    // cos r = 1 + r^2 (-1/2 + r^2 (1/24 + r^2 (-1/720 + r^2 (1/40320 - r^2 / 3628800))))
    float pc = fmaf(r2, -2.755731998149713e-07f, 2.4801587642286904e-05f);
    pc = fmaf(r2, pc, -0.0013888889225199819f);
    pc = fmaf(r2, pc, 0.0416666679084301f);
    pc = fmaf(r2, pc, -0.5f);
    const float c = fmaf(r2, pc, 1.0f);
    const float v = (q & 1) ? c : s;
    return (q & 2) ? -v : v;
}

__device__ __forceinline__ float act_eval(int act, float z) {
    switch (act) {
    case ACT_IDENTITY: return z;
    case ACT_TANH: return act_tanh(z);
    case ACT_SIGMOID: return act_sigmoid(z);
    case ACT_RELU: return act_relu(z);
    case ACT_SIN: return act_sin(z);
    case ACT_GAUSS: return act_gauss(z);
    case ACT_ABS: return fabsf(z);
    }
    return __builtin_nanf("");
}

}  // namespace neat
