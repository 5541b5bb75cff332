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
//   sin(z)     : Cody-Waite reduction by pi (two-constant split with fma),
//                then the Taylor polynomial of sin of degree 13 on
//                [-pi/2, pi/2] (truncation below 7e-10), sign by the parity
//                of the multiple of pi
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
    // k = nearest integer to z / pi; r = z - k pi with pi = fl(pi) - (fl(pi) - pi)
    const float kf = __builtin_rintf(z * 0.31830987334251404f);
    float r = fmaf(kf, -3.1415927410125732f, z);
    r = fmaf(8.742277657347586e-08f, kf, r);
    const int q = (int)kf;
    const float r2 = r * r;
    // sin r = r + r^3 (-1/3! + r^2 (1/5! + r^2 (-1/7! + r^2 (1/9! + r^2 (-1/11! + r^2 / 13!)))))
    float p = fmaf(r2, 1.6059044372074283e-10f, -2.5052107943679403e-08f);
    p = fmaf(r2, p, 2.7557318844628753e-06f);
    p = fmaf(r2, p, -0.00019841270113829523f);
    p = fmaf(r2, p, 0.008333333767950535f);
    p = fmaf(r2, p, -0.1666666716337204f);
    const float s = fmaf(r * r2, p, r);
    // sin(r + k pi) = (-1)^k sin r: odd k flips the sign bit
    return __uint_as_float(__float_as_uint(s) + ((unsigned)q << 31));
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
