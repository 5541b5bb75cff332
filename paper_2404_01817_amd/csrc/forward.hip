// forward.hip -- the calculation stage (Section 3.3) over population x inputs.
//
// Mapping "lane per sample": one 64-lane wave runs one genome's program over
// 64 input vectors, one per lane.  The program is uniform across the wave,
// so its records and edges are read with scalar loads and every branch on
// the node's activation or aggregation is a scalar branch (no divergence).
// The node-value vector v of Section 3.3 lives in LDS as v[position][lane]
// with a row stride of 65 words: reading v[src] for all lanes touches 64
// consecutive banks, and the cooperative input staging (where neighbouring
// lanes hold different inputs of the same sample) is also conflict-free.
//
// Inputs are staged with coalesced loads: the wave's 64 x I input floats are
// one contiguous block that lane l reads at l, l + 64, ...; outputs are
// gathered from LDS and written the same way.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "neat.h"
#include "program.h"
#include "act.h"

namespace neat {
namespace {

constexpr int TILE = 64;        // samples per wave
constexpr int VSTRIDE = TILE + 1;

// The program is read-only for the whole grid: reading it through the
// constant address space lets uniform reads become scalar loads.
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(4))) int32_t cprog_t;
typedef const __attribute__((address_space(4))) i32x4 cint4_t;
typedef const __attribute__((address_space(4))) i32x2 cint2_t;

__device__ __forceinline__ cprog_t *as_const(const int32_t *p) {
    return (cprog_t *)(p);
}

// Run the program of one genome for the lane's sample; v points at the
// lane's column of the value matrix (row stride VSTRIDE).  Positions
// 0..I-1 (the inputs) must already be written.
__device__ __forceinline__ void run_program(cprog_t *prog, int N, int O, int I, float *v) {
    const int nvalid = prog[HDR_NVALID];
    cint4_t *rec = (cint4_t *)(prog + rec_off(O));
    cint2_t *edge = (cint2_t *)(prog + edge_off(N, O));
    int ep = 0;
    for (int k = 0; k < nvalid - I; ++k) {
        const i32x4 r = rec[k];
        const int deg = r.x & 0xffff;
        const int act = (r.x >> 16) & 0xff;
        const int agg = (r.x >> 24) & 0xff;
        const float bias = __int_as_float(r.y);
        const float resp = __int_as_float(r.z);
        const float inv = __int_as_float(r.w);
        float a = 0.0f;
        if (deg > 0) {
            cint2_t *e = edge + ep;
            if (agg == AGG_SUM || agg == AGG_MEAN) {
                float acc = 0.0f;
                for (int i = 0; i < deg; ++i) {
                    const i32x2 ed = e[i];
                    acc = fmaf(__int_as_float(ed.y), v[ed.x * VSTRIDE], acc);
                }
                a = (agg == AGG_MEAN) ? acc * inv : acc;
            } else if (agg == AGG_PRODUCT) {
                float acc = 1.0f;
                for (int i = 0; i < deg; ++i) {
                    const i32x2 ed = e[i];
                    acc *= __int_as_float(ed.y) * v[ed.x * VSTRIDE];
                }
                a = acc;
            } else if (agg == AGG_MAX) {
                const i32x2 e0 = e[0];
                float m = __int_as_float(e0.y) * v[e0.x * VSTRIDE];
                for (int i = 1; i < deg; ++i) {
                    const i32x2 ed = e[i];
                    const float t = __int_as_float(ed.y) * v[ed.x * VSTRIDE];
                    m = (t > m || t != t) ? t : m;
                }
                a = m;
            } else {  // AGG_MIN
                const i32x2 e0 = e[0];
                float m = __int_as_float(e0.y) * v[e0.x * VSTRIDE];
                for (int i = 1; i < deg; ++i) {
                    const i32x2 ed = e[i];
                    const float t = __int_as_float(ed.y) * v[ed.x * VSTRIDE];
                    m = (t < m || t != t) ? t : m;
                }
                a = m;
            }
            ep += deg;
        }
        v[(I + k) * VSTRIDE] = act_eval(act, fmaf(resp, a, bias));
    }
}

struct FwdArgs {
    const int32_t *prog;
    const float *inputs;
    float *outputs;
    long long gstride;  // floats between genomes' input blocks (0 = shared)
    int N, C, I, O, B, tiles, prog_words;
    // grid mode
    int side;
    long long first;
};

// Write the wave's nb x O outputs from the value matrix (coalesced).
__device__ __forceinline__ void store_outputs(cprog_t *prog, const float *sv,
                                              float *out, int nb, int O) {
    const int t = (int)threadIdx.x;
    const int n = nb * O;
    int s = t / O, j = t - (t / O) * O;
    const int ds = TILE / O, dj = TILE - (TILE / O) * O;
    for (int e = t; e < n; e += TILE) {
        out[e] = sv[prog[out_off() + j] * VSTRIDE + s];
        s += ds;
        j += dj;
        if (j >= O) {
            j -= O;
            ++s;
        }
    }
}

// Copy the wave's contiguous block of n = nb * I input floats into the value
// matrix: element e is input e % I of sample e / I, stored at row e % I (the
// inputs occupy positions 0..I-1).  Loads are issued 16 at a time per lane
// before any LDS write, so their latencies overlap.
__device__ __forceinline__ void stage_inputs(const float *__restrict__ in, float *sv, int n, int I) {
    constexpr int K = 16;
    const int t = (int)threadIdx.x;
    int s = t / I, i = t - (t / I) * I;
    const int ds = TILE / I, di = TILE - (TILE / I) * I;
    for (int base = 0; base < n; base += K * TILE) {
        float x[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = base + k * TILE + t;
            x[k] = (e < n) ? __builtin_nontemporal_load(in + e) : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = base + k * TILE + t;
            if (e < n) sv[i * VSTRIDE + s] = x[k];
            s += ds;
            i += di;
            if (i >= I) {
                i -= I;
                ++s;
            }
        }
    }
}

__global__ __launch_bounds__(TILE) void forward_lds_kernel(FwdArgs a) {
    extern __shared__ float sv[];
    const int t = (int)threadIdx.x;
    const int g = (int)(blockIdx.x / (unsigned)a.tiles);
    const int tile = (int)(blockIdx.x - (unsigned)g * (unsigned)a.tiles);
    const int N = a.N, I = a.I, O = a.O, B = a.B;
    cprog_t *prog = as_const(a.prog + (size_t)g * a.prog_words);
    const int b0 = tile * TILE;
    const int nb = min(TILE, B - b0);
    float *out = a.outputs + ((size_t)g * B + b0) * O;

    if (prog[HDR_STATUS] != 0) {
        for (int e = t; e < nb * O; e += TILE) out[e] = __builtin_nanf("");
        return;
    }
    stage_inputs(a.inputs + (size_t)g * a.gstride + (size_t)b0 * I, sv, nb * I, I);
    __syncthreads();
    run_program(prog, N, O, I, sv + t);
    __syncthreads();
    store_outputs(prog, sv, out, nb, O);
}

// CPPN queries: inputs (x1, y1, x2, y2, 1) generated from the query index.
__global__ __launch_bounds__(TILE) void forward_grid_kernel(FwdArgs a) {
    extern __shared__ float sv[];
    const int t = (int)threadIdx.x;
    const int g = (int)(blockIdx.x / (unsigned)a.tiles);
    const int tile = (int)(blockIdx.x - (unsigned)g * (unsigned)a.tiles);
    const int N = a.N, I = a.I, O = a.O, B = a.B;
    cprog_t *prog = as_const(a.prog + (size_t)g * a.prog_words);
    const int b0 = tile * TILE;
    const int nb = min(TILE, B - b0);
    float *out = a.outputs + ((size_t)g * B + b0) * O;

    if (prog[HDR_STATUS] != 0) {
        for (int e = t; e < nb * O; e += TILE) out[e] = __builtin_nanf("");
        return;
    }
    {
        const int side = a.side, pts = side * side;
        const long long q = a.first + b0 + t;
        const int p1 = (int)(q / pts), p2 = (int)(q - (long long)p1 * pts);
        const float den = (float)(side - 1);
        float *v = sv + t;
        v[0 * VSTRIDE] = (float)(2 * (p1 % side) - (side - 1)) / den;
        v[1 * VSTRIDE] = (float)(2 * (p1 / side) - (side - 1)) / den;
        v[2 * VSTRIDE] = (float)(2 * (p2 % side) - (side - 1)) / den;
        v[3 * VSTRIDE] = (float)(2 * (p2 / side) - (side - 1)) / den;
        v[4 * VSTRIDE] = 1.0f;
    }
    run_program(prog, N, O, I, sv + t);
    __syncthreads();
    store_outputs(prog, sv, out, nb, O);
}

}  // namespace

size_t forward_lds_bytes(int N) { return sizeof(float) * (size_t)N * VSTRIDE; }

hipError_t launch_forward(int P, int N, int C, int I, int O, const int32_t *prog,
                          const float *inputs, int64_t gstride, int B, float *outputs,
                          hipStream_t stream) {
    FwdArgs a{};
    a.prog = prog;
    a.inputs = inputs;
    a.outputs = outputs;
    a.gstride = gstride;
    a.N = N, a.C = C, a.I = I, a.O = O, a.B = B;
    a.tiles = (B + TILE - 1) / TILE;
    a.prog_words = prog_words(N, C, O);
    const unsigned blocks = (unsigned)((long long)P * a.tiles);
    hipLaunchKernelGGL(forward_lds_kernel, dim3(blocks), dim3(TILE), forward_lds_bytes(N),
                       stream, a);
    return hipGetLastError();
}

hipError_t launch_forward_grid(int P, int N, int C, int I, int O, const int32_t *prog,
                               int side, int64_t first, int Q, float *outputs,
                               hipStream_t stream) {
    FwdArgs a{};
    a.prog = prog;
    a.outputs = outputs;
    a.N = N, a.C = C, a.I = I, a.O = O, a.B = Q;
    a.tiles = (Q + TILE - 1) / TILE;
    a.prog_words = prog_words(N, C, O);
    a.side = side;
    a.first = first;
    const unsigned blocks = (unsigned)((long long)P * a.tiles);
    hipLaunchKernelGGL(forward_grid_kernel, dim3(blocks), dim3(TILE), forward_lds_bytes(N),
                       stream, a);
    return hipGetLastError();
}

}  // namespace neat
