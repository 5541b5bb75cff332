// forward_reg.hip -- calculation stage (Section 3.3) with the node-value
// vector held in registers, for genomes of up to 64 nodes.
//
// Mapping: one 64-lane wave evaluates one genome on a run of 64-sample
// tiles, one sample per lane.  The genome's program is uniform across the
// wave and is read with scalar loads; the value vector v of Section 3.3 is a
// per-lane array of 32 or 64 VGPRs indexed with the program's (uniform)
// positions through the GPR-indexing mode, so the hot loop touches neither
// LDS nor vector memory: per incoming edge it is one indexed move and one
// fused multiply-add.  The next node's record and first eight edges are
// fetched while the current node computes.
//
// Inputs of the next tile are copied from HBM into LDS by the DMA path of
// global_load_lds (16-byte pieces when aligned) while the current tile
// computes; each lane then moves its own sample's I inputs from LDS into v.
// Outputs are stored straight from registers.
//
// Work items (genome, run of tiles) are spread so that consecutive items of
// a genome land on the same XCD (workgroups are dealt to the 8 XCDs round
// robin), keeping a program's lines in one L2.
#include <hip/hip_runtime.h>

#include "act.h"
#include "launch.h"
#include "neat.h"
#include "program.h"

namespace neat {
namespace {

constexpr int TILE = 64;

typedef float f32x32 __attribute__((ext_vector_type(32)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef const __attribute__((address_space(4))) int32_t cprog_t;
typedef const __attribute__((address_space(4))) i32x4 cint4_t;
typedef const __attribute__((address_space(4))) i32x16 cint16_t;
typedef __attribute__((address_space(1))) const void gvoid;
typedef __attribute__((address_space(3))) void lvoid;

// Value vector of 32 or 64 VGPRs.  Writes go to a half chosen at compile
// time (HI), so that a loop writing one half never merges whole vectors.
template <int NV>
struct VReg;

template <>
struct VReg<32> {
    f32x32 lo;
    __device__ __forceinline__ float get(int i) const { return lo[i]; }
    template <bool HI>
    __device__ __forceinline__ void set(int i, float x) { lo[i] = x; }
};

template <>
struct VReg<64> {
    f32x32 lo, hi;
    __device__ __forceinline__ float get(int i) const {
        if (i < 32) return lo[i];
        return hi[i - 32];
    }
    template <bool HI>
    __device__ __forceinline__ void set(int i, float x) {
        if (HI) hi[i - 32] = x;
        else lo[i] = x;
    }
};

__device__ __forceinline__ float w_of(int bits) { return __int_as_float(bits); }

// max (MAX) or min of the deg >= 1 incoming terms; a NaN term wins.
template <int NV, bool MAX>
__device__ __forceinline__ float extreme(int deg, const i32x16 &e, cprog_t *more,
                                         const VReg<NV> &v) {
    float m = w_of(e[1]) * v.get(e[0]);
#pragma unroll
    for (int i = 1; i < 8; ++i) {
        if (i < deg) {
            const float t = w_of(e[2 * i + 1]) * v.get(e[2 * i]);
            m = ((MAX ? t > m : t < m) || t != t) ? t : m;
        }
    }
    for (int i = 8; i < deg; ++i) {
        const float t = w_of(more[2 * i + 1]) * v.get(more[2 * i]);
        m = ((MAX ? t > m : t < m) || t != t) ? t : m;
    }
    return m;
}

// Aggregate the deg incoming terms w * v[src]: the first eight edges come in
// registers (e), the rest are read from the program (more points at edge 0).
template <int NV>
__device__ __forceinline__ float aggregate(int agg, int deg, const i32x16 &e, cprog_t *more,
                                           const VReg<NV> &v) {
    if (deg == 0) return 0.0f;
    if (agg == AGG_SUM || agg == AGG_MEAN) {
        float acc = 0.0f;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (i < deg) acc = fmaf(w_of(e[2 * i + 1]), v.get(e[2 * i]), acc);
        for (int i = 8; i < deg; ++i) acc = fmaf(w_of(more[2 * i + 1]), v.get(more[2 * i]), acc);
        return acc;
    }
    if (agg == AGG_PRODUCT) {
        float acc = 1.0f;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (i < deg) acc *= w_of(e[2 * i + 1]) * v.get(e[2 * i]);
        for (int i = 8; i < deg; ++i) acc *= w_of(more[2 * i + 1]) * v.get(more[2 * i]);
        return acc;
    }
    return agg == AGG_MAX ? extreme<NV, true>(deg, e, more, v) : extreme<NV, false>(deg, e, more, v);
}

// Program cursor: current record, its first eight edges, first edge index.
struct Cursor {
    i32x4 r;
    i32x16 e;
    int ep;
};

// Evaluate records k0 .. k1-1 (positions I+k0 .. I+k1-1, all in one half).
template <int NV, bool HI>
__device__ __forceinline__ void run_nodes(cint4_t *rec, cprog_t *edges, int I, int k0, int k1,
                                          Cursor &c, VReg<NV> &v) {
    for (int k = k0; k < k1; ++k) {
        const int deg = c.r.x & 0xffff;
        const int act = (c.r.x >> 16) & 0xff;
        const int agg = (c.r.x >> 24) & 0xff;
        const float bias = __int_as_float(c.r.y);
        const float resp = __int_as_float(c.r.z);
        const float inv = __int_as_float(c.r.w);
        const int epn = c.ep + deg;
        // prefetch the next record and its first eight edges (the record
        // array has room for N records and the program ends with slack)
        const i32x4 rn = rec[k + 1];
        const i32x16 en = *(cint16_t *)(edges + 2 * epn);
        float a = aggregate<NV>(agg, deg, c.e, edges + 2 * c.ep, v);
        if (agg == AGG_MEAN) a *= inv;
        v.template set<HI>(I + k, act_eval(act, fmaf(resp, a, bias)));
        c.r = rn;
        c.e = en;
        c.ep = epn;
    }
}

template <int NV>
__device__ __forceinline__ void run_program(cprog_t *prog, int N, int O, int I, VReg<NV> &v) {
    const int ncomp = prog[HDR_NVALID] - I;
    if (ncomp <= 0) return;
    cint4_t *rec = (cint4_t *)(prog + rec_off(O));
    cprog_t *edges = prog + edge_off(N, O);
    Cursor c;
    c.r = rec[0];
    c.e = *(cint16_t *)(edges);
    c.ep = 0;
    if (NV == 32) {
        run_nodes<NV, false>(rec, edges, I, 0, ncomp, c, v);
    } else {
        const int split = min(ncomp, max(0, 32 - I));  // records whose position is < 32
        run_nodes<NV, false>(rec, edges, I, 0, split, c, v);
        run_nodes<NV, true>(rec, edges, I, split, ncomp, c, v);
    }
}

struct RegArgs {
    const int32_t *prog;
    const float *inputs;
    float *outputs;
    long long gstride;
    long long first;  // grid mode: first query
    int N, C, I, O, B, tiles, tpw, chunks, prog_words, side, vec4;
};

// Workgroup b is dealt to XCD b % 8; give each XCD a contiguous range of
// work items so a genome's items share an L2.
__device__ __forceinline__ int xcd_item(unsigned b, unsigned n) {
    const unsigned x = b & 7u, q = b >> 3, per = n >> 3, rem = n & 7u;
    return (int)(x * per + (x < rem ? x : rem) + q);
}

// Issue the DMA of n consecutive floats src[0..n) into lds[0..n).
__device__ __forceinline__ void dma_inputs(const float *src, float *lds, int n, int vec4) {
    const int lane = (int)threadIdx.x;
    if (vec4) {
        const int n4 = n >> 2;
        for (int c = 0; c < n4; c += TILE)
            if (c + lane < n4)
                __builtin_amdgcn_global_load_lds((gvoid *)(src + 4 * (c + lane)),
                                                 (lvoid *)(lds + 4 * c), 16, 0, 0);
        const int rem = n & 3;
        if (lane < rem)
            __builtin_amdgcn_global_load_lds((gvoid *)(src + 4 * n4 + lane),
                                             (lvoid *)(lds + 4 * n4), 4, 0, 0);
    } else {
        for (int c = 0; c < n; c += TILE)
            if (c + lane < n)
                __builtin_amdgcn_global_load_lds((gvoid *)(src + c + lane), (lvoid *)(lds + c), 4,
                                                 0, 0);
    }
}

__device__ __forceinline__ void wait_dma() {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
}

template <int NV, bool GRID>
__global__ __launch_bounds__(TILE) void forward_reg_kernel(RegArgs a) {
    extern __shared__ float stage[];  // GRID ? unused : 2 x TILE x I floats
    const int lane = (int)threadIdx.x;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    const int g = item / a.chunks;
    const int t0 = (item - g * a.chunks) * a.tpw;
    const int t1 = min(a.tiles, t0 + a.tpw);
    const int N = a.N, I = a.I, O = a.O, B = a.B;
    cprog_t *prog = (cprog_t *)(a.prog + (size_t)g * a.prog_words);
    float *out_g = a.outputs + (size_t)g * B * O;
    if (t0 >= t1) return;

    if (prog[HDR_STATUS] != 0) {
        const int e1 = min(B, t1 * TILE) * O;
        for (int e = t0 * TILE * O + lane; e < e1; e += TILE) out_g[e] = __builtin_nanf("");
        return;
    }

    const float *in_g = GRID ? nullptr : a.inputs + (size_t)g * a.gstride;
    float *buf0 = stage, *buf1 = stage + TILE * I;
    if (!GRID) dma_inputs(in_g + (size_t)t0 * TILE * I, buf0, min(TILE, B - t0 * TILE) * I, a.vec4);

    for (int t = t0; t < t1; ++t) {
        const int nb = min(TILE, B - t * TILE);
        VReg<NV> v;
        if (GRID) {
            const int side = a.side, pts = side * side;
            const long long q = a.first + (long long)t * TILE + lane;
            const int p1 = (int)(q / pts), p2 = (int)(q - (long long)p1 * pts);
            const float den = (float)(side - 1);
            v.template set<false>(0, (float)(2 * (p1 % side) - (side - 1)) / den);
            v.template set<false>(1, (float)(2 * (p1 / side) - (side - 1)) / den);
            v.template set<false>(2, (float)(2 * (p2 % side) - (side - 1)) / den);
            v.template set<false>(3, (float)(2 * (p2 / side) - (side - 1)) / den);
            v.template set<false>(4, 1.0f);
        } else {
            wait_dma();
            const float *cur = ((t - t0) & 1) ? buf1 : buf0;
            const int ilo = min(I, 32);
            for (int i = 0; i < ilo; ++i) v.template set<false>(i, cur[lane * I + i]);
            for (int i = ilo; i < I; ++i) v.template set<true>(i, cur[lane * I + i]);
            if (t + 1 < t1) {
                __syncthreads();  // every lane has read cur before the other buffer refills
                dma_inputs(in_g + (size_t)(t + 1) * TILE * I, ((t - t0) & 1) ? buf0 : buf1,
                           min(TILE, B - (t + 1) * TILE) * I, a.vec4);
            }
        }
        run_program<NV>(prog, N, O, I, v);
        if (lane < nb) {
            float *o = out_g + (size_t)(t * TILE + lane) * O;
            for (int j = 0; j < O; ++j) o[j] = v.get(prog[out_off() + j]);
        }
    }
}

int choose_chunks(int P, int tiles, int *tpw) {
    // aim at ~32k work items: enough waves to fill 256 CUs several times over,
    // while a wave still reuses its genome's program across a run of tiles
    const long long target = 32768;
    long long chunks = (target + P - 1) / (P > 0 ? P : 1);
    if (chunks < 1) chunks = 1;
    if (chunks > tiles) chunks = tiles;
    *tpw = (int)((tiles + chunks - 1) / chunks);
    return (tiles + *tpw - 1) / *tpw;
}

template <bool GRID>
hipError_t launch_reg(int P, int N, int C, int I, int O, const int32_t *prog, const float *inputs,
                      int64_t gstride, int64_t first, int side, int B, float *outputs,
                      hipStream_t stream) {
    RegArgs a{};
    a.prog = prog;
    a.inputs = inputs;
    a.outputs = outputs;
    a.gstride = gstride;
    a.first = first;
    a.N = N, a.C = C, a.I = I, a.O = O, a.B = B, a.side = side;
    a.tiles = (B + TILE - 1) / TILE;
    a.chunks = choose_chunks(P, a.tiles, &a.tpw);
    a.prog_words = prog_words(N, C, O);
    a.vec4 = (!GRID && ((uintptr_t)inputs % 16 == 0) && (gstride % 4 == 0)) ? 1 : 0;
    const unsigned blocks = (unsigned)((long long)P * a.chunks);
    const size_t lds = GRID ? 0 : sizeof(float) * 2 * TILE * (size_t)I;
    if (N <= 32)
        hipLaunchKernelGGL((forward_reg_kernel<32, GRID>), dim3(blocks), dim3(TILE), lds, stream,
                           a);
    else
        hipLaunchKernelGGL((forward_reg_kernel<64, GRID>), dim3(blocks), dim3(TILE), lds, stream,
                           a);
    return hipGetLastError();
}

}  // namespace

size_t forward_reg_lds_bytes(int I) { return sizeof(float) * 2 * TILE * (size_t)I; }

hipError_t launch_forward_reg(int P, int N, int C, int I, int O, const int32_t *prog,
                              const float *inputs, int64_t gstride, int B, float *outputs,
                              hipStream_t stream) {
    return launch_reg<false>(P, N, C, I, O, prog, inputs, gstride, 0, 0, B, outputs, stream);
}

hipError_t launch_forward_reg_grid(int P, int N, int C, int I, int O, const int32_t *prog,
                                   int side, int64_t first, int Q, float *outputs,
                                   hipStream_t stream) {
    return launch_reg<true>(P, N, C, I, O, prog, nullptr, 0, first, side, Q, outputs, stream);
}

}  // namespace neat
