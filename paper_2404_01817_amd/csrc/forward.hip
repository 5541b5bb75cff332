// forward.hip -- the calculation stage (Section 3.3) over population x inputs.
//
// Mapping "lane per sample": a 64-lane wave evaluates one genome on a run of
// 64-sample tiles, one sample per lane.  The genome's program is uniform
// across the wave, so it is read with scalar loads and every branch on a
// node's activation or aggregation is a scalar branch.  A workgroup holds up
// to four waves working on the same genome, so they share the CU's scalar
// cache.
//
// Two stores for the value vector v of Section 3.3 (slots, see program.h):
//   AsmStore  64 VGPRs per lane (v0..v63, layout REG, N_max <= 62); the node
//             loop is the assembly of node_loop_asm.h, which indexes the
//             registers in GPR-index mode with the program's uniform slots;
//   LdsStore  one LDS row of 64 lanes per slot (any layout; rows are 256 B,
//             so lane l of every row sits in bank l), node loop in C++.
// Edges come in pairs (the program pads each node to an even count with a
// neutral edge) and the first two pairs sit in the node's record, so the
// inner loops have no per-edge tests.  The next record is fetched while the
// current node computes.
//
// Inputs of the next tile are copied HBM -> LDS by the DMA path of
// global_load_lds (16-byte pieces when aligned) while the current tile
// computes; each lane then moves its own sample's inputs into v.  Outputs
// are stored from v directly.  Workgroups are remapped so consecutive
// genomes share an XCD (workgroups are dealt to the 8 XCDs round robin).
#include <hip/hip_runtime.h>

#include "act.h"
#include "launch.h"
#include "neat.h"
#include "node_loop_asm.h"
#include "program.h"

namespace neat {
namespace {

constexpr int TILE = 64;
constexpr int WAVES = 4;  // waves per workgroup, all on one genome

typedef float f32x32 __attribute__((ext_vector_type(32)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef const __attribute__((address_space(4))) int32_t cprog_t;
typedef const __attribute__((address_space(4))) i32x8 cint8_t;  // unused
typedef const __attribute__((address_space(4))) i32x16 cint16_t;
typedef __attribute__((address_space(1))) const void gvoid;
typedef __attribute__((address_space(3))) void lvoid;

__device__ __forceinline__ float fbits(int b) { return __int_as_float(b); }

// ---------------------------------------------------------------- stores
struct LdsStore {
    float *col;  // this lane's column: slot s at col[s * TILE]
    int layout;
    __device__ __forceinline__ float get_lo(int s) const { return col[s * TILE]; }
    __device__ __forceinline__ float get_hi(int s) const { return col[s * TILE]; }
    template <bool HI>
    __device__ __forceinline__ void set(int s, float x) { col[s * TILE] = x; }
    __device__ __forceinline__ void init(int N) {
        const int z0 = zero_slot(layout, N);
        col[z0 * TILE] = 0.0f;
        col[(z0 + 1) * TILE] = 1.0f;
    }
};

// Value vector pinned to v0..v63 for the assembly node loop
// (node_loop_asm.h).  Slots are absolute (0..63); M0, which the GPR-index
// mode overwrites, is saved and restored around every access.
struct AsmStore {
    f32x32 lo, hi;
    __device__ __forceinline__ float get(int s) const {
        float x;
        asm volatile(
            "s_mov_b32 s91, m0\n\t"
            "s_set_gpr_idx_on %3, gpr_idx(SRC0)\n\t"
            "v_mov_b32_e32 %0, v0\n\t"
            "s_set_gpr_idx_off\n\t"
            "s_mov_b32 m0, s91"
            : "=&v"(x)
            : "{v[0:31]}"(lo), "{v[32:63]}"(hi), "s"(s)
            : "s91");
        return x;
    }
    __device__ __forceinline__ float get_lo(int s) const { return get(s); }
    __device__ __forceinline__ float get_hi(int s) const { return get(s); }
    template <bool HI>
    __device__ __forceinline__ void set(int s, float x) {
        asm volatile(
            "s_mov_b32 s91, m0\n\t"
            "s_set_gpr_idx_on %2, gpr_idx(DST)\n\t"
            "v_mov_b32_e32 v0, %3\n\t"
            "s_set_gpr_idx_off\n\t"
            "s_mov_b32 m0, s91"
            : "+{v[0:31]}"(lo), "+{v[32:63]}"(hi)
            : "s"(s), "v"(x)
            : "s91");
    }
    __device__ __forceinline__ void init(int /*N*/) {
        set<true>(62, 0.0f);
        set<true>(63, 1.0f);
    }
    // all computed nodes of the genome (node_loop_asm.h)
    __device__ __forceinline__ void run(const int32_t *rec, const int32_t *edg, int n) {
        asm volatile(NEAT_NODE_LOOP_ASM
                     : "+{v[0:31]}"(lo), "+{v[32:63]}"(hi)
                     : [rec] "s"(rec), [edg] "s"(edg), [n] "s"(n)
                     : NEAT_NODE_LOOP_CLOBBERS);
    }
};

// ---------------------------------------------------------------- nodes (C++)
// One term w * v[slot] combined into acc (class ACLS); NaN terms of a max
// are remembered in nan (the hardware max ignores NaN).
template <int ACLS, class Store>
__device__ __forceinline__ void combine(float &acc, float &nan, int slot, float w, const Store &v) {
    const float x = v.get_lo(slot);
    if (ACLS == ACLS_SUM) {
        acc = fmaf(w, x, acc);
    } else if (ACLS == ACLS_PROD) {
        acc *= w * x;
    } else {
        const float t = w * x;
        acc = fmaxf(acc, t);
        nan = (t != t) ? t : nan;
    }
}

// pairs edge pairs: the first two from the record (r), then the overflow
// array from e, four words per pair.
template <int ACLS, class Store>
__device__ __forceinline__ float aggregate(const i32x16 &r, cprog_t *e, int pairs,
                                           const Store &v) {
    float acc = ACLS == ACLS_SUM ? 0.0f : (ACLS == ACLS_PROD ? 1.0f : -__builtin_inff());
    float nan = 0.0f;
#pragma unroll
    for (int p = 0; p < REC_INLINE_PAIRS; ++p) {
        if (p < pairs) {
            combine<ACLS>(acc, nan, r[REC_PAIRS + 4 * p], fbits(r[REC_PAIRS + 4 * p + 1]), v);
            combine<ACLS>(acc, nan, r[REC_PAIRS + 4 * p + 2], fbits(r[REC_PAIRS + 4 * p + 3]),
                          v);
        }
    }
    for (int p = 0; p < pairs - REC_INLINE_PAIRS; ++p) {
        combine<ACLS>(acc, nan, e[4 * p], fbits(e[4 * p + 1]), v);
        combine<ACLS>(acc, nan, e[4 * p + 2], fbits(e[4 * p + 3]), v);
    }
    if (ACLS == ACLS_MAX) acc = (nan != nan) ? nan : acc;
    return acc;
}

// Lane select with a uniform 64-bit mask (all ones or zero): mask ? b : a.
__device__ __forceinline__ float sel_mask(float a, float b, unsigned long long mask) {
    float r;
    asm volatile("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(mask));
    return r;
}

template <class Store>
__device__ __forceinline__ void run_program(cprog_t *prog, int N, int O, int I, int /*layout*/,
                                            Store &v) {
    const int ncomp = prog[HDR_NVALID] - I;
    if (ncomp <= 0) return;
    cprog_t *rec = prog + rec_off(O);
    cprog_t *e = prog + edge_off(N, O);
    i32x16 r = *(cint16_t *)rec;
    for (int k = 0; k < ncomp; ++k) {
        const unsigned code = (unsigned)r[REC_CODE];
        const int pairs = (int)(code & 0xffffu), acls = (int)((code >> 16) & 3u);
        const int xcls = (int)((code >> 18) & 3u), dst = (int)(code >> 20);
        const float bias = fbits(r[REC_BIAS]), resp = fbits(r[REC_RESP]);
        const float cf = fbits(r[REC_C]), ea = fbits(r[REC_EA]), eb = fbits(r[REC_EB]);
        const unsigned long long mask =
            ((unsigned long long)(unsigned)r[REC_MASK + 1] << 32) | (unsigned)r[REC_MASK];
        // next record (the record array has room for N records)
        const i32x16 rn = *(cint16_t *)(rec + REC_WORDS * (k + 1));
        float a;
        if (acls == ACLS_SUM) a = aggregate<ACLS_SUM>(r, e, pairs, v);
        else if (acls == ACLS_PROD) a = aggregate<ACLS_PROD>(r, e, pairs, v);
        else a = aggregate<ACLS_MAX>(r, e, pairs, v);
        if (pairs > REC_INLINE_PAIRS) e += 4 * (pairs - REC_INLINE_PAIRS);
        const float z = fmaf(resp, a, bias);
        float y;
        if (xcls == XCLS_PL) {
            // identity, abs, relu: z above 0 (or NaN) passes, else c z or 0
            y = !(z <= 0.0f) ? z : sel_mask(z * cf, 0.0f, mask);
        } else if (xcls == XCLS_EXPO) {
            // sigmoid, tanh: ea + eb / (1 + 2^(c z)); gaussian: 2^(c z z)
            const float ex = exp2_hw(cf * sel_mask(z, z * z, mask));
            y = sel_mask(fmaf(eb, rcp_hw(1.0f + ex), ea), ex, mask);
        } else {
            y = act_sin(z);
        }
        v.template set<false>(dst, y);
        r = rn;
    }
}

__device__ __forceinline__ void run_program(cprog_t *prog, int N, int O, int I, int /*layout*/,
                                            AsmStore &v) {
    const int ncomp = prog[HDR_NVALID] - I;
    const int32_t *p = (const int32_t *)prog;
    v.run(p + rec_off(O), p + edge_off(N, O), ncomp > 0 ? ncomp : 0);
}

// ---------------------------------------------------------------- tiles
struct FwdArgs {
    const int32_t *prog;
    const float *inputs;
    float *outputs;
    long long gstride;  // floats between genomes' input blocks (0 = shared)
    long long first;    // grid mode: first query
    int N, C, I, O, B, tiles, tpw, chunks, wpg, groups, prog_words, side, vec4, layout;
};

// Workgroup b is dealt to XCD b % 8; give each XCD a contiguous range.
__device__ __forceinline__ int xcd_item(unsigned b, unsigned n) {
    const unsigned x = b & 7u, q = b >> 3, per = n >> 3, rem = n & 7u;
    return (int)(x * per + (x < rem ? x : rem) + q);
}

// Issue the DMA of n consecutive floats src[0..n) into lds[0..n).
__device__ __forceinline__ void dma_inputs(const float *src, float *lds, int n, int vec4) {
    const int lane = (int)(threadIdx.x & (TILE - 1));
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

// Wait for this wave's DMA (the waves of a workgroup never share LDS data).
__device__ __forceinline__ void wait_dma() {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <class Store>
__device__ __forceinline__ void place_inputs(Store &v, const float *cur, int I, int /*layout*/,
                                             int lane) {
    for (int i = 0; i < I; ++i) v.template set<false>(i, cur[lane * I + i]);  // slot i
}

template <class Store>
__device__ __forceinline__ void place_grid(Store &v, long long q, int side) {
    const int pts = side * side;
    const int p1 = (int)(q / pts), p2 = (int)(q - (long long)p1 * pts);
    const float den = (float)(side - 1);
    v.template set<false>(0, (float)(2 * (p1 % side) - (side - 1)) / den);
    v.template set<false>(1, (float)(2 * (p1 / side) - (side - 1)) / den);
    v.template set<false>(2, (float)(2 * (p2 % side) - (side - 1)) / den);
    v.template set<false>(3, (float)(2 * (p2 / side) - (side - 1)) / den);
    v.template set<false>(4, 1.0f);
}

// stage: this wave's input staging area (2 x TILE x I floats, unused in GRID)
template <class Store, bool GRID>
__device__ __forceinline__ void forward_body(const FwdArgs &a, float *stage, Store &v) {
    const int lane = (int)(threadIdx.x & (TILE - 1));
    const int wave = (int)(threadIdx.x / TILE);
    const int grp = xcd_item(blockIdx.x, gridDim.x);
    const int g = grp / a.groups;
    const int chunk = (grp - g * a.groups) * a.wpg + wave;
    if (wave >= a.wpg || chunk >= a.chunks) return;
    const int t0 = chunk * a.tpw;
    const int t1 = min(a.tiles, t0 + a.tpw);
    const int N = a.N, I = a.I, O = a.O, B = a.B, L = a.layout;
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
    if (!GRID)
        dma_inputs(in_g + (size_t)t0 * TILE * I, buf0, min(TILE, B - t0 * TILE) * I, a.vec4);
    v.init(N);

    for (int t = t0; t < t1; ++t) {
        const int nb = min(TILE, B - t * TILE);
        if (GRID) {
            place_grid(v, a.first + (long long)t * TILE + lane, a.side);
        } else {
            wait_dma();
            place_inputs(v, ((t - t0) & 1) ? buf1 : buf0, I, L, lane);
            if (t + 1 < t1) {
                // every lane has read its inputs before the other buffer refills
                __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
                __builtin_amdgcn_wave_barrier();
                dma_inputs(in_g + (size_t)(t + 1) * TILE * I, ((t - t0) & 1) ? buf0 : buf1,
                           min(TILE, B - (t + 1) * TILE) * I, a.vec4);
            }
        }
        run_program(prog, N, O, I, L, v);
        if (lane < nb) {
            float *o = out_g + (size_t)(t * TILE + lane) * O;
            for (int j = 0; j < O; ++j) {
                const int s = prog[out_off() + j];
                o[j] = v.get_lo(s);
            }
        }
    }
}

template <bool GRID>
__global__ __launch_bounds__(TILE *WAVES) void forward_asm_kernel(FwdArgs a) {
    extern __shared__ float smem[];
    AsmStore v;
    const size_t stage = GRID ? 0 : (size_t)2 * TILE * a.I;
    forward_body<AsmStore, GRID>(a, smem + (threadIdx.x / TILE) * stage, v);
}

template <bool GRID>
__global__ __launch_bounds__(TILE *WAVES) void forward_lds_kernel(FwdArgs a) {
    extern __shared__ float smem[];
    const size_t stage = GRID ? 0 : (size_t)2 * TILE * a.I;
    const size_t rows = (size_t)n_slots(a.layout, a.N) * TILE;
    float *base = smem + (threadIdx.x / TILE) * (stage + rows);
    LdsStore v;
    v.col = base + stage + (threadIdx.x & (TILE - 1));
    v.layout = a.layout;
    forward_body<LdsStore, GRID>(a, base, v);
}

int choose_chunks(int P, int tiles, int *tpw) {
    // aim at ~32k waves: enough to fill 256 CUs several times over while a
    // wave still reuses its genome's program across a run of tiles
    const long long target = 32768;
    long long chunks = (target + P - 1) / (P > 0 ? P : 1);
    if (chunks < 1) chunks = 1;
    if (chunks > tiles) chunks = tiles;
    *tpw = (int)((tiles + chunks - 1) / chunks);
    return (tiles + *tpw - 1) / *tpw;
}

}  // namespace

size_t forward_lds_bytes(int N, int I, int variant, bool grid) {
    const size_t stage = grid ? 0 : (size_t)2 * TILE * I;
    if (variant == FWD_REG) return sizeof(float) * stage;
    return sizeof(float) * (stage + (size_t)n_slots(layout_of(N), N) * TILE);
}

int forward_default_variant(int N) { return layout_of(N) == LAYOUT_WIDE ? FWD_LDS : FWD_REG; }

size_t forward_launch_lds_bytes(int P, int B, int N, int I, int variant, bool grid) {
    int tpw;
    const int tiles = (B + TILE - 1) / TILE;
    const int chunks = choose_chunks(P, tiles, &tpw);
    const int wpg = chunks < WAVES ? chunks : WAVES;
    return forward_lds_bytes(N, I, variant, grid) * (size_t)wpg;
}

hipError_t launch_forward(int P, int N, int C, int I, int O, const int32_t *prog,
                          const float *inputs, int64_t gstride, int B, float *outputs,
                          int variant, bool grid, int side, int64_t first, hipStream_t stream) {
    FwdArgs a{};
    a.prog = prog;
    a.inputs = inputs;
    a.outputs = outputs;
    a.gstride = gstride;
    a.first = first;
    a.N = N, a.C = C, a.I = I, a.O = O, a.B = B, a.side = side;
    a.layout = layout_of(N);
    a.tiles = (B + TILE - 1) / TILE;
    a.chunks = choose_chunks(P, a.tiles, &a.tpw);
    a.wpg = a.chunks < WAVES ? a.chunks : WAVES;
    a.groups = (a.chunks + a.wpg - 1) / a.wpg;
    a.prog_words = prog_words(N, C, O);
    a.vec4 = (!grid && ((uintptr_t)inputs % 16 == 0) && (gstride % 4 == 0)) ? 1 : 0;
    const unsigned blocks = (unsigned)((long long)P * a.groups);
    const dim3 block(TILE * a.wpg);
    const size_t lds = forward_lds_bytes(N, I, variant, grid) * a.wpg;
    if (variant == FWD_REG) {
        if (grid)
            hipLaunchKernelGGL((forward_asm_kernel<true>), dim3(blocks), block, lds, stream, a);
        else
            hipLaunchKernelGGL((forward_asm_kernel<false>), dim3(blocks), block, lds, stream, a);
    } else {
        if (grid)
            hipLaunchKernelGGL((forward_lds_kernel<true>), dim3(blocks), block, lds, stream, a);
        else
            hipLaunchKernelGGL((forward_lds_kernel<false>), dim3(blocks), block, lds, stream, a);
    }
    return hipGetLastError();
}

}  // namespace neat
