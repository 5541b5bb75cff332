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
//   RegStore  32 or 64 VGPRs per lane, indexed through the GPR-index mode
//             with the program's uniform slot numbers (layouts REG32, REG64);
//   LdsStore  one LDS row of 64 lanes per slot (any layout; rows are 256 B,
//             so lane l of every row sits in bank l).
// Edges come in pairs (the program pads each half to an even count with a
// neutral edge), so the inner loop has no per-edge tests.  The next node's
// record is fetched while the current node computes.
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
#include "program.h"

namespace neat {
namespace {

constexpr int TILE = 64;
constexpr int WAVES = 4;  // waves per workgroup, all on one genome

typedef float f32x32 __attribute__((ext_vector_type(32)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef const __attribute__((address_space(4))) int32_t cprog_t;
typedef const __attribute__((address_space(4))) i32x8 cint8_t;
typedef const __attribute__((address_space(4))) i32x16 cint16_t;
typedef __attribute__((address_space(1))) const void gvoid;
typedef __attribute__((address_space(3))) void lvoid;

__device__ __forceinline__ float fbits(int b) { return __int_as_float(b); }

// ---------------------------------------------------------------- stores
template <int NV>
struct RegStore;

template <>
struct RegStore<32> {
    f32x32 lo;
    __device__ __forceinline__ float get_lo(int s) const { return lo[s]; }
    __device__ __forceinline__ float get_hi(int s) const { return lo[s]; }
    template <bool HI>
    __device__ __forceinline__ void set(int s, float x) { lo[s] = x; }
    __device__ __forceinline__ void init(int /*N*/) {
        lo[30] = 0.0f;
        lo[31] = 1.0f;
    }
};

template <>
struct RegStore<64> {
    f32x32 lo, hi;
    __device__ __forceinline__ float get_lo(int s) const { return lo[s]; }
    __device__ __forceinline__ float get_hi(int s) const { return hi[s - 32]; }
    template <bool HI>
    __device__ __forceinline__ void set(int s, float x) {
        if (HI) hi[s - 32] = x;
        else lo[s] = x;
    }
    __device__ __forceinline__ void init(int /*N*/) {
        lo[30] = 0.0f;
        lo[31] = 1.0f;
        hi[30] = 0.0f;
        hi[31] = 1.0f;
    }
};

struct LdsStore {
    float *col;  // this lane's column: slot s at col[s * TILE]
    int layout;
    __device__ __forceinline__ float get_lo(int s) const { return col[s * TILE]; }
    __device__ __forceinline__ float get_hi(int s) const { return col[s * TILE]; }
    template <bool HI>
    __device__ __forceinline__ void set(int s, float x) { col[s * TILE] = x; }
    __device__ __forceinline__ void init(int N) {
        const int z0 = zero_slot(layout, N, 0);
        col[z0 * TILE] = 0.0f;
        col[(z0 + 1) * TILE] = 1.0f;
        if (layout == LAYOUT_REG64) {
            col[62 * TILE] = 0.0f;
            col[63 * TILE] = 1.0f;
        }
    }
};

// ---------------------------------------------------------------- edges
// Combine n pairs of terms w * v[slot] (edges from e) into acc.
template <int AGG, bool HIGH, class Store>
__device__ __forceinline__ float combine_pairs(float acc, cprog_t *e, int n, const Store &v) {
    for (int p = 0; p < n; p += 4) {
        const i32x16 ch = *(cint16_t *)(e + 4 * p);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (p + q < n) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int slot = ch[4 * q + 2 * u];
                    const float w = fbits(ch[4 * q + 2 * u + 1]);
                    const float x = HIGH ? v.get_hi(slot) : v.get_lo(slot);
                    if (AGG == AGG_SUM) {
                        acc = fmaf(w, x, acc);
                    } else if (AGG == AGG_PRODUCT) {
                        acc *= w * x;
                    } else {
                        const float t = w * x;
                        acc = ((AGG == AGG_MAX ? t > acc : t < acc) || t != t) ? t : acc;
                    }
                }
            }
        }
    }
    return acc;
}

template <int AGG, bool TWO_HALVES, class Store>
__device__ __forceinline__ float aggregate(cprog_t *e, int nlo, int nhi, const Store &v) {
    float acc = AGG == AGG_SUM ? 0.0f
                               : (AGG == AGG_PRODUCT ? 1.0f
                                                     : (AGG == AGG_MAX ? -__builtin_inff()
                                                                       : __builtin_inff()));
    acc = combine_pairs<AGG, false>(acc, e, nlo, v);
    if (TWO_HALVES) acc = combine_pairs<AGG, true>(acc, e + 4 * nlo, nhi, v);
    return acc;
}

// ---------------------------------------------------------------- nodes
// Evaluate records k0 .. k1-1, all writing the same half (DST_HI).
template <bool DST_HI, bool TWO_HALVES, class Store>
__device__ __forceinline__ void run_nodes(cprog_t *rec, cprog_t *edges, int k0, int k1, int &ep,
                                          i32x8 &r, Store &v) {
    for (int k = k0; k < k1; ++k) {
        const int nlo = r[REC_NLO], nhi = r[REC_NHI];
        const int act = r[REC_ACT], agg = r[REC_AGG];
        const float bias = fbits(r[REC_BIAS]), resp = fbits(r[REC_RESP]);
        const float scale = fbits(r[REC_SCALE]);
        const int dst = r[REC_DST];
        // next record (the record array has room for N records)
        const i32x8 rn = *(cint8_t *)(rec + REC_WORDS * (k + 1));
        cprog_t *e = edges + EDGE_WORDS * ep;
        float a = 0.0f;
        if (nlo + nhi > 0) {
            if (agg == AGG_SUM || agg == AGG_MEAN)
                a = aggregate<AGG_SUM, TWO_HALVES>(e, nlo, nhi, v) * scale;
            else if (agg == AGG_PRODUCT)
                a = aggregate<AGG_PRODUCT, TWO_HALVES>(e, nlo, nhi, v);
            else if (agg == AGG_MAX)
                a = aggregate<AGG_MAX, TWO_HALVES>(e, nlo, nhi, v);
            else
                a = aggregate<AGG_MIN, TWO_HALVES>(e, nlo, nhi, v);
        }
        ep += 2 * (nlo + nhi);
        v.template set<DST_HI>(dst, act_eval(act, fmaf(resp, a, bias)));
        r = rn;
    }
}

template <class Store>
__device__ __forceinline__ void run_program(cprog_t *prog, int N, int O, int I, int layout,
                                            Store &v) {
    const int ncomp = prog[HDR_NVALID] - I;
    if (ncomp <= 0) return;
    cprog_t *rec = prog + rec_off(O);
    cprog_t *edges = prog + edge_off(N, O);
    i32x8 r = *(cint8_t *)rec;
    int ep = 0;
    if (layout == LAYOUT_REG64) {
        // records whose position is < 30 write the low half and read only it
        const int split = min(ncomp, max(0, 30 - I));
        run_nodes<false, false>(rec, edges, 0, split, ep, r, v);
        run_nodes<true, true>(rec, edges, split, ncomp, ep, r, v);
    } else {
        run_nodes<false, false>(rec, edges, 0, ncomp, ep, r, v);
    }
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
__device__ __forceinline__ void place_inputs(Store &v, const float *cur, int I, int layout,
                                             int lane) {
    // slot of input i: i, or i + 2 from position 30 on in the REG64 layout
    const int ilo = layout == LAYOUT_REG64 ? min(I, 30) : I;
    for (int i = 0; i < ilo; ++i) v.template set<false>(i, cur[lane * I + i]);
    for (int i = ilo; i < I; ++i) v.template set<true>(i + 2, cur[lane * I + i]);
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
                o[j] = (s < 32) ? v.get_lo(s) : v.get_hi(s);
            }
        }
    }
}

template <int NV, bool GRID>
__global__ __launch_bounds__(TILE *WAVES) void forward_reg_kernel(FwdArgs a) {
    extern __shared__ float smem[];
    RegStore<NV> v;
    const size_t stage = GRID ? 0 : (size_t)2 * TILE * a.I;
    forward_body<RegStore<NV>, GRID>(a, smem + (threadIdx.x / TILE) * stage, v);
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
        if (a.layout == LAYOUT_REG32) {
            if (grid)
                hipLaunchKernelGGL((forward_reg_kernel<32, true>), dim3(blocks), block, lds,
                                   stream, a);
            else
                hipLaunchKernelGGL((forward_reg_kernel<32, false>), dim3(blocks), block, lds,
                                   stream, a);
        } else {
            if (grid)
                hipLaunchKernelGGL((forward_reg_kernel<64, true>), dim3(blocks), block, lds,
                                   stream, a);
            else
                hipLaunchKernelGGL((forward_reg_kernel<64, false>), dim3(blocks), block, lds,
                                   stream, a);
        }
    } else {
        if (grid)
            hipLaunchKernelGGL((forward_lds_kernel<true>), dim3(blocks), block, lds, stream, a);
        else
            hipLaunchKernelGGL((forward_lds_kernel<false>), dim3(blocks), block, lds, stream, a);
    }
    return hipGetLastError();
}

}  // namespace neat
