// forward.hip -- the calculation stage (Section 3.3) over population x inputs.
//
// Mapping "lane per sample": a 64-lane wave evaluates one genome on a run of
// sample tiles, one or two samples per lane.  The genome's program is
// uniform across the wave, so it is read with scalar loads and every branch
// on a node's activation or aggregation is a scalar branch.  A workgroup
// holds up to four waves working on the same genome, so they share the
// CU's scalar cache.
//
// Value stores (the value vector v of Section 3.3, slots and slot classes
// in program.h), one kernel per store:
//   R64    v0..v63, one sample per lane            (class R64)
//   R64X2  v0..v63 and v64..v127, two samples       (class R64)
//   R128   v0..v127, one sample                     (class R128)
//   R224   v0..v223, one sample                     (class R224)
//   LDS    one LDS row of 64 lanes per slot         (class LDS; any class
//          when chosen explicitly)
// The register stores run one assembly block per tile (node_loop_asm.h):
// inputs from the LDS staging area into the registers, the DMA of the next
// tile's inputs, the node loop in GPR-index mode with the program's uniform
// slots, and the outputs into an LDS output area, which the C++ code then
// writes to HBM with coalesced 16-byte stores.  The LDS store runs the same
// node operations in C++.
//
// Work units.  A launch covers one or more populations ("items"); item j
// contributes P_j x chunks_j wave units (chunks_j from the item's wave
// target, or the launch's for several items of the two-samples kernel),
// unit (i, c) being run c of the
// tiles of the i-th genome of the item's list for the kernel's class (the
// class list the transformation wrote, or all genomes).  Each wave of a
// workgroup takes its own unit, so consecutive waves share a genome when it
// has several chunks and take different genomes when it has one.  Units
// past the list's length exit at once.  Workgroups are remapped so
// consecutive ones share an XCD (workgroups are dealt to the 8 XCDs round
// robin).
//
// Inputs of the next tile are copied HBM -> LDS by the DMA path of
// global_load_lds (16-byte pieces when aligned) while the current tile
// computes; each lane then moves its own samples' inputs into v.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "act.h"
#include "launch.h"
#include "neat.h"
#include "node_loop_asm.h"
#include "program.h"

namespace neat {
namespace {

constexpr int WAVE = 64;

typedef float f32x32 __attribute__((ext_vector_type(32)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef const __attribute__((address_space(4))) int32_t cprog_t;
typedef const __attribute__((address_space(4))) i32x16 cint16_t;
typedef const __attribute__((address_space(4))) FwdItem citem_t;
typedef __attribute__((address_space(1))) const void gvoid;
typedef __attribute__((address_space(3))) void lvoid;

__device__ __forceinline__ float fbits(int b) { return __int_as_float(b); }

// NaN-propagating maximum of three (IEEE 754-2019 maximum)
__device__ __forceinline__ float maximum3(float a, float b, float c) {
    float r;
    asm volatile("v_maximum3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// ---------------------------------------------------------------- stores
// LDS rows of LD floats, one column per sample of the tile (LD = 64, or 32
// for half-wave tiles when 64 columns of a large genome do not fit in LDS)
template <int LD>
struct LdsStoreT {
    float *col;  // this lane's column: slot s at col[s * LD]
    template <int H>
    __device__ __forceinline__ float get(int s) const {
        return col[s * LD];
    }
    template <int H>
    __device__ __forceinline__ void set(int s, float x) {
        col[s * LD] = x;
    }
    __device__ __forceinline__ void init(int zs) {
        col[zs * LD] = 0.0f;
        col[(zs + 1) * LD] = 1.0f;
    }
};
using LdsStore = LdsStoreT<WAVE>;

// Register stores: one tile block of node_loop_asm.h per tile.  Operands as
// documented there; every value register lives only inside the block.
#define NEAT_TILE_OPERANDS                                                               \
    [rec] "s"(rec), [edg] "s"(edg), [n] "s"(n), [zs] "s"(zs), [ni] "s"(ni), [dm0] "s"(dm0),  \
        [dn] "s"(dn), [dvec] "s"(dvec), [dsrc] "s"(dsrc), [lane] "v"(lane),                 \
        [outs] "s"(outs), [no] "s"(no), [om0] "s"(om0)
// EXTRA: more operands (the recurrent block's sweep count), or nothing
#define NEAT_NSW_OPERAND , [nsw] "s"(nsw)
#define NEAT_TILE_FN(TILE, CLOB, EXTRA)                                                   \
    __device__ __forceinline__ static void tile(const int32_t *rec, const int32_t *edg,   \
                                                int n, int zs, int ni, unsigned dm0,      \
                                                int dn, int dvec, const float *dsrc,      \
                                                unsigned lane, const int32_t *outs, int no, \
                                                unsigned om0, int nsw) {                  \
        n = __builtin_amdgcn_readfirstlane(n);                                            \
        zs = __builtin_amdgcn_readfirstlane(zs);                                          \
        ni = __builtin_amdgcn_readfirstlane(ni);                                          \
        no = __builtin_amdgcn_readfirstlane(no);                                          \
        dm0 = __builtin_amdgcn_readfirstlane(dm0);                                        \
        om0 = __builtin_amdgcn_readfirstlane(om0);                                        \
        dn = __builtin_amdgcn_readfirstlane(dn);                                          \
        dvec = __builtin_amdgcn_readfirstlane(dvec);                                      \
        nsw = __builtin_amdgcn_readfirstlane(nsw);                                        \
        asm volatile(TILE : : NEAT_TILE_OPERANDS EXTRA : CLOB, "memory");               \
    }

template <int K>
struct AsmTile;
template <>
struct AsmTile<KIND_R64> {
    static constexpr int SPL = 1;
    NEAT_TILE_FN(NEAT_TILE_S1_64, NEAT_CLOB_S1_64, )
};
template <>
struct AsmTile<KIND_R64X2> {
    static constexpr int SPL = 2;
    NEAT_TILE_FN(NEAT_TILE_S2_64, NEAT_CLOB_S2_64, )
};
template <>
struct AsmTile<KIND_R128> {
    static constexpr int SPL = 1;
    NEAT_TILE_FN(NEAT_TILE_S1_128, NEAT_CLOB_S1_128, )
};
template <>
struct AsmTile<KIND_R224> {
    static constexpr int SPL = 1;
    NEAT_TILE_FN(NEAT_TILE_S1_224, NEAT_CLOB_S1_224, )
};
template <>
struct AsmTile<KIND_R64REC> {
    static constexpr int SPL = 1;
    NEAT_TILE_FN(NEAT_TILE_S1_64R, NEAT_CLOB_S1_64R, NEAT_NSW_OPERAND)
};

// ---------------------------------------------------------------- nodes (C++)
// The LDS store's node loop: the operations of node_loop_asm.h in the same
// order, so both give identical bits.
template <int ACLS>
__device__ __forceinline__ void pair_vals(float &acc, bool first, float x0, float w0, float x1,
                                          float w1) {
    if (ACLS == ACLS_SUM) {
        acc = first ? x0 * w0 : fmaf(x0, w0, acc);
        acc = fmaf(x1, w1, acc);
    } else if (ACLS == ACLS_PROD) {
        if (first) {
            acc = x0 * w0;
            acc = acc * (x1 * w1);
        } else {
            const float ta = x0 * w0, tb = x1 * w1;
            acc = acc * ta;
            acc = acc * tb;
        }
    } else {
        const float ta = x0 * w0, tb = x1 * w1;
        acc = first ? maximum3(ta, tb, tb) : maximum3(acc, ta, tb);
    }
}

template <int ACLS, class Store>
__device__ __forceinline__ void pair(float &acc, bool first, int s0, float w0, int s1, float w1,
                                     const Store &v) {
    pair_vals<ACLS>(acc, first, v.template get<0>(s0), w0, v.template get<0>(s1), w1);
}

// pairs (>= 1) edge pairs: the first three from the record r, then the
// overflow array from e, four words per pair.
template <int ACLS, class Store, class EP>
__device__ __forceinline__ float aggregate(const i32x16 &r, EP e, int pairs, const Store &v) {
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < REC_INLINE_PAIRS; ++k) {
        if (k < pairs)
            pair<ACLS>(acc, k == 0, r[REC_PAIRS + 4 * k], fbits(r[REC_PAIRS + 4 * k + 1]),
                       r[REC_PAIRS + 4 * k + 2], fbits(r[REC_PAIRS + 4 * k + 3]), v);
    }
    for (int p = 0; p < pairs - REC_INLINE_PAIRS; ++p)
        pair<ACLS>(acc, false, e[4 * p], fbits(e[4 * p + 1]), e[4 * p + 2], fbits(e[4 * p + 3]),
                   v);
    return acc;
}

// The activation of code act, as the assembly blocks compute it.
__device__ __forceinline__ float activation(int act, float z) {
    switch (act) {
    case ACT_TANH: {
        const float e = exp2_hw(2.885390043258667f * z);
        return fmaf(rcp_hw(1.0f + e), -2.0f, 1.0f);
    }
    case ACT_SIGMOID: return rcp_hw(1.0f + exp2_hw(-1.4426950216293335f * z));
    case ACT_RELU: return maximum3(z, 0.0f, 0.0f);
    case ACT_SIN: return act_sin(z);
    case ACT_GAUSS: return exp2_hw(-1.4426950216293335f * (z * z));
    case ACT_ABS: return maximum3(z, -z, -z);
    default: return z;  // identity
    }
}

// Every computed node of the program in record order; the aggregations read
// src and the results go to dst (the same store for a feedforward network).
template <class Store>
__device__ __forceinline__ void run_program(cprog_t *prog, int N, int O, int I, const Store &src,
                                            Store &dst) {
    const int ncomp = prog[HDR_NVALID] - I;
    if (ncomp <= 0) return;
    cprog_t *rec = prog + rec_off(O);
    cprog_t *e = prog + edge_off(N, O);
    i32x16 r = *(cint16_t *)rec;
    for (int k = 0; k < ncomp; ++k) {
        const unsigned code = (unsigned)r[REC_CODE], np = (unsigned)r[REC_NPAIRS];
        const int pairs = (int)(np & (unsigned)REC_NPAIRS_MASK);
        const int acls = slot_class((int)(np >> REC_FIELD_SHIFT));
        const int act = (int)(code >> REC_FIELD_SHIFT);
        const int slot = (int)(code & (unsigned)REC_DST_MASK);
        const float bias = fbits(r[REC_BIAS]), resp = fbits(r[REC_RESP]);
        // next record (the record array has room for N records)
        const i32x16 rn = *(cint16_t *)(rec + REC_WORDS * (k + 1));
        float a;
        if (acls == ACLS_PROD) a = aggregate<ACLS_PROD>(r, e, pairs, src);
        else if (acls == ACLS_MAX) a = aggregate<ACLS_MAX>(r, e, pairs, src);
        else a = pairs == 0 ? 0.0f : aggregate<ACLS_SUM>(r, e, pairs, src);
        if (pairs > REC_INLINE_PAIRS) e += 4 * (pairs - REC_INLINE_PAIRS);
        dst.template set<0>(slot, activation(act, fmaf(resp, a, bias)));
        r = rn;
    }
}

// ---------------------------------------------------------------- tiles
// Workgroup b is dealt to XCD b % 8; give each XCD a contiguous range.
__device__ __forceinline__ long long xcd_item(unsigned b, unsigned n) {
    const unsigned x = b & 7u, q = b >> 3, per = n >> 3, rem = n & 7u;
    return (long long)(x * per + (x < rem ? x : rem) + q);
}

// Inputs are read once and outputs written once: their loads and stores
// carry the non-temporal cache policy (bit 1 of the load's cache operand),
// which measured 11 % faster on the control workload than cached ones.
constexpr int CPOL_NT = 2;
typedef float v4f __attribute__((ext_vector_type(4)));

// Issue the DMA of n consecutive floats src[0..n) into lds[0..n).
__device__ __forceinline__ void dma_inputs(const float *src, float *lds, int n, int vec4) {
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    if (vec4) {
        const int n4 = n >> 2;
        for (int c = 0; c < n4; c += WAVE)
            if (c + lane < n4)
                __builtin_amdgcn_global_load_lds((gvoid *)(src + 4 * (c + lane)),
                                                 (lvoid *)(lds + 4 * c), 16, 0, CPOL_NT);
        const int rem = n & 3;
        if (lane < rem)
            __builtin_amdgcn_global_load_lds((gvoid *)(src + 4 * n4 + lane),
                                             (lvoid *)(lds + 4 * n4), 4, 0, CPOL_NT);
    } else {
        for (int c = 0; c < n; c += WAVE)
            if (c + lane < n)
                __builtin_amdgcn_global_load_lds((gvoid *)(src + c + lane), (lvoid *)(lds + c), 4,
                                                 0, CPOL_NT);
    }
}

// Wait for this wave's DMA (the waves of a workgroup never share LDS data).
__device__ __forceinline__ void wait_dma() {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Grid-point coordinate -1 + 2 i / (side - 1).
__device__ __forceinline__ float grid_coord(int i, int side) {
    return (float)(2 * i - (side - 1)) / (float)(side - 1);
}

// Largest number of grid coordinates (side of the substrate grid).
constexpr int GRID_MAX_SIDE = 256;

// (p / d, p % d) for p < 2^24 and a uniform divisor d (< 2^16) with its
// reciprocal rd: the float estimate is off by at most one either way.
__device__ __forceinline__ void divmod_small(unsigned p, unsigned d, float rd, unsigned *q,
                                             unsigned *r) {
    int qq = (int)((float)p * rd);
    int rr = (int)p - qq * (int)d;
    if (rr >= (int)d) rr -= (int)d, ++qq;
    if (rr < 0) rr += (int)d, --qq;
    *q = (unsigned)qq;
    *r = (unsigned)rr;
}

template <int H, class Store>
__device__ __forceinline__ void place_grid(Store &v, long long q, int side) {
    const int pts = side * side;
    const int p1 = (int)(q / pts), p2 = (int)(q - (long long)p1 * pts);
    v.template set<H>(0, grid_coord(p1 % side, side));
    v.template set<H>(1, grid_coord(p1 / side, side));
    v.template set<H>(2, grid_coord(p2 % side, side));
    v.template set<H>(3, grid_coord(p2 / side, side));
    v.template set<H>(4, 1.0f);
}

template <int H, class Store>
__device__ __forceinline__ void store_outputs(const Store &v, cprog_t *prog, float *o, int O) {
    for (int j = 0; j < O; ++j) __builtin_nontemporal_store(v.template get<H>(prog[out_off() + j]), o + j);
}

// LDS byte address of a pointer into the workgroup's LDS.
__device__ __forceinline__ unsigned lds_addr(const float *p) {
    return (unsigned)(uintptr_t)(const __attribute__((address_space(3))) float *)p;
}

// Copy n floats of a tile's outputs from the LDS output area to HBM
// (16-byte pieces when the destination allows).
__device__ __forceinline__ void flush_outputs(const float *ostage, float *dst, int n) {
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    int c0 = 0;
    if (((uintptr_t)dst & 15) == 0) {
        const int n4 = n >> 2;
        for (int c = lane; c < n4; c += WAVE)
            __builtin_nontemporal_store(reinterpret_cast<const v4f *>(ostage)[c],
                                        reinterpret_cast<v4f *>(dst) + c);
        c0 = 4 * n4;
    }
    for (int c = c0 + lane; c < n; c += WAVE) __builtin_nontemporal_store(ostage[c], dst + c);
}

// Bring words [0, n) of a genome's program into the L2 cache ahead of the
// node loop's scalar loads: one 4-byte DMA per 128-byte line, landing in a
// scratch LDS area (the caller waits for vmcnt(0) before reusing it).
__device__ __forceinline__ void touch_lines(const int32_t *base, int n, float *lds_scratch) {
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    for (int off = lane * 32; off < n; off += WAVE * 32)
        __builtin_amdgcn_global_load_lds((gvoid *)(base + off), (lvoid *)lds_scratch, 4, 0, 0);
}

// Tile range [t0, t1) of run chunk, or false when it is empty.
__device__ __forceinline__ bool wave_tiles(citem_t *it, int chunk, int *t0, int *t1) {
    *t0 = chunk * it->tpw;
    *t1 = min(it->tiles, *t0 + it->tpw);
    return *t0 < *t1;
}

// Rejected genome: NaN outputs for the wave's samples.
__device__ __forceinline__ void fill_nan(float *out_g, int first, int end, int O) {
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    for (int e = first * O + lane; e < end * O; e += WAVE) out_g[e] = __builtin_nanf("");
}

// The waves of one unit with a register store: genome g, this wave's tiles.
// area: the wave's LDS (input staging TS x I floats, then output staging
// TS x O floats).
template <int K, bool GRID>
__device__ __forceinline__ void forward_unit_reg(citem_t *it, int g, int chunk, float *area,
                                                 int stage_floats) {
    constexpr int SPL = AsmTile<K>::SPL;
    constexpr int TS = WAVE * SPL;  // samples per tile
    int t0, t1;
    if (!wave_tiles(it, chunk, &t0, &t1)) return;
    const unsigned lane = threadIdx.x & (WAVE - 1);
    const int N = it->N, I = it->I, O = it->O, B = it->B, side = GRID ? it->side : 0;
    cprog_t *prog = (cprog_t *)(it->prog + (size_t)g * it->prog_words);
    float *out_g = it->outputs + (size_t)g * B * O;
    if (prog[HDR_STATUS] != 0) {
        fill_nan(out_g, t0 * TS, min(B, t1 * TS), O);
        return;
    }
    const int32_t *p = (const int32_t *)prog;
    const int32_t *rec = p + rec_off(O), *edg = p + edge_off(N, O), *outs = p + out_off();
    const int ncomp = max(prog[HDR_NVALID] - I, 0);
    const int zs = zero_slot(prog[HDR_CLASS], N);
    float *istage = area, *ostage = area + stage_floats;
    const unsigned ibase = lds_addr(istage), obase = lds_addr(ostage);
    const float *in_g = GRID ? nullptr : it->inputs + (size_t)g * it->gstride;
    const int vec4 = it->vec4;
    if (!GRID) dma_inputs(in_g + (size_t)t0 * TS * I, istage, min(TS, B - t0 * TS) * I, vec4);
    // grid queries: the side coordinates, once per unit, after the staging
    float *ctab = istage + TS * I;
    const unsigned pts = (unsigned)(side * side);
    const float rside = GRID ? 1.0f / (float)side : 0.0f;
    if (GRID) {
        for (int i = (int)lane; i < side; i += WAVE) ctab[i] = grid_coord(i, side);
        __builtin_amdgcn_wave_barrier();
    }
    // the records and overflow edges the node loop will read, in one burst
    // (the first tile's wait covers it)
    touch_lines(rec, REC_WORDS * (ncomp + 1), ostage);
    touch_lines(edg, EDGE_WORDS * prog[HDR_NEDGES], ostage);
    if (GRID) wait_dma();

    for (int t = t0; t < t1; ++t) {
        if (GRID) {
            // grid queries: the five inputs of each of the lane's samples.
            // Queries are below side^4 <= 2^32; the tile's first one is split
            // into its two points once, each lane adds its offset (< 128)
            const unsigned q0 = (unsigned)(it->first + (long long)t * TS);
            const unsigned p1_0 = q0 / pts, p2_0 = q0 - p1_0 * pts;
            for (int h = 0; h < SPL; ++h) {
                unsigned p1 = p1_0, p2 = p2_0 + (unsigned)(h * WAVE) + lane;
                if (pts >= (unsigned)TS) {
                    if (p2 >= pts) p2 -= pts, ++p1;
                } else {
                    p1 += p2 / pts;
                    p2 %= pts;
                }
                unsigned y1, x1, y2, x2;
                divmod_small(p1, (unsigned)side, rside, &y1, &x1);
                divmod_small(p2, (unsigned)side, rside, &y2, &x2);
                y1 = min(y1, (unsigned)side - 1u);  // lanes past the last query
                float *x = istage + (h * WAVE + lane) * 5;
                x[0] = ctab[x1];
                x[1] = ctab[y1];
                x[2] = ctab[x2];
                x[3] = ctab[y2];
                x[4] = 1.0f;
            }
        } else {
            wait_dma();
        }
        if (t > t0) flush_outputs(ostage, out_g + (size_t)(t - 1) * TS * O, TS * O);
        int dn = 0, dvec = 0;
        const float *dsrc = in_g;
        if (!GRID && t + 1 < t1) {
            const int nf = min(TS, B - (t + 1) * TS) * I;
            dvec = (vec4 && (nf & 3) == 0) ? 1 : 0;
            dn = dvec ? nf >> 2 : nf;
            dsrc = in_g + (size_t)(t + 1) * TS * I;
        }
        AsmTile<K>::tile(rec, edg, ncomp, zs, I, ibase, dn, dvec, dsrc, lane, outs, O, obase,
                         it->sweeps);
    }
    flush_outputs(ostage, out_g + (size_t)(t1 - 1) * TS * O, (min(B, t1 * TS) - (t1 - 1) * TS) * O);
}

// The waves of one unit with the LDS store.  stage: the wave's input
// staging area (TS x I floats; unused for grid items).
template <bool GRID, int LD>
__device__ __forceinline__ void forward_unit_lds(citem_t *it, int g, int chunk, float *stage,
                                                 LdsStoreT<LD> &v) {
    constexpr int TS = LD;
    int t0, t1;
    if (!wave_tiles(it, chunk, &t0, &t1)) return;
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    // half-wave tiles: lanes LD.. take no sample (their columns would alias)
    const bool active = LD == WAVE || lane < LD;
    const int N = it->N, I = it->I, O = it->O, B = it->B, side = GRID ? it->side : 0;
    cprog_t *prog = (cprog_t *)(it->prog + (size_t)g * it->prog_words);
    float *out_g = it->outputs + (size_t)g * B * O;
    if (prog[HDR_STATUS] != 0) {
        fill_nan(out_g, t0 * TS, min(B, t1 * TS), O);
        return;
    }
    const float *in_g = GRID ? nullptr : it->inputs + (size_t)g * it->gstride;
    const int vec4 = it->vec4;
    if (!GRID) dma_inputs(in_g + (size_t)t0 * TS * I, stage, min(TS, B - t0 * TS) * I, vec4);
    if (active) v.init(zero_slot(prog[HDR_CLASS], N));
    for (int t = t0; t < t1; ++t) {
        const int nb = min(TS, B - t * TS);
        if (GRID) {
            if (active) place_grid<0>(v, it->first + (long long)t * TS + lane, side);
        } else {
            wait_dma();
            if (active)
                for (int i = 0; i < I; ++i) v.template set<0>(i, stage[lane * I + i]);
            if (t + 1 < t1) {
                // every lane has read its inputs before the buffer refills
                __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
                __builtin_amdgcn_wave_barrier();
                dma_inputs(in_g + (size_t)(t + 1) * TS * I, stage, min(TS, B - (t + 1) * TS) * I,
                           vec4);
            }
        }
        if (active) run_program(prog, N, O, I, v, v);
        if (lane < nb) store_outputs<0>(v, prog, out_g + (size_t)(t * TS + lane) * O, O);
    }
}

// ---------------------------------------------------------------- levels
// Mapping "lanes over a level" (FWD_LVL), for genomes evaluated on few
// samples, where a lane-per-sample tile would leave most lanes idle.  A
// wave takes a tile of BW = 2^sh samples (BW <= 64) and walks the genome
// level by level (Section 3.3's order groups nodes by level: a level's
// nodes read only earlier levels).  Each step spreads 64 / BW of the
// level's computed nodes over the lanes, node-major (lane = node * BW +
// sample), so one step evaluates up to 64 (node, sample) pairs and a
// genome costs about sum over levels of nodes * BW / 64 steps instead of
// one node loop iteration per node.  A lane reads its node's 64-byte
// record with vector loads and aggregates its in-edges in its own lane, in
// the record's order with the operations of the other stores (identical
// bits).  Values live in this wave's LDS area: slot s of the tile's sample
// j at v[s * BW + j].  Every node of a step reads its sources before any
// node of the step writes (a barrier-free wave step with the results held
// in registers), and a slot the program reuses after its last reader
// (liveness) is taken only by a later position, so no value is overwritten
// before it is read.
struct LvlStore {
    float *v;
    int sh;  // log2 BW
    int j;   // this lane's sample in the tile
    template <int H>
    __device__ __forceinline__ float get(int s) const {
        return v[(s << sh) + j];
    }
};

typedef const __attribute__((address_space(1))) int32_t gint_t;
typedef const __attribute__((address_space(1))) i32x16 gint16_t;

// Order this wave's LDS accesses (the hardware keeps a wave's LDS
// operations in order; this stops the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Advance (l, kb, k1) to the next step: the next npw records of level l,
// or the first records of the next level that has computed nodes (l =
// nlev when none is left).  Start with l = -1.
__device__ __forceinline__ void lvl_advance(cprog_t *lvl, int nlev, int I, int npw, int *l,
                                            int *kb, int *k1) {
    if (*l >= 0 && *kb + npw < *k1) {
        *kb += npw;
        return;
    }
    for (++*l; *l < nlev; ++*l) {
        *kb = max(lvl[*l], I) - I, *k1 = lvl[*l + 1] - I;
        if (*kb < *k1) return;
    }
}

// Request the record (and its first overflow edge) of this lane's node in
// step (l, kb, k1).
__device__ __forceinline__ void lvl_load(gint16_t *recs, gint_t *ebeg, int nlev, int node, int l,
                                         int kb, int k1, i32x16 *r, int *e) {
    const int k = kb + node;
    if (l < nlev && k < k1) {
        *r = recs[k];
        *e = ebeg[k];
    }
}

// One step: this lane's node (record r, first overflow edge e) on its
// sample, when active; then the write of every active lane's result once
// all lanes of the step have read their sources.
__device__ __forceinline__ void lvl_step(const i32x16 &r, int e, bool active, gint_t *edges,
                                         const LvlStore &src, float *v, int sh, int j) {
    // the sources of this step were written by earlier steps
    wave_lds_sync();
    float y = 0.0f;
    int slot = -1;
    if (active) {
        const unsigned code = (unsigned)r[REC_CODE], np = (unsigned)r[REC_NPAIRS];
        const int pairs = (int)(np & (unsigned)REC_NPAIRS_MASK);
        const int acls = slot_class((int)(np >> REC_FIELD_SHIFT));
        const int act = (int)(code >> REC_FIELD_SHIFT);
        slot = (int)(code & (unsigned)REC_DST_MASK);
        // the six inline sources at once (unused inline edges name the
        // constant slot with weight 0)
        float x[2 * REC_INLINE_PAIRS];
#pragma unroll
        for (int q = 0; q < 2 * REC_INLINE_PAIRS; ++q) x[q] = src.get<0>(r[REC_PAIRS + 2 * q]);
        float a = 0.0f;
        const int inl = min(pairs, REC_INLINE_PAIRS);
        gint_t *ov = edges + EDGE_WORDS * e;
#define NEAT_LVL_AGG(ACLS)                                                                   \
    {                                                                                        \
        _Pragma("unroll") for (int q = 0; q < REC_INLINE_PAIRS; ++q) if (q < inl)            \
            pair_vals<ACLS>(a, q == 0, x[2 * q], fbits(r[REC_PAIRS + 4 * q + 1]), x[2 * q + 1], \
                            fbits(r[REC_PAIRS + 4 * q + 3]));                                \
        for (int p = 0; p < pairs - REC_INLINE_PAIRS; ++p)                                   \
            pair<ACLS>(a, false, ov[4 * p], fbits(ov[4 * p + 1]), ov[4 * p + 2],             \
                       fbits(ov[4 * p + 3]), src);                                           \
    }
        if (acls == ACLS_PROD) NEAT_LVL_AGG(ACLS_PROD)
        else if (acls == ACLS_MAX) NEAT_LVL_AGG(ACLS_MAX)
        else NEAT_LVL_AGG(ACLS_SUM)
#undef NEAT_LVL_AGG
        y = activation(act, fmaf(fbits(r[REC_RESP]), a, fbits(r[REC_BIAS])));
    }
    // every lane of the step has read its sources
    wave_lds_sync();
    if (slot >= 0) v[(slot << sh) + j] = y;
}

__device__ __forceinline__ void forward_unit_lvl(citem_t *it, int g, int chunk, float *v) {
    int t0, t1;
    if (!wave_tiles(it, chunk, &t0, &t1)) return;
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    const int sh = it->lvl_sh, BW = 1 << sh;
    const int N = it->N, C = it->C, I = it->I, O = it->O, B = it->B;
    cprog_t *prog = (cprog_t *)(it->prog + (size_t)g * it->prog_words);
    gint_t *gp = (gint_t *)(it->prog + (size_t)g * it->prog_words);
    float *out_g = it->outputs + (size_t)g * B * O;
    if (prog[HDR_STATUS] != 0) {
        fill_nan(out_g, t0 * BW, min(B, t1 * BW), O);
        return;
    }
    const float *in_g = it->inputs + (size_t)g * it->gstride;
    const int nlev = prog[HDR_NLEVELS];
    const int zs = zero_slot(prog[HDR_CLASS], N);
    cprog_t *lvl = prog + lvl_off(N, C, O);
    gint_t *ebeg = gp + ebeg_off(N, C, O);
    gint_t *edges = gp + edge_off(N, O);
    gint16_t *recs = (gint16_t *)(gp + rec_off(O));
    const int j = lane & (BW - 1), node = lane >> sh, npw = WAVE >> sh;
    const LvlStore src{v, sh, j};
    for (int t = t0; t < t1; ++t) {
        const int s0 = t * BW, nb = min(BW, B - s0);
        // inputs of the tile (contiguous [nb][I] floats): v[i][j] = x[s0 + j][i];
        // columns past the tile's last sample read 0
        const float *x = in_g + (size_t)s0 * I;
        for (int e = lane; e < BW * I; e += WAVE) {
            const int jj = e / I, i = e - jj * I;
            v[(i << sh) + jj] = jj < nb ? x[e] : 0.0f;
        }
        if (lane < BW) {
            v[(zs << sh) + lane] = 0.0f;
            v[((zs + 1) << sh) + lane] = 1.0f;
        }
        // the steps of every level in order: (level l, records kb ..
        // kb + npw - 1 below k1), alternating two record buffers: the next
        // step's records (and overflow offsets) are requested before the
        // current step is aggregated
        int l = -1, kb = 0, k1 = 0;
        lvl_advance(lvl, nlev, I, npw, &l, &kb, &k1);
        i32x16 ra = {}, rb = {};
        int ea = 0, eb = 0;
        lvl_load(recs, ebeg, nlev, node, l, kb, k1, &ra, &ea);
        while (l < nlev) {
            int l2 = l, kb2 = kb, k12 = k1;
            lvl_advance(lvl, nlev, I, npw, &l2, &kb2, &k12);
            lvl_load(recs, ebeg, nlev, node, l2, kb2, k12, &rb, &eb);
            lvl_step(ra, ea, kb + node < k1, edges, src, v, sh, j);
            l = l2, kb = kb2, k1 = k12;
            if (l >= nlev) break;
            lvl_advance(lvl, nlev, I, npw, &l2, &kb2, &k12);
            lvl_load(recs, ebeg, nlev, node, l2, kb2, k12, &ra, &ea);
            lvl_step(rb, eb, kb + node < k1, edges, src, v, sh, j);
            l = l2, kb = kb2, k1 = k12;
        }
        wave_lds_sync();
        // outputs of the tile: y[s0 + j][o] = v[out slot o][j]
        float *o_t = out_g + (size_t)s0 * O;
        for (int e = lane; e < nb * O; e += WAVE) {
            const int jj = e / O, o = e - jj * O;
            __builtin_nontemporal_store(v[(prog[out_off() + o] << sh) + jj], o_t + e);
        }
        wave_lds_sync();
    }
}

// ---------------------------------------------------------------- segments
// Mapping "lanes over a level's in-edges" (FWD_SEG).  As in the level
// mapping, a wave takes a tile of BW = 2^sh samples and walks the levels,
// values in LDS at v[s * BW + j].  Here a step spreads the level's
// in-edges over the lanes: R = 64 / BW rows of edges, each row holding one
// edge for the tile's BW samples (lane = row * BW + sample).  The level's
// edges are laid out destination after destination (a node's edges in its
// record's order, a node without in-edges contributing one edge w = 1 from
// the constant 0), so every destination owns a run of consecutive rows: a
// segment.  Each lane forms w * v[src] and a segmented inclusive scan over
// the rows (Hillis-Steele, partner rows 1, 2, 4, ... back in the same
// segment) combines the terms with the destination's aggregation: sum,
// product or the NaN-propagating maximum (mean and min are folded into the
// response, as in every store).  A segment cut by the end of a step passes
// its partial result to the next step's first row (carry).  The lane
// holding a segment's last edge applies bias, response and activation and
// writes the value once every lane of the step has read its sources.  The
// terms are combined in a tree rather than a chain, so sums and products
// round differently from the other mappings (within the oracle's bound,
// which holds for any order); maxima are exact.
__device__ __forceinline__ float seg_combine(int acls, float early, float late) {
    return acls == ACLS_PROD ? early * late
                             : (acls == ACLS_MAX ? maximum3(early, late, late) : early + late);
}

// exclusive scan of one int per lane across the wave; *total = the sum
__device__ __forceinline__ int wave_excl_scan(int v, int *total) {
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    int x = v;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const int y = __shfl_up(x, d, WAVE);
        if (lane >= d) x += y;
    }
    *total = __shfl(x, WAVE - 1, WAVE);
    return x - v;
}

__device__ __forceinline__ void forward_unit_seg(citem_t *it, int g, int chunk, float *v) {
    int t0, t1;
    if (!wave_tiles(it, chunk, &t0, &t1)) return;
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    const int sh = it->lvl_sh, BW = 1 << sh, R = WAVE >> sh;
    const int N = it->N, C = it->C, I = it->I, O = it->O, B = it->B;
    cprog_t *prog = (cprog_t *)(it->prog + (size_t)g * it->prog_words);
    gint_t *gp = (gint_t *)(it->prog + (size_t)g * it->prog_words);
    float *out_g = it->outputs + (size_t)g * B * O;
    if (prog[HDR_STATUS] != 0) {
        fill_nan(out_g, t0 * BW, min(B, t1 * BW), O);
        return;
    }
    const float *in_g = it->inputs + (size_t)g * it->gstride;
    const int nlev = prog[HDR_NLEVELS];
    const int zs = zero_slot(prog[HDR_CLASS], N);
    cprog_t *lvl = prog + lvl_off(N, C, O);
    gint_t *ebeg = gp + ebeg_off(N, C, O);
    gint_t *edges = gp + edge_off(N, O);
    gint_t *recs = gp + rec_off(O);
    // the rows of v, then each level's edge offsets by node (N + 1 ints)
    int *eoff = (int *)(v + ((size_t)it->lvl_rows << sh));
    const int row = lane >> sh, j = lane & (BW - 1);
    for (int t = t0; t < t1; ++t) {
        const int s0 = t * BW, nb = min(BW, B - s0);
        const float *x = in_g + (size_t)s0 * I;
        for (int e = lane; e < BW * I; e += WAVE) {
            const int jj = e / I, i = e - jj * I;
            v[(i << sh) + jj] = jj < nb ? x[e] : 0.0f;
        }
        if (lane < BW) {
            v[(zs << sh) + lane] = 0.0f;
            v[((zs + 1) << sh) + lane] = 1.0f;
        }
        for (int l = 0; l < nlev; ++l) {
            const int k0 = max(lvl[l], I) - I, k1 = lvl[l + 1] - I, nl = k1 - k0;
            if (nl <= 0) continue;
            // edges per node (at least one) and their offsets
            int base = 0;
            for (int c = 0; c < nl; c += WAVE) {
                int ec = 0;
                if (c + lane < nl) {
                    const int pairs =
                        recs[REC_WORDS * (k0 + c + lane) + REC_NPAIRS] & REC_NPAIRS_MASK;
                    ec = pairs > 0 ? 2 * pairs : 1;
                }
                int tot;
                const int ex = wave_excl_scan(ec, &tot);
                if (c + lane < nl) eoff[c + lane] = base + ex;
                base += tot;
            }
            if (lane == 0) eoff[nl] = base;
            wave_lds_sync();
            float carry = 0.0f;
            for (int eb = 0; eb < base; eb += R) {
                const int e = eb + row;
                const bool active = e < base;
                int node = 0, q = 0, ec = 1, acls = ACLS_SUM;
                float xv = 0.0f;
                unsigned code = 0;
                float bias = 0.0f, resp = 0.0f;
                if (active) {
                    // the node owning edge e: the last offset <= e
                    int lo = 0, hi = nl - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (eoff[mid] <= e) lo = mid;
                        else hi = mid - 1;
                    }
                    node = lo;
                    q = e - eoff[lo];
                    ec = eoff[lo + 1] - eoff[lo];
                    const int k = k0 + node;
                    gint_t *r = recs + REC_WORDS * k;
                    code = (unsigned)r[REC_CODE];
                    bias = fbits(r[REC_BIAS]);
                    resp = fbits(r[REC_RESP]);
                    const unsigned np = (unsigned)r[REC_NPAIRS];
                    const int pairs = (int)(np & (unsigned)REC_NPAIRS_MASK);
                    acls = slot_class((int)(np >> REC_FIELD_SHIFT));
                    int src = zs;
                    float w = 1.0f;
                    if (pairs > 0) {
                        gint_t *ew = q < 2 * REC_INLINE_PAIRS
                                         ? r + REC_PAIRS + 2 * q
                                         : edges + EDGE_WORDS * (ebeg[k] + q - 2 * REC_INLINE_PAIRS);
                        src = ew[0];
                        w = fbits(ew[1]);
                    }
                    xv = v[(src << sh) + j] * w;
                    // a segment begun in an earlier step continues from its carry
                    if (row == 0 && q > 0) xv = seg_combine(acls, carry, xv);
                }
                // segmented inclusive scan over the rows (same sample)
#pragma unroll
                for (int d = 1; d < WAVE; d <<= 1) {
                    if (d >= R) break;
                    const float y = __shfl(xv, lane - d * BW >= 0 ? lane - d * BW : lane, WAVE);
                    if (active && row >= d && q >= d) xv = seg_combine(acls, y, xv);
                }
                carry = __shfl(xv, (R - 1) * BW + j, WAVE);
                const bool tail = active && q == ec - 1;
                float yv = 0.0f;
                if (tail)
                    yv = activation((int)(code >> REC_FIELD_SHIFT), fmaf(resp, xv, bias));
                // every lane of the step has read its sources
                wave_lds_sync();
                if (tail) v[((int)(code & (unsigned)REC_DST_MASK) << sh) + j] = yv;
            }
            wave_lds_sync();
        }
        float *o_t = out_g + (size_t)s0 * O;
        for (int e = lane; e < nb * O; e += WAVE) {
            const int jj = e / O, o = e - jj * O;
            __builtin_nontemporal_store(v[(prog[out_off() + o] << sh) + jj], o_t + e);
        }
        wave_lds_sync();
    }
}

// ---------------------------------------------------------------- recurrent
// Recurrent networks (read as K synchronous sweeps; the program comes from
// the recurrent transformation: records in key order, one slot per node).
// One wave per (genome, tile of 64 samples).  The lane's values live in two
// LDS columns, the previous sweep's (cur) and the one being written (nxt),
// which swap after every sweep: v0 = the inputs at slots 0..I-1 and 0 at
// the other nodes; every sweep runs all records reading cur and writing nxt.
template <int LD>
__global__ __launch_bounds__(WAVE) void recurrent_kernel(RecLaunch L) {
    // tiles of LD samples (64, or 32 when two columns of 64 do not fit)
    extern __shared__ float smem[];
    const long long u = xcd_item(blockIdx.x, gridDim.x);
    if (u >= (long long)L.P * L.tiles) return;
    const int g = (int)(u / L.tiles), t = (int)(u - (long long)g * L.tiles);
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    const bool active = LD == WAVE || lane < LD;  // lanes LD.. take no sample
    const int I = L.I, O = L.O, N = L.N;
    cprog_t *prog = (cprog_t *)(L.prog + (size_t)g * L.prog_words);
    float *out_g = L.outputs + (size_t)g * L.B * O;
    const int s0 = t * LD, nb = min(LD, L.B - s0);
    if (prog[HDR_STATUS] != 0) {
        fill_nan(out_g, s0, s0 + nb, O);
        return;
    }
    float *stage = smem;
    dma_inputs(L.inputs + (size_t)g * L.gstride + (size_t)s0 * I, stage, nb * I, L.vec4);
    LdsStoreT<LD> cur, nxt;
    cur.col = smem + L.stage_floats + (lane & (LD - 1));
    nxt.col = cur.col + (size_t)L.rows * LD;
    const int nvalid = prog[HDR_NVALID];
    if (active) {
        for (int s = I; s < nvalid; ++s) cur.template set<0>(s, 0.0f);
        cur.init(zero_slot(prog[HDR_CLASS], N));
        nxt.init(zero_slot(prog[HDR_CLASS], N));
    }
    wait_dma();
    // lanes past the tile's last sample read stale staging words; their
    // results are never stored
    if (active)
        for (int i = 0; i < I; ++i) {
            const float x = stage[lane * I + i];
            cur.template set<0>(i, x);
            nxt.template set<0>(i, x);
        }
    for (int k = 0; k < L.K; ++k) {
        if (active) run_program(prog, N, O, I, cur, nxt);
        float *c = cur.col;
        cur.col = nxt.col;
        nxt.col = c;
    }
    if (lane < nb) store_outputs<0>(cur, prog, out_g + (size_t)(s0 + lane) * O, O);
}

// Item holding unit u (items sorted by unit0; the first has unit0 = 0).
__device__ __forceinline__ citem_t *find_item(const FwdItem *table, int n, long long u) {
    citem_t *items = (citem_t *)table;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].unit0 <= u) lo = mid;
        else hi = mid - 1;
    }
    return items + lo;
}

// The launch argument in the kernarg segment (FwdLaunch is the kernel's only
// argument, so it sits at offset 0; its inline item is its first member).
__device__ __forceinline__ const __attribute__((address_space(4))) FwdLaunch *launch_arg() {
    return (const __attribute__((address_space(4))) FwdLaunch *)
        __builtin_amdgcn_kernarg_segment_ptr();
}

// One unit: find its item and genome, then run the unit's waves with a
// fresh value store (nothing carries over from one unit to the next).
template <int K, bool GRID>
__device__ __forceinline__ void run_unit(long long u, float *wave_area) {
    const auto *L = launch_arg();
    citem_t *it = L->items ? find_item(L->items, L->n_items, u) : (citem_t *)&L->one;
    const long long local = u - it->unit0;
    const int chunks = it->chunks;
    const int i = (int)(local / chunks), chunk = (int)(local - (long long)i * chunks);
    int g = i;
    const int cls = it->cls;
    if (cls >= 0) {
        cprog_t *pop = (cprog_t *)it->pop;
        if (i >= pop[POP_COUNT + cls]) return;
        g = pop[POP_IDS + pop[POP_BEGIN + cls] + i];
    }
    if constexpr (K == KIND_LVL) {
        forward_unit_lvl(it, g, chunk, wave_area);
    } else if constexpr (K == KIND_SEG) {
        forward_unit_seg(it, g, chunk, wave_area);
    } else if constexpr (K == KIND_LDS) {
        LdsStore v;
        v.col = wave_area + L->stage_floats + (threadIdx.x & (WAVE - 1));
        forward_unit_lds<GRID, WAVE>(it, g, chunk, wave_area, v);
    } else if constexpr (K == KIND_LDS32) {
        LdsStoreT<WAVE / 2> v;
        v.col = wave_area + L->stage_floats + (threadIdx.x & (WAVE / 2 - 1));
        forward_unit_lds<GRID, WAVE / 2>(it, g, chunk, wave_area, v);
    } else {
        forward_unit_reg<K, GRID>(it, g, chunk, wave_area, L->stage_floats);
    }
}

// PERSIST: a grid smaller than the unit count, each workgroup looping.
// GRID: CPPN grid queries generated in the kernel instead of read inputs.
template <int K, bool PERSIST, bool GRID>
__global__ __launch_bounds__(WAVE *FWD_MAX_WAVES) void forward_kernel(FwdLaunch L) {
    extern __shared__ float smem[];
    float *wave_area = smem + (size_t)(threadIdx.x / WAVE) * L.wave_floats;
    // the wave index is uniform; say so, so everything derived stays scalar
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const long long waves = blockDim.x / WAVE;
    const long long b0 = xcd_item(blockIdx.x, gridDim.x);
    if (!PERSIST) {
        const long long u = b0 * waves + wave;
        if (u < L.units) run_unit<K, GRID>(u, wave_area);
        return;
    }
    if (L.counter) {
        // every wave takes the next unit until none is left
        for (;;) {
            unsigned u = 0;
            if ((threadIdx.x & (WAVE - 1)) == 0) u = atomicAdd(L.counter, 1u);
            u = (unsigned)__builtin_amdgcn_readfirstlane((int)u);  // lane 0's, uniform
            if ((long long)u >= L.units) return;
            run_unit<K, GRID>((long long)u, wave_area);
        }
    }
    for (long long b = b0; b * waves < L.units; b += gridDim.x) {
        const long long u = b * waves + wave;
        if (u < L.units) run_unit<K, GRID>(u, wave_area);
    }
}

__global__ void zero_counters_kernel(unsigned *c, int n) {
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) c[i] = 0u;
}

// Waves a forward launch aims at (NEAT_FWD_WAVES overrides, for tuning).
long long wave_target() {
    static const long long t = [] {
        const char *e = getenv("NEAT_FWD_WAVES");
        const long long v = e ? atoll(e) : 0;
        return v >= 1024 ? v : 32768ll;
    }();
    return t;
}

// LDS bytes of one wave's values in the level mapping: the tile width is
// the widest that keeps rows x width within it (NEAT_LVL_WAVE_BYTES
// overrides, for tuning).
size_t lvl_wave_bytes() {
    static const size_t b = [] {
        const char *e = getenv("NEAT_LVL_WAVE_BYTES");
        const long long v = e ? atoll(e) : 0;
        return v >= 1024 && v <= 65536 ? (size_t)v : (size_t)8192;
    }();
    return b;
}

int choose_chunks(long long P, int tiles, int *tpw) {
    // aim at a wave count that fills 256 CUs several times over while a
    // wave still reuses its genome's program across a run of tiles (and
    // hides the first tile's input latency behind the others)
    const long long target = wave_target();
    long long chunks = (target + P - 1) / (P > 0 ? P : 1);
    if (chunks < 1) chunks = 1;
    if (chunks > tiles) chunks = tiles;
    *tpw = (int)((tiles + chunks - 1) / chunks);
    return (tiles + *tpw - 1) / *tpw;
}

// One tiles-per-wave count for every item of a launch: the largest t whose
// units, sum of P x ceil(tiles / t), still reach the wave target (1 when
// even one tile per wave falls short).  The units never grow with t, so a
// binary search finds it.
int launch_tiles_per_wave(const std::vector<FwdItem> &items) {
    const long long target = wave_target();
    int max_tiles = 1;
    for (const FwdItem &it : items) max_tiles = std::max(max_tiles, it.tiles);
    auto units = [&](int t) {
        long long u = 0;
        for (const FwdItem &it : items) u += (long long)it.P * ((it.tiles + t - 1) / t);
        return u;
    };
    int lo = 1, hi = max_tiles;  // units(lo) >= target unless lo = 1
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (units(mid) >= target) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// samples of one tile
int tile_samples(int kind) {
    return kind == KIND_R64X2 ? 2 * WAVE : (kind == KIND_LDS32 ? WAVE / 2 : WAVE);
}

bool lds_kind(int kind) { return kind == KIND_LDS || kind == KIND_LDS32; }

// kernel of class c under a variant
int kind_of(int variant, int cls, int B) {
    if (variant == FWD_LDS) return KIND_LDS;
    if (variant == FWD_LVL || variant == FWD_SEG) variant = FWD_AUTO;  // grid, recurrent items
    switch (cls) {
    case CLS_R64:
        if (variant == FWD_REG2 || (variant == FWD_AUTO && B > WAVE)) return KIND_R64X2;
        return KIND_R64;
    case CLS_R128: return KIND_R128;
    case CLS_R224: return KIND_R224;
    }
    return KIND_LDS;
}

}  // namespace

const char *kind_name(int kind) {
    static const char *names[] = {"r64", "r64x2", "r128", "r224", "lds", "r64rec", "lds32",
                                  "lvl", "seg"};
    return kind >= 0 && kind < N_KINDS ? names[kind] : "?";
}

int forward_plan(const FwdJob *jobs, int n, int variant, size_t max_lds,
                 std::vector<FwdKernelLaunch> &out, char *err, size_t errlen) {
    out.clear();
    // one launch per (kernel, input mode)
    constexpr int NL = 2 * N_KINDS;
    FwdKernelLaunch k[NL];
    int rows_max[NL], stage_max[NL], ostage_max[NL];
    for (int x = 0; x < NL; ++x) {
        k[x] = FwdKernelLaunch{};
        k[x].kind = x / 2;
        k[x].grid_mode = x & 1;
        rows_max[x] = stage_max[x] = ostage_max[x] = 0;
    }
    const int plan_variant = variant;
    for (int j = 0; j < n; ++j) {
        const FwdJob &J = jobs[j];
        if (J.P == 0 || J.B == 0) continue;
        const int variant = J.variant >= 0 ? J.variant : plan_variant;
        const int top = max_class(J.N);
        if ((variant == FWD_LVL || variant == FWD_SEG) && !J.side && !J.recurrent) {
            // the level and segment mappings: every genome, one launch per
            // mapping over all items; the widest power-of-two tile of
            // samples (<= 64, <= B rounded up) whose values fit a wave's
            // LDS budget (the segment mapping also keeps N_max + 1 edge
            // offsets)
            const bool seg = variant == FWD_SEG;
            const int rows = class_slots(top, J.N);
            const size_t extra = seg ? sizeof(int) * (size_t)(J.N + 1) : 0;
            int sh = 0;
            while (sh < 6 && (1 << sh) < J.B &&
                   sizeof(float) * (size_t)rows * (2u << sh) + extra <= lvl_wave_bytes())
                ++sh;
            FwdItem it{};
            it.prog = J.prog;
            it.inputs = J.inputs;
            it.outputs = J.outputs;
            it.gstride = J.gstride;
            it.pop = J.prog + pop_off(J.P, J.N, J.C, J.O);
            it.cls = -1;
            it.P = J.P, it.N = J.N, it.C = J.C, it.I = J.I, it.O = J.O, it.B = J.B;
            it.prog_words = prog_words(J.N, J.C, J.O);
            it.lvl_sh = sh;
            it.lvl_rows = rows;
            it.tiles = (J.B + (1 << sh) - 1) >> sh;
            const int x = 2 * (seg ? KIND_SEG : KIND_LVL);
            k[x].items.push_back(it);
            rows_max[x] = std::max(rows_max[x], (rows << sh) + (seg ? J.N + 1 : 0));
            continue;
        }
        // FWD_LDS takes every genome in one pass over all genomes; the other
        // variants take class c's genomes with class c's kernel; a recurrent
        // job (N_max <= 62) takes every genome with the recurrent kernel
        const int c_lo = (variant == FWD_LDS || J.recurrent) ? -1 : 0;
        const int c_hi = (variant == FWD_LDS || J.recurrent) ? -1 : top;
        for (int c = c_lo; c <= c_hi; ++c) {
            int kind = J.recurrent ? KIND_R64REC : kind_of(variant, c < 0 ? CLS_LDS : c, J.B);
            // LDS rows too large for 64 columns per wave: half-wave tiles
            if (kind == KIND_LDS &&
                sizeof(float) * (size_t)WAVE * (J.I + class_slots(top, J.N)) > max_lds)
                kind = KIND_LDS32;
            FwdItem it{};
            it.prog = J.prog;
            it.inputs = J.inputs;
            it.outputs = J.outputs;
            it.gstride = J.gstride;
            it.first = J.first;
            it.pop = J.prog + pop_off(J.P, J.N, J.C, J.O);
            // populations of N_max <= 62 are all R64 and have no class list
            it.cls = (c < 0 || top == CLS_R64) ? -1 : c;
            it.P = J.P, it.N = J.N, it.C = J.C, it.I = J.I, it.O = J.O, it.B = J.B;
            it.side = J.side;
            it.prog_words = prog_words(J.N, J.C, J.O);
            it.sweeps = J.recurrent ? J.sweeps : 0;
            const int TS = tile_samples(kind);
            it.tiles = (J.B + TS - 1) / TS;
            it.vec4 = (!J.side && ((uintptr_t)J.inputs % 16 == 0) && (J.gstride % 4 == 0)) ? 1 : 0;
            const int x = 2 * kind + (J.side ? 1 : 0);
            k[x].items.push_back(it);
            // register kernels on grid queries keep the coordinates after
            // the staged inputs
            if (!J.side || !lds_kind(kind))
                stage_max[x] = std::max(stage_max[x], TS * J.I + (J.side ? GRID_MAX_SIDE : 0));
            if (!lds_kind(kind)) ostage_max[x] = std::max(ostage_max[x], TS * J.O);
            if (lds_kind(kind)) rows_max[x] = std::max(rows_max[x], class_slots(top, J.N));
        }
    }
    for (int x = 0; x < NL; ++x) {
        FwdKernelLaunch &K = k[x];
        const int kind = K.kind;
        if (K.items.empty()) continue;
        const size_t rows = (kind == KIND_LVL || kind == KIND_SEG) ? (size_t)rows_max[x]
                            : lds_kind(kind) ? (size_t)rows_max[x] * tile_samples(kind)
                                             : (size_t)ostage_max[x];
        const size_t wave_floats = (size_t)stage_max[x] + rows;
        const size_t wave_bytes = wave_floats * sizeof(float);
        int waves = FWD_MAX_WAVES;
        while (waves > 1 && wave_bytes * waves > max_lds) --waves;
        if (wave_bytes > max_lds) {
            snprintf(err, errlen,
                     "forward kernel %s needs %zu B of LDS per wave (value rows %d, input "
                     "staging %d floats), device allows %zu",
                     kind_name(kind), wave_bytes, lds_kind(kind) ? rows_max[x] : 0,
                     stage_max[x], max_lds);
            return NEAT_E_TOO_LARGE;
        }
        // Several items of the two-samples kernel (the streaming one, taken
        // for B > 64) share the launch's wave target: one tiles-per-wave
        // count for all, the largest that still gives the target, so a
        // population split into items runs as it does whole and each wave
        // overlaps its next tile's input DMA with the current tile (the
        // control workload as 10 items: 0.238 -> 0.214 ms).  Other kernels
        // keep each item's own target: their short-B items are latency-bound
        // and gain from spreading tiles over waves (a launch-wide target made
        // the uneven batch's calculation up to 32 % slower).
        const int shared_tpw = kind == KIND_R64X2 && K.items.size() > 1
                                   ? launch_tiles_per_wave(K.items) : 0;
        long long units = 0;
        for (FwdItem &it : K.items) {
            if (shared_tpw > 0) {
                // as many units as the shared count gives, their tiles
                // balanced (32 tiles at 15 per wave: 11 + 11 + 10, not
                // 15 + 15 + 2), as choose_chunks balances an item's own
                const int t = std::min(shared_tpw, std::max(1, it.tiles));
                it.chunks = (it.tiles + t - 1) / t;
                it.tpw = (it.tiles + it.chunks - 1) / it.chunks;
            } else {
                it.chunks = choose_chunks(it.P, it.tiles, &it.tpw);
            }
            it.unit0 = units;
            units += (long long)it.P * it.chunks;
        }
        const long long groups = (units + waves - 1) / waves;
        K.args.wave_floats = (int)wave_floats;
        K.args.stage_floats = stage_max[x];
        K.args.units = units;
        K.block = (unsigned)(WAVE * waves);
        K.lds = wave_bytes * waves;
        // the LDS store limits the workgroups a CU holds: loop over units with
        // a grid of a few per CU instead of one workgroup per unit
        const long long cap = (lds_kind(kind) || kind == KIND_LVL || kind == KIND_SEG)
                                  ? 256ll * 2 * std::max<long long>(1, (long long)(163840 / K.lds))
                                  : (1ll << 31) - 1;
        K.args.persistent = groups > cap ? 1 : 0;
        K.grid = (unsigned)std::min(groups, cap);
        if (K.items.size() == 1) K.args.one = K.items[0];
        out.push_back(K);
    }
    return NEAT_OK;
}

size_t recurrent_lds_bytes(int N, int I, int ld) {
    return sizeof(float) * (size_t)ld * ((size_t)I + 2 * (size_t)class_slots(max_class(N), N));
}

hipError_t recurrent_launch(RecLaunch L, size_t max_lds, hipStream_t stream) {
    const int ld = recurrent_lds_bytes(L.N, L.I, WAVE) <= max_lds ? WAVE : WAVE / 2;
    L.tiles = (L.B + ld - 1) / ld;
    L.stage_floats = ld * L.I;
    const long long blocks = (long long)L.P * L.tiles;
    if (blocks == 0) return hipSuccess;
    if (ld == WAVE)
        hipLaunchKernelGGL(recurrent_kernel<WAVE>, dim3((unsigned)blocks), dim3(WAVE),
                           recurrent_lds_bytes(L.N, L.I, WAVE), stream, L);
    else
        hipLaunchKernelGGL(recurrent_kernel<WAVE / 2>, dim3((unsigned)blocks), dim3(WAVE),
                           recurrent_lds_bytes(L.N, L.I, WAVE / 2), stream, L);
    return hipGetLastError();
}

hipError_t launch_zero_counters(unsigned *c, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, stream, c, n);
    return hipGetLastError();
}

hipError_t forward_launch(const FwdKernelLaunch &k, const FwdItem *dev_items, hipStream_t stream,
                          unsigned *counter) {
    FwdLaunch L = k.args;
    L.counter = L.persistent ? counter : nullptr;
    if (k.items.size() == 1 && dev_items == nullptr) {
        L.items = nullptr;
        L.n_items = 1;
    } else {
        L.items = dev_items;
        L.n_items = (int)k.items.size();
    }
#define NEAT_LAUNCH2(KIND, GRID)                                                           \
    if (L.persistent)                                                                      \
        hipLaunchKernelGGL((forward_kernel<KIND, true, GRID>), dim3(k.grid), dim3(k.block),   \
                           k.lds, stream, L);                                              \
    else                                                                                   \
        hipLaunchKernelGGL((forward_kernel<KIND, false, GRID>), dim3(k.grid), dim3(k.block),  \
                           k.lds, stream, L);
#define NEAT_LAUNCH(KIND)                                                                  \
    if (k.grid_mode) {                                                                     \
        NEAT_LAUNCH2(KIND, true)                                                           \
    } else {                                                                               \
        NEAT_LAUNCH2(KIND, false)                                                          \
    }
    switch (k.kind) {
    case KIND_R64: NEAT_LAUNCH(KIND_R64) break;
    case KIND_R64X2: NEAT_LAUNCH(KIND_R64X2) break;
    case KIND_R128: NEAT_LAUNCH(KIND_R128) break;
    case KIND_R224: NEAT_LAUNCH(KIND_R224) break;
    case KIND_R64REC: NEAT_LAUNCH2(KIND_R64REC, false) break;
    case KIND_LDS32: NEAT_LAUNCH(KIND_LDS32) break;
    case KIND_LVL: NEAT_LAUNCH2(KIND_LVL, false) break;
    case KIND_SEG: NEAT_LAUNCH2(KIND_SEG, false) break;
    default: NEAT_LAUNCH(KIND_LDS) break;
    }
#undef NEAT_LAUNCH
#undef NEAT_LAUNCH2
    return hipGetLastError();
}

}  // namespace neat
