// topo.hip -- the transformation stage (Section 3.3) for a whole population.
//
// One workgroup per genome; thread t owns node row t (the block has
// round_up(N_max, 64) threads).  Everything of one genome lives in LDS:
//
//   1. node rows: presence (key not NaN), key / act / agg validity; every
//      well-formed key goes into an open-addressing key -> row table;
//   2. a stable rank of every well-formed key (the number of smaller
//      (key, row) words), which gives the keys in sorted order and detects
//      duplicate keys; presence of the input/output keys;
//   3. connection rows, read as one float4 each: padding and disabled rows
//      are dropped, enabled rows are resolved through the table into
//      (source row, destination row);
//   4. adjacency: groups of more than one wave count degrees, scan them and
//      scatter in-lists (source keys) and out-lists (destination rows); an
//      edge's index among its destination's in-edges is the number of
//      smaller source keys there, and an equal one is a duplicate edge.
//      One-wave groups (N_max <= 64) keep each row's sources as a 64-bit
//      mask over key ranks instead: setting a bit already set is a
//      duplicate edge, and an edge's index is a popcount;
//   5. level-synchronous Kahn: every round, the nodes whose sources have all
//      been emitted form the frontier; lanes are assigned to nodes in
//      key-rank order, so a ballot + mbcnt prefix count gives each frontier
//      node its position in (level, key) order; nodes never emitted mean a
//      cycle.  One-wave groups test their masks against the ranks emitted
//      so far; larger groups decrement in-degrees with LDS atomics;
//   6. value slots (position, or by liveness in parallel when the largest
//      genomes need more than 64 slots), then the program (program.h):
//      records in topological order, in-edges sorted by source key, source
//      slots, level starts.
//
// In recurrent mode (networks with cycles, evaluated by synchronous sweeps)
// self-loops are not flagged, step 5 is skipped (position = key rank, level
// 0) and step 6 gives every node its own slot (position).
//
// classify_kernel then lists the genomes of a population by slot class.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "neat.h"
#include "program.h"

namespace neat {
namespace {

constexpr float KEY_LIMIT = 16777216.0f;  // 2^24

__device__ __forceinline__ bool is_int_in(float x, float lo, float hi_excl) {
    // NaN fails every comparison
    return x >= lo && x < hi_excl && x == floorf(x);
}

// Key -> row table: open addressing with linear probing in H = hash_size(N)
// slots (a power of two, at least twice the rows, so probes end at an empty
// slot).  Every well-formed key is inserted with the smallest row holding it.
constexpr int HASH_EMPTY = -1;
__host__ __device__ constexpr int hash_size(int N) {
    int h = 64;
    while (h < 2 * N) h *= 2;
    return h;
}
__device__ __forceinline__ int hash_slot(int key, int H) {
    return (int)(((unsigned)key * 2654435761u) >> 8) & (H - 1);
}
// Returns the key's slot.
__device__ __forceinline__ int hash_insert(int *hkey, int *hrow, int H, int key, int row) {
    int h = hash_slot(key, H);
    for (;;) {
        const int old = atomicCAS(&hkey[h], HASH_EMPTY, key);
        if (old == HASH_EMPTY || old == key) {
            atomicMin(&hrow[h], row);
            return h;
        }
        h = (h + 1) & (H - 1);
    }
}
// k as a well-formed key (an integer in [0, 2^24)), else -1, without
// branches: the clamp keeps the conversion in range (NaN becomes -1), and
// the conversion back must give k again.
__device__ __forceinline__ int key_of(float k) {
    const int i = (int)fminf(fmaxf(k, -1.0f), KEY_LIMIT);
    return ((float)i == k && (unsigned)i < (1u << 24)) ? i : -1;
}

// Table word of the well-formed key equal to k, or -1.  The word's low 16
// bits are the first row among duplicates; one-wave groups later add the
// key's rank above them.
__device__ __forceinline__ int find_row(float k, const int *hkey, const int *hrow, int H) {
    if (!is_int_in(k, 0.0f, KEY_LIMIT)) return -1;
    const int key = (int)k;
    for (int h = hash_slot(key, H);; h = (h + 1) & (H - 1)) {
        const int kk = hkey[h];
        if (kk == key) return hrow[h];
        if (kk == HASH_EMPTY) return -1;
    }
}

// Threads of a genome's group, and the connection rows kept in LDS: none
// when every row stays in a thread's registers (at most four per thread).
__host__ __device__ constexpr int group_threads(int N) { return N <= 64 ? 64 : (N + 63) & ~63; }
__host__ __device__ constexpr int stored_conns(int N, int C) {
    return C > 4 * group_threads(N) ? C : 0;
}

// Ranks by merging sorted per-wave lists take fewer instructions than
// counting all N words for more than MERGE_MIN rows.
constexpr int MERGE_MIN = 128;

// Packed (key, row) words in LDS: a multiple of 4 (read four at a time), or
// whole 64-word lists when ranks come from merging per-wave lists.
__host__ __device__ constexpr int stack_words(int N) {
    return N <= MERGE_MIN ? (N + 3) & ~3 : (N + 63) & ~63;
}

// The number of words below mine over nl sorted lists of 64 words at sl:
// branch-free binary searches, G lists side by side (a group's lists past
// the last search the last one again and are not counted).
template <int G>
__device__ __forceinline__ int merged_rank(const unsigned *sl, int nl, unsigned mine) {
    int rank = 0;
    for (int w0 = 0; w0 < nl; w0 += G) {
        int pos[G];
#pragma unroll
        for (int w = 0; w < G; ++w) pos[w] = 0;
#pragma unroll
        for (int d = 64; d > 0; d >>= 1) {
            unsigned v[G];
#pragma unroll
            for (int w = 0; w < G; ++w) v[w] = sl[min(w0 + w, nl - 1) * 64 + min(pos[w] + d - 1, 63)];
#pragma unroll
            for (int w = 0; w < G; ++w) pos[w] += (pos[w] + d <= 64 && v[w] < mine) ? d : 0;
        }
#pragma unroll
        for (int w = 0; w < G; ++w) rank += w0 + w < nl ? pos[w] : 0;
    }
    return rank;
}

// The two rows of a resolved connection, packed in one LDS word (-1: none).
__device__ __forceinline__ int src_of(int sd) { return (int)(short)(sd & 0xffff); }
__device__ __forceinline__ int dst_of(int sd) { return sd >> 16; }

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x >> 6); }

// number of set bits of m below this lane
__device__ __forceinline__ int mbcnt(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Inclusive prefix sum and minimum over the 64 lanes of a wave, by DPP
// (no LDS traffic): row shifts by 1, 2, 4 and 8 within each row of 16
// lanes, then the row results carried on by broadcasts of lanes 15 (to
// rows 1 and 3) and 31 (to rows 2 and 3).  A lane whose source is out of
// its row, or whose row is masked, takes the identity.
__device__ __forceinline__ int wave_incl_add(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}
__device__ __forceinline__ int wave_incl_min(int x) {
    constexpr int ID = 0x7fffffff;
    x = min(x, __builtin_amdgcn_update_dpp(ID, x, 0x111, 0xf, 0xf, false));
    x = min(x, __builtin_amdgcn_update_dpp(ID, x, 0x112, 0xf, 0xf, false));
    x = min(x, __builtin_amdgcn_update_dpp(ID, x, 0x114, 0xf, 0xf, false));
    x = min(x, __builtin_amdgcn_update_dpp(ID, x, 0x118, 0xf, 0xf, false));
    x = min(x, __builtin_amdgcn_update_dpp(ID, x, 0x142, 0xa, 0xf, false));
    x = min(x, __builtin_amdgcn_update_dpp(ID, x, 0x143, 0xc, 0xf, false));
    return x;
}

// Block-wide exclusive scan of one value per thread; *total receives the sum.
// Contains two barriers; every thread of the block must call it.
__device__ int block_excl_scan(int v, int *s_wave, int *total) {
    const int lane = lane_id(), wave = wave_id(), nw = (int)(blockDim.x >> 6);
    const int x = wave_incl_add(v);
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    // lane w reads wave w's sum; a wave scan adds them up
    const int incl = wave_incl_add(lane < nw ? s_wave[lane] : 0);
    const int base = wave > 0 ? __builtin_amdgcn_readlane(incl, wave - 1) : 0;
    *total = __builtin_amdgcn_readlane(incl, nw - 1);
    __syncthreads();
    return base + x - v;
}

// The threads transforming one genome (one workgroup of at least
// round_up(N_max, 64) threads).  When N_max <= 64 the group is one wave:
// it needs no s_barrier (its lanes run together and its LDS operations
// complete in order), only a fence that keeps the compiler from moving
// memory operations across the synchronisation point, and its scans stay
// in the wave.  (Packing several one-wave genomes into a workgroup was
// measured slower on the control workload: 61 and 62.5 us for two and four
// per workgroup against 59 us for one.)
template <bool ONE>
struct Grp {
    int t, W;        // thread in the group, group size
    int lane, wave;  // lane and wave within the group
    int nw;          // waves in the group (1 when ONE)
    int *sh;         // the group's scalars (SH_*) and per-wave partials
};
constexpr int SH_STATUS = 0, SH_NVALID = 1, SH_USED = 2, SH_WIDE = 3, SH_WAVE = 4, SH_WORDS = 20;

template <bool ONE>
__device__ __forceinline__ void gsync(const Grp<ONE> &G) {
    if (ONE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <bool ONE>
__device__ __forceinline__ bool gsync_or(const Grp<ONE> &G, bool x) {
    if (ONE) {
        gsync(G);
        return __ballot(x) != 0ull;
    }
    return __syncthreads_or(x);
}

// The sum of the per-wave values in G.sh[SH_WAVE + w] over the waves before
// this one (*before) and over all (*total): lane w reads wave w's value, and a
// wave scan adds them up.
template <bool ONE>
__device__ __forceinline__ void wave_partials(const Grp<ONE> &G, int *before, int *total) {
    const int part = G.lane < G.nw ? G.sh[SH_WAVE + G.lane] : 0;
    const int incl = wave_incl_add(part);
    *before = G.wave > 0 ? __builtin_amdgcn_readlane(incl, G.wave - 1) : 0;
    *total = __builtin_amdgcn_readlane(incl, G.nw - 1);
}

// Exclusive scan of one value per thread over the group; *total receives
// the sum.  Every thread of the group must call it.
template <bool ONE>
__device__ __forceinline__ int group_excl_scan(const Grp<ONE> &G, int v, int *total) {
    const int x = wave_incl_add(v);
    if (ONE) {
        *total = __builtin_amdgcn_readlane(x, 63);
        return x - v;
    }
    if (G.lane == 63) G.sh[SH_WAVE + G.wave] = x;
    gsync(G);
    int base;
    wave_partials(G, &base, total);
    gsync(G);
    return base + x - v;
}

// Inclusive prefix minimum of one value per thread over the group.
template <bool ONE>
__device__ __forceinline__ int group_incl_min(const Grp<ONE> &G, int v) {
    const int x = wave_incl_min(v);
    if (ONE) return x;
    if (G.lane == 63) G.sh[SH_WAVE + G.wave] = x;
    gsync(G);
    // the minimum over the waves before this one
    const int part = G.lane < G.wave ? G.sh[SH_WAVE + G.lane] : 0x7fffffff;
    const int before = __builtin_amdgcn_readlane(wave_incl_min(part), 63);
    gsync(G);
    return min(before, x);
}

// Transformation of genome g of population a by group G (at least
// round_up(N_max, 64) threads), in the LDS words at smem.
template <bool ONE>
__device__ __forceinline__ void topo_genome(const TopoItem &a, size_t g, const Grp<ONE> &G,
                                            int *smem) {
    unsigned &s_status = *reinterpret_cast<unsigned *>(&G.sh[SH_STATUS]);
    int &s_nvalid = G.sh[SH_NVALID];

    const int N = a.N, C = a.C, I = a.I, O = a.O;
    const int t = G.t, W = G.W;

    // 32-bit words first (keys, atomics, packed words), then 16-bit arrays
    // (rows, positions, slots, offsets: all below 2^15).  s_stack comes
    // first so that it is 16-byte aligned for the rank's vector reads.
    const int H = hash_size(N);
    const int NS = stack_words(N);
    const bool merge = !ONE && N > MERGE_MIN;
    int *s_stack = smem;          // [NS] packed (key, row) words: by row (padding
                                  //      -1), or sorted per wave when merging; slot
                                  //      allocation scratch
    int *s_key = s_stack + NS;    // [N] key of row, -1 absent, -2 malformed
    int *s_skey = s_key + N;      // [N] well-formed keys by stable rank; later level of row
    int *s_indeg = s_skey + N;    // [N] in-degree, consumed by Kahn
    int *s_deg = s_indeg + N;     // [N] in-degree kept for the program
    int *s_curo = s_deg + N;      // [N] out-degree, out cursor, later edge begin by row
    int *s_curi = s_curo + N;     // [N] io presence, in cursor, later row by position
    const int CE = stored_conns(N, C);
    int *e_sd = s_curi + N;       // [CE] connection row: source row | destination row << 16,
                                  //      -1 if unused (rows < 2^10): the rows a thread
                                  //      does not keep in registers
    int *h_key = e_sd + CE;       // [H] key -> row table: keys; after the lookups
                                  //     (larger groups) the key rank of every row
    int *h_row = h_key + H;       // [H] rows
    int16_t *s_srow = reinterpret_cast<int16_t *>(h_row + H);  // [N] row by rank
    int16_t *s_inoff = s_srow + N;      // [N+1] in-edge offsets (<= C_max <= 2^14)
    int16_t *s_outoff = s_inoff + N + 1;  // [N+1] out-edge offsets
    int16_t *s_pos = s_outoff + N + 1;  // [N] position of row
    int16_t *s_slot = s_pos + N;        // [N] value slot of row
    int16_t *s_oval = s_slot + N;       // [N] slot allocation scratch
    uint16_t *out_list = reinterpret_cast<uint16_t *>(s_oval + N);  // [C] destination rows
                                        //     grouped by source
    int16_t *in_rank = reinterpret_cast<int16_t *>(out_list + C);  // [C] source key ranks of
                                        //     the in-edges, grouped by destination
    int16_t *s_rnk = reinterpret_cast<int16_t *>(h_key);  // [N] key rank of row (-1: none)

    const float *nodes = a.nodes + g * (size_t)N * 5;
    const float *conns = a.conns + g * (size_t)C * 4;
    const float4 *conns4 = reinterpret_cast<const float4 *>(conns);

    // the first connection rows of this thread and its node row, requested
    // together before anything waits on memory
    constexpr int CPRE = 4;
    float4 cpre[CPRE];
#pragma unroll
    for (int k = 0; k < CPRE; ++k) {
        const float nan = __builtin_nanf("");
        cpre[k] = make_float4(nan, nan, nan, nan);  // past C_max: a padding row
        if (t + k * W < C) cpre[k] = conns4[t + k * W];
    }
    float nrow[5];
    if (t < N) {
#pragma unroll
        for (int k = 0; k < 5; ++k) nrow[k] = nodes[(size_t)t * 5 + k];
    }

    if (t == 0) {
        s_status = 0u;
        s_nvalid = 0;
        G.sh[SH_WIDE] = 0;
    }
    for (int i = t; i < N; i += W) {
        if (!ONE) {  // one-wave groups write these before any read
            s_indeg[i] = 0;
            s_curo[i] = 0;
            s_pos[i] = -1;
        }
        s_curi[i] = 0;
        s_skey[i] = -1;
    }
    for (int i = t; i < H; i += W) {
        h_key[i] = HASH_EMPTY;
        h_row[i] = 0x7fffffff;
    }
    if (!merge && t >= N && t < NS) s_stack[t] = -1;
    gsync(G);

    // ---- 1. node rows
    const int rb = N <= 256 ? 8 : 10;  // row bits of the packed (key, row) words
    unsigned st = 0u;
    int key = -1, act = 0, agg = 0, my_h = -1;
    float bias = 0.0f, resp = 0.0f;
    if (t < N) {
        const float kf = nrow[0];
        bias = nrow[1];
        resp = nrow[2];
        const float af = nrow[3], gf = nrow[4];
        if (!isnan(kf)) {
            atomicAdd(&s_nvalid, 1);
            const bool key_ok = is_int_in(kf, 0.0f, KEY_LIMIT);
            if (!key_ok) st |= NEAT_ST_BAD_VALUE;
            if (!is_int_in(af, 0.0f, (float)N_ACT) || !is_int_in(gf, 0.0f, (float)N_AGG))
                st |= NEAT_ST_BAD_VALUE;
            else {
                act = (int)af;
                agg = (int)gf;
            }
            key = key_ok ? (int)kf : -2;
            if (key_ok) my_h = hash_insert(h_key, h_row, H, key, t);
        }
        s_key[t] = key;
        // (key, row) in one word: rows take rb bits, keys the rest (always
        // room when rows fit in 8 bits, keys being below 2^24; with 10 row
        // bits a key of 2^22 or more marks the genome as wide)
        if (key >= 0 && rb == 10 && key >= (1 << 22)) G.sh[SH_WIDE] = 1;
        if (!merge) s_stack[t] = key >= 0 ? (int)(((unsigned)key << rb) | (unsigned)t) : -1;
    }
    gsync(G);

    // ---- 2. stable key rank (by key, then row), duplicate keys,
    // input/output presence
    int rank = -1;
    const bool packed = G.sh[SH_WIDE] == 0;
    if (merge && packed) {
        // Every wave sorts its rows' (key, row) words in
        // registers (bitonic network; absent rows and lanes beyond N_max hold
        // the largest word) into its own list, and a row's rank is the sum
        // over the lists of the number of words below its own (binary
        // searches, all lists side by side).
        const unsigned mine =
            (t < N && key >= 0) ? (((unsigned)key << rb) | (unsigned)t) : 0xffffffffu;
        unsigned x = mine;
#pragma unroll
        for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                const unsigned y = (unsigned)__shfl_xor((int)x, j, 64);
                x = (((G.lane & j) == 0) == ((G.lane & k) == 0)) ? min(x, y) : max(x, y);
            }
        const int nl = (N + 63) >> 6;  // lists (waves holding rows)
        if (G.wave < nl) s_stack[G.wave * 64 + G.lane] = (int)x;
        gsync(G);
        if (key >= 0) {
            const unsigned *sl = reinterpret_cast<const unsigned *>(s_stack);
            rank = nl <= 4 ? merged_rank<4>(sl, nl, mine) : merged_rank<8>(sl, nl, mine);
        }
    }
    if (key >= 0) {
        if (merge && packed) {
            // ranked above
        } else if (packed) {
            // rank = number of (key, row) words below this row's (the words
            // are distinct; absent and malformed rows and the padding hold
            // the largest), read four at a time (every lane the same address)
            const unsigned mine = ((unsigned)key << rb) | (unsigned)t;
            const uint4 *comp = reinterpret_cast<const uint4 *>(s_stack);
            int less = 0;
#pragma unroll 4
            for (int q = 0; q < (NS >> 2); ++q) {
                const uint4 v = comp[q];
                less += (v.x < mine) + (v.y < mine) + (v.z < mine) + (v.w < mine);
            }
            rank = less;
        } else {
            int less = 0, eq_before = 0;
            for (int q = 0; q < N; ++q) {
                const int kq = s_key[q];
                if (kq < 0) continue;
                less += (kq < key);
                eq_before += (kq == key && q < t);
            }
            rank = less + eq_before;
        }
        s_skey[rank] = key;
        s_srow[rank] = t;
        if (key < I + O) s_curi[key] = 1;
    }
    gsync(G);
    // equal keys hold neighbouring ranks (the other entries are -1)
    if (rank >= 0 && ((rank > 0 && s_skey[rank - 1] == key) ||
                      (rank + 1 < N && s_skey[rank + 1] == key)))
        st |= NEAT_ST_DUP_KEY;
    if (t < I + O && s_curi[t] == 0) st |= NEAT_ST_MISSING_IO;
    // One-wave groups hold the graph as bit masks over key ranks (at most
    // 64): row d's sources, bits 0-31 in s_stack[d] and 32-63 in s_skey[d]
    // (both free until Kahn's levels are written).  Every key's table word
    // gets the key's rank above its row.
    if constexpr (ONE) {
        gsync(G);  // the duplicate-key check has read s_skey
        // (with duplicated keys the last writer wins; such a genome is
        // rejected, and its other status bits depend on keys only)
        if (key >= 0) h_row[my_h] = t | (rank << 16);
        if (t < N) {
            s_stack[t] = 0;
            s_skey[t] = 0;
        }
        gsync(G);
    }

    // ---- 3. connection rows.  A resolved row counts into the degrees (in
    // one-wave groups: sets its source's bit in the destination's mask, and
    // a bit already set is a duplicate edge); the thread keeps its
    // prefetched rows (rows packed as in e_sd, source key) in registers, the
    // others go to e_sd.  One-wave groups pack the source's rank too:
    // source | rank << 8 | destination << 16.
    auto resolved = [&](int ws, int wd, int kd) {
        if (ws < 0 || wd < 0) {
            st |= NEAT_ST_BAD_REF;
            return -1;
        }
        const int s = ws & 0xffff, d = wd & 0xffff;
        // d holds key kd (the table maps a key to a row holding it)
        if (kd < I) st |= NEAT_ST_INTO_INPUT;
        if (s == d && !a.recurrent) st |= NEAT_ST_CYCLE;
        if constexpr (ONE) {
            const int rs = ws >> 16;
            const unsigned bit = 1u << (rs & 31);
            unsigned *mask = reinterpret_cast<unsigned *>(rs < 32 ? s_stack : s_skey);
            if (atomicOr(&mask[d], bit) & bit) st |= NEAT_ST_DUP_EDGE;
            return s | (rs << 8) | (d << 16);
        } else {
            atomicAdd(&s_indeg[d], 1);
            atomicAdd(&s_curo[s], 1);
            return s | (d << 16);
        }
    };
    // an enabled row's endpoint keys, or false (padding, disabled, or a bad
    // enabled flag, which is flagged)
    auto enabled = [&](const float4 row) {
        if (isnan(row.x) || row.z == 0.0f) return false;
        if (row.z != 1.0f) {
            st |= NEAT_ST_BAD_VALUE;
            return false;
        }
        return true;
    };
    int sdp[CPRE], ksp[CPRE];
    {
        // all endpoints of the prefetched rows: first probes read together,
        // then the (rare) further probes, then the rows together
        int key2[2 * CPRE], hs[2 * CPRE], hk[2 * CPRE];
#pragma unroll
        for (int k = 0; k < CPRE; ++k) {
            // enabled (flag 1), padding or disabled (NaN source, flag 0), or a
            // bad flag; branch-free
            const float4 r = cpre[k];
            const bool live = !isnan(r.x) & (r.z != 0.0f);
            const bool bad = live & (r.z != 1.0f);
            st |= bad ? (unsigned)NEAT_ST_BAD_VALUE : 0u;
            const bool on = live & !bad;
            key2[k] = on ? key_of(r.x) : -1;
            key2[CPRE + k] = on ? key_of(r.y) : -1;
            sdp[k] = on ? -2 : -1;  // -2: enabled, endpoints to resolve
        }
#pragma unroll
        for (int i = 0; i < 2 * CPRE; ++i) {
            hs[i] = key2[i] >= 0 ? hash_slot(key2[i], H) : 0;
            hk[i] = h_key[hs[i]];
        }
        for (;;) {
            bool more = false;
#pragma unroll
            for (int i = 0; i < 2 * CPRE; ++i) {
                const bool go = key2[i] >= 0 && hk[i] != key2[i] && hk[i] != HASH_EMPTY;
                if (go) hs[i] = (hs[i] + 1) & (H - 1);
                more |= go;
            }
            if (!more) break;
#pragma unroll
            for (int i = 0; i < 2 * CPRE; ++i) hk[i] = h_key[hs[i]];
        }
        int r2[2 * CPRE];
#pragma unroll
        for (int i = 0; i < 2 * CPRE; ++i) r2[i] = h_row[hs[i]];
        // every read is needed as issued (a select on a fresh load would
        // otherwise become a branch around it, and the reads one wait each)
#pragma unroll
        for (int i = 0; i < 2 * CPRE; ++i) asm volatile("" : "+v"(r2[i]));
#pragma unroll
        for (int i = 0; i < 2 * CPRE; ++i) r2[i] = (key2[i] >= 0 && hk[i] == key2[i]) ? r2[i] : -1;
        if constexpr (ONE) {
            // the mask updates of all four rows in flight together; a row
            // without an edge ORs 0 into row 0's mask
            unsigned bits[CPRE], old[CPRE];
#pragma unroll
            for (int k = 0; k < CPRE; ++k) {
                const int ws = r2[k], wd = r2[CPRE + k];
                const bool ok = sdp[k] == -2 && ws >= 0 && wd >= 0;
                if (sdp[k] == -2 && !ok) st |= NEAT_ST_BAD_REF;
                const int s = ws & 0xffff, d = wd & 0xffff, rs = (ws >> 16) & 0xff;
                if (ok && key2[CPRE + k] < I) st |= NEAT_ST_INTO_INPUT;
                if (ok && s == d && !a.recurrent) st |= NEAT_ST_CYCLE;
                bits[k] = ok ? 1u << (rs & 31) : 0u;
                unsigned *mask = reinterpret_cast<unsigned *>(ok && rs >= 32 ? s_skey : s_stack);
                old[k] = atomicOr(&mask[ok ? d : 0], bits[k]);
                sdp[k] = ok ? s | (rs << 8) | (d << 16) : -1;
            }
#pragma unroll
            for (int k = 0; k < CPRE; ++k)
                if (old[k] & bits[k]) st |= NEAT_ST_DUP_EDGE;
        } else {
#pragma unroll
            for (int k = 0; k < CPRE; ++k)
                if (sdp[k] == -2) sdp[k] = resolved(r2[k], r2[CPRE + k], key2[CPRE + k]);
        }
#pragma unroll
        for (int k = 0; k < CPRE; ++k) ksp[k] = key2[k];
    }
    for (int c = t + CPRE * W; c < C; c += W) {
        const float4 row = conns4[c];
        int sd = -1;
        if (enabled(row))
            sd = resolved(find_row(row.x, h_key, h_row, H), find_row(row.y, h_key, h_row, H),
                          is_int_in(row.y, 0.0f, KEY_LIMIT) ? (int)row.y : -1);
        e_sd[c] = sd;
    }
    gsync(G);

    // ---- 4. adjacency (one-wave groups: in-degrees and indices from the
    // masks; other groups: counting sort by destination and by source)
    int jp[CPRE];     // index of each prefetched edge among its destination's
                      // in-edges by source key
    int deg1 = 0;     // one-wave groups: in-degree of row t
    int nreal = 0;    // one-wave groups: edges
    if constexpr (ONE) {
        // ranks follow keys, so an edge's index is the number of its
        // destination's sources of smaller rank
        auto below = [&](int d, int rs) {
            const unsigned lo = (unsigned)s_stack[d], hi = (unsigned)s_skey[d];
            return rs < 32 ? __popc(lo & ((1u << rs) - 1u))
                           : __popc(lo) + __popc(hi & ((1u << (rs - 32)) - 1u));
        };
        if (t < N) deg1 = __popc((unsigned)s_stack[t]) + __popc((unsigned)s_skey[t]);
        group_excl_scan(G, deg1, &nreal);
#pragma unroll
        for (int k = 0; k < CPRE; ++k)
            jp[k] = sdp[k] >= 0 ? below(sdp[k] >> 16, (sdp[k] >> 8) & 0xff) : 0;
        // the other rows keep their index in place of the rank
        for (int c = t + CPRE * W; c < C; c += W) {
            const int sd = e_sd[c];
            if (sd >= 0) e_sd[c] = (sd & ~0xff00) | (below(sd >> 16, (sd >> 8) & 0xff) << 8);
        }
    } else {
        // the key table is done with: it now holds every row's key rank, and
        // the in-lists compare ranks (the same order as keys, 16 bits)
        if (t < N) s_rnk[t] = (int16_t)rank;
        {
            const int din = (t < N) ? s_indeg[t] : 0;
            const int dout = (t < N) ? s_curo[t] : 0;
            int tin, tout;
            const int ein = group_excl_scan(G, din, &tin);
            const int eout = group_excl_scan(G, dout, &tout);
            if (t < N) {
                s_inoff[t] = ein;
                s_outoff[t] = eout;
                s_deg[t] = din;
                s_curo[t] = 0;
                s_curi[t] = 0;
            }
            if (t == 0) {
                s_inoff[N] = tin;
                s_outoff[N] = tout;
            }
        }
        gsync(G);
        // scatter: a destination's in-list holds the source key ranks, a
        // source's out-list the destination rows
        auto scatter = [&](int sd, int rs) {
            const int s = src_of(sd), d = dst_of(sd);
            in_rank[s_inoff[d] + atomicAdd(&s_curi[d], 1)] = (int16_t)rs;
            out_list[s_outoff[s] + atomicAdd(&s_curo[s], 1)] = (uint16_t)d;
        };
#pragma unroll
        for (int k = 0; k < CPRE; ++k) ksp[k] = sdp[k] >= 0 ? s_rnk[src_of(sdp[k])] : -1;
#pragma unroll
        for (int k = 0; k < CPRE; ++k)
            if (sdp[k] >= 0) scatter(sdp[k], ksp[k]);
        for (int c = t + CPRE * W; c < C; c += W) {
            const int sd = e_sd[c];
            if (sd >= 0) scatter(sd, s_rnk[src_of(sd)]);
        }
        gsync(G);
        // every edge's index among its destination's in-edges by source key (the
        // number of smaller source ranks) and duplicate edges (an equal source
        // rank besides its own).  The prefetched rows walk their in-lists side
        // by side, so their reads overlap; their indices stay in registers.
        {
            int base[CPRE], cnt[CPRE], eq[CPRE];
            int m = 0;
#pragma unroll
            for (int k = 0; k < CPRE; ++k) {
                base[k] = 0;
                cnt[k] = 0;
                if (sdp[k] >= 0) {
                    const int d = dst_of(sdp[k]);
                    base[k] = s_inoff[d];
                    cnt[k] = s_inoff[d + 1] - base[k];
                }
                m = max(m, cnt[k]);
                jp[k] = 0;
                eq[k] = 0;
            }
            for (int i = 0; i < m; ++i) {
#pragma unroll
                for (int k = 0; k < CPRE; ++k) {
                    // an exhausted list re-reads its last entry (or entry 0 of
                    // a row with no list, which exists since m > 0)
                    const int q = in_rank[base[k] + min(i, max(cnt[k] - 1, 0))];
                    const bool v = i < cnt[k];
                    jp[k] += (v && q < ksp[k]) ? 1 : 0;
                    eq[k] += (v && q == ksp[k]) ? 1 : 0;
                }
            }
#pragma unroll
            for (int k = 0; k < CPRE; ++k)
                if (eq[k] > 1) st |= NEAT_ST_DUP_EDGE;
        }
        for (int c = t + CPRE * W; c < C; c += W) {
            const int sd = e_sd[c];
            if (sd < 0) continue;
            const int d = dst_of(sd), rs = s_rnk[src_of(sd)];
            int eq = 0;
            for (int k = s_inoff[d]; k < s_inoff[d + 1]; ++k) eq += in_rank[k] == rs;
            if (eq > 1) st |= NEAT_ST_DUP_EDGE;
        }
    }
    if (st) atomicOr(&s_status, st);
    gsync(G);
    unsigned status = s_status;
    const int nvalid = s_nvalid;

    // ---- 5. level-synchronous Kahn over key ranks (a recurrent network has
    // no order to find: every node takes its key rank as position, level 0)
    int n_levels = 0;
    int my_level = -1;
    const int my_row = (status == 0u && t < nvalid) ? s_srow[t] : -1;
    if (status == 0u && a.recurrent) {
        if (my_row >= 0) {
            s_pos[my_row] = t;
            my_level = 0;
        }
        n_levels = nvalid > 0 ? 1 : 0;
    } else if (status == 0u) {
        int base = 0;
        if constexpr (ONE) {
            // a node is ready once every source's rank bit is in done (the
            // ranks emitted so far); lane t holds rank t
            unsigned long long pm = 0ull, done = 0ull;
            if (my_row >= 0)
                pm = (unsigned long long)(unsigned)s_stack[my_row] |
                     ((unsigned long long)(unsigned)s_skey[my_row] << 32);
            bool emitted = false;
            int my_pos = -1;
            for (;;) {
                const bool ready = my_row >= 0 && !emitted && (pm & ~done) == 0ull;
                const unsigned long long m = __ballot(ready);
                if (m == 0ull) break;
                if (ready) {
                    my_pos = base + mbcnt(m);
                    my_level = n_levels;
                    emitted = true;
                }
                done |= m;
                base += __popcll(m);
                ++n_levels;
            }
            if (emitted) s_pos[my_row] = my_pos;
        } else {
            const int lane = G.lane, wave = G.wave;
            bool emitted = false;
            const int ob = my_row >= 0 ? s_outoff[my_row] : 0;
            const int oe = my_row >= 0 ? s_outoff[my_row + 1] : 0;
            for (;;) {
                const bool ready = my_row >= 0 && !emitted && s_indeg[my_row] == 0;
                const unsigned long long m = __ballot(ready);
                if (lane == 0) G.sh[SH_WAVE + wave] = __popcll(m);
                gsync(G);
                int wbase, total;
                wave_partials(G, &wbase, &total);
                if (total == 0) break;  // uniform across the block
                if (ready) {
                    s_pos[my_row] = base + wbase + mbcnt(m);
                    my_level = n_levels;
                    emitted = true;
                    // successors read four at a time, then decremented
                    int k = ob;
                    for (; k + 3 < oe; k += 4) {
                        const int d0 = out_list[k], d1 = out_list[k + 1];
                        const int d2 = out_list[k + 2], d3 = out_list[k + 3];
                        atomicSub(&s_indeg[d0], 1);
                        atomicSub(&s_indeg[d1], 1);
                        atomicSub(&s_indeg[d2], 1);
                        atomicSub(&s_indeg[d3], 1);
                    }
                    for (; k < oe; ++k) atomicSub(&s_indeg[out_list[k]], 1);
                }
                gsync(G);
                base += total;
                ++n_levels;
            }
        }
        if (base < nvalid) status |= NEAT_ST_CYCLE;
    }
    gsync(G);  // s_pos complete; s_skey is free and now holds levels
    if (my_row >= 0) s_skey[my_row] = my_level;
    if (status == 0u && t < N && s_key[t] != -1) s_curi[s_pos[t]] = t;  // row by position
    gsync(G);

    // ---- outputs: order, level, status
    const bool ok = status == 0u;
    if (a.order) {
        if (t < N && (!ok || t >= nvalid)) a.order[g * N + t] = -1;
        if (ok && t < N && s_key[t] != -1) a.order[g * N + s_pos[t]] = t;
    }
    if (a.level && t < N) a.level[g * N + t] = (ok && s_key[t] != -1) ? s_skey[t] : -1;
    if (a.status && t == 0) a.status[g] = status;
    if (!a.prog) return;

    // ---- 6. value slots, then the program (layout in program.h)
    int &s_used = G.sh[SH_USED];
    int32_t *prog = a.prog + g * (size_t)a.prog_words;
    float *progf = reinterpret_cast<float *>(prog);
    if (!ok) {
        if (t == 0) {
            prog[HDR_NVALID] = 0;
            prog[HDR_NEDGES] = 0;
            prog[HDR_STATUS] = (int32_t)status;
            prog[HDR_NLEVELS] = 0;
            prog[HDR_I] = I;
            prog[HDR_O] = O;
            prog[HDR_CLASS] = CLS_R64;
            prog[HDR_NREAL] = 0;
            prog[HDR_SLOTS] = 0;
        }
        return;  // uniform
    }
    if (max_class(N) == CLS_R64 || a.recurrent) {
        // every genome fits the 64-slot class, or every value stays live
        // from one sweep to the next: slot = position
        if (t < nvalid) s_slot[s_curi[t]] = t;
        if (t == 0) s_used = nvalid;
    } else {
        // last reading position of every value (s_indeg is free after
        // Kahn, and unused by one-wave groups); outputs are read after the
        // last node
        int *s_last = s_indeg;
        if constexpr (ONE) {
            // every edge raises its source's last position to its own
            if (t < N && s_key[t] != -1)
                s_last[t] = (s_key[t] >= I && s_key[t] < I + O) ? nvalid : (int)s_pos[t];
            gsync(G);
#pragma unroll
            for (int k = 0; k < CPRE; ++k)
                if (sdp[k] >= 0) atomicMax(&s_last[sdp[k] & 0xff], (int)s_pos[sdp[k] >> 16]);
            for (int c = t + CPRE * W; c < C; c += W) {
                const int sd = e_sd[c];
                if (sd >= 0) atomicMax(&s_last[sd & 0xff], (int)s_pos[sd >> 16]);
            }
        } else if (t < N && s_key[t] != -1) {
            int last = s_pos[t];
            for (int k = s_outoff[t]; k < s_outoff[t + 1]; ++k)
                last = max(last, (int)s_pos[out_list[k]]);
            if (s_key[t] >= I && s_key[t] < I + O) last = nvalid;
            s_last[t] = last;
        }
        gsync(G);
        // Slots by liveness, in parallel.  A value frees its slot for the
        // position free_at: its last reader (which reads before writing),
        // the next position when nothing reads it, I for unread inputs;
        // outputs never.  Position p >= I takes a slot freed at p when there
        // is one (the smallest such row), else the earliest-ranked slot freed
        // before p and not yet taken, else a new slot.  Rank order is valid:
        // a close that finds a free slot is preceded by more frees than
        // earlier matched closes, so the free of its rank has happened.  A
        // new slot is made only when none is free, so the count is the
        // largest live set.  Each value hands its slot on at most once, so
        // slots follow chains, resolved by pointer jumping.
        int *s_free = s_last;     // by row: free position (INT_MAX: never)
        int *s_dc = s_stack;      // by position: frees there (+ cursor << 16); later ancestor
        int *s_pair = s_deg;      // by position: smallest row freed there
        int *s_obase = s_curo;    // by position: rank of its first extra free
        const int NEVER = 0x7fffffff;
        if (t < N) {
            s_dc[t] = 0;
            s_pair[t] = NEVER;
        }
        gsync(G);
        if (t < N && s_key[t] != -1) {
            const int p = s_pos[t], last = s_last[t];
            const bool out = s_key[t] >= I && s_key[t] < I + O;
            const int fa = out ? NEVER : (last > p ? last : (p < I ? I : p + 1));
            s_free[t] = fa;
            if (fa < nvalid) {
                atomicAdd(&s_dc[fa], 1);
                atomicMin(&s_pair[fa], t);
            }
        }
        gsync(G);
        // per position: pairing, or an open (extra frees) / close (birth
        // without a free at its position) event; clamped depth by scans
        const bool vp = t >= I && t < nvalid;
        const int d = vp ? (s_dc[t] & 0xffff) : 0;
        const int pairrow = vp ? s_pair[t] : -1;
        const int n_open = d > 1 ? d - 1 : 0, n_close = (vp && d == 0) ? 1 : 0;
        int tot_open, tot_close;
        const int ob = group_excl_scan(G, n_open, &tot_open);
        const int cb = group_excl_scan(G, n_close, &tot_close);
        const int u_before = -group_incl_min(G, ob - cb);  // unmatched closes before
        const int s_incl = ob + n_open - cb - n_close;
        const int u_incl = max(u_before, -s_incl);
        const bool unmatched = n_close && u_incl > u_before;
        const int close_rank = cb - u_before;  // matched closes before this one
        if (vp) s_obase[t] = ob;
        if (t == nvalid - 1) s_used = I + u_incl;
        gsync(G);
        // extra frees get their open ranks
        if (t < N && s_key[t] != -1) {
            const int fa = s_free[t];
            if (fa < nvalid && s_pair[fa] != t) {
                const int k = atomicAdd(&s_dc[fa], 0x10000) >> 16;
                s_oval[s_obase[fa] + k] = t;
            }
        }
        gsync(G);
        // ancestors: the value whose slot a birth takes; roots get slots
        int *s_anc = s_dc;
        if (t < nvalid) {
            const int b = s_curi[t];
            int anc = -1;
            if (t < I) s_slot[b] = t;
            else if (d > 0) anc = pairrow;
            else if (!unmatched) anc = s_oval[close_rank];
            else s_slot[b] = I + u_incl - 1;
            s_anc[b] = anc;
        }
        gsync(G);
        bool more = true;
        while (more) {
            int anc = -1, slot = 0;
            bool changed = false;
            if (t < N && s_key[t] != -1) {
                anc = s_anc[t];
                if (anc >= 0) {
                    const int aa = s_anc[anc];
                    if (aa < 0) slot = s_slot[anc];
                    changed = true;
                    anc = aa;
                }
            }
            gsync(G);
            if (changed) {
                s_anc[t] = anc;
                if (anc < 0) s_slot[t] = slot;
            }
            more = gsync_or(G, changed);
        }
    }
    gsync(G);
    const int used = s_used;
    const int cls = class_of(used);
    const int zs = zero_slot(cls, N);
    if (t == 0) {
        prog[HDR_NVALID] = nvalid;
        prog[HDR_STATUS] = 0;
        prog[HDR_NLEVELS] = n_levels;
        prog[HDR_I] = I;
        prog[HDR_O] = O;
        prog[HDR_CLASS] = cls;
        prog[HDR_NREAL] = ONE ? nreal : (int)s_inoff[N];
        prog[HDR_SLOTS] = used;
    }
    // output slots: rank I + j holds key I + j
    if (t < O) prog[out_off() + t] = s_slot[s_srow[I + t]];
    // owner of a computed row: in-degree, pairs after padding to an even
    // count, overflow edges beyond the record
    const bool computed = t < N && s_key[t] >= 0 && s_pos[t] >= I;
    const int deg = !computed ? 0 : (ONE ? deg1 : s_inoff[t + 1] - s_inoff[t]);
    const int pairs = (deg + 1) >> 1;
    const int over = pairs > REC_INLINE_PAIRS ? 2 * (pairs - REC_INLINE_PAIRS) : 0;
    if (computed) s_deg[t] = over;
    gsync(G);
    // first overflow edge of every position, in topological order; level starts
    {
        const int row = (t < nvalid) ? s_curi[t] : -1;
        const int cnt = (t >= I && t < nvalid) ? s_deg[row] : 0;
        int tot;
        const int eb = group_excl_scan(G, cnt, &tot);
        if (t >= I && t < nvalid) {
            prog[ebeg_off(N, C, O) + (t - I)] = eb;
            s_curo[row] = eb;  // overflow begin by row
        }
        if (t < nvalid) {
            const int lv = s_skey[row];
            if (t == 0 || s_skey[s_curi[t - 1]] != lv) prog[lvl_off(N, C, O) + lv] = t;
        }
        if (t == 0) {
            prog[lvl_off(N, C, O) + n_levels] = nvalid;
            prog[HDR_NEDGES] = tot;
        }
        // the sentinel record after the last node (the record array holds
        // N records and at most N - I of them are nodes)
        if (t < REC_WORDS) {
            const int rs = rec_off(O) + REC_WORDS * (nvalid - I) + t;
            prog[rs] = t == REC_CODE     ? (int32_t)REC_SENTINEL_CODE
                       : t == REC_NPAIRS ? (int32_t)REC_SENTINEL_NPAIRS
                                         : 0;
        }
    }
    gsync(G);
    const int eoff = edge_off(N, O);
    if (computed) {
        const int k = s_pos[t] - I;
        const int r0 = rec_off(O) + REC_WORDS * k;
        const int ob = s_curo[t];
        const int acls = deg == 0 ? ACLS_SUM
                                  : (agg == AGG_PRODUCT ? ACLS_PROD
                                                        : ((agg == AGG_MAX || agg == AGG_MIN)
                                                               ? ACLS_MAX
                                                               : ACLS_SUM));
        // response folded with the mean's 1 / degree and min's sign
        const float rp = deg == 0 ? resp
                                  : (agg == AGG_MEAN ? resp * (1.0f / (float)deg)
                                                     : (agg == AGG_MIN ? -resp : resp));
        prog[r0 + REC_CODE] = (int32_t)rec_code(act, s_slot[t]);
        progf[r0 + REC_BIAS] = bias;
        progf[r0 + REC_RESP] = rp;
        prog[r0 + REC_NPAIRS] = (int32_t)rec_npairs(acls, pairs);
        // unused inline edges: a harmless (constant slot, 0) pair
        for (int j = 2 * pairs; j < 2 * REC_INLINE_PAIRS; ++j) {
            prog[r0 + REC_PAIRS + 2 * j] = zs;
            progf[r0 + REC_PAIRS + 2 * j + 1] = 0.0f;
        }
        // neutral padding edge when the in-degree is odd: the constant 0
        // (sum, mean) or 1 (product); for max and min the writer of the first
        // in-edge repeats it
        if ((deg & 1) && agg != AGG_MAX && agg != AGG_MIN) {
            const int widx = deg < 2 * REC_INLINE_PAIRS ? r0 + REC_PAIRS + 2 * deg
                                                         : eoff + EDGE_WORDS * (ob + deg - 2 * REC_INLINE_PAIRS);
            prog[widx] = agg == AGG_PRODUCT ? zs + 1 : zs;
            progf[widx + 1] = 1.0f;
        }
    }
    // aggregation code and in-degree by row for the edge writers (the
    // overflow begin by row is in s_curo)
    int *s_agg = s_deg;
    if (computed) s_agg[t] = agg | (deg << 8);
    gsync(G);
    // real edges at their index j among the destination's in-edges (found
    // above; source keys are unique here): j < 6 in the record, the rest in
    // the overflow array.  The thread that read a connection row writes its
    // edge (the prefetched rows' weights are still in registers).
    auto edge = [&](int sd, int j, float w) {
        const int s = src_of(sd), d = dst_of(sd);
        const int ad = s_agg[d], aggd = ad & 0xff, degd = ad >> 8;
        const int rd = rec_off(O) + REC_WORDS * (s_pos[d] - I);
        const int ob = s_curo[d];
        const int slot = s_slot[s];
        // min is stored as max over negated weights (negation is exact)
        const float wv = aggd == AGG_MIN ? -w : w;
        auto put = [&](int jj) {
            const int widx = jj < 2 * REC_INLINE_PAIRS ? rd + REC_PAIRS + 2 * jj
                                                        : eoff + EDGE_WORDS * (ob + jj - 2 * REC_INLINE_PAIRS);
            prog[widx] = slot;
            progf[widx + 1] = wv;
        };
        put(j);
        // max / min of an odd in-degree: the first edge once more
        if (j == 0 && (degd & 1) && (aggd == AGG_MAX || aggd == AGG_MIN)) put(degd);
    };
    // (one-wave groups pack a rank or an index in bits 8-15)
#pragma unroll
    for (int k = 0; k < CPRE; ++k)
        if (sdp[k] >= 0) edge(ONE ? sdp[k] & ~0xff00 : sdp[k], jp[k], cpre[k].w);
    for (int c = t + CPRE * W; c < C; c += W) {
        const int sd = e_sd[c];
        if (sd < 0) continue;
        int j = 0;
        if constexpr (ONE) {
            j = (sd >> 8) & 0xff;
        } else {
            const int d = dst_of(sd), rs = s_rnk[src_of(sd)];
            for (int k = s_inoff[d]; k < s_inoff[d + 1]; ++k) j += in_rank[k] < rs;
        }
        edge(ONE ? sd & ~0xff00 : sd, j, conns[(size_t)c * 4 + 3]);
    }
}

// Genome g by the workgroup (ONE: a single wave, N_max <= 64).
template <bool ONE>
__device__ __forceinline__ void topo_group(const TopoItem &a, long long g) {
    extern __shared__ __align__(16) int smem[];
    Grp<ONE> G;
    G.t = (int)threadIdx.x, G.W = ONE ? 64 : (int)blockDim.x, G.lane = G.t & 63;
    G.wave = ONE ? 0 : G.t >> 6, G.nw = ONE ? 1 : G.W >> 6;
    G.sh = smem;
    topo_genome(a, (size_t)g, G, smem + SH_WORDS);
}

template <bool ONE>
__global__ __launch_bounds__(1024) void topo_kernel(TopoItem a) {
    topo_group<ONE>(a, blockIdx.x);
}

// Many populations: workgroup b transforms genome b - block0 of the item
// whose range holds b (items sorted by block0).
template <bool ONE>
__global__ __launch_bounds__(1024) void topo_batch_kernel(const TopoItem *items, int n) {
    int lo = 0, hi = n - 1;
    const long long b = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    const TopoItem it = items[lo];
    topo_group<ONE>(it, b - it.block0);
}

// List the genomes of a population by slot class (one workgroup of 1024
// threads; thread t takes a contiguous run of genomes, so the lists are in
// genome order).  Rejected genomes go with R64: every forward kernel writes
// their NaN rows.
__device__ __forceinline__ void classify_pop(const int32_t *prog, int prog_words, int P,
                                             int32_t *pop) {
    __shared__ int s_wave[16];
    const int t = (int)threadIdx.x, W = (int)blockDim.x;
    const int per = (P + W - 1) / W;
    const int g0 = min(P, t * per), g1 = min(P, g0 + per);
    int cnt[N_CLASSES] = {0, 0, 0, 0};
    for (int g = g0; g < g1; ++g) {
        const int c = prog[(size_t)g * prog_words + HDR_CLASS];
#pragma unroll
        for (int k = 0; k < N_CLASSES; ++k) cnt[k] += (c == k) || (k == 0 && (c < 0 || c >= N_CLASSES));
    }
    int base[N_CLASSES], tot[N_CLASSES];
#pragma unroll
    for (int c = 0; c < N_CLASSES; ++c) base[c] = block_excl_scan(cnt[c], s_wave, &tot[c]);
    int begin = 0;
#pragma unroll
    for (int c = 0; c < N_CLASSES; ++c) {
        if (t == 0) {
            pop[POP_COUNT + c] = tot[c];
            pop[POP_BEGIN + c] = begin;
        }
        base[c] += begin;
        begin += tot[c];
    }
    for (int g = g0; g < g1; ++g) {
        int c = prog[(size_t)g * prog_words + HDR_CLASS];
        c = c < 0 || c >= N_CLASSES ? 0 : c;
        // select the class's cursor without dynamic register indexing
        int pos = base[0];
#pragma unroll
        for (int k = 1; k < N_CLASSES; ++k) pos = (c == k) ? base[k] : pos;
        pop[POP_IDS + pos] = g;
#pragma unroll
        for (int k = 0; k < N_CLASSES; ++k) base[k] += (c == k);
    }
}

__global__ __launch_bounds__(1024) void classify_kernel(const int32_t *prog, int prog_words,
                                                        int P, int32_t *pop) {
    classify_pop(prog, prog_words, P, pop);
}

// One workgroup per item (items of N_max <= 62 have no class list).
__global__ __launch_bounds__(1024) void classify_batch_kernel(const TopoItem *items) {
    const TopoItem it = items[blockIdx.x];
    if (!it.prog || max_class(it.N) == CLS_R64) return;
    classify_pop(it.prog, it.prog_words, it.P, it.prog + pop_off(it.P, it.N, it.C, it.O));
}

}  // namespace

size_t topo_lds_bytes(int N, int C) {
    // 32-bit: 7 N node words (the packed words padded, stack_words), the
    // connection rows kept in LDS (stored_conns), the key table (2 H);
    // 16-bit: 6 N + 2 node entries, 2 C connection entries
    return sizeof(int) * ((size_t)SH_WORDS + (size_t)stack_words(N) + (size_t)6 * N +
                          (size_t)stored_conns(N, C) + 2 * (size_t)hash_size(N)) +
           sizeof(int16_t) * ((size_t)6 * N + 2 + (size_t)2 * C);
}


int topo_block_threads(int N) {
    int w = round_up(N, 64);
    return w < 64 ? 64 : w;
}

hipError_t launch_topo(int P, int N, int C, int I, int O, const float *nodes,
                       const float *conns, int32_t *order, int32_t *level,
                       uint32_t *status, int32_t *prog, hipStream_t stream, int recurrent) {
    TopoItem a{nodes,   conns, order, level, status, prog, P, N, C, I, O, prog_words(N, C, O),
               0,       recurrent ? 1 : 0};
    const size_t L = topo_lds_bytes(N, C);
    if (P > 0) {
        const dim3 grid((unsigned)P), block((unsigned)topo_block_threads(N));
        if (N <= 64)
            hipLaunchKernelGGL(topo_kernel<true>, grid, block, L, stream, a);
        else
            hipLaunchKernelGGL(topo_kernel<false>, grid, block, L, stream, a);
    }
    if (prog && max_class(N) != CLS_R64) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(classify_kernel, dim3(1), dim3(1024), 0, stream, prog, a.prog_words, P,
                           prog + pop_off(P, N, C, O));
    }
    return hipGetLastError();
}

hipError_t launch_topo_batch(const TopoItem *dev_items, int n, long long blocks, int threads,
                             size_t lds, hipStream_t stream) {
    // one-wave groups when every genome fits a wave (the 64-thread bucket)
    if (threads == 64)
        hipLaunchKernelGGL(topo_batch_kernel<true>, dim3((unsigned)blocks), dim3(64u), lds, stream,
                           dev_items, n);
    else
        hipLaunchKernelGGL(topo_batch_kernel<false>, dim3((unsigned)blocks),
                           dim3((unsigned)threads), lds, stream, dev_items, n);
    return hipGetLastError();
}

hipError_t launch_classify_batch(const TopoItem *dev_items, int n, hipStream_t stream) {
    hipLaunchKernelGGL(classify_batch_kernel, dim3((unsigned)n), dim3(1024), 0, stream, dev_items);
    return hipGetLastError();
}

}  // namespace neat
