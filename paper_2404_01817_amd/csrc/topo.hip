// topo.hip -- the transformation stage (Section 3.3) for a whole population.
//
// One workgroup per genome; thread t owns node row t (the block has
// round_up(N_max, 64) threads).  Everything of one genome lives in LDS:
//
//   1. node rows: presence (key not NaN), key / act / agg validity;
//   2. key -> row map: a stable rank of every well-formed key (counting the
//      smaller keys), which gives the keys in sorted order for binary search
//      and detects duplicate keys; presence of the input/output keys;
//   3. connection rows, read as one float4 each: padding and disabled rows
//      are dropped, enabled rows are resolved through the key map into
//      (source row, destination row) and counted into in/out degrees;
//   4. exclusive scans of the degrees (wave shuffles + a cross-wave pass) and
//      a scatter into in- and out-adjacency lists; duplicate edges are found
//      inside each destination's in-list;
//   5. level-synchronous Kahn: every round, the nodes with in-degree 0 form
//      the frontier; lanes are assigned to nodes in key-rank order, so a
//      ballot + mbcnt prefix count gives each frontier node its position in
//      (level, key) order; emitted nodes decrement their successors' in-degree
//      with LDS atomics; nodes never emitted mean a cycle;
//   6. value slots by liveness (a sequential scan over the positions that
//      hands each value a free slot and frees it after its last reader),
//      then the program (program.h): records in topological order, in-edges
//      sorted by source key, source slots, level starts.
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
__device__ __forceinline__ void hash_insert(int *hkey, int *hrow, int H, int key, int row) {
    int h = hash_slot(key, H);
    for (;;) {
        const int old = atomicCAS(&hkey[h], HASH_EMPTY, key);
        if (old == HASH_EMPTY || old == key) {
            atomicMin(&hrow[h], row);
            return;
        }
        h = (h + 1) & (H - 1);
    }
}
// Row of the well-formed key equal to k (first row among duplicates), or -1.
__device__ __forceinline__ int find_row(float k, const int *hkey, const int *hrow, int H) {
    if (!is_int_in(k, 0.0f, KEY_LIMIT)) return -1;
    const int key = (int)k;
    for (int h = hash_slot(key, H);; h = (h + 1) & (H - 1)) {
        const int kk = hkey[h];
        if (kk == key) return hrow[h];
        if (kk == HASH_EMPTY) return -1;
    }
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

// Block-wide exclusive scan of one value per thread; *total receives the sum.
// Contains two barriers; every thread of the block must call it.
__device__ int block_excl_scan(int v, int *s_wave, int *total) {
    const int lane = lane_id(), wave = wave_id(), nw = (int)(blockDim.x >> 6);
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    int base = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        const int c = s_wave[w];
        base += (w < wave) ? c : 0;
        tot += c;
    }
    __syncthreads();
    *total = tot;
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

// Exclusive scan of one value per thread over the group; *total receives
// the sum.  Every thread of the group must call it.
template <bool ONE>
__device__ __forceinline__ int group_excl_scan(const Grp<ONE> &G, int v, int *total) {
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (G.lane >= d) x += y;
    }
    if (ONE) {
        *total = __shfl(x, 63, 64);
        return x - v;
    }
    if (G.lane == 63) G.sh[SH_WAVE + G.wave] = x;
    gsync(G);
    int base = 0, tot = 0;
    for (int w = 0; w < G.nw; ++w) {
        const int c = G.sh[SH_WAVE + w];
        base += (w < G.wave) ? c : 0;
        tot += c;
    }
    gsync(G);
    *total = tot;
    return base + x - v;
}

// Inclusive prefix minimum of one value per thread over the group.
template <bool ONE>
__device__ __forceinline__ int group_incl_min(const Grp<ONE> &G, int v) {
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (G.lane >= d) x = min(x, y);
    }
    if (ONE) return x;
    if (G.lane == 63) G.sh[SH_WAVE + G.wave] = x;
    gsync(G);
    int before = 0x7fffffff;
    for (int w = 0; w < G.wave; ++w) before = min(before, G.sh[SH_WAVE + w]);
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
    // (rows, positions, slots, offsets: all below 2^15)
    const int H = hash_size(N);
    int *s_key = smem;            // [N] key of row, -1 absent, -2 malformed
    int *s_skey = s_key + N;      // [N] well-formed keys by stable rank; later level of row
    int *s_indeg = s_skey + N;    // [N] in-degree, consumed by Kahn
    int *s_deg = s_indeg + N;     // [N] in-degree kept for the program
    int *s_curo = s_deg + N;      // [N] out-degree, out cursor, later edge begin by row
    int *s_curi = s_curo + N;     // [N] io presence, in cursor, later row by position
    int *s_stack = s_curi + N;    // [N] packed (key, row) words; slot allocation scratch
    int *e_sd = s_stack + N;      // [C] connection row: source row | destination row << 16,
                                  //     -1 if unused (rows < 2^10)
    int *out_list = e_sd + C;     // [C] destination rows grouped by source; later the
                                  //     source key of every in-edge
    int *h_key = out_list + C;    // [H] key -> row table: keys
    int *h_row = h_key + H;       // [H] rows
    int16_t *s_srow = reinterpret_cast<int16_t *>(h_row + H);  // [N] row by rank
    int16_t *s_inoff = s_srow + N;      // [N+1] in-edge offsets (<= C_max <= 2^14)
    int16_t *s_outoff = s_inoff + N + 1;  // [N+1] out-edge offsets
    int16_t *s_pos = s_outoff + N + 1;  // [N] position of row
    int16_t *s_slot = s_pos + N;        // [N] value slot of row
    int16_t *s_oval = s_slot + N;       // [N] slot allocation scratch
    uint16_t *in_list = reinterpret_cast<uint16_t *>(s_oval + N);  // [C] connection rows
                                        //     grouped by destination (rows < 2^14)

    const float *nodes = a.nodes + g * (size_t)N * 5;
    const float *conns = a.conns + g * (size_t)C * 4;
    const float4 *conns4 = reinterpret_cast<const float4 *>(conns);

    // the first connection rows of this thread and its node row, requested
    // together before anything waits on memory
    constexpr int CPRE = 4;
    float4 cpre[CPRE];
#pragma unroll
    for (int k = 0; k < CPRE; ++k)
        if (t + k * W < C) cpre[k] = conns4[t + k * W];
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
        s_indeg[i] = 0;
        s_curo[i] = 0;
        s_curi[i] = 0;
        s_pos[i] = -1;
        s_skey[i] = -1;
    }
    for (int i = t; i < H; i += W) {
        h_key[i] = HASH_EMPTY;
        h_row[i] = 0x7fffffff;
    }
    gsync(G);

    // ---- 1. node rows
    const int rb = N <= 256 ? 8 : 10;  // row bits of the packed (key, row) words
    unsigned st = 0u;
    int key = -1, act = 0, agg = 0;
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
            if (key_ok) hash_insert(h_key, h_row, H, key, t);
        }
        s_key[t] = key;
        // (key, row) in one word: rows take rb bits, keys the rest (always
        // room when rows fit in 8 bits, keys being below 2^24; with 10 row
        // bits a key of 2^22 or more marks the genome as wide)
        if (key >= 0 && rb == 10 && key >= (1 << 22)) G.sh[SH_WIDE] = 1;
        s_stack[t] = key >= 0 ? (int)(((unsigned)key << rb) | (unsigned)t) : -1;
    }
    gsync(G);

    // ---- 2. stable key rank (by key, then row), duplicate keys,
    // input/output presence
    int rank = -1;
    const bool packed = G.sh[SH_WIDE] == 0;
    if (key >= 0) {
        if (packed) {
            // rank = number of (key, row) words below this row's (the words
            // are distinct; absent and malformed rows hold the largest)
            const unsigned mine = ((unsigned)key << rb) | (unsigned)t;
            const unsigned *comp = reinterpret_cast<const unsigned *>(s_stack);
            int less = 0;
#pragma unroll 8
            for (int q = 0; q < N; ++q) less += comp[q] < mine;
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

    // ---- 3. connection rows (the prefetched ones first)
    auto connection = [&](int c, const float4 row) {
        int src = -1, dst = -1;
        if (!isnan(row.x) && row.z != 0.0f) {
            if (row.z != 1.0f) {
                st |= NEAT_ST_BAD_VALUE;
            } else {
                const int s = find_row(row.x, h_key, h_row, H);
                const int d = find_row(row.y, h_key, h_row, H);
                if (s < 0 || d < 0) {
                    st |= NEAT_ST_BAD_REF;
                } else {
                    if (s_key[d] < I) st |= NEAT_ST_INTO_INPUT;
                    if (s == d && !a.recurrent) st |= NEAT_ST_CYCLE;
                    src = s;
                    dst = d;
                    atomicAdd(&s_indeg[d], 1);
                    atomicAdd(&s_curo[s], 1);
                }
            }
        }
        e_sd[c] = src < 0 ? -1 : (src | (dst << 16));
    };
#pragma unroll
    for (int k = 0; k < CPRE; ++k)
        if (t + k * W < C) connection(t + k * W, cpre[k]);
    for (int c = t + CPRE * W; c < C; c += W) connection(c, conns4[c]);
    gsync(G);

    // ---- 4. adjacency lists (counting sort by destination and by source)
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
    for (int c = t; c < C; c += W) {
        const int sd = e_sd[c];
        const int s = src_of(sd);
        if (s < 0) continue;
        const int d = dst_of(sd);
        in_list[s_inoff[d] + atomicAdd(&s_curi[d], 1)] = (uint16_t)c;
        out_list[s_outoff[s] + atomicAdd(&s_curo[s], 1)] = d;
    }
    gsync(G);
    for (int c = t; c < C; c += W) {
        const int sd = e_sd[c];
        const int s = src_of(sd);
        if (s < 0) continue;
        const int d = dst_of(sd);
        for (int k = s_inoff[d]; k < s_inoff[d + 1]; ++k) {
            const int c2 = in_list[k];
            if (c2 != c && src_of(e_sd[c2]) == s) st |= NEAT_ST_DUP_EDGE;
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
        const int lane = G.lane, wave = G.wave, nw = G.nw;
        bool emitted = false;
        int base = 0;
        for (;;) {
            const bool ready = my_row >= 0 && !emitted && s_indeg[my_row] == 0;
            const unsigned long long m = __ballot(ready);
            if (lane == 0) G.sh[SH_WAVE + wave] = __popcll(m);
            gsync(G);
            int wbase = 0, total = 0;
            for (int w = 0; w < nw; ++w) {
                const int c = G.sh[SH_WAVE + w];
                wbase += (w < wave) ? c : 0;
                total += c;
            }
            if (total == 0) break;  // uniform across the block
            if (ready) {
                s_pos[my_row] = base + wbase + mbcnt(m);
                my_level = n_levels;
                emitted = true;
                for (int k = s_outoff[my_row]; k < s_outoff[my_row + 1]; ++k)
                    atomicSub(&s_indeg[out_list[k]], 1);
            }
            gsync(G);
            base += total;
            ++n_levels;
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
    // last reading position of every value (s_indeg is free after Kahn);
    // outputs are read after the last node
    int *s_last = s_indeg;
    if (t < N && s_key[t] != -1) {
        int last = s_pos[t];
        for (int k = s_outoff[t]; k < s_outoff[t + 1]; ++k) last = max(last, s_pos[out_list[k]]);
        if (s_key[t] >= I && s_key[t] < I + O) last = nvalid;
        s_last[t] = last;
    }
    gsync(G);
    if (max_class(N) == CLS_R64 || a.recurrent) {
        // every genome fits the 64-slot class, or every value stays live
        // from one sweep to the next: slot = position
        if (t < nvalid) s_slot[s_curi[t]] = t;
        if (t == 0) s_used = nvalid;
    } else {
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
    // source key of every in-edge (the out lists are no longer needed), for
    // the per-node scans below
    int *in_key = out_list;
    for (int k = t; k < s_inoff[N]; k += W) in_key[k] = s_key[src_of(e_sd[in_list[k]])];
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
        prog[HDR_NREAL] = s_inoff[N];
        prog[HDR_SLOTS] = used;
    }
    // output slots: rank I + j holds key I + j
    if (t < O) prog[out_off() + t] = s_slot[s_srow[I + t]];
    // owner of a computed row: in-degree, first in-edge (min source key),
    // pairs after padding to an even count, overflow edges beyond the record
    const bool computed = t < N && s_key[t] >= 0 && s_pos[t] >= I;
    int deg = 0, first = -1;
    if (computed) {
        int kmin = 0x7fffffff;
        for (int k = s_inoff[t]; k < s_inoff[t + 1]; ++k) {
            const int ks = in_key[k];
            ++deg;
            if (ks < kmin) kmin = ks, first = in_list[k];
        }
    }
    const int pairs = (deg + 1) >> 1;
    const int over = pairs > REC_INLINE_PAIRS ? 2 * (pairs - REC_INLINE_PAIRS) : 0;
    gsync(G);
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
        // neutral padding edge when the in-degree is odd
        if (deg & 1) {
            int slot;
            float w = 1.0f;
            if (agg == AGG_SUM || agg == AGG_MEAN) {
                slot = zs;
            } else if (agg == AGG_PRODUCT) {
                slot = zs + 1;
            } else {  // max / min: the first edge again (min stores -w)
                slot = s_slot[src_of(e_sd[first])];
                w = conns[(size_t)first * 4 + 3];
                if (agg == AGG_MIN) w = -w;
            }
            const int widx = deg < 2 * REC_INLINE_PAIRS ? r0 + REC_PAIRS + 2 * deg
                                                         : eoff + EDGE_WORDS * (ob + deg - 2 * REC_INLINE_PAIRS);
            prog[widx] = slot;
            progf[widx + 1] = w;
        }
    }
    // aggregation code and overflow begin by row for the edge writers
    int *s_agg = s_deg;
    if (computed) s_agg[t] = agg;
    gsync(G);
    // real edges: index j = number of in-edges of the destination with a
    // smaller source key (keys are unique here); j < 6 in the record, the
    // rest in the overflow array.  The thread that read a connection row
    // writes its edge (weights of the prefetched rows are still in registers)
    auto edge = [&](int c, float w) {
        const int sd = e_sd[c];
        const int s = src_of(sd);
        if (s < 0) return;
        const int d = dst_of(sd);
        const int ks = s_key[s];
        int j = 0;
        for (int k = s_inoff[d]; k < s_inoff[d + 1]; ++k) j += (in_key[k] < ks);
        const int rd = rec_off(O) + REC_WORDS * (s_pos[d] - I);
        const int widx = j < 2 * REC_INLINE_PAIRS ? rd + REC_PAIRS + 2 * j
                                                   : eoff + EDGE_WORDS * (s_curo[d] + j - 2 * REC_INLINE_PAIRS);
        // min is stored as max over negated weights (negation is exact)
        prog[widx] = s_slot[s];
        progf[widx + 1] = s_agg[d] == AGG_MIN ? -w : w;
    };
#pragma unroll
    for (int k = 0; k < CPRE; ++k)
        if (t + k * W < C) edge(t + k * W, cpre[k].w);
    for (int c = t + CPRE * W; c < C; c += W) edge(c, conns[(size_t)c * 4 + 3]);
}

// Genome g by the workgroup (ONE: a single wave, N_max <= 64).
template <bool ONE>
__device__ __forceinline__ void topo_group(const TopoItem &a, long long g) {
    extern __shared__ int smem[];
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
    // 32-bit: 7 N node words, 2 C connection words, the key table (2 H);
    // 16-bit: 6 N + 2 node entries, C connection entries
    return sizeof(int) * ((size_t)SH_WORDS + (size_t)7 * N + (size_t)2 * C +
                          2 * (size_t)hash_size(N)) +
           sizeof(int16_t) * ((size_t)6 * N + 2 + (size_t)C);
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
