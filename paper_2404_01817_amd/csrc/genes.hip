// genes.hip -- gene-level population operators: NEAT's compatibility
// distance and crossover.
//
// Compatibility distance of every genome of a population to every species
// representative (speciation divides the
// population by distances between networks: the NEAT algorithm of the
// paper's appendix; Appendix A names the disjoint and homologous
// coefficients).  Per pair (genome A, representative B):
//   genes: node rows with a key, connection rows with an in key;
//   an A gene is homologous when B has a gene with the same key (nodes) or
//   the same (in, out) keys (connections), its partner being the first
//   such B row; node distance |bias - bias'| + |resp - resp'| + [act !=
//   act'] + [agg != agg'], connection distance |w - w'| + [enabled !=
//   enabled'];
//   per kind (cd (|A| + |B| - 2 h) + ch sum) / max(|A|, |B|), 0 when both
//   are empty; the distance is the node part plus the connection part.
//
// A workgroup takes eight genomes (two per wave) and loops over the
// representatives: B's genes go into LDS hash tables (key bits -> first
// row, by atomic min), built once for the eight, then every lane probes the
// tables with its A genes and each wave sums counts and attribute
// distances.  Keys are compared as floats: -0 is folded into +0
// before hashing, and a connection whose out key is NaN never matches.
#include <hip/hip_runtime.h>

#include "genes.h"

namespace neat {
namespace {

constexpr int WAVE = 64;
constexpr unsigned long long EMPTY64 = ~0ull;

__device__ __forceinline__ unsigned key_bits(float k) {
    return __float_as_uint(k == 0.0f ? 0.0f : k);  // -0 -> +0
}

__device__ __forceinline__ unsigned mix(unsigned long long x, int H) {
    x ^= x >> 29;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 32;
    return (unsigned)x & (unsigned)(H - 1);
}

__device__ __forceinline__ int wave_sum(int v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Wave sums on the DPP lane network (register-to-register, no LDS round
// trips): lanes pair up within rows of 16 (swap neighbours, swap pairs,
// mirror each half row, mirror the row), after which every lane of a row
// holds the row's sum; the four row sums are read out into scalars.  Called
// with the whole wave active.
constexpr int DPP_SWAP1 = 0xB1;      // quad_perm [1, 0, 3, 2]
constexpr int DPP_SWAP2 = 0x4E;      // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;

__device__ __forceinline__ int row_sums(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, DPP_SWAP1, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, DPP_SWAP2, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, DPP_HALF_MIRROR, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, DPP_MIRROR, 0xF, 0xF, false);
    return v;
}
__device__ __forceinline__ float row_sums(float v) {
#define NEAT_DPP_ADD(CTRL) \
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false))
    NEAT_DPP_ADD(DPP_SWAP1);
    NEAT_DPP_ADD(DPP_SWAP2);
    NEAT_DPP_ADD(DPP_HALF_MIRROR);
    NEAT_DPP_ADD(DPP_MIRROR);
#undef NEAT_DPP_ADD
    return v;
}
__device__ __forceinline__ int wave_total(int v) {
    v = row_sums(v);
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
           __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}
__device__ __forceinline__ float wave_total(float v) {
    v = row_sums(v);
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}

// insert key -> row (keeping the smallest row for a key)
__device__ __forceinline__ void insert(unsigned long long *hk, int *hr, int H,
                                       unsigned long long key, int row) {
    unsigned s = mix(key, H);
    for (;;) {
        const unsigned long long prev = atomicCAS(hk + s, EMPTY64, key);
        if (prev == EMPTY64 || prev == key) {
            atomicMin(hr + s, row);
            return;
        }
        s = (s + 1) & (unsigned)(H - 1);
    }
}

__device__ __forceinline__ int lookup_from(const unsigned long long *hk, const int *hr, int H,
                                           unsigned long long key, unsigned s) {
    for (;;) {
        const unsigned long long k = hk[s];
        if (k == key) return hr[s];
        if (k == EMPTY64) return -1;
        s = (s + 1) & (unsigned)(H - 1);
    }
}

__device__ __forceinline__ int lookup(const unsigned long long *hk, const int *hr, int H,
                                      unsigned long long key) {
    unsigned s = mix(key, H);
    for (;;) {
        const unsigned long long k = hk[s];
        if (k == key) return hr[s];
        if (k == EMPTY64) return -1;
        s = (s + 1) & (unsigned)(H - 1);
    }
}

// DIST_WAVES waves per workgroup, DIST_PER_WAVE genomes per wave: a
// representative's tables are built once for DIST_WAVES * DIST_PER_WAVE
// genomes.
constexpr int DIST_WAVES = 4, DIST_PER_WAVE = 2;
constexpr int DIST_GENOMES = DIST_WAVES * DIST_PER_WAVE;

// SMALL (N_max <= 64, C_max <= 256): every lane keeps its genes' keys,
// attributes and first hash slots in registers for the whole loop over the
// representatives (one node row and up to four connection rows per genome),
// B's rows are copied into LDS beside the tables (a partner's attributes
// are an LDS read away, not a cache round trip), and the per-pair sums run
// on the DPP lane network.
constexpr int SMALL_CONN_ROWS = 4;

template <bool SMALL>
__global__ __launch_bounds__(WAVE *DIST_WAVES) void distance_kernel(DistLaunch L) {
    extern __shared__ unsigned long long dsm[];
    const int N = L.N, C = L.C, HN = L.hn, HC = L.hc;
    unsigned long long *nk = dsm;            // node table: keys [HN]
    unsigned long long *ck = nk + HN;        // connection table: keys [HC]
    int *nr = (int *)(ck + HC);              // rows [HN]
    int *cr = nr + HN;                       // rows [HC]
    int *bcount = cr + HC;                   // B's node and connection genes
    float *bn_s = (float *)(bcount + 2);     // SMALL: B's rows [N][5], [C][4]
    float *bc_s = bn_s + (SMALL ? N * 5 : 0);
    const int t = (int)threadIdx.x, lane = t & (WAVE - 1), wave = t / WAVE;
    const int T = WAVE * DIST_WAVES;

    // this wave's genomes and their gene counts (once)
    long long gs[DIST_PER_WAVE];
    int na[DIST_PER_WAVE], ca[DIST_PER_WAVE];
    // SMALL: the lane's genes (node row lane, connection rows lane + 64 m)
    float xn[DIST_PER_WAVE][5];
    unsigned xns[DIST_PER_WAVE];
    float xc[DIST_PER_WAVE][SMALL_CONN_ROWS][4];
    unsigned xcs[DIST_PER_WAVE][SMALL_CONN_ROWS];
#pragma unroll
    for (int i = 0; i < DIST_PER_WAVE; ++i) {
        gs[i] = (long long)blockIdx.x * DIST_GENOMES + wave * DIST_PER_WAVE + i;
        int a = 0, c = 0;
        if (gs[i] < L.P) {
            const float *An = L.nodes + (size_t)gs[i] * N * 5;
            const float *Ac = L.conns + (size_t)gs[i] * C * 4;
            for (int r = lane; r < N; r += WAVE) a += !isnan(An[(size_t)r * 5]);
            for (int r = lane; r < C; r += WAVE) c += !isnan(Ac[(size_t)r * 4]);
            if constexpr (SMALL) {
                const bool in = lane < N;
#pragma unroll
                for (int f = 0; f < 5; ++f)
                    xn[i][f] = in ? An[(size_t)lane * 5 + f] : __builtin_nanf("");
                xns[i] = mix(key_bits(xn[i][0]), HN);
#pragma unroll
                for (int m = 0; m < SMALL_CONN_ROWS; ++m) {
                    const int r = lane + WAVE * m;
#pragma unroll
                    for (int f = 0; f < 4; ++f)
                        xc[i][m][f] = r < C ? Ac[(size_t)r * 4 + f] : __builtin_nanf("");
                    xcs[i][m] = mix(((unsigned long long)key_bits(xc[i][m][0]) << 32) |
                                        key_bits(xc[i][m][1]),
                                    HC);
                }
            }
        }
        na[i] = wave_sum(a);
        ca[i] = wave_sum(c);
    }

    for (int q = 0; q < L.Q; ++q) {
        const float *Bn = L.rnodes + (size_t)q * N * 5;
        const float *Bc = L.rconns + (size_t)q * C * 4;
        for (int s = t; s < HN; s += T) nk[s] = EMPTY64, nr[s] = 0x7fffffff;
        for (int s = t; s < HC; s += T) ck[s] = EMPTY64, cr[s] = 0x7fffffff;
        if (t < 2) bcount[t] = 0;
        __syncthreads();
        int nb = 0, cb = 0;
        for (int r = t; r < N; r += T) {
            const float k = Bn[(size_t)r * 5];
            if constexpr (SMALL) {
#pragma unroll
                for (int f = 0; f < 5; ++f) bn_s[r * 5 + f] = Bn[(size_t)r * 5 + f];
            }
            if (isnan(k)) continue;
            ++nb;
            insert(nk, nr, HN, key_bits(k), r);
        }
        for (int r = t; r < C; r += T) {
            const float ki = Bc[(size_t)r * 4], ko = Bc[(size_t)r * 4 + 1];
            if constexpr (SMALL) {
#pragma unroll
                for (int f = 0; f < 4; ++f) bc_s[r * 4 + f] = Bc[(size_t)r * 4 + f];
            }
            if (isnan(ki)) continue;
            ++cb;
            if (isnan(ko)) continue;  // can never match
            insert(ck, cr, HC, ((unsigned long long)key_bits(ki) << 32) | key_bits(ko), r);
        }
        nb = wave_sum(nb);
        cb = wave_sum(cb);
        if (lane == 0) {
            atomicAdd(bcount, nb);
            atomicAdd(bcount + 1, cb);
        }
        __syncthreads();
        nb = bcount[0];
        cb = bcount[1];
#pragma unroll
        for (int i = 0; i < DIST_PER_WAVE; ++i) {
            if (gs[i] >= L.P) continue;  // uniform across the wave
            const float *An = L.nodes + (size_t)gs[i] * N * 5;
            const float *Ac = L.conns + (size_t)gs[i] * C * 4;
            int hn = 0, hc = 0;
            float sn = 0.0f, sc = 0.0f;
            if constexpr (SMALL) {
                const float *x = xn[i];
                if (!isnan(x[0])) {
                    const int j = lookup_from(nk, nr, HN, key_bits(x[0]), xns[i]);
                    if (j >= 0) {
                        const float *y = bn_s + j * 5;
                        ++hn;
                        sn += fabsf(x[1] - y[1]) + fabsf(x[2] - y[2]) + (float)(x[3] != y[3]) +
                              (float)(x[4] != y[4]);
                    }
                }
#pragma unroll
                for (int m = 0; m < SMALL_CONN_ROWS; ++m) {
                    const float *xm = xc[i][m];
                    if (isnan(xm[0]) || isnan(xm[1])) continue;
                    const int j = lookup_from(
                        ck, cr, HC, ((unsigned long long)key_bits(xm[0]) << 32) | key_bits(xm[1]),
                        xcs[i][m]);
                    if (j < 0) continue;
                    const float *y = bc_s + j * 4;
                    ++hc;
                    sc += fabsf(xm[3] - y[3]) + (float)(xm[2] != y[2]);
                }
            } else {
                for (int r = lane; r < N; r += WAVE) {
                    const float *x = An + (size_t)r * 5;
                    if (isnan(x[0])) continue;
                    const int j = lookup(nk, nr, HN, key_bits(x[0]));
                    if (j < 0) continue;
                    const float *y = Bn + (size_t)j * 5;
                    ++hn;
                    sn += fabsf(x[1] - y[1]) + fabsf(x[2] - y[2]) + (float)(x[3] != y[3]) +
                          (float)(x[4] != y[4]);
                }
                for (int r = lane; r < C; r += WAVE) {
                    const float *x = Ac + (size_t)r * 4;
                    if (isnan(x[0]) || isnan(x[1])) continue;
                    const int j = lookup(ck, cr, HC,
                                         ((unsigned long long)key_bits(x[0]) << 32) | key_bits(x[1]));
                    if (j < 0) continue;
                    const float *y = Bc + (size_t)j * 4;
                    ++hc;
                    sc += fabsf(x[3] - y[3]) + (float)(x[2] != y[2]);
                }
            }
            hn = wave_total(hn);
            hc = wave_total(hc);
            sn = wave_total(sn);
            sc = wave_total(sc);
            if (lane == 0) {
                const int mn = max(na[i], nb), mc = max(ca[i], cb);
                const float dn =
                    mn ? (L.cd * (float)(na[i] + nb - 2 * hn) + L.ch * sn) / (float)mn : 0.0f;
                const float dc =
                    mc ? (L.cd * (float)(ca[i] + cb - 2 * hc) + L.ch * sc) / (float)mc : 0.0f;
                L.out[(size_t)gs[i] * L.Q + q] = dn + dc;
            }
        }
        __syncthreads();  // the tables are cleared for the next representative
    }
}

// Crossover (Section 3.2: the genetic operators become row and attribute
// writes of the tensors; the gene alignment is NEAT's): the child of
// (p1, p2) keeps p1's rows; a p1 gene homologous in p2 (same node key, or
// same (in, out) keys; partner = p2's first such row) takes the partner's
// non-key columns when its uniform number is below 0.5.  One wave per
// child, four children per workgroup while their tables fit in 64 KB of LDS
// (else one): p2's genes go into the wave's own LDS hash tables, every lane
// writes its p1 rows (connection rows as 16-byte loads and stores when the
// tensor is 16-byte aligned).
constexpr int CROSS_WAVES = 4;

__global__ __launch_bounds__(WAVE *CROSS_WAVES) void crossover_kernel(CrossLaunch L) {
    extern __shared__ unsigned long long dsm[];
    const int N = L.N, C = L.C, HN = L.hn, HC = L.hc;
    const int lane = (int)threadIdx.x & (WAVE - 1), wave = (int)threadIdx.x / WAVE;
    const int waves = (int)blockDim.x / WAVE;
    unsigned long long *nk = dsm + (size_t)wave * L.words;  // this wave's tables
    unsigned long long *ck = nk + HN;
    int *nr = (int *)(ck + HC);
    int *cr = nr + HN;
    const long long k = (long long)blockIdx.x * waves + wave;
    const bool live = k < L.Pc;
    int a = 0, b = 0;
    if (live) a = L.pairs[2 * k], b = L.pairs[2 * k + 1];
    // uniform across the wave; every wave reaches both barriers
    const bool ok = live && a >= 0 && a < L.P && b >= 0 && b < L.P;
    if (live && !ok) {
        for (int e = lane; e < N * 5; e += WAVE) L.cn[(size_t)k * N * 5 + e] = __builtin_nanf("");
        for (int e = lane; e < C * 4; e += WAVE) L.cc[(size_t)k * C * 4 + e] = __builtin_nanf("");
    }
    if (!ok) a = b = 0;
    const float *An = L.nodes + (size_t)a * N * 5, *Ac = L.conns + (size_t)a * C * 4;
    const float *Bn = L.nodes + (size_t)b * N * 5, *Bc = L.conns + (size_t)b * C * 4;
    if (ok) {
        for (int s = lane; s < HN; s += WAVE) nk[s] = EMPTY64, nr[s] = 0x7fffffff;
        for (int s = lane; s < HC; s += WAVE) ck[s] = EMPTY64, cr[s] = 0x7fffffff;
    }
    __syncthreads();
    if (ok) {
        for (int r = lane; r < N; r += WAVE) {
            const float key = Bn[(size_t)r * 5];
            if (!isnan(key)) insert(nk, nr, HN, key_bits(key), r);
        }
        for (int r = lane; r < C; r += WAVE) {
            const float ki = Bc[(size_t)r * 4], ko = Bc[(size_t)r * 4 + 1];
            if (!isnan(ki) && !isnan(ko))
                insert(ck, cr, HC, ((unsigned long long)key_bits(ki) << 32) | key_bits(ko), r);
        }
    }
    __syncthreads();
    if (!ok) return;
    float *On = L.cn + (size_t)k * N * 5, *Oc = L.cc + (size_t)k * C * 4;
    for (int r = lane; r < N; r += WAVE) {
        const float *x = An + (size_t)r * 5;
        const float *src = x;
        if (!isnan(x[0]) && L.rn[(size_t)k * N + r] < 0.5f) {
            const int j = lookup(nk, nr, HN, key_bits(x[0]));
            if (j >= 0) src = Bn + (size_t)j * 5;
        }
        float *o = On + (size_t)r * 5;
        o[0] = x[0];
#pragma unroll
        for (int c = 1; c < 5; ++c) o[c] = src[c];
    }
    for (int r = lane; r < C; r += WAVE) {
        const float *x = Ac + (size_t)r * 4;
        float4 v;
        if (L.vec) v = *reinterpret_cast<const float4 *>(x);
        else v = make_float4(x[0], x[1], x[2], x[3]);
        if (!isnan(v.x) && !isnan(v.y) && L.rc[(size_t)k * C + r] < 0.5f) {
            const int j = lookup(ck, cr, HC,
                                 ((unsigned long long)key_bits(v.x) << 32) | key_bits(v.y));
            if (j >= 0) {
                const float *y = Bc + (size_t)j * 4;
                if (L.vec) {
                    const float2 w = *reinterpret_cast<const float2 *>(y + 2);
                    v.z = w.x, v.w = w.y;
                } else {
                    v.z = y[2], v.w = y[3];
                }
            }
        }
        *reinterpret_cast<float4 *>(Oc + (size_t)r * 4) = v;
    }
}

// Tensorized edits (Section 3.2): additions at the first NaN row, NaN
// removals, attribute writes; a genome's edits in their order, genomes in
// parallel.  One wave per genome finds its edits by a 64-way search over
// the genome-sorted list, loads up to 64 records at once (one per lane, read
// out in order) and keeps its rows' key columns in LDS (the first-NaN
// searches read only keys).  Column c of a row is always written by lane c,
// so two edits of one address are ordered by that lane's program order.
__global__ __launch_bounds__(256) void edit_clear_kernel(int32_t *applied, int n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) applied[i] = 0;
}

// First index whose genome is >= g in edits sorted by genome: each step
// lets every lane probe one of 64 evenly spaced positions and narrows the
// range to the gap the ballot points at (about three steps for 10^5 edits,
// against seventeen dependent loads of a binary search).  Every probe
// stays inside [0, n) whatever the order of the edits.
__device__ __forceinline__ int edits_lower_bound(const EditRec *e, int n, int g, int lane) {
    int lo = 0, hi = n;  // the answer lies in [lo, hi]
    while (hi - lo > WAVE) {
        const int step = (hi - lo + WAVE - 1) / WAVE;
        const long long p = lo + (long long)(lane + 1) * step - 1;
        const bool less = p < hi && e[p].genome < g;
        const int cnt = __popcll(__ballot(less));
        const long long top = lo + (long long)(cnt + 1) * step - 1;  // first probe >= g
        if (top < hi) hi = (int)top;
        lo += cnt * step;
    }
    const bool less = lo + lane < hi && e[lo + lane].genome < g;
    return lo + __popcll(__ballot(less));
}

// Edits of genome g from lo on: the run of records whose genome is g,
// counted 64 at a time.
__device__ __forceinline__ int edits_run_end(const EditRec *e, int n, int g, int lo, int lane) {
    int hi = lo;
    for (;;) {
        const bool same = hi + lane < n && e[hi + lane].genome == g;
        const int c = __popcll(__ballot(same));
        hi += c;
        if (c < WAVE) return hi;
    }
}

__device__ __forceinline__ int lane_int(int v, int i) { return __builtin_amdgcn_readlane(v, i); }
__device__ __forceinline__ float lane_float(float v, int i) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
}

__global__ __launch_bounds__(WAVE) void edit_kernel(EditLaunch L) {
    extern __shared__ float ks[];  // node keys [N], then connection in keys [C]
    const int g = (int)blockIdx.x, lane = (int)threadIdx.x;
    const int N = L.N, C = L.C;
    const int lo = edits_lower_bound(L.edits, L.n, g, lane);
    const int hi = edits_run_end(L.edits, L.n, g, lo, lane);
    if (lo >= hi) return;
    float *gn = L.nodes + (size_t)g * N * 5, *gc = L.conns + (size_t)g * C * 4;
    for (int r = lane; r < N; r += WAVE) ks[r] = gn[(size_t)r * 5];
    for (int r = lane; r < C; r += WAVE) ks[N + r] = gc[(size_t)r * 4];
    __syncthreads();
    for (int c0 = lo; c0 < hi; c0 += WAVE) {
        // up to 64 records at once, one per lane, then taken in order
        const int cn = min(WAVE, hi - c0);
        EditRec mine{};
        if (lane < cn) mine = L.edits[c0 + lane];
        for (int i = 0; i < cn; ++i) {
            const int e = c0 + i;
            EditRec d;
            d.genome = lane_int(mine.genome, i);
            d.op = lane_int(mine.op, i);
            d.row = lane_int(mine.row, i);
            d.column = lane_int(mine.column, i);
#pragma unroll
            for (int f = 0; f < 5; ++f) d.v[f] = lane_float(mine.v[f], i);
            // this lane's column value of an added row (selects, not an
            // indexed private array)
            const float vl = lane == 0 ? d.v[0] : lane == 1 ? d.v[1] : lane == 2 ? d.v[2]
                           : lane == 3 ? d.v[3] : d.v[4];
            const bool node = d.op == 0 || d.op == 1 || d.op == 4;
            float *t = node ? gn : gc;
            const int rows = node ? N : C, w = node ? 5 : 4, kb = node ? 0 : N;
            int row = -1;
            if (d.genome == g && (d.op == 0 || d.op == 2)) {
                // first NaN key, 64 rows at a time
                for (int r0 = 0; r0 < rows && row < 0; r0 += WAVE) {
                    const bool nan_row = r0 + lane < rows && isnan(ks[kb + r0 + lane]);
                    const unsigned long long m = __ballot(nan_row);
                    if (m) row = r0 + __ffsll((long long)m) - 1;
                }
                if (row >= 0) {
                    if (lane < w) t[(size_t)row * w + lane] = vl;
                    if (lane == 0) ks[kb + row] = d.v[0];
                }
            } else if (d.genome == g && (d.op == 1 || d.op == 3)) {
                if (d.row >= 0 && d.row < rows) {
                    row = d.row;
                    if (lane < w) t[(size_t)row * w + lane] = __builtin_nanf("");
                    if (lane == 0) ks[kb + row] = __builtin_nanf("");
                }
            } else if (d.genome == g && (d.op == 4 || d.op == 5)) {
                const bool ok = d.row >= 0 && d.row < rows &&
                                (node ? (d.column >= 1 && d.column <= 4)
                                      : (d.column >= 2 && d.column <= 3));
                if (ok) {
                    row = d.row;
                    if (lane == d.column) t[(size_t)row * w + lane] = d.v[0];
                }
            }
            if (lane == 0 && row >= 0) L.applied[e] = 1;
            __syncthreads();  // key updates visible to the next edit's search
        }
    }
}

int pow2_at_least(int x) {
    int h = 64;
    while (h < x) h <<= 1;
    return h;
}

}  // namespace

// the two hash tables and two counters
size_t gene_tables_lds_bytes(int N, int C) {
    const int hn = pow2_at_least(2 * N), hc = pow2_at_least(2 * C);
    return (size_t)(hn + hc) * (sizeof(unsigned long long) + sizeof(int)) + 2 * sizeof(int);
}

static bool distance_small(int N, int C) { return N <= WAVE && C <= WAVE * SMALL_CONN_ROWS; }

size_t distance_lds_bytes(int N, int C) {
    return gene_tables_lds_bytes(N, C) +
           (distance_small(N, C) ? sizeof(float) * (size_t)(5 * N + 4 * C) : 0);
}

hipError_t crossover_launch(CrossLaunch L, hipStream_t stream) {
    L.hn = pow2_at_least(2 * L.N);
    L.hc = pow2_at_least(2 * L.C);
    L.words = L.hn + L.hc + (L.hn + L.hc) / 2;  // keys, then rows (hn + hc even)
    L.vec = ((uintptr_t)L.conns % 16) == 0;
    if (L.Pc == 0) return hipSuccess;
    // four children per workgroup while their tables stay small (≤ 64 KB)
    const size_t wave_bytes = sizeof(unsigned long long) * (size_t)L.words;
    const int waves = 4 * wave_bytes <= 65536 ? CROSS_WAVES : 1;
    hipLaunchKernelGGL(crossover_kernel, dim3((unsigned)((L.Pc + waves - 1) / waves)),
                       dim3(WAVE * waves), waves * wave_bytes, stream, L);
    return hipGetLastError();
}

hipError_t edit_launch(EditLaunch L, hipStream_t stream) {
    if (L.n == 0) return hipSuccess;
    hipLaunchKernelGGL(edit_clear_kernel, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0,
                       stream, L.applied, L.n);
    if (L.P == 0) return hipGetLastError();
    hipLaunchKernelGGL(edit_kernel, dim3((unsigned)L.P), dim3(WAVE),
                       sizeof(float) * (size_t)(L.N + L.C), stream, L);
    return hipGetLastError();
}

hipError_t distance_launch(DistLaunch L, hipStream_t stream) {
    L.hn = pow2_at_least(2 * L.N);
    L.hc = pow2_at_least(2 * L.C);
    if (L.P == 0 || L.Q == 0) return hipSuccess;
    const dim3 grid((unsigned)((L.P + DIST_GENOMES - 1) / DIST_GENOMES)), block(WAVE * DIST_WAVES);
    if (distance_small(L.N, L.C))
        hipLaunchKernelGGL(distance_kernel<true>, grid, block, distance_lds_bytes(L.N, L.C), stream,
                           L);
    else
        hipLaunchKernelGGL(distance_kernel<false>, grid, block, distance_lds_bytes(L.N, L.C),
                           stream, L);
    return hipGetLastError();
}

}  // namespace neat
