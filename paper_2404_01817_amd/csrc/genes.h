// genes.h -- launch interfaces of the gene-level population operators in
// genes.hip: compatibility distance and crossover.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace neat {

// out [P][Q] = distance of genome p (nodes/conns [P][N][5] / [P][C][4]) to
// representative q (rnodes/rconns [Q][N][5] / [Q][C][4]); hn, hc are set by
// distance_launch (hash table sizes).
struct DistLaunch {
    const float *nodes;
    const float *conns;
    const float *rnodes;
    const float *rconns;
    float *out;
    int P, Q, N, C;
    float cd, ch;
    int hn, hc;
};

size_t distance_lds_bytes(int N, int C);
// LDS of the two gene hash tables alone (what crossover uses)
size_t gene_tables_lds_bytes(int N, int C);
hipError_t distance_launch(DistLaunch L, hipStream_t stream);

// children cn/cc [Pc][N][5] / [Pc][C][4] of the parent pairs [Pc][2] of
// nodes/conns [P][N][5] / [P][C][4], with uniform numbers rn [Pc][N], rc
// [Pc][C] per first-parent row; a pair with an index outside [0, P) gives
// an all-NaN child; hn, hc as for DistLaunch (words: one wave's LDS tables
// in 8-byte words; vec: conns is 16-byte aligned).  Both are set by
// crossover_launch.
struct CrossLaunch {
    const float *nodes;
    const float *conns;
    const int32_t *pairs;
    const float *rn;
    const float *rc;
    float *cn;
    float *cc;
    int Pc, P, N, C;
    int hn, hc;
    int words, vec;
};

hipError_t crossover_launch(CrossLaunch L, hipStream_t stream);

// One tensorized edit (layout of neat_edit in neat.h).
struct EditRec {
    int32_t genome, op, row, column;
    float v[5];
};

// edits [n] sorted by genome (application order within a genome) applied
// in place to nodes/conns [P][N][5] / [P][C][4]; applied [n] written.
struct EditLaunch {
    float *nodes;
    float *conns;
    const EditRec *edits;
    int32_t *applied;
    int n, P, N, C;
};

hipError_t edit_launch(EditLaunch L, hipStream_t stream);

}  // namespace neat
