// program.h -- layout of the per-genome program that the transformation
// kernel writes and the calculation kernels read.
//
// The program replaces the paper's dense expanded-connection tensor C_exp
// (|N|max x |N|max cells, Section 3.3) by a compressed form in topological
// order: nodes are renumbered by their position p in the (level, key) order,
// so that the inputs, which have level 0 and the smallest keys, sit at
// positions 0..I-1, and every computed node p >= I has one record; its
// incoming edges follow each other in ascending source-key order, and the
// edges of consecutive records are consecutive.
//
// All fields are 32-bit words; one genome's program is prog_words() words,
// a multiple of 64 (256 bytes), so every genome starts on its own lines.
#pragma once

#include <cstddef>
#include <cstdint>

namespace neat {

// header words
constexpr int HDR_NVALID = 0;   // node positions in use (0 when rejected)
constexpr int HDR_NEDGES = 1;   // enabled edges
constexpr int HDR_STATUS = 2;   // status bit-mask (NEAT_ST_*)
constexpr int HDR_NLEVELS = 3;  // number of levels
constexpr int HDR_I = 4;
constexpr int HDR_O = 5;
constexpr int HDR_WORDS = 16;

// node record (4 words), record k describes position I + k:
//   w0 = in-degree | act << 16 | agg << 24
//   w1 = bias, w2 = response, w3 = 1 / in-degree (0 when the in-degree is 0)
constexpr int REC_WORDS = 4;
// edge record (2 words): source position, weight
constexpr int EDGE_WORDS = 2;

__host__ __device__ constexpr int round_up(int x, int m) { return (x + m - 1) / m * m; }

// output positions: O words (padded to 4)
__host__ __device__ constexpr int out_off() { return HDR_WORDS; }
__host__ __device__ constexpr int rec_off(int O) { return HDR_WORDS + round_up(O, 4); }
__host__ __device__ constexpr int edge_off(int N, int O) { return rec_off(O) + REC_WORDS * N; }
// first edge index of record k (N words)
__host__ __device__ constexpr int ebeg_off(int N, int C, int O) {
    return edge_off(N, O) + EDGE_WORDS * C;
}
// first position of level l, l = 0..n_levels (N + 1 words)
__host__ __device__ constexpr int lvl_off(int N, int C, int O) { return ebeg_off(N, C, O) + N; }
// 16 words of slack after the last array: the forward kernels read edge
// records 8 at a time (16 words) and may run past the last edge.
constexpr int PROG_SLACK = 16;
__host__ __device__ constexpr int prog_words(int N, int C, int O) {
    return round_up(lvl_off(N, C, O) + N + 1 + PROG_SLACK, 64);
}

__host__ __device__ inline uint32_t pack_rec(int deg, int act, int agg) {
    return (uint32_t)deg | ((uint32_t)act << 16) | ((uint32_t)agg << 24);
}

enum Act { ACT_IDENTITY = 0, ACT_TANH, ACT_SIGMOID, ACT_RELU, ACT_SIN, ACT_GAUSS, ACT_ABS };
enum Agg { AGG_SUM = 0, AGG_PRODUCT, AGG_MAX, AGG_MIN, AGG_MEAN };
constexpr int N_ACT = 7;
constexpr int N_AGG = 5;

}  // namespace neat
