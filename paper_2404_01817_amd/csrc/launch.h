// launch.h -- host-side launchers of the kernels (internal to the library).
// Each returns a hipError_t from the launch; arguments are checked by the
// C-ABI layer before any launcher is called.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace neat {

// Dynamic LDS bytes the transformation kernel needs for one genome.
size_t topo_lds_bytes(int N, int C);
// Threads per block of the transformation kernel (one thread per node row).
int topo_block_threads(int N);

hipError_t launch_topo(int P, int N, int C, int I, int O, const float *nodes,
                       const float *conns, int32_t *order, int32_t *level,
                       uint32_t *status, int32_t *prog, hipStream_t stream);

// Forward variants (value store of the lane-per-sample mapping).
constexpr int FWD_AUTO = 0;
constexpr int FWD_REG = 1;  // value vector in VGPRs, node loop in assembly (N_max <= 62)
constexpr int FWD_LDS = 2;  // value vector in LDS rows (any N_max)

int forward_default_variant(int N);
// LDS bytes of one forward launch (all waves of a workgroup).
size_t forward_launch_lds_bytes(int P, int B, int N, int I, int variant, bool grid);

// inputs: per-genome stride in floats (0 = shared); B vectors per genome.
// grid: CPPN queries generated in the kernel (I == 5, side, first).
hipError_t launch_forward(int P, int N, int C, int I, int O, const int32_t *prog,
                          const float *inputs, int64_t gstride, int B, float *outputs,
                          int variant, bool grid, int side, int64_t first, hipStream_t stream);

}  // namespace neat
