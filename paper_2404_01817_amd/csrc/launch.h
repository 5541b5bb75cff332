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

// Dynamic LDS bytes of the lane-per-sample forward for N node positions.
size_t forward_lds_bytes(int N);

// inputs: per-genome stride in floats (0 = shared); B vectors per genome.
hipError_t launch_forward(int P, int N, int C, int I, int O, const int32_t *prog,
                          const float *inputs, int64_t gstride, int B, float *outputs,
                          hipStream_t stream);

// CPPN grid queries generated in the kernel (I == 5).
hipError_t launch_forward_grid(int P, int N, int C, int I, int O, const int32_t *prog,
                               int side, int64_t first, int Q, float *outputs,
                               hipStream_t stream);

// Register-resident forward (N_max <= 64): LDS bytes per wave, launchers.
size_t forward_reg_lds_bytes(int I);
hipError_t launch_forward_reg(int P, int N, int C, int I, int O, const int32_t *prog,
                              const float *inputs, int64_t gstride, int B, float *outputs,
                              hipStream_t stream);
hipError_t launch_forward_reg_grid(int P, int N, int C, int I, int O, const int32_t *prog,
                                   int side, int64_t first, int Q, float *outputs,
                                   hipStream_t stream);

// Largest N_max the register-resident forward handles.
constexpr int REG_MAX_NODES = 64;

}  // namespace neat
