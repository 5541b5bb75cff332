// abi.h -- helpers shared by the C-ABI entry points (internal): error
// reporting into neat_last_error(), argument checks, device limits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "launch.h"
#include "neat.h"

namespace neat {
namespace abi {

// Record a formatted message for neat_last_error() and return code.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
// NEAT_E_HIP with the runtime's message.
int hip_fail(hipError_t e, const char *what);
// Largest dynamic LDS allocation of one workgroup on the current device.
size_t max_lds_bytes();
bool aligned(const void *p, size_t a);
// NEAT_OK or NEAT_E_INVALID (message set) for a population's dims.
int check_dims(const neat_dims *d);
// Arguments of the transformation of one population (dims already checked).
int check_topo_args(const neat_dims *d, const float *nodes, const float *conns,
                    const void *program);
// Arguments of the calculation of one population (dims already checked);
// grid: CPPN queries (B = Q) instead of inputs.
int check_forward_args(const neat_dims *d, const void *program, const float *inputs,
                       int64_t stride, int32_t B, float *outputs, bool grid, int32_t side,
                       int64_t first);
FwdJob make_job(const neat_dims *d, const void *program, const float *inputs, int64_t stride,
                int32_t B, float *outputs, int32_t side, int64_t first);

}  // namespace abi
}  // namespace neat
