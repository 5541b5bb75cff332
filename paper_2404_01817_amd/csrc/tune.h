// tune.h -- the forward autotuner's table (defined in api.hip): the variant
// measured fastest per bucket of (N_max, C_max, B), for calls that ask for
// NEAT_FWD_TUNED and for the batched path.
#pragma once

namespace neat {

// The variant recorded for the bucket of (N, C, B); FWD_AUTO when none is.
int tuned_variant(int N, int C, int B);

}  // namespace neat
