// tune.h -- the forward autotuner's table (defined in api.hip): the variant
// measured fastest per bucket of (N_max, C_max, B, input mode), for calls
// that ask for NEAT_FWD_TUNED, the batched path and the server.
#pragma once

namespace neat {

// The variant recorded for the bucket of (N, C, B, grid): the fastest for a
// call alone, or (throughput) the one with the most genome-inputs per
// second on a full GPU; FWD_AUTO when none is recorded.
int tuned_variant(int N, int C, int B, int grid, int throughput);
// Changes whenever a recorded variant changes (plans built from the table
// compare it to know they are stale).
unsigned tune_generation();
// Read the tune cache file at path into the table and keep writing the
// table there after every tuning (nothing happens for a NULL or empty path).
int tune_cache_use(const char *path);

}  // namespace neat
