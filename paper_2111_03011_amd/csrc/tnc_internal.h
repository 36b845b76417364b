// Hooks between the host runtime (tnc.cpp) and the no-allocation entry point
// (noalloc.hip); internal to libtnc.
#pragma once
#include <stdint.h>

#include "tnc.h"

namespace tnc {

// Record an error message for tnc_last_error() and return `code`.
tnc_status report_error(tnc_status code, const char* msg);

// HIP device of a plan.
tnc_status plan_device(tnc_plan plan, int* device);

// tnc_sample with every device buffer it needs (closed bits, open qubit ids, running sums,
// draws) carved from `scratch` (device memory of `scratch_bytes` bytes, 256-byte aligned)
// instead of the plan's workspace.  Allocates nothing; synchronous on the stream.
tnc_status sample_in_scratch(tnc_plan plan, uint8_t* scratch, uint64_t scratch_bytes,
                             const double* amps, uint64_t seed, int64_t n_samples,
                             uint64_t* h_bits, void* stream);

}  // namespace tnc
