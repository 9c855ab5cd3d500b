// Hooks of the context used by the serving loop (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "../../include/helmdd.h"

namespace helmdd_internal {

// Moves a context to another stream (waits for the work on the old one).
hh_status set_stream(hh_ctx* c, hipStream_t s);

// Device bytes the context holds (factors, coarse data, work buffers).
size_t resident_bytes(const hh_ctx* c);

// Host-side estimate of the device bytes of a context for q right-hand sides
// of hh_solve with GMRES(restart): leaf factors (FP64 during the set-up, plus
// complex64 copies when mixed), coarse data at the given ranks, level buffers
// and the Krylov bases.  Returns 0 for an invalid decomposition.
size_t estimate_bytes(const hh_operator* A, const hh_decomposition* d, const int32_t* rank, int32_t oversample,
                      int32_t q, int32_t restart, int32_t precision);

}  // namespace helmdd_internal
