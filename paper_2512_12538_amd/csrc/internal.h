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

// Returns the level work buffers to the device cache (they are regrown by the
// next call that needs them); factors and coarse data stay.
void release_work(hh_ctx* c);

// Host-side estimate of the device bytes of an operator and of hh_solve with
// GMRES(restart): leaf factors (FP64 during the set-up, plus complex64 copies
// when mixed) and coarse data at the given ranks; level buffers and Krylov
// bases per right-hand side; level buffers for the sketch columns during the
// set-up.  All zero for an invalid decomposition.
struct Footprint {
  size_t op = 0;       // a prepared operator
  size_t per_rhs = 0;  // solve work space per right-hand side
  size_t setup = 0;    // transient work space of the coarse-space construction
};
Footprint estimate_bytes(const hh_operator* A, const hh_decomposition* d, const int32_t* rank,
                         int32_t oversample, int32_t restart, int32_t precision);

}  // namespace helmdd_internal
