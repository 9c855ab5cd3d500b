// Process-wide caching allocator for device memory.
//
// hipMalloc / hipFree of the large per-solve buffers (Krylov bases of several
// GB, level work space) cost milliseconds each and hipFree synchronises the
// device.  Contexts therefore take their buffers from this pool and hand them
// back on release; a block is reused for a request of the same rounded size
// class.  A block released on stream s carries an event recorded on s at the
// release: a later request on the same stream reuses it at once (stream
// order), a request on another stream first waits for that event.  The
// functions ignore HIP errors of their own calls and leave none in the
// thread's last-error slot.  Cached
// bytes are capped (HH_POOL_CAP_GB, default a quarter of the device memory);
// when hipMalloc fails, the cached blocks of the device are freed and the
// allocation is retried once.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace devpool {

// Size class of a request: 256-byte multiples up to 1 MiB, 2 MiB multiples above.
size_t size_class(size_t bytes);

// A block of at least `bytes` on the current device, usable by work enqueued
// on `stream`; nullptr if the device is out of memory.
void* acquire(size_t bytes, hipStream_t stream);

// Returns a block obtained from acquire (same byte count); work already
// enqueued on `stream` may still use it (unless idle: nothing pending on the
// stream uses the block, so no event is recorded).
void release(void* p, size_t bytes, hipStream_t stream, bool idle = false);

// Waits for and drops the events recorded on `stream` by earlier releases, so
// that no cached block refers to the stream any more.  Call it before the
// stream is destroyed (an event recorded on a destroyed stream must not be
// waited for).
void forget_stream(hipStream_t stream);

// Frees every cached block of the current device; returns the bytes freed.
size_t trim();

// Bytes currently cached (not handed out) on the current device.
size_t cached_bytes();

}  // namespace devpool
