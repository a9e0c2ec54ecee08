// vr_cache.h -- the library's own device memory: a stream-ordered caching
// allocator used when the caller supplies no allocator.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

// Device memory of at least `bytes` usable on stream s in stream order
// (nullptr when the device is out of memory even after dropping the cache).
void *cache_get(size_t bytes, hipStream_t s);

// Return p (from cache_get) once the work enqueued on s so far is done with
// it.  Nothing is released to the driver.
void cache_put(void *p, hipStream_t s);

// Release the cached blocks of the current device that are not in use
// (synchronises the device).  Returns the bytes released.
size_t cache_trim();

// Bytes held from the driver on the current device (in use plus cached).
size_t cache_held();
