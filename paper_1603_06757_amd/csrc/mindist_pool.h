// mindist_pool.h -- process-wide caches of device memory, pinned host memory,
// streams and events.  Contexts come and go per code (and per request in the
// server); hipMalloc/hipHostMalloc/hipStreamCreate cost tens of microseconds
// to milliseconds each, so released resources are kept for reuse instead of
// being returned to the runtime.  All functions are thread-safe.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace md {

// device memory of the current device; nullptr if the device is out of memory
void *dev_alloc(size_t bytes);
void dev_free(void *p);
// page-locked host memory
void *pinned_alloc(size_t bytes);
void pinned_free(void *p);
// page-locked, coherent host memory mapped into the device's address space
// (device writes reach the host without copies); *device receives the
// address kernels use
void *mapped_alloc(size_t bytes, void **device);
void mapped_free(void *p);
// non-blocking streams at the default priority, and timing events
hipStream_t stream_get();
void stream_put(hipStream_t s);
hipEvent_t event_get();
void event_put(hipEvent_t e);
// the binomial table C(x, t), x < kBinomX, t < kBinomT, on the current
// device (copied from host_table on the first call per device)
const uint64_t *device_binom_from(const uint64_t *host_table);
// a small immutable device array identified by `key` (key_bytes bytes): the
// first call per device and key copies `bytes` bytes from `host` and waits
// for the copy; later calls return the same device address.  Held until the
// process ends.  nullptr if allocation or copy fails.
const void *device_const(const void *key, size_t key_bytes, const void *host, size_t bytes);
// bytes currently held in the device cache (not handed out)
size_t dev_cached_bytes();

}  // namespace md
