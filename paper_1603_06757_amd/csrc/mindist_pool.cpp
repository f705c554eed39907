// mindist_pool.cpp -- caches of device/pinned memory, streams and events.
#include "mindist_pool.h"

#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "mindist_internal.h"

namespace md {
namespace {

std::mutex g_mu;
std::mutex &g_const_mu() { static std::mutex m; return m; }

// sizes are rounded so repeated requests of nearby sizes share blocks
size_t round_size(size_t b) {
    if (b < 4096) return 4096;
    if (b <= (1u << 20)) {
        size_t r = 4096;
        while (r < b) r <<= 1;
        return r;
    }
    const size_t q = 1u << 20;
    return (b + q - 1) / q * q;
}

struct Block { int dev; size_t size; bool pinned; };
std::unordered_map<void *, Block> g_live;
std::map<std::pair<int, size_t>, std::vector<void *>> g_dev_free;   // (device, size)
std::map<size_t, std::vector<void *>> g_pin_free;
size_t g_dev_cached = 0;
std::vector<hipStream_t> g_streams[64];
std::vector<hipEvent_t> g_events[64];
const uint64_t *g_binom[64] = {nullptr};
std::map<std::pair<int, std::string>, void *> g_const;   // (device, key) -> device copy

int cur_dev() {
    int d = 0;
    (void)hipGetDevice(&d);
    return d < 0 ? 0 : (d > 63 ? 63 : d);
}

void release_cached_device(int dev) {
    for (auto it = g_dev_free.begin(); it != g_dev_free.end();) {
        if (it->first.first == dev) {
            for (void *p : it->second) {
                (void)hipFree(p);
                g_dev_cached -= it->first.second;
            }
            it = g_dev_free.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace

void *dev_alloc(size_t bytes) {
    const size_t sz = round_size(bytes);
    const int dev = cur_dev();
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev_free.find({dev, sz});
    if (it != g_dev_free.end() && !it->second.empty()) {
        void *p = it->second.back();
        it->second.pop_back();
        g_dev_cached -= sz;
        g_live[p] = {dev, sz, false};
        return p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) {
        (void)hipGetLastError();
        release_cached_device(dev);
        if (hipMalloc(&p, sz) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    g_live[p] = {dev, sz, false};
    return p;
}

void dev_free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    g_dev_free[{it->second.dev, it->second.size}].push_back(p);
    g_dev_cached += it->second.size;
    g_live.erase(it);
}

void *pinned_alloc(size_t bytes) {
    const size_t sz = round_size(bytes);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_pin_free.find(sz);
    if (it != g_pin_free.end() && !it->second.empty()) {
        void *p = it->second.back();
        it->second.pop_back();
        g_live[p] = {-1, sz, true};
        return p;
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    g_live[p] = {-1, sz, true};
    return p;
}

void pinned_free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    g_pin_free[it->second.size].push_back(p);
    g_live.erase(it);
}

namespace {
struct Mapped { size_t size; void *dev; };
std::unordered_map<void *, Mapped> g_mapped_live;
std::map<size_t, std::vector<std::pair<void *, void *>>> g_mapped_free;
}  // namespace

void *mapped_alloc(size_t bytes, void **device) {
    const size_t sz = round_size(bytes);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_mapped_free.find(sz);
    if (it != g_mapped_free.end() && !it->second.empty()) {
        auto pr = it->second.back();
        it->second.pop_back();
        g_mapped_live[pr.first] = {sz, pr.second};
        *device = pr.second;
        return pr.first;
    }
    void *p = nullptr, *d = nullptr;
    if (hipHostMalloc(&p, sz, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(p);
        return nullptr;
    }
    g_mapped_live[p] = {sz, d};
    *device = d;
    return p;
}

void mapped_free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_mapped_live.find(p);
    if (it == g_mapped_live.end()) return;
    g_mapped_free[it->second.size].push_back({p, it->second.dev});
    g_mapped_live.erase(it);
}

hipStream_t stream_get() {
    const int dev = cur_dev();
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_streams[dev].empty()) {
            hipStream_t s = g_streams[dev].back();
            g_streams[dev].pop_back();
            return s;
        }
    }
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    return s;
}

void stream_put(hipStream_t s) {
    if (!s) return;
    const int dev = cur_dev();
    std::lock_guard<std::mutex> lk(g_mu);
    g_streams[dev].push_back(s);
}

hipEvent_t event_get() {
    const int dev = cur_dev();
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_events[dev].empty()) {
            hipEvent_t e = g_events[dev].back();
            g_events[dev].pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void event_put(hipEvent_t e) {
    if (!e) return;
    const int dev = cur_dev();
    std::lock_guard<std::mutex> lk(g_mu);
    g_events[dev].push_back(e);
}

const uint64_t *device_binom_from(const uint64_t *host_table) {
    const int dev = cur_dev();
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_binom[dev]) return g_binom[dev];
    }
    const size_t bytes = sizeof(uint64_t) * kBinomX * kBinomT;
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    if (hipMemcpy(p, host_table, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(p);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_binom[dev]) {          // another thread won the race
        (void)hipFree(p);
        return g_binom[dev];
    }
    g_binom[dev] = static_cast<const uint64_t *>(p);
    return g_binom[dev];
}

const void *device_const(const void *key, size_t key_bytes, const void *host, size_t bytes) {
    const int dev = cur_dev();
    const std::pair<int, std::string> k(dev, std::string(static_cast<const char *>(key), key_bytes));
    std::lock_guard<std::mutex> lk(g_const_mu());
    auto it = g_const.find(k);
    if (it != g_const.end()) return it->second;
    void *p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) return nullptr;
    // synchronous: once this returns, the copy is visible to kernels on
    // every stream (the streams handed out here are non-blocking, so this
    // does not wait for their work)
    if (bytes && hipMemcpy(p, host, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(p);
        return nullptr;
    }
    g_const.emplace(k, p);
    return p;
}

size_t dev_cached_bytes() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_dev_cached;
}

}  // namespace md
