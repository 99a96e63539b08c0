// Caching device allocator for handle and batch buffers.
//
// Creating and destroying hundreds of scenario handles (a planning sweep,
// surrogate training data) would otherwise map and unmap device memory for
// every buffer, and hipFree synchronises the whole device.  Freed blocks are
// kept here per device and size class and handed out again; the cache holds
// at most a bounded number of bytes (FEDFEM_DEVICE_CACHE_MB, default 16384)
// and fedfem_release_cached_memory returns all of it.  Callers return a
// block only once no stream still uses it.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/fedfem.h"
#include "internal.h"

namespace fedfem {

namespace {

struct Cache {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void*>> free;  // (device, class)
    size_t bytes = 0;
    size_t limit = 0;
    Cache() {
        const char* s = std::getenv("FEDFEM_DEVICE_CACHE_MB");
        const long long mb = s ? std::atoll(s) : 16384;
        limit = mb > 0 ? (size_t)mb << 20 : 0;
    }
};

Cache& cache() {
    static Cache* c = new Cache();  // never destroyed: outlives every handle
    return *c;
}

// 1 KiB granules up to 64 KiB, then 8 classes per octave (< 12.5% waste)
size_t size_class(size_t bytes) {
    bytes = bytes < 256 ? 256 : bytes;
    if (bytes <= (size_t(64) << 10)) return (bytes + 1023) / 1024 * 1024;
    int k = 0;
    while ((size_t(1) << (k + 1)) <= bytes) k++;  // 2^k <= bytes < 2^(k+1)
    const size_t step = size_t(1) << (k - 3);
    return (bytes + step - 1) / step * step;
}

size_t trim_locked(Cache& c, size_t keep) {
    size_t released = 0;
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (auto it = c.free.begin(); it != c.free.end() && c.bytes > keep;) {
        auto& v = it->second;
        if (!v.empty()) (void)hipSetDevice(it->first.first);
        while (!v.empty() && c.bytes > keep) {
            (void)hipFree(v.back());
            v.pop_back();
            c.bytes -= it->first.second;
            released += it->first.second;
        }
        it = v.empty() ? c.free.erase(it) : std::next(it);
    }
    if (cur >= 0) (void)hipSetDevice(cur);
    return released;
}

}  // namespace

hipError_t cached_malloc(void** p, size_t bytes, size_t* granted) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const size_t cls = size_class(bytes);
    Cache& c = cache();
    {
        std::lock_guard<std::mutex> lock(c.mu);
        auto it = c.free.find({dev, cls});
        if (it != c.free.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            c.bytes -= cls;
            *granted = cls;
            return hipSuccess;
        }
    }
    e = hipMalloc(p, cls);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lock(c.mu);
            trim_locked(c, 0);
        }
        (void)hipSetDevice(dev);
        e = hipMalloc(p, cls);
    }
    if (e == hipSuccess) *granted = cls;
    return e;
}

void cached_free(void* p, size_t granted) {
    if (!p) return;
    Cache& c = cache();
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lock(c.mu);
    if (c.bytes + granted > c.limit) {
        (void)hipFree(p);
        return;
    }
    c.free[{dev, granted}].push_back(p);
    c.bytes += granted;
}

}  // namespace fedfem

extern "C" size_t fedfem_release_cached_memory(void) {
    fedfem::Cache& c = fedfem::cache();
    std::lock_guard<std::mutex> lock(c.mu);
    return fedfem::trim_locked(c, 0);
}
