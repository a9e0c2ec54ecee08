// vr_cache.hip -- stream-ordered caching allocator for the library's device
// memory.
//
// Builds of different shapes need workspaces and output blocks of sizes that
// change with every request.  Blocks come from hipMalloc once and are kept:
// a freed block records an event on the freeing stream and joins a free list
// ordered by size.  A request takes the smallest free block of the same
// device that holds it and is at most twice its size (so a huge block does
// not serve a tiny request); when that block was last used on another
// stream, the requesting stream first waits on the block's event, which keeps
// every reuse in stream order without any host synchronisation.  Sizes are
// rounded to 512 B below 1 MiB and to 2 MiB above, so neighbouring sizes
// share blocks.
#include "vr_cache.h"

#include <map>
#include <mutex>
#include <unordered_map>

namespace {

struct Block {
    void *p = nullptr;
    size_t size = 0;
    int dev = 0;
    hipStream_t stream = nullptr;  // stream of the last use
    hipEvent_t ev = nullptr;       // recorded on `stream` when freed
};

struct Cache {
    std::mutex mu;
    std::multimap<size_t, Block> free_;       // by size
    std::unordered_map<void *, Block> live_;  // by address
    std::unordered_map<int, size_t> held_;    // per device

    static size_t round(size_t b) {
        if (b == 0) b = 1;
        if (b < (1u << 20)) return (b + 511) & ~(size_t)511;
        return (b + (2u << 20) - 1) & ~((size_t)(2u << 20) - 1);
    }

    void *get(size_t bytes, hipStream_t s) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return nullptr;
        const size_t r = round(bytes);
        {
            std::lock_guard<std::mutex> g(mu);
            for (auto it = free_.lower_bound(r); it != free_.end() && it->first <= 2 * r; ++it) {
                if (it->second.dev != dev) continue;
                Block b = it->second;
                free_.erase(it);
                if (b.stream != s && b.ev) (void)hipStreamWaitEvent(s, b.ev, 0);
                b.stream = s;
                live_[b.p] = b;
                return b.p;
            }
        }
        Block b;
        b.size = r;
        b.dev = dev;
        b.stream = s;
        if (hipMalloc(&b.p, r) != hipSuccess) {
            (void)hipGetLastError();
            trim(dev);  // drop what the cache holds on this device, then try once more
            if (hipMalloc(&b.p, r) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
        }
        std::lock_guard<std::mutex> g(mu);
        live_[b.p] = b;
        held_[dev] += r;
        return b.p;
    }

    void put(void *p, hipStream_t s) {
        if (!p) return;
        std::lock_guard<std::mutex> g(mu);
        auto it = live_.find(p);
        if (it == live_.end()) return;
        Block b = it->second;
        live_.erase(it);
        if (!b.ev && hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            b.ev = nullptr;
        }
        b.stream = s;
        if (b.ev && hipEventRecord(b.ev, s) != hipSuccess) {
            (void)hipGetLastError();
            // without an event the block is only safe once the device is idle
            (void)hipDeviceSynchronize();
        }
        free_.emplace(b.size, b);
    }

    size_t trim(int dev) {
        // the device's outstanding work may still use freed blocks
        (void)hipDeviceSynchronize();
        std::lock_guard<std::mutex> g(mu);
        size_t rel = 0;
        for (auto it = free_.begin(); it != free_.end();) {
            if (it->second.dev != dev) {
                ++it;
                continue;
            }
            if (it->second.ev) (void)hipEventDestroy(it->second.ev);
            (void)hipFree(it->second.p);
            rel += it->second.size;
            held_[dev] -= it->second.size;
            it = free_.erase(it);
        }
        return rel;
    }
};

// Never destroyed: blocks live until the process ends, and the HIP runtime
// may already be torn down when static destructors run.
Cache &cache() {
    static Cache *c = new Cache();
    return *c;
}

}  // namespace

void *cache_get(size_t bytes, hipStream_t s) { return cache().get(bytes, s); }

void cache_put(void *p, hipStream_t s) { cache().put(p, s); }

size_t cache_trim() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    return cache().trim(dev);
}

size_t cache_held() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    Cache &c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.held_.find(dev);
    return it == c.held_.end() ? 0 : it->second;
}
