// Caching device allocator for the library's temporaries and factors.
//
// Driver allocations and frees are slow on this stack (a free costs hundreds
// of microseconds and synchronises), and one HSS build allocates and releases
// dozens of buffers per tree level.  Blocks are therefore kept in per-device
// size-class bins after their first allocation.  A freed block is tagged with
// the stream it was released on and is only handed out again for work on that
// same stream, so stream order guarantees its previous users have finished.  A
// block released with no work pending on it (dev_free_idle) may be handed out
// for any stream: the factors of a destroyed HSS object are allocated on the
// build's second stream and released on the caller's, and would otherwise
// never be reused.
//
// The cache is bounded, so that the memory of one large problem does not stay
// out of other users' reach (the process's own framework allocations among
// them): free blocks are kept up to kCacheMaxBytes per device (the environment
// variable BMHSS_CACHE_MAX_GIB overrides it); a block released beyond that is
// returned to the driver once its stream has drained, and a failed driver
// allocation returns every cached block of the device (after a device
// synchronisation) and tries once more.
#include <cstdlib>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace bm {

namespace {

struct CachedBlock {
    void* p;
    hipStream_t s;
    bool idle;   // no work pending: reusable on any stream
};

struct DeviceCache {
    std::map<size_t, std::vector<CachedBlock>> free_bins;   // size class -> free blocks
    std::unordered_map<void*, size_t> size_of;        // live and cached blocks
    size_t cached = 0;                                 // bytes in free_bins
};

std::mutex g_mu;
std::unordered_map<int, DeviceCache> g_cache;

constexpr size_t kCacheMaxBytes = size_t{16} << 30;

size_t cache_max_bytes() {
    static const size_t v = [] {
        const char* e = std::getenv("BMHSS_CACHE_MAX_GIB");
        if (!e) return kCacheMaxBytes;
        const double g = std::atof(e);
        return g >= 0.0 && g < 1e6 ? static_cast<size_t>(g * static_cast<double>(size_t{1} << 30)) : kCacheMaxBytes;
    }();
    return v;
}

// every cached block of the device back to the driver (the caller has
// synchronised the device)
void trim_device(int dev) {
    std::vector<void*> blocks;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        DeviceCache& dc = g_cache[dev];
        for (auto& bin : dc.free_bins)
            for (const CachedBlock& b : bin.second) {
                blocks.push_back(b.p);
                dc.size_of.erase(b.p);
            }
        dc.free_bins.clear();
        dc.cached = 0;
    }
    for (void* q : blocks) (void)hipFree(q);
}

size_t size_class(size_t bytes) {
    size_t c = 256;
    while (c < bytes) c <<= 1;
    return c;
}

}  // namespace

hipError_t dev_alloc(void** p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const size_t c = size_class(bytes == 0 ? 1 : bytes);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        DeviceCache& dc = g_cache[dev];
        auto it = dc.free_bins.find(c);
        if (it != dc.free_bins.end()) {
            std::vector<CachedBlock>& v = it->second;
            for (size_t i = v.size(); i-- > 0;) {
                if (v[i].idle || v[i].s == s) {
                    *p = v[i].p;
                    v.erase(v.begin() + static_cast<std::ptrdiff_t>(i));
                    dc.cached -= c;
                    return hipSuccess;
                }
            }
        }
    }
    e = hipMalloc(p, c);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        if ((e = hipDeviceSynchronize()) != hipSuccess) {
            *p = nullptr;
            return e;
        }
        trim_device(dev);
        e = hipMalloc(p, c);
    }
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[dev].size_of[*p] = c;
    return hipSuccess;
}

namespace {

void release_block(void* p, hipStream_t s, bool idle) {
    if (!p) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        DeviceCache& dc = g_cache[dev];
        auto it = dc.size_of.find(p);
        if (it == dc.size_of.end()) return;   // not ours
        if (dc.cached + it->second <= cache_max_bytes()) {
            dc.cached += it->second;
            dc.free_bins[it->second].push_back(CachedBlock{p, s, idle});
            return;
        }
        dc.size_of.erase(it);
    }
    // beyond the cache bound: back to the driver once its users have finished
    if (!idle) (void)hipStreamSynchronize(s);
    (void)hipFree(p);
}

}  // namespace

void dev_free(void* p, hipStream_t s) { release_block(p, s, false); }

void dev_free_idle(void* p) { release_block(p, nullptr, true); }

}  // namespace bm
