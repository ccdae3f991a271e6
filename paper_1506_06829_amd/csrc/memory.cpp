// Workspace memory of the library.  Freeing device memory costs about 0.1 ms
// per buffer on this platform (a d1 solver's 40 buffers: ~4 ms, more than a
// tenth of a complete solve, and the stream-ordered pools of the runtime cost
// the same), so freed workspace is cached: dev_free keeps a block in a free
// list and dev_alloc reuses the smallest cached block of the same device that
// is at least the requested size and at most a quarter larger.  The cache is
// capped (older blocks are released beyond 64 GiB) and dropped when an
// allocation fails.  Pinned host staging buffers are kept in a free list for
// the same reason.  Cached memory is held until the process ends.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace gplhr {
namespace {

struct Block {
    void *p;
    size_t bytes;
    int dev;
};

constexpr size_t CACHE_CAP = (size_t)64 << 30;

std::mutex g_mu;
std::vector<Block> g_free;                        // cached device blocks, oldest first
size_t g_cached = 0;
std::unordered_map<void *, Block> g_live;         // blocks handed out
struct PinnedBuf {
    void *p;
    size_t bytes;
};
std::vector<PinnedBuf> g_pinned;                  // free pinned buffers

// with g_mu held
void release_cached(int dev) {
    for (size_t i = 0; i < g_free.size();) {
        if (dev < 0 || g_free[i].dev == dev) {
            (void)hipFree(g_free[i].p);
            g_cached -= g_free[i].bytes;
            g_free.erase(g_free.begin() + i);
        } else {
            ++i;
        }
    }
}

}  // namespace

void *dev_alloc(size_t bytes, hipStream_t st) {
    (void)st;
    if (bytes == 0) bytes = 1;
    bytes = (bytes + 255) & ~(size_t)255;
    int dev = 0;
    GPLHR_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    size_t best = g_free.size();
    for (size_t i = 0; i < g_free.size(); ++i) {
        const Block &b = g_free[i];
        if (b.dev == dev && b.bytes >= bytes && b.bytes - bytes <= bytes / 4 &&
            (best == g_free.size() || b.bytes < g_free[best].bytes))
            best = i;
    }
    if (best < g_free.size()) {
        Block b = g_free[best];
        g_free.erase(g_free.begin() + best);
        g_cached -= b.bytes;
        g_live[b.p] = b;
        return b.p;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release_cached(dev);
        e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(-2, "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                            hipGetErrorString(e));
    }
    g_live[p] = Block{p, bytes, dev};
    return p;
}

void dev_free(void *p, hipStream_t st) {
    if (!p) return;
    // the block may be handed to another stream next: let this one finish
    (void)hipStreamSynchronize(st);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    g_free.push_back(it->second);
    g_cached += it->second.bytes;
    g_live.erase(it);
    while (g_cached > CACHE_CAP && !g_free.empty()) {
        (void)hipFree(g_free.front().p);
        g_cached -= g_free.front().bytes;
        g_free.erase(g_free.begin());
    }
}

void *pinned_alloc(size_t bytes) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (size_t i = 0; i < g_pinned.size(); ++i) {
            if (g_pinned[i].bytes >= bytes) {
                void *p = g_pinned[i].p;
                g_pinned.erase(g_pinned.begin() + i);
                return p;
            }
        }
    }
    void *p = nullptr;
    GPLHR_HIP_CHECK(hipHostMalloc(&p, bytes, hipHostMallocDefault));
    return p;
}

void pinned_free(void *p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_pinned.push_back(PinnedBuf{p, bytes});
}

}  // namespace gplhr
