// Caching device allocator behind DBuf (see common.h).
#include <mutex>
#include <vector>

#include "common.h"

namespace h2 {
namespace {

constexpr size_t CACHE_MIN = (size_t)64 << 20;  // blocks from 64 MiB up are cached

struct Block {
    void* p;
    size_t bytes;
};

std::mutex g_mu;
std::vector<Block> g_cache;

void* raw_alloc(size_t bytes)
{
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

}  // namespace

void* dev_alloc(size_t bytes)
{
    if (bytes >= CACHE_MIN) {
        std::lock_guard<std::mutex> lk(g_mu);
        // smallest cached block that fits without wasting more than a quarter
        int best = -1;
        for (int i = 0; i < (int)g_cache.size(); ++i)
            if (g_cache[i].bytes >= bytes && g_cache[i].bytes <= bytes + bytes / 4 &&
                (best < 0 || g_cache[i].bytes < g_cache[best].bytes))
                best = i;
        if (best >= 0) {
            void* p = g_cache[best].p;
            g_cache.erase(g_cache.begin() + best);
            return p;
        }
    }
    void* p = raw_alloc(bytes);
    if (!p) {
        dev_cache_trim();
        p = raw_alloc(bytes);
    }
    if (!p) fail(H2_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
}

void dev_free(void* p, size_t bytes, hipStream_t s)
{
    if (!p) return;
    if (bytes >= CACHE_MIN) {
        // work queued on s may still read or write the block
        if (hipStreamSynchronize(s) == hipSuccess) {
            std::lock_guard<std::mutex> lk(g_mu);
            g_cache.push_back({p, bytes});
            return;
        }
        (void)hipGetLastError();
    }
    (void)hipFree(p);
}

void dev_cache_trim()
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& b : g_cache) (void)hipFree(b.p);
    g_cache.clear();
}

}  // namespace h2
