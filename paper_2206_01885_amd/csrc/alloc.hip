// Caching device allocator behind DBuf (see common.h).
//
// Every freed block is kept for reuse: blocks below LARGE bytes in power-of-
// two size classes, larger ones reused best-fit within 25 % waste.  A block
// remembers the stream it was last used on and an event recorded there when
// it was freed; reusing it on another stream makes that stream wait for the
// event (no host synchronisation, no device-wide hipFree on the hot path).
// When hipMalloc fails the cache is released (after each block's event) and
// the allocation retried.  The environment variable H2_DEVICE_MEMORY_CAP
// (bytes) caps what the library holds from hipMalloc, cache included: an
// allocation beyond it fails as hipMalloc would (a test of the H2_ENOMEM
// path).
#include <cstdlib>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace h2 {
namespace {

constexpr size_t LARGE = (size_t)32 << 20;
constexpr size_t MIN_CLASS = 512;

struct Block {
    void* p;
    size_t bytes;
    hipStream_t s;
    hipEvent_t ev;
};

std::mutex g_mu;
std::vector<Block> g_cache;
std::vector<hipEvent_t> g_events;
std::mutex g_raw_mu;
size_t g_raw_bytes = 0;                       // held from hipMalloc
std::unordered_map<void*, size_t> g_raw_size;  // its blocks (under a cap)

size_t memory_cap()
{
    static const size_t cap = [] {
        const char* v = std::getenv("H2_DEVICE_MEMORY_CAP");
        return v ? (size_t)std::strtoull(v, nullptr, 10) : (size_t)0;
    }();
    return cap;
}

size_t class_bytes(size_t bytes)
{
    if (bytes >= LARGE) return bytes;
    size_t c = MIN_CLASS;
    while (c < bytes) c <<= 1;
    return c;
}

void* raw_alloc(size_t bytes)
{
    std::lock_guard<std::mutex> lk(g_raw_mu);
    const size_t cap = memory_cap();
    if (cap && g_raw_bytes + bytes > cap) return nullptr;
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (cap) {
        g_raw_bytes += bytes;
        g_raw_size[p] = bytes;
    }
    return p;
}

hipEvent_t take_event()
{
    if (!g_events.empty()) {
        hipEvent_t e = g_events.back();
        g_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

}  // namespace

void* dev_alloc(size_t bytes, hipStream_t s)
{
    const size_t cb = class_bytes(bytes);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        int best = -1;
        for (int i = (int)g_cache.size() - 1; i >= 0; --i) {
            const size_t b = g_cache[i].bytes;
            const bool fits = cb < LARGE ? b == cb : (b >= cb && b <= cb + cb / 4);
            if (fits && (best < 0 || b < g_cache[best].bytes)) {
                best = i;
                if (cb < LARGE) break;
            }
        }
        if (best >= 0) {
            Block blk = g_cache[best];
            g_cache.erase(g_cache.begin() + best);
            if (blk.ev) {
                if (blk.s != s) H2_HIP(hipStreamWaitEvent(s, blk.ev, 0));
                g_events.push_back(blk.ev);
            }
            return blk.p;
        }
    }
    void* p = raw_alloc(cb);
    if (!p) {
        dev_cache_trim();
        p = raw_alloc(cb);
    }
    if (!p) fail(H2_ENOMEM, "device allocation of " + std::to_string(cb) + " bytes failed");
    return p;
}

thread_local int g_idle = 0;
IdleFree::IdleFree() { ++g_idle; }
IdleFree::~IdleFree() { --g_idle; }

void dev_free(void* p, size_t bytes, hipStream_t s)
{
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_idle) {
        g_cache.push_back({p, class_bytes(bytes), nullptr, nullptr});
        return;
    }
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, s) != hipSuccess) {
        (void)hipGetLastError();
        g_events.push_back(e);
        e = nullptr;
    }
    if (!e) {
        // no event: wait here so that the block is idle when reused
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
    }
    g_cache.push_back({p, class_bytes(bytes), s, e});
}

void dev_cache_trim()
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& b : g_cache) {
        if (b.ev) {
            (void)hipEventSynchronize(b.ev);
            g_events.push_back(b.ev);
        }
        (void)hipFree(b.p);
        std::lock_guard<std::mutex> lk2(g_raw_mu);
        auto it = g_raw_size.find(b.p);
        if (it != g_raw_size.end()) {
            g_raw_bytes -= it->second;
            g_raw_size.erase(it);
        }
    }
    (void)hipGetLastError();
    g_cache.clear();
}

}  // namespace h2
