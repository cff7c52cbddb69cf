// pool.cpp -- device memory pool for circuit set-up.
//
// Blocks of up to 16 MiB are rounded up to a power of two (at least 4 KiB)
// and carved from slabs; freed blocks go to a per-class free list and are
// reused.  Slabs start at 64 MiB and double up to 2 GiB, so a serving run
// that sets up thousands of fresh circuits calls hipMalloc a handful of
// times rather than once per 64 MiB (each such call stalls the thread that
// makes it, and with it the requests that thread is launching).  Larger
// blocks are plain hipMalloc allocations.  One pool per device; thread-safe.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <vector>

#include "host_internal.h"

namespace lofp {
namespace host {
namespace {

constexpr size_t kSlabMin = size_t(64) << 20;
constexpr size_t kSlabMax = size_t(2) << 30;
constexpr size_t kMinBlock = size_t(4) << 10;
constexpr size_t kMaxPooled = size_t(16) << 20;

struct Pool {
    std::map<size_t, std::vector<void *>> free_lists;   // class size -> blocks
    char *slab = nullptr;
    size_t cap = 0;            // bytes of the current slab
    size_t used = 0;
    size_t next = kSlabMin;    // bytes of the next slab
};

std::mutex g_mu;
std::map<int, Pool> g_pools;

size_t size_class(size_t bytes)
{
    size_t c = kMinBlock;
    while (c < bytes) c <<= 1;
    return c;
}

}  // namespace

void *pool_alloc(size_t bytes, int device)
{
    if (bytes > kMaxPooled) {
        void *p = nullptr;
        return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
    }
    const size_t c = size_class(bytes);
    std::lock_guard<std::mutex> lk(g_mu);
    Pool &pl = g_pools[device];
    std::vector<void *> &fl = pl.free_lists[c];
    if (!fl.empty()) {
        void *p = fl.back();
        fl.pop_back();
        return p;
    }
    if (pl.used + c > pl.cap) {
        void *s = nullptr;
        if (hipMalloc(&s, pl.next) != hipSuccess) {
            // the doubled slab does not fit: fall back to the smallest
            if (pl.next == kSlabMin || hipMalloc(&s, kSlabMin) != hipSuccess) return nullptr;
            pl.next = kSlabMin;
        }
        pl.slab = static_cast<char *>(s);
        pl.cap = pl.next;
        pl.used = 0;
        pl.next = pl.next < kSlabMax ? pl.next * 2 : kSlabMax;
    }
    void *p = pl.slab + pl.used;
    pl.used += c;
    return p;
}

void pool_free(void *p, size_t bytes, int device)
{
    if (!p) return;
    if (bytes > kMaxPooled) {
        (void)hipFree(p);
        return;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_pools[device].free_lists[size_class(bytes)].push_back(p);
}

}  // namespace host
}  // namespace lofp
