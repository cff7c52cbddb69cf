// Host model of the split contraction's grouping buffers over a sequence of
// calls on one circuit (test infrastructure).
//
// It replays on host memory what the insert and jobs kernels do to the hash
// table and the slot hulls, through the same index functions the kernels use
// (key_layout.h), for a list of batch sizes.  Before each claim of a slot it
// checks that the slot's table entry and hull row are empty, and after each
// call that every key's hull equals the hull of its members' intervals.
// Memory that a buffer gets when it grows holds a non-empty pattern, as new
// device memory may.
//
// Two layouts can be replayed:
//   stride   the library's: rows per half = the largest capacity so far,
//            cleared when laid out anew (plan_key_layout);
//   per-call rows per half = each call's own capacity, cleared only when a
//            buffer is reallocated (the layout that let a smaller call read
//            the upper bounds of its hulls from another call's lower bounds).
//
// Usage: key_layout_check stride|per-call SPAN B1 [B2 ...]
// Exit status 0 when every call saw empty rows and exact hulls; 1 otherwise,
// with the first violation printed.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "key_layout.h"

using namespace lofp;

namespace {

struct Buffers {
    std::vector<unsigned long long> table;
    std::vector<int> hull;
    bool grew = false;
    void ensure(size_t table_n, size_t hull_n)
    {
        grew = false;
        if (table_n > table.size()) { table.assign(table_n, 0xA5A5A5A5A5A5A5A5ULL); grew = true; }
        if (hull_n > hull.size()) { hull.assign(hull_n, 0x5A5A5A5A); grew = true; }
    }
};

uint64_t mix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int fail_at(int call, const char *what, long long a, long long b)
{
    std::printf("call %d: %s (%lld, %lld)\n", call, what, a, b);
    return 1;
}

}  // namespace

int main(int argc, char **argv)
{
    if (argc < 4) {
        std::fprintf(stderr, "usage: %s stride|per-call SPAN B1 [B2 ...]\n", argv[0]);
        return 2;
    }
    const bool per_call = std::strcmp(argv[1], "per-call") == 0;
    const int span = std::atoi(argv[2]);
    Buffers buf;
    KeyLayoutState st;           // stride layout
    bool legacy_clean = false;   // per-call layout: cleared only on reallocation
    for (int call = 0; call + 3 < argc; ++call) {
        const int B = std::atoi(argv[call + 3]);
        int64_t cap = 1;
        while (cap < 4 * (int64_t)B) cap <<= 1;
        int64_t stride;
        bool clear;
        if (per_call) {
            stride = cap;
            buf.ensure((size_t)2 * cap, (size_t)2 * 2 * cap * span);
            if (buf.grew) legacy_clean = false;
            clear = !legacy_clean;
        } else {
            const KeyLayoutPlan p = plan_key_layout(st, cap, span);
            stride = p.stride;
            buf.ensure(p.table_bytes / sizeof(unsigned long long), p.hull_bytes / sizeof(int));
            clear = p.clear;
        }
        const int64_t hi_off = key_hull_hi_offset(stride, span);
        if (clear) {
            for (int64_t i = 0; i < 2 * stride; ++i) buf.table[i] = kKeyEmpty;
            for (int64_t i = 0; i < 2 * stride * span; ++i) {
                buf.hull[i] = kHullEmptyLo;
                buf.hull[hi_off + i] = kHullEmptyHi;
            }
        }
        if (per_call) legacy_clean = false; else st.clean = false;
        // rows: B patterns, about B/4 distinct rows per half; random intervals
        std::vector<int64_t> claimed[2];
        std::vector<std::vector<int>> want_lo[2], want_hi[2];
        for (int half = 0; half < 2; ++half) {
            std::vector<int64_t> slot_of_key((size_t)B, -1);
            for (int p = 0; p < B; ++p) {
                const uint64_t key = mix((uint64_t)call * 1000003u + (uint64_t)half * 7919u + (uint64_t)(p % (B / 4 + 1)));
                int64_t j = (int64_t)(key & (uint64_t)(cap - 1));
                for (int64_t probe = 0;; ++probe) {
                    if (probe >= cap) return fail_at(call, "table full", half, p);
                    unsigned long long &e = buf.table[key_slot_index(half, stride, j)];
                    if (e == kKeyEmpty) {
                        const int64_t row = key_hull_row(half, stride, j, span);
                        for (int i = 0; i < span; ++i)
                            if (buf.hull[row + i] != kHullEmptyLo || buf.hull[hi_off + row + i] != kHullEmptyHi)
                                return fail_at(call, "claimed slot has a stale hull row (lo, hi)", buf.hull[row + i],
                                               buf.hull[hi_off + row + i]);
                        e = key;
                        claimed[half].push_back(j);
                        want_lo[half].push_back(std::vector<int>(span, kHullEmptyLo));
                        want_hi[half].push_back(std::vector<int>(span, kHullEmptyHi));
                        break;
                    }
                    if (e == key) break;
                    j = (j + 1) & (cap - 1);
                }
                size_t k = 0;
                while (claimed[half][k] != j) ++k;
                const int64_t row = key_hull_row(half, stride, j, span);
                for (int i = 0; i < span; ++i) {
                    const int lo = (int)(mix((uint64_t)p * 131 + i) % 5), hi = lo + (int)(mix((uint64_t)p * 137 + i) % 4);
                    buf.hull[row + i] = std::min(buf.hull[row + i], lo);
                    buf.hull[hi_off + row + i] = std::max(buf.hull[hi_off + row + i], hi);
                    want_lo[half][k][i] = std::min(want_lo[half][k][i], lo);
                    want_hi[half][k][i] = std::max(want_hi[half][k][i], hi);
                }
            }
        }
        // jobs kernel: read each key's hull, then empty its row and entry
        for (int half = 0; half < 2; ++half)
            for (size_t k = 0; k < claimed[half].size(); ++k) {
                const int64_t j = claimed[half][k];
                const int64_t row = key_hull_row(half, stride, j, span);
                for (int i = 0; i < span; ++i) {
                    if (buf.hull[row + i] != want_lo[half][k][i] || buf.hull[hi_off + row + i] != want_hi[half][k][i])
                        return fail_at(call, "key hull differs from its members' hull (lo, hi)", buf.hull[row + i],
                                       buf.hull[hi_off + row + i]);
                    buf.hull[row + i] = kHullEmptyLo;
                    buf.hull[hi_off + row + i] = kHullEmptyHi;
                }
                buf.table[key_slot_index(half, stride, j)] = kKeyEmpty;
            }
        if (per_call) legacy_clean = true; else st.clean = true;
        std::printf("call %d: B=%d cap=%lld stride=%lld cleared=%d keys=%zu+%zu ok\n", call, B, (long long)cap,
                    (long long)stride, (int)clear, claimed[0].size(), claimed[1].size());
    }
    return 0;
}
