// key_layout.h -- where the grouping of a split contraction keeps its hash
// table, slot hulls and slot key numbers, and when they must be cleared.
//
// The grouping (keys.hip) has one open-addressing table per half of T.  A
// call probes modulo its own capacity `cap` (a power of two >= 4 x its
// batch), but the rows of the two halves sit `stride` rows apart, where
// `stride` is the largest capacity laid out so far on this circuit: a call
// with a smaller batch then uses the first `cap` rows of each half of the
// same layout, and every row it can touch is one that the earlier calls
// left empty.  (Laying the halves out by each call's own cap would put the
// second half's rows, and the upper hull bounds, on memory that a larger
// earlier call used for something else.)
//
// Host and device code share the index functions below; the planning
// function is host-only and has no HIP dependence, so a CPU build can check
// the bookkeeping on its own.
#pragma once
#include <stddef.h>
#include <stdint.h>

#if defined(__HIP__)
#define LOFP_KL_HD __host__ __device__
#else
#define LOFP_KL_HD
#endif

namespace lofp {

// Empty hull row: lo = +large (a min identity), hi = -1 (a max identity, and
// "no feasible member" when still -1 after the insert kernel).
constexpr int kHullEmptyLo = 0x7f7f7f7f;
constexpr int kHullEmptyHi = -1;
constexpr unsigned long long kKeyEmpty = ~0ULL;   // an empty hash slot

// Index of slot j of a half in the table and in the slot-key array.
LOFP_KL_HD inline int64_t key_slot_index(int half, int64_t stride, int64_t j)
{
    return (int64_t)half * stride + j;
}
// First int of the hull row of slot j of a half (lower bounds; the upper
// bounds sit key_hull_hi_offset further on).
LOFP_KL_HD inline int64_t key_hull_row(int half, int64_t stride, int64_t j, int span)
{
    return key_slot_index(half, stride, j) * span;
}
LOFP_KL_HD inline int64_t key_hull_hi_offset(int64_t stride, int span)
{
    return 2 * stride * (int64_t)span;
}

// What the host keeps per circuit about the layout.
struct KeyLayoutState {
    int64_t stride = 0;   // rows per half laid out (0: none yet)
    int span = 0;         // ints per hull row of that layout
    bool clean = false;   // every row of the layout empty, counts zero
};

// What one call must do before its insert kernel.
struct KeyLayoutPlan {
    int64_t stride;       // rows per half for this call (>= cap)
    bool clear;           // set every row of the layout empty first
    size_t table_bytes;   // uint64 [2][stride]
    size_t slot_key_bytes;// int32 [2][stride]
    size_t hull_bytes;    // int32 [2 (lo, hi)][2][stride][span]
};

// Plan a call with probe capacity cap (a power of two) and hull rows of span
// ints.  A larger capacity or another span lays the buffers out anew (they
// are then cleared whatever their allocation holds); otherwise the call uses
// the existing layout and clears it only if an earlier call stopped before
// emptying it.  The caller marks the state unclean when it launches the
// insert kernel and clean again once the kernel that empties the rows it
// claimed is enqueued.
inline KeyLayoutPlan plan_key_layout(KeyLayoutState &st, int64_t cap, int span)
{
    if (cap > st.stride || span != st.span) {
        st.stride = cap > st.stride ? cap : st.stride;
        st.span = span;
        st.clean = false;
    }
    KeyLayoutPlan p;
    p.stride = st.stride;
    p.clear = !st.clean;
    p.table_bytes = (size_t)2 * (size_t)st.stride * sizeof(unsigned long long);
    p.slot_key_bytes = (size_t)2 * (size_t)st.stride * sizeof(int32_t);
    p.hull_bytes = (size_t)2 * (size_t)key_hull_hi_offset(st.stride, span) * sizeof(int32_t);
    return p;
}

}  // namespace lofp
