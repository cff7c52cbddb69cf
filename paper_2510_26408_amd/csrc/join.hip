// join.hip -- the join of a split contraction (Sec. II.C): each pattern's
// amplitude as the sum, over the versions of the cuts that cross the split,
// of the product of its top-half and bottom-half key states.
#include <utility>

#include "lofp_device.h"

namespace lofp {

// Join of a split contraction, one wave per pattern: the sum over the
// pattern's own box of crossing versions of TOP(versions) * BOT(versions),
// each state addressed by value through its key's interval layout.  Both
// states list the crossing versions in the same order, so neighbouring lanes
// read neighbouring entries of both.  Boxes hold hundreds to a few thousand
// entries (580 on average for 16 modes, 8 photons, depth 8); the reads of
// the two states, written by other XCDs in the contraction kernel, mostly
// miss L2 and bound the kernel, so the per-entry index work is kept small
// (see the loop).
// NS: the number of crossing versions (a compile-time count, so the set-up
// loads are all issued together and the digit loops have no branches).
constexpr int kJoinWaves = 4;
constexpr int kJoinBlock = 64 * kJoinWaves;
template <int NS>
__global__ __launch_bounds__(kJoinBlock) void k_join(JoinArgs g)
{
    if (g.split_flag && !*g.split_flag) return;   // contracted per pattern instead
    const int p = blockIdx.x * kJoinWaves + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (p >= g.B) return;
    const int nc = g.m - 1, span = (g.D + 1) * nc;
    if (g.infeasible[p]) {
        if (lane == 0) g.out[p] = make_double2(0.0, 0.0);
        return;
    }
    const int tk = g.slot_key[key_slot_index(0, g.stride, g.slot[p])];
    const int bk = g.slot_key[key_slot_index(1, g.stride, g.slot[g.B + p])];
    const int16_t *plo = g.lo + (int64_t)p * span, *phi = g.hi + (int64_t)p * span;
    const int16_t *tlo = g.tlo + (int64_t)tk * span, *thi = g.thi + (int64_t)tk * span;
    const int16_t *blo = g.blo + (int64_t)bk * span, *bhi = g.bhi + (int64_t)bk * span;
    // per crossing variable (both states in the top order): pattern box,
    // top stride/offset, bottom stride/offset
    int pl[NS > 0 ? NS : 1], ph[NS > 0 ? NS : 1], tl[NS > 0 ? NS : 1], th[NS > 0 ? NS : 1];
    int bl[NS > 0 ? NS : 1], bh[NS > 0 ? NS : 1];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int i = g.cidx[q];
        pl[q] = plo[i]; ph[q] = phi[i]; tl[q] = tlo[i]; th[q] = thi[i]; bl[q] = blo[i]; bh[q] = bhi[i];
    }
    int pstr[NS > 0 ? NS : 1], toff[NS > 0 ? NS : 1], tstr[NS > 0 ? NS : 1], boff[NS > 0 ? NS : 1];
    int bstr[NS > 0 ? NS : 1];
    float pinv[NS > 0 ? NS : 1];
    int box = 1;
    int64_t ts = 1, bs = 1;
    bool fits = !g.top_ovf[tk] && !g.bot_ovf[bk];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        pstr[q] = box;
        pinv[q] = 1.0f / (float)box;
        toff[q] = pl[q] - tl[q];          // state digit = pattern digit + offset
        boff[q] = pl[q] - bl[q];
        tstr[q] = (int)ts;
        bstr[q] = (int)bs;
        ts *= th[q] >= tl[q] ? th[q] - tl[q] + 1 : 0;
        bs *= bh[q] >= bl[q] ? bh[q] - bl[q] + 1 : 0;
        ts = ts < (1LL << 40) ? ts : (1LL << 40);
        bs = bs < (1LL << 40) ? bs : (1LL << 40);
        box *= ph[q] >= pl[q] ? ph[q] - pl[q] + 1 : 0;
        box = box < (1 << 30) ? box : (1 << 30);
        // a feasible pattern's box lies inside both keys' boxes (each key's
        // box is the hull of its members' boxes)
        fits = fits && (ph[q] < pl[q] || (pl[q] >= tl[q] && ph[q] <= th[q] && pl[q] >= bl[q] && ph[q] <= bh[q]));
    }
    // both states must be as large as their keys' boxes say
    fits = fits && ts <= g.state_cap && bs <= g.state_cap;
    if (!fits) {
        if (lane == 0) g.out[p] = nan2();
        return;
    }
    const gdouble *TS = (const gdouble *)(g.top_state + (int64_t)tk * g.state_cap);
    const gdouble *BS_ = (const gdouble *)(g.bot_state + (int64_t)bk * g.state_cap);
    // Lane l takes entries l, l + 64, ...: its first entry is decoded once,
    // then each step adds 64 in the box's mixed radix digit by digit (inc:
    // the digits of 64), moving both state indices by selected constants
    // instead of a decode per entry.
    int rad[NS > 0 ? NS : 1], inc[NS > 0 ? NS : 1], dg[NS > 0 ? NS : 1];
    int tinc[NS > 0 ? NS : 1], twrap[NS > 0 ? NS : 1], binc[NS > 0 ? NS : 1], bwrap[NS > 0 ? NS : 1];
    int ti = 0, bi = 0;
    {
        int rem = lane;
#pragma unroll
        for (int q = NS - 1; q >= 0; --q) {
            rad[q] = ph[q] - pl[q] + 1;
            const int d = q > 0 ? qdiv(rem, pstr[q], pinv[q]) : rem;
            rem -= d * pstr[q];
            dg[q] = d;
            ti += (d + toff[q]) * tstr[q];
            bi += (d + boff[q]) * bstr[q];
            const int hi64 = q > 0 ? qdiv(64, pstr[q], pinv[q]) : 64;
            const int up = q + 1 < NS ? qdiv(64, pstr[q + 1 < NS ? q + 1 : q], pinv[q + 1 < NS ? q + 1 : q]) : 0;
            inc[q] = hi64 - rad[q] * up;
            tinc[q] = inc[q] * tstr[q];
            twrap[q] = rad[q] * tstr[q];
            binc[q] = inc[q] * bstr[q];
            bwrap[q] = rad[q] * bstr[q];
        }
    }
    CSum sr{0.0, 0.0}, si{0.0, 0.0};
#pragma unroll 2
    for (int e = lane; e < box; e += 64) {
        const double2 c = cmul(make_double2(TS[2 * ti], TS[2 * ti + 1]), make_double2(BS_[2 * bi], BS_[2 * bi + 1]));
        csum_add(sr, c.x);
        csum_add(si, c.y);
        bool carry = false;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int d = dg[q] + inc[q] + (carry ? 1 : 0);
            const bool w = d >= rad[q];
            dg[q] = w ? d - rad[q] : d;
            ti += tinc[q] + (carry ? tstr[q] : 0) - (w ? twrap[q] : 0);
            bi += binc[q] + (carry ? bstr[q] : 0) - (w ? bwrap[q] : 0);
            carry = w;
        }
    }
    // the lanes' partial sums, merged in a fixed butterfly order
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        CSum b{__shfl_xor(sr.s, off, 64), __shfl_xor(sr.c, off, 64)};
        CSum c{__shfl_xor(si.s, off, 64), __shfl_xor(si.c, off, 64)};
        if (lane & off) { CSum t = sr; sr = b; b = t; t = si; si = c; c = t; }
        csum_merge(sr, b);
        csum_merge(si, c);
    }
    if (lane == 0) g.out[p] = make_double2(sr.s + sr.c, si.s + si.c);
}

template <int... N>
static void launch_join_ns(const JoinArgs &a, hipStream_t stream, std::integer_sequence<int, N...>)
{
    using K = void (*)(JoinArgs);
    static const K table[] = {k_join<N>...};
    hipLaunchKernelGGL(table[a.nshared], dim3((a.B + kJoinWaves - 1) / kJoinWaves), dim3(kJoinBlock), 0, stream, a);
}

hipError_t launch_join(const JoinArgs &a, hipStream_t stream)
{
    if (a.B == 0) return hipSuccess;
    if (a.nshared < 0 || a.nshared > kMaxActive) return hipErrorInvalidValue;
    launch_join_ns(a, stream, std::make_integer_sequence<int, kMaxActive + 1>{});
    return hipGetLastError();
}

}  // namespace lofp
