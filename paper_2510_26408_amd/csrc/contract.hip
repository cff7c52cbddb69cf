// contract.hip -- mode-axis contraction of the path sum (Sec. II.C).
//
// The paper cuts the circuit into horizontal contraction blocks and carries,
// from one block to the next, the photon numbers of the waveguides crossing
// the boundary together with their summed amplitudes.  Here the boundary
// between modes r and r+1 is the cut r, and what crosses it over the whole
// circuit is the sequence of values A_t(r): it changes only at the beam
// splitters on that cut, so the state of cut r is the tuple of its values
// between consecutive splitters (its "versions"; the first is fixed by S, the
// last by T).  In a brickwork circuit a cut changes once per block of two
// layers.  A beam splitter on cut r reads the current versions of cuts r-1,
// r and r+1, so the sweep keeps the pair (state of cut r-1, state of cut r):
//
//   V_{r+1}(a_r, a_{r+1}) = sum_{a_{r-1}} V_r(a_{r-1}, a_r) Phi_r(a_{r-1}, a_r, a_{r+1})
//
// where Phi_r is the product of the transition amplitudes of every splitter on
// cut r, and pairs that violate the order A_t(r) <= A_t(r+1) at some time are
// zero.  The amplitude is the sum of V after the last cut.  With unit weights
// the same sweep counts the valid paths.
//
// One 256-thread block per pattern; V lives in a per-pattern global workspace
// (two buffers), each step is one pass over the target pairs, and the final
// sum is compensated and done in a fixed order.
#include "lofp_device.h"

namespace lofp {

constexpr int kMaxVer = 16;  // versions per cut (splitters on one cut + 1)

struct CutState {
    int nv;               // number of versions (gates on the cut + 1)
    int val[kMaxVer];     // value of each version
};

// Decode the state index of cut r (mixed radix over the free versions, first
// free version fastest).  Versions 0 and nv-1 are fixed by S and T.
__device__ __forceinline__ void decode_cut(const ContractArgs &g, int r, int idx, int spre, int tpre,
                                           const int16_t *lo, const int16_t *hi, CutState &cs)
{
    const int nc = g.m - 1;
    if (r < 0 || r >= nc) {
        cs.nv = 1;
        cs.val[0] = r < 0 ? 0 : g.n;
        return;
    }
    const int k = g.cut_ngates[r];
    cs.nv = k + 1;
    cs.val[0] = spre;
#pragma unroll
    for (int j = 1; j < kMaxVer; ++j) {
        if (j < k) {
            const int t = g.gate_layer[g.cut_gates[r * g.D + j - 1]] + 1;
            const int L = lo[t * nc + r], H = hi[t * nc + r];
            const int rad = H - L + 1;
            const int q = idx / rad;
            cs.val[j] = L + (idx - q * rad);
            idx = q;
        }
    }
    if (k > 0) cs.val[k] = tpre;
}

__device__ __forceinline__ int cut_domain(const ContractArgs &g, int r, const int16_t *lo, const int16_t *hi)
{
    const int nc = g.m - 1;
    if (r < 0 || r >= nc) return 1;
    const int k = g.cut_ngates[r];
    int dom = 1;
    for (int j = 1; j < k; ++j) {
        const int t = g.gate_layer[g.cut_gates[r * g.D + j - 1]] + 1;
        const int rad = hi[t * nc + r] - lo[t * nc + r] + 1;
        dom *= rad > 0 ? rad : 0;
    }
    return dom;
}

// value of cut (r) at time t, from its decoded versions
__device__ __forceinline__ int value_at(const ContractArgs &g, int r, int t, const CutState &cs)
{
    const int nc = g.m - 1;
    if (r < 0) return 0;
    if (r >= nc) return g.n;
    return cs.val[g.ver_at[t * nc + r]];
}

__device__ __forceinline__ bool ordered(const ContractArgs &g, int r, const CutState &lo_c, const CutState &hi_c)
{
    // A_t(r) <= A_t(r+1) for every time t
    for (int t = 0; t <= g.D; ++t)
        if (value_at(g, r, t, lo_c) > value_at(g, r + 1, t, hi_c)) return false;
    return true;
}

template <bool COUNT>
__global__ __launch_bounds__(256) void k_contract(ContractArgs g)
{
    const int p = blockIdx.x;
    const int nc = g.m - 1, span = (g.D + 1) * nc;
    const int16_t *lo = g.lo + (int64_t)p * span, *hi = g.hi + (int64_t)p * span;
    const int32_t *Tp = g.T + (int64_t)p * g.m;
    double2 *bufA = g.ws + (int64_t)p * 2 * g.max_states;
    double2 *bufB = bufA + g.max_states;
    __shared__ CSum part[2][4];
    if (g.infeasible[p]) {
        if (threadIdx.x == 0) g.out[p] = make_double2(0.0, 0.0);
        return;
    }
    // prefix sums of S and T for the fixed versions
    __shared__ int spre[kMaxCuts + 1], tpre[kMaxCuts + 1];
    if (threadIdx.x == 0) {
        int s = 0, t = 0;
        for (int r = 0; r < nc; ++r) { s += g.S[r]; t += Tp[r]; spre[r] = s; tpre[r] = t; }
    }
    __syncthreads();

    // V_0(a_{-1}, a_0) = 1 on every state of cut 0 (cut -1 has one state)
    int dom_prev = 1, dom_cur = cut_domain(g, 0, lo, hi);
    if ((int64_t)dom_prev * dom_cur > g.max_states) { if (threadIdx.x == 0) atomicOr(g.overflow, 1); return; }
    for (int i = threadIdx.x; i < dom_cur; i += blockDim.x) bufA[i] = make_double2(1.0, 0.0);
    __syncthreads();
    unsigned long long trans = 0;

    for (int r = 0; r < nc; ++r) {
        const int dom_next = cut_domain(g, r + 1, lo, hi);
        const int64_t ntgt = (int64_t)dom_cur * dom_next;
        if (ntgt > g.max_states) { if (threadIdx.x == 0) atomicOr(g.overflow, 1); return; }
        const int k = g.cut_ngates[r];
        for (int64_t q = threadIdx.x; q < ntgt; q += blockDim.x) {
            const int ar = (int)(q / dom_next), an = (int)(q - (int64_t)ar * dom_next);
            CutState cr, cn, cp;
            decode_cut(g, r, ar, spre[r], tpre[r], lo, hi, cr);
            decode_cut(g, r + 1, an, r + 1 < nc ? spre[r + 1] : 0, r + 1 < nc ? tpre[r + 1] : 0, lo, hi, cn);
            double2 acc = make_double2(0.0, 0.0);
            if (ordered(g, r, cr, cn)) {
                for (int ap = 0; ap < dom_prev; ++ap) {
                    const double2 vprev = bufA[(int64_t)ap * dom_cur + ar];
                    if (vprev.x == 0.0 && vprev.y == 0.0) continue;
                    decode_cut(g, r - 1, ap, r > 0 ? spre[r - 1] : 0, r > 0 ? tpre[r - 1] : 0, lo, hi, cp);
                    double2 phi = make_double2(1.0, 0.0);
                    bool ok = true;
                    for (int j = 1; j <= k; ++j) {
                        const int gid = g.cut_gates[r * g.D + j - 1];
                        const int l = g.gate_layer[gid];
                        const int vm = value_at(g, r - 1, l, cp), vp = value_at(g, r + 1, l, cn);
                        const int x1 = cr.val[j - 1] - vm, y1 = cr.val[j] - vm, N = vp - vm;
                        if (x1 < 0 || y1 < 0 || x1 > N || y1 > N) { ok = false; break; }
                        if (!COUNT)
                            phi = cmul(phi, g.table[(int64_t)gid * g.tab_stride + sector_offset(N) + x1 * (N + 1) + y1]);
                    }
                    if (!ok) continue;
                    ++trans;
                    acc = COUNT ? make_double2(acc.x + vprev.x, 0.0) : cfma(vprev, phi, acc);
                }
            }
            bufB[q] = acc;
        }
        __syncthreads();
        double2 *t = bufA; bufA = bufB; bufB = t;
        dom_prev = dom_cur;
        dom_cur = dom_next;
    }
    // amplitude = sum over the states of cut m-2 (cut m-1 has one state)
    CSum sr{0.0, 0.0}, si{0.0, 0.0};
    for (int i = threadIdx.x; i < dom_prev; i += blockDim.x) {
        const double2 x = bufA[i];
        csum_add(sr, x.x);
        csum_add(si, x.y);
    }
    // fixed-order block combine
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        CSum b{__shfl_xor(sr.s, off, 64), __shfl_xor(sr.c, off, 64)};
        CSum c{__shfl_xor(si.s, off, 64), __shfl_xor(si.c, off, 64)};
        if (threadIdx.x & off) { CSum t = sr; sr = b; b = t; t = si; si = c; c = t; }
        csum_merge(sr, b);
        csum_merge(si, c);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { part[0][wv] = sr; part[1][wv] = si; }
    __syncthreads();
    if (threadIdx.x == 0) {
        CSum a = part[0][0], b = part[1][0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) { csum_merge(a, part[0][w]); csum_merge(b, part[1][w]); }
        g.out[p] = make_double2(a.s + a.c, b.s + b.c);
    }
    atomicAdd(g.stat_transitions, trans);
}

hipError_t launch_contract(const ContractArgs &a, hipStream_t stream)
{
    if (a.B == 0) return hipSuccess;
    if (a.count_only) hipLaunchKernelGGL((k_contract<true>), dim3(a.B), dim3(256), 0, stream, a);
    else hipLaunchKernelGGL((k_contract<false>), dim3(a.B), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace lofp
