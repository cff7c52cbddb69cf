// lofp_core.h -- host/device logic shared by the planner and the kernels.
//
// Representation.  A Fock configuration of m modes holding n photons is kept as
// its m-1 cut values A(r) = number of photons in modes 0..r (r = 0..m-2), with
// A(-1) = 0 and A(m-1) = n implied.  Occupations are A(r) - A(r-1) >= 0, so a
// configuration is a nondecreasing sequence.  A beam splitter on modes
// (a, a+1) changes only A(a): photon conservation at the splitter (Sec. II,
// "valid path") leaves every other cut untouched.  Its inputs are
// x1 = A(a) - A(a-1), x2 = A(a+1) - A(a) and its outputs y1 = A'(a) - A(a-1),
// y2 = A(a+1) - A'(a).
//
// Valid paths (Eq. (1)) are therefore the sequences of nondecreasing cut
// vectors A_0 = prefix(S), ..., A_D = prefix(T) in which a cut only changes in
// a layer that has a beam splitter on it.  The light cones of Sec. II.B give
// starting intervals lo_t(r) <= A_t(r) <= hi_t(r); propagating the two
// constraint kinds above (order between neighbouring cuts, equality across a
// layer without a splitter on the cut) tightens them.  Both constraint kinds
// are closed under max and min, so after propagation every value left in an
// interval lies on some valid path.
//
// State spaces.  Between beam splitters ("stages") each cut sits at a known
// time, so the configurations of a stage are the nondecreasing sequences with
// A(r) in [L(r), H(r)].  They are ranked densely in lexicographic order by
//   rank(A) = sum_r ( C[r][A(r)] - C[r][A(r-1)] ),
// C[r][v] = number of valid sequences that agree on cuts < r and have
// L(r) <= A(r) < v, summed over completions; equivalently
//   rank(A) = sum_r E[r][A(r)],  E[r][v] = C[r][v] - C[r+1][v]  (C[m-1] = 0).
// Dense ranks let merged frontiers live in flat arrays with no hashing or
// sorting, and let a kernel find any neighbour configuration's slot with one
// table lookup per changed cut.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define LOFP_HD __host__ __device__ inline

namespace lofp {

constexpr int kMaxModes = 32;
constexpr int kMaxCuts = kMaxModes - 1;
constexpr int kMaxPhotons = 64;

// Offset of photon-number sector N inside one beam splitter's table:
// sum_{k<N} (k+1)^2.
LOFP_HD int sector_offset(int N) { return N * (N + 1) * (2 * N + 1) / 6; }

// Row stride of the per-stage tables C and E (values v = 0..n+1).
LOFP_HD int table_cols(int n) { return n + 2; }

// ---------------------------------------------------------------- bounds
// lo/hi: (D+1) x (m-1) arrays, row t = after t layers.  cut_gate[t*(m-1)+r]
// is nonzero when layer t has a beam splitter on cut r.  On entry lo/hi hold
// the light-cone intervals (or 0..n); on exit they are propagated to the
// fixed point.  Returns 1 if some interval is empty (no valid path), else 0.
//
// The passes run until one changes nothing.  They terminate: every value
// lies in [0, n] (the light-cone sums are photon counts, and the first pass
// clamps the ends), lower bounds only grow and upper bounds only shrink, so
// a pass that changes something moves one of the 2 (D+1)(m-1) values by at
// least one, which can happen at most 2 (D+1)(m-1) n times.
LOFP_HD int bound_pass_limit(int m, int D, int n) { return 2 * (D + 1) * (m - 1) * (n + 1) + 2; }

LOFP_HD int propagate_bounds(int m, int D, int n, const uint8_t *cut_gate, int16_t *lo, int16_t *hi)
{
    const int nc = m - 1;
    const int limit = bound_pass_limit(m, D, n);
    for (int it = 0; it < limit; ++it) {
        int changed = 0;
        for (int t = 0; t <= D; ++t) {
            int16_t *L = lo + t * nc, *H = hi + t * nc;
            if (L[0] < 0) { L[0] = 0; changed = 1; }
            if (H[nc - 1] > n) { H[nc - 1] = (int16_t)n; changed = 1; }
            for (int r = 1; r < nc; ++r)
                if (L[r] < L[r - 1]) { L[r] = L[r - 1]; changed = 1; }
            for (int r = nc - 2; r >= 0; --r)
                if (H[r] > H[r + 1]) { H[r] = H[r + 1]; changed = 1; }
        }
        for (int t = 0; t < D; ++t) {
            for (int r = 0; r < nc; ++r) {
                if (cut_gate[t * nc + r]) continue;
                int16_t &l0 = lo[t * nc + r], &l1 = lo[(t + 1) * nc + r];
                int16_t &h0 = hi[t * nc + r], &h1 = hi[(t + 1) * nc + r];
                int16_t l = l0 > l1 ? l0 : l1, h = h0 < h1 ? h0 : h1;
                if (l != l0 || l != l1 || h != h0 || h != h1) { l0 = l1 = l; h0 = h1 = h; changed = 1; }
            }
        }
        if (!changed) break;
    }
    for (int i = 0; i < (D + 1) * nc; ++i)
        if (lo[i] > hi[i]) return 1;
    return 0;
}

// Light-cone starting intervals from the photons of S (forward reach) and of T
// (backward reach).  fr_lo/fr_hi[t*m+s]: modes that input mode s can reach
// after t layers; br_lo/br_hi[t*m+o]: modes after t layers from which output
// mode o can be reached.  A photon whose reach lies wholly in modes <= r is
// certainly counted by A_t(r); one whose reach starts above r certainly is not.
LOFP_HD void light_cone_bounds(int m, int D, const int32_t *S, const int32_t *T, const int8_t *fr_lo,
                               const int8_t *fr_hi, const int8_t *br_lo, const int8_t *br_hi,
                               int16_t *lo, int16_t *hi)
{
    const int nc = m - 1;
    for (int t = 0; t <= D; ++t) {
        for (int r = 0; r < nc; ++r) {
            int ls = 0, hs = 0, lt = 0, ht = 0;
            for (int s = 0; s < m; ++s) {
                int x = S[s], y = T[s];
                if (fr_hi[t * m + s] <= r) ls += x;
                if (fr_lo[t * m + s] <= r) hs += x;
                if (br_hi[t * m + s] <= r) lt += y;
                if (br_lo[t * m + s] <= r) ht += y;
            }
            lo[t * nc + r] = (int16_t)(ls > lt ? ls : lt);
            hi[t * nc + r] = (int16_t)(hs < ht ? hs : ht);
        }
    }
}

// ------------------------------------------------------------ state spaces
// Interval of cut r at a stage: the time index of the cut is stage_time[r].
// C, E: (m-1) x (n+2) int32, row-major by cut.  Returns the number of states
// (or -1 if it exceeds 2^31-1).
LOFP_HD int64_t build_stage_tables(int m, int n, const uint8_t *stage_time, const int16_t *lo,
                                   const int16_t *hi, int32_t *C, int32_t *E)
{
    const int nc = m - 1, W = table_cols(n);
    int64_t tot_next = 1;  // completions beyond the last cut: A(m-1) = n is fixed
    for (int r = nc - 1; r >= 0; --r) {
        const int t = stage_time[r];
        const int L = lo[t * nc + r], H = hi[t * nc + r];
        int32_t *Cr = C + r * W;
        const int32_t *Cn = (r + 1 < nc) ? C + (r + 1) * W : nullptr;
        int64_t run = 0;
        for (int v = 0; v <= n + 1; ++v) {
            Cr[v] = (int32_t)run;
            if (v >= L && v <= H) {
                int64_t c = (r + 1 < nc) ? (tot_next - (int64_t)Cn[v]) : 1;
                run += c;
                if (run > 0x7fffffffLL) return -1;
            }
        }
        tot_next = run;
    }
    for (int r = 0; r < nc; ++r)
        for (int v = 0; v <= n + 1; ++v)
            E[r * W + v] = C[r * W + v] - ((r + 1 < nc) ? C[(r + 1) * W + v] : 0);
    return tot_next;
}

// Unrank a dense index into cut values (A[r] for r < m-1) given the stage's C
// table and intervals.
LOFP_HD void unrank_state(int m, int n, const uint8_t *stage_time, const int16_t *lo, const int16_t *hi,
                          const int32_t *C, int64_t idx, uint8_t *A)
{
    const int nc = m - 1, W = table_cols(n);
    int prev = 0;
    for (int r = 0; r < nc; ++r) {
        const int t = stage_time[r];
        const int L = lo[t * nc + r], H = hi[t * nc + r];
        const int32_t *Cr = C + r * W;
        const int64_t base = Cr[prev];
        int v = prev > L ? prev : L;
        while (v < H && (int64_t)Cr[v + 1] - base <= idx) ++v;
        idx -= (int64_t)Cr[v] - base;
        A[r] = (uint8_t)v;
        prev = v;
    }
}

LOFP_HD int64_t rank_state(int m, int n, const int32_t *E, const uint8_t *A)
{
    const int W = table_cols(n);
    int64_t s = 0;
    for (int r = 0; r < m - 1; ++r) s += E[r * W + A[r]];
    return s;
}

}  // namespace lofp
