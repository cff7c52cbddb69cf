// plan.hip -- per-pattern cut bounds (light cones of Sec. II.B tightened by
// photon conservation) and the dense rank tables of every needed stage.
#include "lofp_device.h"

namespace lofp {

// One wave per pattern.  The light-cone intervals of every (time, cut) are
// computed in parallel into LDS; the propagation then alternates row passes
// (order between neighbouring cuts: prefix max / suffix min, one lane per
// time) and column passes (equality across layers without a splitter on the
// cut, one lane per cut) until nothing changes.
constexpr int kBoundsLds = 4096;   // int16 entries per array: (D+1)(m-1) <= 4096

// Bounds of one pattern by one 64-thread wave: light cones into LDS, then
// row and column passes until nothing changes (a wave vote decides).  S and
// Tp: this pattern's input and output; results to Lg/Hg and *inf.
__device__ void bounds_wave(int m, int D, int n, const int32_t *__restrict__ S, const int32_t *__restrict__ Tp,
                            const int8_t *__restrict__ fr_lo, const int8_t *__restrict__ fr_hi,
                            const int8_t *__restrict__ br_lo, const int8_t *__restrict__ br_hi,
                            const uint8_t *__restrict__ cut_gate, int16_t *__restrict__ Lg, int16_t *__restrict__ Hg,
                            int32_t *__restrict__ inf)
{
    // the two interval arrays in dynamic LDS sized to the largest span of
    // the launch (a few hundred bytes), so a CU holds as many waves as it can
    extern __shared__ int16_t bounds_lds[];
    const int nc_ = m - 1, span_ = (D + 1) * nc_;
    int16_t *L = bounds_lds, *H = bounds_lds + span_;
    __shared__ int sS[kMaxModes], sT[kMaxModes];
    __shared__ int s_bad;
    const int tid = threadIdx.x;
    const int nc = m - 1, span = (D + 1) * nc;
    if (tid == 0) {
        int nT = 0, bad = 0;
        for (int i = 0; i < m; ++i) { nT += Tp[i]; bad |= Tp[i] < 0; sS[i] = S[i]; sT[i] = Tp[i]; }
        s_bad = bad || nT != n;
    }
    __syncthreads();
    if (s_bad) {
        for (int i = tid; i < span; i += 64) { Lg[i] = 1; Hg[i] = 0; }
        if (tid == 0) *inf = 1;
        return;
    }
    for (int i = tid; i < span; i += 64) {
        const int t = i / nc, r = i - t * nc;
        int ls = 0, hs = 0, lt = 0, ht = 0;
        for (int s = 0; s < m; ++s) {
            const int x = sS[s], y = sT[s];
            ls += fr_hi[t * m + s] <= r ? x : 0;
            hs += fr_lo[t * m + s] <= r ? x : 0;
            lt += br_hi[t * m + s] <= r ? y : 0;
            ht += br_lo[t * m + s] <= r ? y : 0;
        }
        int l = ls > lt ? ls : lt, h = hs < ht ? hs : ht;
        l = l < 0 ? 0 : l;
        h = h > n ? n : h;
        L[i] = (int16_t)l;
        H[i] = (int16_t)h;
    }
    __syncthreads();
    // until a pass changes nothing (bound_pass_limit is never reached: it
    // bounds how many passes can change a value)
    const int limit = bound_pass_limit(m, D, n);
    for (int it = 0; it < limit; ++it) {
        int ch = 0;
        for (int t = tid; t <= D; t += 64) {          // rows: order between cuts
            int16_t *Lr = L + t * nc, *Hr = H + t * nc;
            for (int r = 1; r < nc; ++r)
                if (Lr[r] < Lr[r - 1]) { Lr[r] = Lr[r - 1]; ch = 1; }
            for (int r = nc - 2; r >= 0; --r)
                if (Hr[r] > Hr[r + 1]) { Hr[r] = Hr[r + 1]; ch = 1; }
        }
        __syncthreads();
        for (int r = tid; r < nc; r += 64) {          // columns: no splitter, no change
            for (int t = 0; t < D; ++t) {
                if (cut_gate[t * nc + r]) continue;
                const int a = t * nc + r, b = a + nc;
                const int16_t l = L[a] > L[b] ? L[a] : L[b], h = H[a] < H[b] ? H[a] : H[b];
                if (l != L[a] || l != L[b] || h != H[a] || h != H[b]) { L[a] = L[b] = l; H[a] = H[b] = h; ch = 1; }
            }
            for (int t = D - 1; t >= 0; --t) {
                if (cut_gate[t * nc + r]) continue;
                const int a = t * nc + r, b = a + nc;
                const int16_t l = L[a] > L[b] ? L[a] : L[b], h = H[a] < H[b] ? H[a] : H[b];
                if (l != L[a] || l != L[b] || h != H[a] || h != H[b]) { L[a] = L[b] = l; H[a] = H[b] = h; ch = 1; }
            }
        }
        __syncthreads();
        // the block is one wave: a wave vote gives every lane the same answer
        if (!__any(ch)) break;
    }
    int bad = 0;
    for (int i = tid; i < span; i += 64) {
        Lg[i] = L[i];
        Hg[i] = H[i];
        bad |= L[i] > H[i];
    }
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();
    if (tid == 0) *inf = s_bad;
}

__global__ __launch_bounds__(64) void k_bounds(int B, int m, int D, int n, const int32_t *__restrict__ S,
                                               const int32_t *__restrict__ T, const int8_t *__restrict__ fr_lo,
                                               const int8_t *__restrict__ fr_hi, const int8_t *__restrict__ br_lo,
                                               const int8_t *__restrict__ br_hi, const uint8_t *__restrict__ cut_gate,
                                               int16_t *__restrict__ lo, int16_t *__restrict__ hi,
                                               int32_t *__restrict__ infeasible)
{
    const int p = blockIdx.x;
    const int span = (D + 1) * (m - 1);
    bounds_wave(m, D, n, S, T + (int64_t)p * m, fr_lo, fr_hi, br_lo, br_hi, cut_gate, lo + (int64_t)p * span,
                hi + (int64_t)p * span, infeasible + p);
}

// Fallback for circuits with more than 4096 (time, cut) entries: one thread
// per pattern on global memory.
__global__ void k_bounds_big(int B, int m, int D, int n, const int32_t *__restrict__ S,
                             const int32_t *__restrict__ T, const int8_t *__restrict__ fr_lo,
                             const int8_t *__restrict__ fr_hi, const int8_t *__restrict__ br_lo,
                             const int8_t *__restrict__ br_hi, const uint8_t *__restrict__ cut_gate,
                             int16_t *__restrict__ lo, int16_t *__restrict__ hi, int32_t *__restrict__ infeasible)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= B) return;
    const int nc = m - 1, span = (D + 1) * nc;
    const int32_t *Tp = T + (int64_t)p * m;
    int16_t *L = lo + (int64_t)p * span, *H = hi + (int64_t)p * span;
    int nT = 0, bad = 0;
    for (int i = 0; i < m; ++i) { nT += Tp[i]; bad |= Tp[i] < 0; }
    if (bad || nT != n) {
        for (int i = 0; i < span; ++i) { L[i] = 1; H[i] = 0; }
        infeasible[p] = 1;
        return;
    }
    light_cone_bounds(m, D, S, Tp, fr_lo, fr_hi, br_lo, br_hi, L, H);
    infeasible[p] = propagate_bounds(m, D, n, cut_gate, L, H);
}

hipError_t launch_bounds(int B, int m, int D, int n, const int32_t *S, const int32_t *T,
                         const int8_t *fr_lo, const int8_t *fr_hi, const int8_t *br_lo,
                         const int8_t *br_hi, const uint8_t *cut_gate, int16_t *lo, int16_t *hi,
                         int32_t *infeasible, hipStream_t stream)
{
    if (B == 0) return hipSuccess;
    const int span = (D + 1) * (m - 1);
    if (span <= kBoundsLds) {
        hipLaunchKernelGGL(k_bounds, dim3(B), dim3(64), (size_t)2 * span * sizeof(int16_t), stream, B, m, D, n, S,
                           T, fr_lo, fr_hi, br_lo, br_hi, cut_gate, lo, hi, infeasible);
    } else {
        hipLaunchKernelGGL(k_bounds_big, dim3((B + 63) / 64), dim3(64), 0, stream, B, m, D, n, S, T, fr_lo, fr_hi,
                           br_lo, br_hi, cut_gate, lo, hi, infeasible);
    }
    return hipGetLastError();
}

// One wave per job of a multi-circuit batch (a job whose (time, cut) grid
// exceeds the LDS arrays is propagated by one thread on global memory).
__global__ __launch_bounds__(64) void k_bounds_multi(int count, const BoundsJob *__restrict__ jobs)
{
    const BoundsJob j = jobs[blockIdx.x];
    const int nc = j.m - 1, span = (j.D + 1) * nc;
    if (span <= kBoundsLds) {
        bounds_wave(j.m, j.D, j.n, j.S, j.T, j.fr_lo, j.fr_hi, j.br_lo, j.br_hi, j.cut_gate, j.lo, j.hi,
                    j.infeasible);
        return;
    }
    if (threadIdx.x != 0) return;
    int nT = 0, bad = 0;
    for (int k = 0; k < j.m; ++k) { nT += j.T[k]; bad |= j.T[k] < 0; }
    if (bad || nT != j.n) {
        for (int k = 0; k < span; ++k) { j.lo[k] = 1; j.hi[k] = 0; }
        *j.infeasible = 1;
        return;
    }
    light_cone_bounds(j.m, j.D, j.S, j.T, j.fr_lo, j.fr_hi, j.br_lo, j.br_hi, j.lo, j.hi);
    *j.infeasible = propagate_bounds(j.m, j.D, j.n, j.cut_gate, j.lo, j.hi);
}

hipError_t launch_bounds_multi(int count, const BoundsJob *jobs, int max_span, hipStream_t stream)
{
    if (count == 0) return hipSuccess;
    const int lds_span = max_span < kBoundsLds ? max_span : kBoundsLds;
    hipLaunchKernelGGL(k_bounds_multi, dim3(count), dim3(64), (size_t)2 * lds_span * sizeof(int16_t), stream, count,
                       jobs);
    return hipGetLastError();
}

// One thread per (stage slot, pattern).
__global__ void k_stage_tables(int B, int m, int D, int n, int nslots, const int32_t *__restrict__ slot_stage,
                               const uint8_t *__restrict__ stage_time, const int16_t *__restrict__ lo,
                               const int16_t *__restrict__ hi, const int32_t *__restrict__ infeasible,
                               int32_t *__restrict__ C, int32_t *__restrict__ E, int32_t *__restrict__ count,
                               int32_t *__restrict__ overflow)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)nslots * B) return;
    const int slot = (int)(k / B), p = (int)(k - (int64_t)slot * B);
    const int nc = m - 1, span = (D + 1) * nc, tsz = nc * table_cols(n);
    const int s = slot_stage[slot];
    int32_t *Cp = C + k * tsz, *Ep = E + k * tsz;
    if (infeasible[p]) {
        for (int i = 0; i < tsz; ++i) { Cp[i] = 0; Ep[i] = 0; }
        count[k] = 0;
        return;
    }
    const int64_t c = build_stage_tables(m, n, stage_time + (int64_t)s * nc, lo + (int64_t)p * span,
                                         hi + (int64_t)p * span, Cp, Ep);
    if (c < 0) { atomicOr(overflow, 1); count[k] = -1; return; }
    count[k] = (int32_t)c;
}

hipError_t launch_stage_tables(int B, int m, int D, int n, int nslots, const int32_t *slot_stage,
                               const uint8_t *stage_time, const int16_t *lo, const int16_t *hi,
                               const int32_t *infeasible, int32_t *C, int32_t *E, int32_t *count,
                               int32_t *overflow, hipStream_t stream)
{
    const int64_t total = (int64_t)nslots * B;
    if (total == 0) return hipSuccess;
    const int block = 64;
    hipLaunchKernelGGL(k_stage_tables, dim3((unsigned)((total + block - 1) / block)), dim3(block), 0, stream,
                       B, m, D, n, nslots, slot_stage, stage_time, lo, hi, infeasible, C, E, count, overflow);
    return hipGetLastError();
}

}  // namespace lofp
