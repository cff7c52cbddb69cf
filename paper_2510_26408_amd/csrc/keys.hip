// keys.hip -- grouping of a batch's patterns by the halves of T that the two
// halves of a split contraction depend on (Sec. II.C contracted from both
// ends): the top half of the circuit sees T only through modes 0..rs+1, the
// bottom half only through modes rs+1..m-1.  Patterns with equal halves share
// one contraction of that half.
//
// Per half: an open-addressing hash table over the sub-rows of T (equal rows
// found by comparing hashes, then values).  The wave that claims a slot numbers the key;
// every member folds its intervals into the slot's hull (feasible members
// only) and its index into the slot's representative, the lowest-indexed
// member whose photon number is right, else the lowest member.  The jobs
// kernel reads each key's slot and leaves the table and the hulls empty for
// the next call.
#include "lofp_device.h"

namespace lofp {

// splitmix64 finalizer (Steele, Lea and Flood), used per row entry
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// The hull entries a half's keys use: every time of the cuts its program
// reads, its own cuts and the two crossing ones (top: cuts 0..rs+1, bottom:
// cuts rs..m-2).  Entries outside stay empty in every slot.
struct HullRegion {
    int r0, w, n;
    float winv;
};
__device__ __forceinline__ HullRegion hull_region(const KeyArgs &a, int half)
{
    const int nc = a.m - 1;
    HullRegion h;
    h.r0 = half ? a.rs : 0;
    h.w = half ? nc - a.rs : a.rs + 2;
    h.n = (a.span / nc) * h.w;
    h.winv = 1.0f / (float)h.w;
    return h;
}
// Entry j (0 <= j < n) of the region as an index into a hull row.
__device__ __forceinline__ int hull_at(const HullRegion &h, int nc, int j)
{
    const int t = qdiv(j, h.w, h.winv);
    return t * nc + h.r0 + (j - t * h.w);
}

// One wave per (pattern, half); lane i holds row entry i (m <= 32).  The
// hash is the XOR of per-entry mixes (order-free, so the same on every run).
// A slot holds the row's 32-bit hash above p (right photon number) or p + B
// (otherwise), all ones when empty: a probe compares hashes first and the
// rows lane by lane only when they agree, and the minimum over a group (one
// hash) is its representative.
__global__ __launch_bounds__(256) void k_key_insert(KeyArgs a)
{
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (gw >= 2 * (int64_t)a.B) return;
    const int half = (int)(gw / a.B), p = (int)(gw - (int64_t)half * a.B);
    const int c0 = half ? a.rs + 1 : 0, c1 = half ? a.m - 1 : a.rs + 1;
    const bool mine = lane >= c0 && lane <= c1;
    const int x = lane < a.m ? a.T[(int64_t)p * a.m + lane] : 0;
    int tot = x;
    uint64_t h = mine ? mix64((uint64_t)(uint32_t)x + 0x9E3779B97F4A7C15ULL * (uint64_t)(lane + 1)) : 0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        tot += __shfl_xor(tot, o, 64);
        h ^= __shfl_xor(h, o, 64);
    }
    const unsigned v = (unsigned)(tot == a.n ? p : p + a.B);
    const unsigned long long hv = (h >> 32) << 32;
    const unsigned long long mine_e = hv | v;
    unsigned long long *tab = a.table + key_slot_index(half, a.stride, 0);
    uint32_t j = (uint32_t)h & (uint32_t)(a.cap - 1);
    // at most B rows per half and cap >= 4B slots: a free slot is always found
    for (int probe = 0; probe < a.cap; ++probe) {
        unsigned long long cur = tab[j];
        if (cur == kKeyEmpty) {
            unsigned long long won = 0;
            if (lane == 0) won = atomicCAS(&tab[j], kKeyEmpty, mine_e);
            cur = __shfl(won, 0, 64);
            if (cur == kKeyEmpty) {
                // claimed: list the slot under its sub-counter (the keys
                // are numbered by the jobs kernel, through the counts)
                if (lane == 0) {
                    const int sub = (int)(j & (kKeySubs - 1));
                    const int local = atomicAdd(&a.count[half * kKeySubs + sub], 1);   // < B
                    if (local < a.B) a.key_slot[((int64_t)half * kKeySubs + sub) * a.B + local] = (int)j;
                }
                break;
            }
        }
        if ((cur >> 32) == (hv >> 32)) {
            const unsigned cv = (unsigned)cur;
            const int occ = (int)(cv >= (unsigned)a.B ? cv - a.B : cv);
            const int y = mine ? a.T[(int64_t)occ * a.m + lane] : x;
            if (__all(y == x)) {
                if (lane == 0) atomicMin(&tab[j], mine_e);
                break;
            }
        }
        j = (j + 1) & (uint32_t)(a.cap - 1);
    }
    if (lane == 0) a.slot[gw] = (int)j;
    if (a.infeasible[p]) return;
    // the slot's hull of its feasible members' intervals
    const int64_t row = key_hull_row(half, a.stride, j, a.span);
    const HullRegion hr = hull_region(a, half);
    for (int e = lane; e < hr.n; e += 64) {
        const int i = hull_at(hr, a.m - 1, e);
        atomicMin(&a.hlo[row + i], (int)a.lo[(int64_t)p * a.span + i]);
        atomicMax(&a.hhi[row + i], (int)a.hi[(int64_t)p * a.span + i]);
    }
}

// Slot of key k of a half (whole wave): keys are numbered through the
// sub-counters in order, so key k is entry k - (claims of earlier
// sub-counters) of its sub-counter's list.
__device__ __forceinline__ int key_slot_of(const KeyArgs &a, int half, int k)
{
    const int lane = threadIdx.x & 63;
    const int c = a.count[half * kKeySubs + lane];
    int incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    const int excl = incl - c;
    const unsigned long long hit = __ballot(k >= excl && k < incl);
    const int sub = hit ? __ffsll((long long)hit) - 1 : 0;
    const int local = k - __shfl(excl, sub, 64);
    return a.key_slot[((int64_t)half * kKeySubs + sub) * a.B + local];
}

// One wave per key (top keys, then bottom keys; wave w is job w): the key's
// 16-bit interval rows from its slot's hull, its contraction job and the
// bucket of its work, the sum over its steps of the state entries times the
// summed versions' radii (lanes over steps).  Then the slot's hull and table
// entry are reset, and the key counts zeroed, for the next call.
__global__ __launch_bounds__(256) void k_key_jobs(KeyArgs a, int ntop, int nbot, ContractJob top, ContractJob bot,
                                                  ContractJob *jobs, int32_t *kinf)
{
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int w = (int)(gt >> 6);
    const int lane = threadIdx.x & 63;
    if (gt < 8) a.counters[gt] = 0;   // the contraction's counters for this call
    if (w >= ntop + nbot) return;
    const int half = w >= ntop, k = half ? w - ntop : w;
    const int sl = key_slot_of(a, half, k);
    if (lane == 0) a.slot_key[key_slot_index(half, a.stride, sl)] = k;
    const int64_t srow = key_hull_row(half, a.stride, sl, a.span);
    const int64_t krow = ((int64_t)half * a.B + k) * a.span;
    for (int i = lane; i < a.span; i += 64) {
        int l = a.hlo[srow + i], h = a.hhi[srow + i];
        if (h < 0) { l = 1; h = 0; }   // no feasible member: empty interval
        a.klo[krow + i] = (int16_t)l;
        a.khi[krow + i] = (int16_t)h;
    }
    const ContractJob &tmpl = half ? bot : top;
    const int nc = a.m - 1;
    float work = 0.0f;
    for (int si = lane; si < tmpl.nsteps; si += 64) {
        const ContractStep &st = tmpl.steps[si];
        float e = 1.0f;
        for (int q = 0; q < st.n_new; ++q) {
            const int v = st.new_vars[q];
            const int64_t i = srow + tmpl.var_time[v] * nc + tmpl.var_cut[v];
            e *= (float)max(0, a.hhi[i] - a.hlo[i] + 1);
        }
        for (int q = 0; q < st.n_sum; ++q) {
            const int v = st.sum_vars[q];
            const int64_t i = srow + tmpl.var_time[v] * nc + tmpl.var_cut[v];
            e *= (float)max(1, a.hhi[i] - a.hlo[i] + 1);
        }
        work += e;
    }
    // (the reduction consumes every lane's loads before the hull is reset)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) work += __shfl_xor(work, o, 64);
    {
        const HullRegion hr = hull_region(a, half);
        for (int e = lane; e < hr.n; e += 64) {
            const int i = hull_at(hr, a.m - 1, e);
            a.hlo[srow + i] = kHullEmptyLo;
            a.hhi[srow + i] = kHullEmptyHi;
        }
    }
    if (lane != 0) return;
    unsigned long long *tab = a.table + key_slot_index(half, a.stride, 0);
    const int rv = (int)(unsigned)tab[sl];
    tab[sl] = kKeyEmpty;
    a.job_bucket[w] = work > 1.0f ? min(255, (int)(8.0f * log2f(work))) : 0;
    ContractJob J = tmpl;
    J.T = a.T + (int64_t)(rv >= a.B ? rv - a.B : rv) * a.m;
    J.lo = a.klo + krow;
    J.hi = a.khi + krow;
    J.infeasible = kinf + w;
    kinf[w] = 0;
    J.ovf = kinf + ntop + nbot + w;   // the join reads it
    kinf[ntop + nbot + w] = 0;
    J.out = nullptr;
    jobs[w] = J;
}

// One wave per key: empties the key's slot (hull and table entry), for a
// call that groups the batch but then contracts per pattern (the counts are
// cleared after it).
__global__ __launch_bounds__(256) void k_key_reset(KeyArgs a, int ntop, int nbot)
{
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int w = (int)(gt >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= ntop + nbot) return;
    const int half = w >= ntop, k = half ? w - ntop : w;
    const int sl = key_slot_of(a, half, k);
    const int64_t srow = key_hull_row(half, a.stride, sl, a.span);
    {
        const HullRegion hr = hull_region(a, half);
        for (int e = lane; e < hr.n; e += 64) {
            const int i = hull_at(hr, a.m - 1, e);
            a.hlo[srow + i] = kHullEmptyLo;
            a.hhi[srow + i] = kHullEmptyHi;
        }
    }
    if (lane == 0) a.table[key_slot_index(half, a.stride, sl)] = kKeyEmpty;
}

// Totals of claimed keys per half (whole wave).
__device__ __forceinline__ void key_totals(const KeyArgs &a, int &ntop, int &nbot)
{
    const int lane = threadIdx.x & 63;
    int t = a.count[lane], b = a.count[kKeySubs + lane];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        t += __shfl_xor(t, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    ntop = t;
    nbot = b;
}

// Device-decided jobs (launch_key_jobs_dev): 2B waves, wave w serves key w
// of the keys that were claimed.
__global__ __launch_bounds__(256) void k_key_jobs_dev(KeyArgs a, ContractJob top, ContractJob bot, ContractJob *jobs,
                                                      int32_t *kinf, double2 *state_base, int state_cap)
{
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int w = (int)(gt >> 6);
    const int lane = threadIdx.x & 63;
    if (gt < 8) a.counters[gt] = 0;   // the contraction's counters for this call
    int ntop, nbot;
    key_totals(a, ntop, nbot);
    const bool split = (int64_t)(ntop + nbot) * 4 <= (int64_t)a.B * 3 || (a.B >= a.small_min && a.B <= a.small_max);
    if (gt == 0) {
        a.ctl[0] = split;
        a.ctl[1] = split ? ntop + nbot : 0;
        a.ctl[2] = ntop;
        a.ctl[3] = nbot;
        a.ctl[4] = 0;   // the contraction's job counter
    }
    if (w >= ntop + nbot) return;
    const int half = w >= ntop, k = half ? w - ntop : w;
    const int sl = key_slot_of(a, half, k);
    const int64_t srow = key_hull_row(half, a.stride, sl, a.span);
    if (!split) {
        // one contraction per pattern: only empty the slot
        const HullRegion hr = hull_region(a, half);
        for (int e = lane; e < hr.n; e += 64) {
            const int i = hull_at(hr, a.m - 1, e);
            a.hlo[srow + i] = kHullEmptyLo;
            a.hhi[srow + i] = kHullEmptyHi;
        }
        if (lane == 0) a.table[key_slot_index(half, a.stride, sl)] = kKeyEmpty;
        return;
    }
    if (lane == 0) a.slot_key[key_slot_index(half, a.stride, sl)] = k;
    const int64_t krow = ((int64_t)half * a.B + k) * a.span;
    for (int i = lane; i < a.span; i += 64) {
        int l = a.hlo[srow + i], h = a.hhi[srow + i];
        if (h < 0) { l = 1; h = 0; }   // no feasible member: empty interval
        a.klo[krow + i] = (int16_t)l;
        a.khi[krow + i] = (int16_t)h;
    }
    const ContractJob &tmpl = half ? bot : top;
    const int nc = a.m - 1;
    float work = 0.0f;
    for (int si = lane; si < tmpl.nsteps; si += 64) {
        const ContractStep &st = tmpl.steps[si];
        float e = 1.0f;
        for (int q = 0; q < st.n_new; ++q) {
            const int v = st.new_vars[q];
            const int64_t i = srow + tmpl.var_time[v] * nc + tmpl.var_cut[v];
            e *= (float)max(0, a.hhi[i] - a.hlo[i] + 1);
        }
        for (int q = 0; q < st.n_sum; ++q) {
            const int v = st.sum_vars[q];
            const int64_t i = srow + tmpl.var_time[v] * nc + tmpl.var_cut[v];
            e *= (float)max(1, a.hhi[i] - a.hlo[i] + 1);
        }
        work += e;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) work += __shfl_xor(work, o, 64);
    {
        const HullRegion hr = hull_region(a, half);
        for (int e = lane; e < hr.n; e += 64) {
            const int i = hull_at(hr, a.m - 1, e);
            a.hlo[srow + i] = kHullEmptyLo;
            a.hhi[srow + i] = kHullEmptyHi;
        }
    }
    if (lane != 0) return;
    unsigned long long *tab = a.table + key_slot_index(half, a.stride, 0);
    const int rv = (int)(unsigned)tab[sl];
    tab[sl] = kKeyEmpty;
    a.job_bucket[w] = work > 1.0f ? min(255, (int)(8.0f * log2f(work))) : 0;
    const int place = half ? a.B + k : k;   // fixed by the half, not by the key counts
    ContractJob J = tmpl;
    J.T = a.T + (int64_t)(rv >= a.B ? rv - a.B : rv) * a.m;
    J.lo = a.klo + krow;
    J.hi = a.khi + krow;
    J.infeasible = kinf + w;
    kinf[w] = 0;
    J.ovf = kinf + 2 * (int64_t)a.B + place;
    kinf[2 * (int64_t)a.B + place] = 0;
    J.out = nullptr;
    J.state_out = state_base + (int64_t)place * state_cap;
    J.state_cap = state_cap;
    jobs[w] = J;
}

// One block: the jobs in decreasing work bucket (a counting sort; the order
// inside a bucket is arbitrary and changes no result).
__global__ __launch_bounds__(1024) void k_key_order(KeyArgs a, int nj)
{
    __shared__ int hist[256], start[256];
    __shared__ int wsum[4];
    const int t = threadIdx.x;
    if (a.ctl) nj = a.ctl[1];   // decided on the device (0 when not split)
    if (t < 2 * kKeySubs) a.count[t] = 0;   // the jobs kernel has read them
    if (t < 256) hist[t] = 0;
    __syncthreads();
    for (int j = t; j < nj; j += blockDim.x) atomicAdd(&hist[255 - a.job_bucket[j]], 1);
    __syncthreads();
    // exclusive scan of the 256 counts (largest bucket first), four waves
    if (t < 256) {
        const int lane = t & 63, w = t >> 6;
        int x = hist[t];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
        start[t] = x - hist[t];
    }
    __syncthreads();
    if (t < 256) {
        int before = 0;
        for (int w = 0; w < (t >> 6); ++w) before += wsum[w];
        start[t] += before;
    }
    __syncthreads();
    for (int j = t; j < nj; j += blockDim.x) a.order[atomicAdd(&start[255 - a.job_bucket[j]], 1)] = j;
}

hipError_t launch_keys(const KeyArgs &a, hipStream_t stream)
{
    if (a.B == 0) return hipSuccess;
    const int64_t n2 = 2 * (int64_t)a.B;
    hipLaunchKernelGGL(k_key_insert, dim3((unsigned)((n2 * 64 + 255) / 256)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_key_jobs(const KeyArgs &a, int ntop, int nbot, const ContractJob &top, const ContractJob &bot,
                           ContractJob *jobs, int32_t *kinf, hipStream_t stream)
{
    const int64_t threads = (int64_t)(ntop + nbot) * 64;
    hipLaunchKernelGGL(k_key_jobs, dim3((unsigned)(threads > 0 ? (threads + 255) / 256 : 1)), dim3(256), 0, stream,
                       a, ntop, nbot, top, bot, jobs, kinf);
    hipLaunchKernelGGL(k_key_order, dim3(1), dim3(1024), 0, stream, a, ntop + nbot);
    return hipGetLastError();
}

hipError_t launch_key_jobs_dev(const KeyArgs &a, const ContractJob &top, const ContractJob &bot, ContractJob *jobs,
                               int32_t *kinf, double2 *state_base, int state_cap, hipStream_t stream)
{
    if (!a.ctl) return hipErrorInvalidValue;
    const int64_t threads = 2 * (int64_t)a.B * 64;
    hipLaunchKernelGGL(k_key_jobs_dev, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, stream, a, top, bot, jobs,
                       kinf, state_base, state_cap);
    hipLaunchKernelGGL(k_key_order, dim3(1), dim3(1024), 0, stream, a, 0);
    return hipGetLastError();
}

hipError_t launch_key_reset(const KeyArgs &a, int ntop, int nbot, hipStream_t stream)
{
    const int64_t threads = (int64_t)(ntop + nbot) * 64;
    hipLaunchKernelGGL(k_key_reset, dim3((unsigned)(threads > 0 ? (threads + 255) / 256 : 1)), dim3(256), 0, stream,
                       a, ntop, nbot);
    return hipGetLastError();
}

}  // namespace lofp
