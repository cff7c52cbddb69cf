// keys.hip -- grouping of a batch's patterns by the halves of T that the two
// halves of a split contraction depend on (Sec. II.C contracted from both
// ends): the top half of the circuit sees T only through modes 0..rs+1, the
// bottom half only through modes rs+1..m-1.  Patterns with equal halves share
// one contraction of that half.
//
// Per half: an open-addressing hash table over the sub-rows of T (equal rows
// found by comparing values), numbered in order of each group's
// representative -- the lowest-indexed member whose photon number is right,
// else the lowest member -- so key numbers do not depend on thread timing.
// The group's cut intervals are the hull of its feasible members' intervals.
#include "lofp_device.h"

namespace lofp {

// splitmix64 finalizer (Steele, Lea and Flood), used per row entry
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// One wave per (pattern, half); lane i holds row entry i (m <= 32).  The
// hash is the XOR of per-entry mixes (order-free, so the same on every run);
// equal hashes are confirmed by comparing the rows lane by lane.  A slot
// holds p (right photon number) or p + B (otherwise); the minimum over a
// group is its representative.
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
    const int v = tot == a.n ? p : p + a.B;
    // reset hull row (half, p): key numbers are below B, so the rows of all
    // keys get reset
    {
        const int64_t row = ((int64_t)half * a.B + p) * a.span;
        for (int i = lane; i < a.span; i += 64) {
            a.hlo[row + i] = 0x7f7f7f7f;
            a.hhi[row + i] = -1;
        }
    }
    int *tab = a.table + (int64_t)half * a.cap;
    uint32_t j = (uint32_t)(h ^ (h >> 32)) & (uint32_t)(a.cap - 1);
    for (int probe = 0; probe < a.cap; ++probe) {
        int cur = tab[j];
        if (cur < 0) {
            int won = 0;
            if (lane == 0) won = atomicCAS(&tab[j], -1, v);
            cur = __shfl(won, 0, 64);
            if (cur < 0) {
                if (lane == 0) a.slot[gw] = (int)j;
                return;
            }
        }
        const int occ = cur >= a.B ? cur - a.B : cur;
        const int y = mine ? a.T[(int64_t)occ * a.m + lane] : x;
        if (__all(y == x)) {
            if (lane == 0) {
                atomicMin(&tab[j], v);
                a.slot[gw] = (int)j;
            }
            return;
        }
        j = (j + 1) & (uint32_t)(a.cap - 1);
    }
    if (lane == 0) a.slot[gw] = -1;   // unreachable: the table has twice as many slots as rows
}

// Representative of the group in table slot sl (a pattern that found no
// slot, which a table twice the batch size rules out, stands alone).
__device__ __forceinline__ int rep_of_slot(const int *tab, int sl, int p, int B)
{
    if (sl < 0) return p;
    const int v = tab[sl];
    return v >= B ? v - B : v;
}

// One block per half: number the groups in order of their representatives
// (a block-wide scan over the patterns), then give every pattern its key and
// every key its representative.
__global__ __launch_bounds__(1024) void k_key_number(KeyArgs a)
{
    const int half = blockIdx.x;
    const int *tab = a.table + (int64_t)half * a.cap;
    const int *slot = a.slot + (int64_t)half * a.B;
    int *key_of = a.key_of + (int64_t)half * a.B;
    int *rep_of = a.rep_of + (int64_t)half * a.B;
    __shared__ int wsum[16];
    __shared__ int base_s;
    if (threadIdx.x == 0) base_s = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int c = 0; c < a.B; c += blockDim.x) {
        const int p = c + threadIdx.x;
        int is_rep = 0;
        if (p < a.B) is_rep = rep_of_slot(tab, slot[p], p, a.B) == p;
        // exclusive scan of is_rep over the block
        int x = is_rep;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        int before = base_s;
        for (int w = 0; w < wid; ++w) before += wsum[w];
        if (is_rep) key_of[p] = before + x - 1;   // the representative's key number
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int w = 0; w < nw; ++w) t += wsum[w];
            base_s += t;
        }
        __syncthreads();
    }
    const int nkeys = base_s;
    if (threadIdx.x == 0) a.count[half] = nkeys;
    __syncthreads();
    // representatives hold their key numbers; members copy theirs
    for (int p = threadIdx.x; p < a.B; p += blockDim.x)
        if (rep_of_slot(tab, slot[p], p, a.B) == p) rep_of[key_of[p]] = p;
    __syncthreads();
    for (int p = threadIdx.x; p < a.B; p += blockDim.x) {
        const int r = rep_of_slot(tab, slot[p], p, a.B);
        if (r != p) key_of[p] = key_of[r];
    }
    // leave the table empty for the next call (every used slot is some
    // pattern's slot)
    __syncthreads();
    int *wtab = a.table + (int64_t)half * a.cap;
    for (int p = threadIdx.x; p < a.B; p += blockDim.x)
        if (slot[p] >= 0) wtab[slot[p]] = -1;
}

// Hull of the feasible members' intervals, one thread per (pattern, half, entry).
__global__ void k_key_hull(KeyArgs a)
{
    const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)a.B * a.span;
    if (gi >= 2 * per) return;
    const int half = (int)(gi / per);
    const int64_t r = gi - half * per;
    const int p = (int)(r / a.span), i = (int)(r - (int64_t)p * a.span);
    if (a.infeasible[p]) return;
    const int k = a.key_of[(int64_t)half * a.B + p];
    const int64_t o = ((int64_t)half * a.B + k) * a.span + i;
    atomicMin(&a.hlo[o], (int)a.lo[(int64_t)p * a.span + i]);
    atomicMax(&a.hhi[o], (int)a.hi[(int64_t)p * a.span + i]);
}

// One wave per (half, key): the key's 16-bit interval rows, its contraction
// job (top keys first, then bottom keys) and the bucket of its work, the sum
// over its steps of the state entries times the summed versions' radii
// (lanes over steps).
__global__ __launch_bounds__(256) void k_key_jobs(KeyArgs a, ContractJob top, ContractJob bot, ContractJob *jobs,
                                                  int32_t *kinf)
{
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gw = gt >> 6;
    const int lane = threadIdx.x & 63;
    if (gt < 8) a.counters[gt] = 0;   // the contraction's counters for this call
    if (gw >= 2 * (int64_t)a.B) return;
    const int half = (int)(gw / a.B), k = (int)(gw - (int64_t)half * a.B);
    if (k >= a.count[half]) return;
    const int64_t row = ((int64_t)half * a.B + k) * a.span;
    for (int i = lane; i < a.span; i += 64) {
        int l = a.hlo[row + i], h = a.hhi[row + i];
        if (h < 0) { l = 1; h = 0; }   // no feasible member: empty interval
        a.klo[row + i] = (int16_t)l;
        a.khi[row + i] = (int16_t)h;
    }
    const ContractJob &tmpl = half ? bot : top;
    const int nc = a.m - 1;
    float work = 0.0f;
    for (int si = lane; si < tmpl.nsteps; si += 64) {
        const ContractStep &st = tmpl.steps[si];
        float e = 1.0f;
        for (int q = 0; q < st.n_new; ++q) {
            const int v = st.new_vars[q];
            const int64_t i = row + tmpl.var_time[v] * nc + tmpl.var_cut[v];
            e *= (float)max(0, a.hhi[i] - a.hlo[i] + 1);
        }
        for (int q = 0; q < st.n_sum; ++q) {
            const int v = st.sum_vars[q];
            const int64_t i = row + tmpl.var_time[v] * nc + tmpl.var_cut[v];
            e *= (float)max(1, a.hhi[i] - a.hlo[i] + 1);
        }
        work += e;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) work += __shfl_xor(work, o, 64);
    if (lane != 0) return;
    const int j = half ? a.count[0] + k : k;
    a.job_bucket[j] = work > 1.0f ? min(255, (int)(8.0f * log2f(work))) : 0;
    ContractJob J = tmpl;
    J.T = a.T + (int64_t)a.rep_of[(int64_t)half * a.B + k] * a.m;
    J.lo = a.klo + row;
    J.hi = a.khi + row;
    J.infeasible = kinf + j;
    kinf[j] = 0;
    J.out = nullptr;
    jobs[j] = J;
}

// One block: the jobs in decreasing work bucket (a counting sort; the order
// inside a bucket is arbitrary and changes no result).
__global__ __launch_bounds__(1024) void k_key_order(KeyArgs a)
{
    __shared__ int hist[256], start[256];
    __shared__ int wsum[4];
    const int nj = a.count[0] + a.count[1];
    const int t = threadIdx.x;
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
    hipLaunchKernelGGL(k_key_number, dim3(2), dim3(1024), 0, stream, a);
    const int64_t nh = n2 * a.span;
    hipLaunchKernelGGL(k_key_hull, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_key_jobs(const KeyArgs &a, const ContractJob &top, const ContractJob &bot, ContractJob *jobs,
                           int32_t *kinf, hipStream_t stream)
{
    const int64_t threads = 2 * (int64_t)a.B * 64;
    hipLaunchKernelGGL(k_key_jobs, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, stream, a, top, bot, jobs,
                       kinf);
    hipLaunchKernelGGL(k_key_order, dim3(1), dim3(1024), 0, stream, a);
    return hipGetLastError();
}

}  // namespace lofp
