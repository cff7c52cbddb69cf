// frontier.hip -- merged frontiers (Schroedinger-Feynman interpolation, Sec. I):
// the amplitudes of every configuration reachable at a stage, expanded one
// beam splitter at a time from S (forward) or from T (backward).  Each thread
// produces two consecutive configurations of the target stage, each by
// gathering the (at most N+1) configurations of the source stage that differ
// from it on the split cut, so the summation order is fixed and the result
// deterministic.
#include <climits>

#include "lofp_device.h"

namespace lofp {

__global__ void k_seed(int B, const int64_t *__restrict__ off, double2 *__restrict__ vec)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= B) return;
    if (off[p + 1] > off[p]) vec[off[p]] = make_double2(1.0, 0.0);
}

hipError_t launch_seed(int B, const int64_t *off, double2 *vec, hipStream_t stream)
{
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seed, dim3((B + 255) / 256), dim3(256), 0, stream, B, off, vec);
    return hipGetLastError();
}

constexpr int kScan = 3;          // candidates one pass of the unranking scan reads
constexpr int kGateThreads = kGateChunk / 2;   // two consecutive target ranks per thread

// One cut of the unranking: the value v of cut r for the remaining rank rem
// given the previous cut's value pv; rem becomes the rank within the
// configurations that share cuts 0..r.  Row Cr (of the target rank table) is
// non-decreasing up to the cut's upper bound and INT_MAX past it, so the
// scan reads kScan candidates at fixed offsets per pass and needs no bound
// test.  flip: the next rank (same cuts before r) moves this cut, i.e. the
// first candidate above the target is exactly one above it.
__device__ __forceinline__ int unrank_cut(const int32_t *Cr, int L, int pv, int &rem, bool &flip)
{
    const int base = Cr[pv];
    int v = pv > L ? pv : L;
    const int tgt = base + rem;   // the last v with Cr[v] <= tgt
    int above;
    while (true) {
        const int32_t *c = Cr + v;
        const int c1 = c[1], c2 = c[2], c3 = c[3];
        const int st = (c1 <= tgt) + (c2 <= tgt) + (c3 <= tgt);
        v += st;
        if (st < kScan) {
            above = st == 0 ? c1 : (st == 1 ? c2 : c3);
            break;
        }
    }
    flip = above == tgt + 1;
    rem = tgt - Cr[v];
    return v;
}

// One block per chunk of kGateChunk consecutive target states of one pattern,
// two consecutive ranks per thread; the pattern's rank tables and intervals
// are staged in LDS once per block.  The target rank table is staged with
// rows of W + kScan entries, every entry past the cut's upper bound set to
// INT_MAX (see unrank_cut).  Ranks follow the lexicographic order of the cut
// values, so the second rank shares every cut before the first one that
// moves at the next rank (flip): it is unranked from that cut on only
// (ranks within a pattern are below 2^31: the planner refuses larger state
// spaces, so the rank arithmetic is 32-bit).
template <int NCM, bool FWD>
__global__ __launch_bounds__(kGateThreads) void k_gate(GateArgs g)
{
    extern __shared__ __align__(16) int32_t gate_lds[];
    __shared__ int16_t sL[kMaxCuts], sH[kMaxCuts];
    __shared__ int s_p, s_ch, s_Ls, s_Hs;
    const int nc = g.m - 1, W = table_cols(g.n), span = (g.D + 1) * nc, tsz = nc * W;
    const int WP = W + kScan;
    int32_t *sC = gate_lds, *sE = gate_lds + nc * WP;
    if (threadIdx.x == 0) {
        int pp = -1, ch = 0;
        if (!xcd_chunk(g.xoff, g.nbx, g.B, blockIdx.x, pp, ch)) pp = -1;
        s_p = pp;
        s_ch = ch;
    }
    __syncthreads();
    const int p = s_p;
    if (p < 0) return;
    const int16_t *lo = g.lo + (int64_t)p * span, *hi = g.hi + (int64_t)p * span;
    const int32_t *Ct = g.C_tgt + (int64_t)p * tsz;
    const int32_t *Es = g.E_src + (int64_t)p * tsz;
    for (int i = threadIdx.x; i < tsz; i += blockDim.x) sE[i] = Es[i];
    for (int r = threadIdx.x; r < nc; r += blockDim.x) {
        const int t = g.st_tgt[r];
        sL[r] = lo[t * nc + r];
        sH[r] = hi[t * nc + r];
    }
    const int a = g.cut;
    if (threadIdx.x == 0) {
        const int ts = g.st_src[a];
        s_Ls = lo[ts * nc + a];
        s_Hs = hi[ts * nc + a];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nc * WP; i += blockDim.x) {
        const int r = i / WP, v = i - r * WP;
        sC[i] = v <= sH[r] ? Ct[r * W + v] : INT_MAX;
    }
    __syncthreads();
    const int64_t i0 = (int64_t)s_ch * kGateChunk + 2 * threadIdx.x;
    const int64_t base_t = g.off_tgt[p], count = g.off_tgt[p + 1] - base_t;
    if (i0 >= count) return;
    const int Ls = s_Ls, Hs = s_Hs;
    const double2 *src = g.src + g.off_src[p];
    const int32_t *Ea = sE + a * W;
    // the splitter's sum for one target: its source states differ from it on cut a
    auto gather = [&](int prev, int next, int cur, int K, int64_t i) {
        const int N = next - prev;
        const int ulo = Ls > prev ? Ls : prev, uhi = Hs < next ? Hs : next;
        const double2 *Wn = g.W + sector_offset(N);
        double2 acc = make_double2(0.0, 0.0);
        for (int u = ulo; u <= uhi; ++u) {
            const double2 w = FWD ? Wn[(u - prev) * (N + 1) + (cur - prev)] : Wn[(cur - prev) * (N + 1) + (u - prev)];
            acc = cfma(w, src[K + Ea[u]], acc);
        }
        g.dst[base_t + i] = acc;
    };

    // first rank: every cut; keep each cut's value and remaining rank
    int vr[NCM], rin[NCM];
    unsigned flips = 0;
    int prev = 0, next = g.n, cur = 0;
    int rem = (int)i0, K = 0;
    int pv = 0;
#pragma unroll
    for (int r = 0; r < NCM; ++r) {
        if (r < nc) {
            rin[r] = rem;
            bool f;
            const int v = unrank_cut(sC + r * WP, sL[r], pv, rem, f);
            flips |= (unsigned)f << r;
            vr[r] = v;
            pv = v;
            if (r == a - 1) prev = v;
            if (r == a + 1) next = v;
            if (r == a) cur = v;
            else K += sE[r * W + v];
        }
    }
    gather(prev, next, cur, K, i0);
    if (i0 + 1 >= count) return;

    // second rank: the cuts before the first flip are the first rank's
    const int rs = flips ? __ffs(flips) - 1 : 0;   // (a flip always exists below count)
#pragma unroll
    for (int r = 0; r < NCM; ++r) {
        if (r >= rs && r < nc) {
            if (r == rs) {
                rem = rin[r] + 1;
                pv = r > 0 ? vr[r > 0 ? r - 1 : 0] : 0;
            }
            bool f;
            const int v = unrank_cut(sC + r * WP, sL[r], pv, rem, f);
            pv = v;
            if (r == a - 1) prev = v;
            if (r == a + 1) next = v;
            if (r == a) cur = v;
            else K += sE[r * W + v] - sE[r * W + vr[r]];
        }
    }
    gather(prev, next, cur, K, i0 + 1);
}

hipError_t launch_gate(const GateArgs &a, bool forward, hipStream_t stream)
{
    if (a.total_tgt == 0) return hipSuccess;
    const int block = kGateThreads;
    if (a.grid <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.grid);
    const int nc = a.m - 1;
    // rank rows (padded) and source offsets of every cut
    const size_t dyn = (size_t)nc * (2 * table_cols(a.n) + kScan) * sizeof(int32_t);
    if (nc <= 15) {
        if (forward) hipLaunchKernelGGL((k_gate<15, true>), grid, dim3(block), dyn, stream, a);
        else hipLaunchKernelGGL((k_gate<15, false>), grid, dim3(block), dyn, stream, a);
    } else {
        if (forward) hipLaunchKernelGGL((k_gate<31, true>), grid, dim3(block), dyn, stream, a);
        else hipLaunchKernelGGL((k_gate<31, false>), grid, dim3(block), dyn, stream, a);
    }
    return hipGetLastError();
}

}  // namespace lofp
