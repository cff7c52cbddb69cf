// frontier.hip -- merged frontiers (Schroedinger-Feynman interpolation, Sec. I):
// the amplitudes of every configuration reachable at a stage, expanded one
// beam splitter at a time from S (forward) or from T (backward).  Each thread
// produces one configuration of the target stage by gathering the (at most
// N+1) configurations of the source stage that differ from it on the split
// cut, so the summation order is fixed and the result deterministic.
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

constexpr int kTabMax = kMaxCuts * (kMaxPhotons + 2);
constexpr int kScan = 3;   // candidates one pass of the unranking scan reads
constexpr int kTabPadMax = kMaxCuts * (kMaxPhotons + 2 + kScan);

// One block per chunk of kGateChunk consecutive target states of one pattern;
// the pattern's rank tables and intervals are staged in LDS once per block.
// The target rank table is staged with rows of W + kScan entries, every
// entry past the cut's upper bound set to INT_MAX, so the unranking scan
// needs no bound test: it reads kScan candidates at fixed offsets and stops
// at the first one above the remaining rank.
template <int NCM, bool FWD>
__global__ __launch_bounds__(kGateChunk) void k_gate(GateArgs g)
{
    __shared__ int32_t sC[kTabPadMax], sE[kTabMax];
    __shared__ int16_t sL[kMaxCuts], sH[kMaxCuts];
    __shared__ int s_p, s_ch, s_Ls, s_Hs;
    const int nc = g.m - 1, W = table_cols(g.n), span = (g.D + 1) * nc, tsz = nc * W;
    const int WP = W + kScan;
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
    const int64_t i = (int64_t)s_ch * kGateChunk + threadIdx.x;
    const int64_t base_t = g.off_tgt[p];
    if (i >= g.off_tgt[p + 1] - base_t) return;

    // unrank the target configuration; collect the neighbours of cut a and
    // the source rank contributed by every cut other than a (ranks within a
    // pattern are below 2^31: the planner refuses larger state spaces, so
    // the rank arithmetic is 32-bit)
    int prev = 0, next = g.n, cur = 0;
    int rem = (int)i, K = 0;
    int pv = 0;
#pragma unroll
    for (int r = 0; r < NCM; ++r) {
        if (r < nc) {
            const int L = sL[r];
            const int32_t *Cr = sC + r * WP;
            const int base = Cr[pv];
            int v = pv > L ? pv : L;
            // the last v <= H (the cut's upper bound) with Cr[v] <= tgt: Cr
            // is non-decreasing up to H and INT_MAX past it
            const int tgt = base + rem;
            while (true) {
                const int32_t *c = Cr + v;
                const int st = (c[1] <= tgt) + (c[2] <= tgt) + (c[3] <= tgt);
                v += st;
                if (st < kScan) break;
            }
            rem = tgt - Cr[v];
            pv = v;
            if (r == a - 1) prev = v;
            if (r == a + 1) next = v;
            if (r == a) cur = v;
            else K += sE[r * W + v];
        }
    }
    const int N = next - prev;
    const int Ls = s_Ls, Hs = s_Hs;
    const int ulo = Ls > prev ? Ls : prev, uhi = Hs < next ? Hs : next;
    const double2 *Wn = g.W + sector_offset(N);
    const double2 *src = g.src + g.off_src[p];
    const int32_t *Ea = sE + a * W;
    double2 acc = make_double2(0.0, 0.0);
    for (int u = ulo; u <= uhi; ++u) {
        const double2 w = FWD ? Wn[(u - prev) * (N + 1) + (cur - prev)] : Wn[(cur - prev) * (N + 1) + (u - prev)];
        acc = cfma(w, src[K + Ea[u]], acc);
    }
    g.dst[base_t + i] = acc;
}

hipError_t launch_gate(const GateArgs &a, bool forward, hipStream_t stream)
{
    if (a.total_tgt == 0) return hipSuccess;
    const int block = kGateChunk;
    if (a.grid <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.grid);
    const int nc = a.m - 1;
    if (nc <= 15) {
        if (forward) hipLaunchKernelGGL((k_gate<15, true>), grid, dim3(block), 0, stream, a);
        else hipLaunchKernelGGL((k_gate<15, false>), grid, dim3(block), 0, stream, a);
    } else {
        if (forward) hipLaunchKernelGGL((k_gate<31, true>), grid, dim3(block), 0, stream, a);
        else hipLaunchKernelGGL((k_gate<31, false>), grid, dim3(block), 0, stream, a);
    }
    return hipGetLastError();
}

}  // namespace lofp
