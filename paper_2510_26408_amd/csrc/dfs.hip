// dfs.hip -- depth-first enumeration of Feynman paths (Eq. (1)) through the
// middle beam splitters, between the forward merged frontier (stage s_f) and
// the backward merged frontier (stage s_b).
//
// Each lane owns one forward-frontier configuration at a time and walks every
// sequence of beam-splitter outputs that leads from it to a configuration of
// stage s_b, so that lanes of a wave advance independently and stay busy
// whatever the shape of their subtrees.  One loop pass takes every leaf of a
// last-level range, climbs out of the levels it has used up and steps down
// one edge, so the lanes of a wave run the same bodies in step.  Per edge: one transition-table read (from LDS, or through
// the vector caches where LDS tables would cost resident blocks) and one
// complex FP64 product; at a leaf the backward-frontier amplitude of the reached
// configuration is found by its dense rank, which is kept up to date with two
// table lookups per changed cut.  Ranges come from the per-pattern cut bounds,
// so every edge taken leads to at least one valid leaf.
//
// The per-lane stack (prefix product, choice, range end, previous cut value,
// prefix rank) lives in LDS as [level][lane], and so do the lane's cut values
// as bytes, [cut][lane]: a cut is read or written by one LDS access at the
// lane's own address (held as packed words in registers, each access was a
// chain of selects over the words, several per edge).  A lane's leaves are
// accumulated with a compensated (TwoSum) complex sum, multiplied by the
// frontier amplitude and written back in place of it; the per-pattern total
// is formed by the reduction kernel in a fixed order, so results do not
// depend on which lane took which entry.
#include "lofp_device.h"

namespace lofp {

constexpr int kTabMax = kMaxCuts * (kMaxPhotons + 2);

// ---------------------------------------------------------------- annotate
// One block per chunk of consecutive frontier entries of one pattern.
__global__ __launch_bounds__(kDfsChunk) void k_annotate(AnnotateArgs g)
{
    __shared__ int32_t sC[kTabMax], sE[kTabMax];
    __shared__ int16_t sL[kMaxCuts], sH[kMaxCuts];
    __shared__ int s_p, s_ch;
    const int nc = g.m - 1, W = table_cols(g.n), span = (g.D + 1) * nc, tsz = nc * W;
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
    for (int i = threadIdx.x; i < tsz; i += blockDim.x) {
        sC[i] = g.C_front[(int64_t)p * tsz + i];
        sE[i] = g.E_back[(int64_t)p * tsz + i];
    }
    for (int r = threadIdx.x; r < nc; r += blockDim.x) {
        const int t = g.st_front[r];
        sL[r] = lo[t * nc + r];
        sH[r] = hi[t * nc + r];
    }
    __syncthreads();
    const int64_t i = (int64_t)s_ch * kDfsChunk + threadIdx.x;
    const int64_t base = g.off_front[p];
    if (i >= g.off_front[p + 1] - base) return;
    int64_t rem = i;
    int pv = 0, rank = 0;
    uint32_t w = 0;
    uint32_t *out = g.cfg + (base + i) * g.cfg_words;
    for (int r = 0; r < nc; ++r) {
        const int L = sL[r], H = sH[r];
        const int32_t *Cr = sC + r * W;
        const int64_t b0 = Cr[pv];
        int v = pv > L ? pv : L;
        while (v < H && (int64_t)Cr[v + 1] - b0 <= rem) ++v;
        rem -= (int64_t)Cr[v] - b0;
        pv = v;
        w |= (uint32_t)v << ((r & 3) * 8);
        if ((r & 3) == 3) { out[r >> 2] = w; w = 0; }
        rank += sE[r * W + v];
    }
    if (nc & 3) out[(nc - 1) >> 2] = w;
    for (int q = (nc + 3) >> 2; q < g.cfg_words; ++q) out[q] = 0;
    g.rank_back[base + i] = rank;
}

hipError_t launch_annotate(const AnnotateArgs &a, hipStream_t stream)
{
    if (a.nchunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_annotate, dim3(a.nchunks), dim3(kDfsChunk), 0, stream, a);
    return hipGetLastError();
}

// --------------------------------------------------------------------- dfs
constexpr int kMaxLevels = 128;

// Dynamic LDS layout of k_dfs.
struct DfsLds {
    size_t tab, lev, stP, stM, E, LH, cut, total;
};
__host__ __device__ inline DfsLds dfs_layout(int tab_len, int levels, int tsz, int nc)
{
    DfsLds L;
    size_t o = 0;
    // the stacks hold levels 0 .. levels-2: the last level's outputs are
    // leaves, summed in place, never pushed
    const size_t depth = levels > 1 ? (size_t)(levels - 1) : 0;
    L.tab = o; o += (size_t)tab_len * 16;
    L.stP = o; o += depth * kDfsBlock * 16;
    L.lev = o; o += (size_t)levels * 16;
    L.stM = o; o += depth * kDfsBlock * 8;
    L.LH = o; o += (size_t)levels * 8;
    L.E = o; o += (size_t)tsz * 4;
    L.cut = o; o += (size_t)nc * kDfsBlock;
    L.total = (o + 15) & ~(size_t)15;
    return L;
}

// Four waves per block share the middle gates' tables.  The block takes
// chunks of kDfsChunk consecutive frontier entries of one pattern; the
// pattern's backward rank table and the cut intervals of the levels are staged
// in LDS when the pattern changes, and lanes pull entries from an LDS counter.
template <int NW, bool FP32, bool TAB_LDS>
__global__ __launch_bounds__(kDfsBlock) void k_dfs(DfsArgs g)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int nc = g.m - 1, W = table_cols(g.n), span = (g.D + 1) * nc, tsz = nc * W;
    const DfsLds Ly = dfs_layout(TAB_LDS ? g.tab_len : 0, g.levels, tsz, nc);
    double2 *tab_s = reinterpret_cast<double2 *>(smem + Ly.tab);
    const double2 *tab = TAB_LDS ? tab_s : g.tab;
    int4 *lev = reinterpret_cast<int4 *>(smem + Ly.lev);
    double2 *stP = reinterpret_cast<double2 *>(smem + Ly.stP);
    int2 *stM = reinterpret_cast<int2 *>(smem + Ly.stM);
    int32_t *sE = reinterpret_cast<int32_t *>(smem + Ly.E);
    int2 *sLH = reinterpret_cast<int2 *>(smem + Ly.LH);
    unsigned char *cut8 = smem + Ly.cut + threadIdx.x;   // cut r of this lane at cut8[r * kDfsBlock]
    __shared__ int s_p, s_cnt, s_beg, s_end;
    const int tid = threadIdx.x, bd = kDfsBlock;

    if (TAB_LDS)
        for (int i = tid; i < g.tab_len; i += bd) tab_s[i] = g.tab[i];
    for (int i = tid; i < g.levels; i += bd) lev[i] = g.level_info[i];
    __syncthreads();

    const int last = g.levels - 1;
    unsigned long long leaves = 0, edges = 0;
    int cur_p = -1;

    // blocks take chunks from their own XCD's list first (patterns p with
    // p % 8 == XCD share its L2), then help the other lists
    const int home = blockIdx.x % kXcds;
    int lst = 0;
    while (true) {
        if (tid == 0) {
            int pp = -1, beg = 0, end = 0;
            while (lst < kXcds) {
                const int x = (home + lst) % kXcds;
                const int32_t *xo = g.xoff + (size_t)x * (g.nbx + 1);
                const int j = (int)atomicAdd(g.work_counter + x, 1ull);
                if (j < xo[g.nbx]) {
                    int lo = 0, hi = g.nbx - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (xo[mid] <= j) lo = mid; else hi = mid - 1;
                    }
                    pp = x + kXcds * lo;
                    const int64_t cnt = g.off_front[pp + 1] - g.off_front[pp];
                    const int64_t b = (int64_t)(j - xo[lo]) * kDfsChunk;
                    beg = (int)b;
                    end = (int)(b + kDfsChunk < cnt ? b + kDfsChunk : cnt);
                    break;
                }
                ++lst;
            }
            s_p = pp;
            s_beg = beg;
            s_end = end;
            s_cnt = 0;
        }
        __syncthreads();
        if (s_p < 0) break;
        __syncthreads();
        const int p = s_p;
        if (p != cur_p) {
            const int16_t *plo = g.lo + (int64_t)p * span, *phi = g.hi + (int64_t)p * span;
            for (int i = tid; i < tsz; i += bd) sE[i] = g.E_back[(int64_t)p * tsz + i];
            for (int d = tid; d < g.levels; d += bd) {
                const int4 L = lev[d];
                const int t = L.y + 1;
                sLH[d] = make_int2(plo[t * nc + L.x], phi[t * nc + L.x]);
            }
            cur_p = p;
        }
        __syncthreads();
        const int beg = s_beg, end = s_end;
        const int64_t kbase = g.off_front[p];
        const double2 *Bp = g.back + g.off_back[p];

        int64_t k = 0;
        int d = 0, v = 0, vhi = -1, old = 0, prev = 0, N = 0, x1 = 0, a = 0, tb = 0, rank = 0;
        double2 P = make_double2(1.0, 0.0);
        float2 Pf = make_float2(1.f, 0.f);
        CSum sr{0.0, 0.0}, si{0.0, 0.0};

        auto init_level = [&]() {
            const int4 L = lev[d];
            a = L.x;
            tb = L.z;
            prev = a > 0 ? cut8[(a - 1) * kDfsBlock] : 0;
            const int next = a + 1 < nc ? cut8[(a + 1) * kDfsBlock] : g.n;
            old = cut8[a * kDfsBlock];
            x1 = old - prev;
            N = next - prev;
            const int2 LH = sLH[d];
            v = LH.x > prev ? LH.x : prev;
            vhi = LH.y < next ? LH.y : next;
        };
        // the lane's next entry of the chunk (false once the chunk is used up)
        auto fetch = [&]() -> bool {
            const int e = beg + atomicAdd(&s_cnt, 1);
            if (e >= end) return false;
            k = kbase + e;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                const uint32_t wq = g.cfg[k * g.cfg_words + q];
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (4 * q + b < nc) cut8[(4 * q + b) * kDfsBlock] = (unsigned char)(wq >> (8 * b));
            }
            rank = g.rank_back[k];
            d = 0;
            P = make_double2(1.0, 0.0);
            Pf = make_float2(1.f, 0.f);
            sr = CSum{0.0, 0.0};
            si = CSum{0.0, 0.0};
            init_level();
            return true;
        };

        // One pass: every leaf of a last-level range, then the climb out of
        // the exhausted levels, then one step down.  A wave runs each of the
        // three bodies once per pass with its lanes in step, where a pass of
        // one body per lane ran the three one after another for the wave's
        // lanes in different phases.
        bool live = fetch();
        while (live) {
            if (d == last && v <= vhi) {
                // the whole leaf range: independent loads
                const int wrow = tb + sector_offset(N) + x1 * (N + 1) - prev;
                const int32_t *Ea = sE + a * W;
                const int rbase = rank - Ea[old];
                for (; v <= vhi; ++v) {
                    const double2 w = tab[wrow + v];
                    const double2 b = Bp[rbase + Ea[v]];
                    double2 c2;
                    if (FP32) {
                        const float2 Pn = make_float2(Pf.x * (float)w.x - Pf.y * (float)w.y,
                                                      Pf.x * (float)w.y + Pf.y * (float)w.x);
                        c2 = cmul(make_double2((double)Pn.x, (double)Pn.y), b);
                    } else {
                        c2 = cmul(cmul(P, w), b);
                    }
                    csum_add(sr, c2.x);
                    csum_add(si, c2.y);
                    ++leaves;
                }
            }
            while (v > vhi && d > 0) {
                cut8[a * kDfsBlock] = (unsigned char)old;
                --d;
                const int2 M = stM[d * bd + tid];
                if (FP32) {
                    const double2 q = stP[d * bd + tid];
                    Pf = make_float2((float)q.x, (float)q.y);
                } else {
                    P = stP[d * bd + tid];
                }
                rank = M.y;
                v = (M.x & 0xff) + 1;
                vhi = (M.x >> 8) & 0xff;
                old = (M.x >> 16) & 0xff;
                const int4 L = lev[d];
                a = L.x;
                tb = L.z;
                prev = a > 0 ? cut8[(a - 1) * kDfsBlock] : 0;
                const int next = a + 1 < nc ? cut8[(a + 1) * kDfsBlock] : g.n;
                x1 = old - prev;
                N = next - prev;
            }
            if (v > vhi) {
                // level 0 used up: the entry is done
                const double2 f = g.front[k];
                const double2 sm = make_double2(sr.s + sr.c, si.s + si.c);
                g.front[k] = cmul(f, sm);
                live = fetch();
                continue;
            }
            // one step down (d < last here: a last-level range is used up above)
            const int wrow = tb + sector_offset(N) + x1 * (N + 1) - prev;
            const int32_t *Ea = sE + a * W;
            const int rbase = rank - Ea[old];
            const double2 w = tab[wrow + v];
            const int rn = rbase + Ea[v];
            ++edges;
            stM[d * bd + tid] = make_int2(v | (vhi << 8) | (old << 16), rank);
            if (FP32) {
                stP[d * bd + tid] = make_double2((double)Pf.x, (double)Pf.y);
                Pf = make_float2(Pf.x * (float)w.x - Pf.y * (float)w.y, Pf.x * (float)w.y + Pf.y * (float)w.x);
            } else {
                stP[d * bd + tid] = P;
                P = cmul(P, w);
            }
            cut8[a * kDfsBlock] = (unsigned char)v;
            ++d;
            rank = rn;
            init_level();
        }
        __syncthreads();
    }
    atomicAdd(g.stat_leaves, leaves);
    atomicAdd(g.stat_edges, edges + leaves);
}

// Resident blocks per CU of the k_dfs instantiation a launch would use, with
// `lds` bytes of dynamic LDS (0 when the runtime cannot say).
template <bool FP32, bool TAB_LDS>
static int dfs_occupancy_t(const DfsArgs &a, size_t lds)
{
    const int nc = a.m - 1;
    int nb = 0;
    hipError_t e;
    if (nc <= 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_dfs<2, FP32, TAB_LDS>, kDfsBlock, lds);
    else if (nc <= 16) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_dfs<4, FP32, TAB_LDS>, kDfsBlock, lds);
    else if (nc <= 24) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_dfs<6, FP32, TAB_LDS>, kDfsBlock, lds);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_dfs<8, FP32, TAB_LDS>, kDfsBlock, lds);
    return e == hipSuccess ? nb : 0;
}

static int dfs_occupancy(const DfsArgs &a, bool tab_lds, size_t lds)
{
    if (a.fp32_products) return tab_lds ? dfs_occupancy_t<true, true>(a, lds) : dfs_occupancy_t<true, false>(a, lds);
    return tab_lds ? dfs_occupancy_t<false, true>(a, lds) : dfs_occupancy_t<false, false>(a, lds);
}

// The middle gates' tables go to LDS only when that costs no resident
// blocks: the walk is bound by the latency of its reads, and more waves per
// CU hide more of it than the faster LDS table read saves (tables read
// through the vector caches with 7 blocks per CU ran the c2 middle 1.57x
// faster than LDS tables with 4).
static bool dfs_tables_in_lds(const DfsArgs &a)
{
    const int tsz = (a.m - 1) * table_cols(a.n);
    const size_t with = dfs_layout(a.tab_len, a.levels, tsz, a.m - 1).total;
    if (with > 64 * 1024) return false;
    const size_t without = dfs_layout(0, a.levels, tsz, a.m - 1).total;
    return dfs_occupancy(a, true, with) >= dfs_occupancy(a, false, without);
}

int dfs_blocks_per_cu(const DfsArgs &a)
{
    const bool tl = dfs_tables_in_lds(a);
    return dfs_occupancy(a, tl, dfs_layout(tl ? a.tab_len : 0, a.levels, (a.m - 1) * table_cols(a.n), a.m - 1).total);
}

size_t dfs_lds_bytes(const DfsArgs &a)
{
    return dfs_layout(dfs_tables_in_lds(a) ? a.tab_len : 0, a.levels, (a.m - 1) * table_cols(a.n), a.m - 1).total;
}

template <bool FP32, bool TAB_LDS>
static void launch_dfs_t(const DfsArgs &a, dim3 gr, size_t lds, hipStream_t stream)
{
    const int nc = a.m - 1;
    const dim3 bl(kDfsBlock);
    if (nc <= 8) hipLaunchKernelGGL((k_dfs<2, FP32, TAB_LDS>), gr, bl, lds, stream, a);
    else if (nc <= 16) hipLaunchKernelGGL((k_dfs<4, FP32, TAB_LDS>), gr, bl, lds, stream, a);
    else if (nc <= 24) hipLaunchKernelGGL((k_dfs<6, FP32, TAB_LDS>), gr, bl, lds, stream, a);
    else hipLaunchKernelGGL((k_dfs<8, FP32, TAB_LDS>), gr, bl, lds, stream, a);
}

hipError_t launch_dfs(const DfsArgs &a, int grid, hipStream_t stream)
{
    if (a.total == 0 || a.levels == 0) return hipSuccess;
    if (a.levels > kMaxLevels) return hipErrorInvalidValue;
    const size_t lds = dfs_lds_bytes(a);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    const bool in_lds = dfs_tables_in_lds(a);
    const dim3 gr(grid);
    if (a.fp32_products) {
        if (in_lds) launch_dfs_t<true, true>(a, gr, lds, stream);
        else launch_dfs_t<true, false>(a, gr, lds, stream);
    } else {
        if (in_lds) launch_dfs_t<false, true>(a, gr, lds, stream);
        else launch_dfs_t<false, false>(a, gr, lds, stream);
    }
    return hipGetLastError();
}

}  // namespace lofp
