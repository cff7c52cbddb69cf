// dfs.hip -- depth-first enumeration of Feynman paths (Eq. (1)) through the
// middle beam splitters, between the forward merged frontier (stage s_f) and
// the backward merged frontier (stage s_b).
//
// Each lane owns one forward-frontier configuration at a time and walks every
// sequence of beam-splitter outputs that leads from it to a configuration of
// stage s_b, one tree edge per loop iteration (push, leaf or pop), so that
// lanes of a wave advance independently and stay busy whatever the shape of
// their subtrees.  Per edge: one transition-table read from LDS and one complex
// FP64 product; at a leaf the backward-frontier amplitude of the reached
// configuration is found by its dense rank, which is kept up to date with two
// table lookups per changed cut.  Ranges come from the per-pattern cut bounds,
// so every edge taken leads to at least one valid leaf.
//
// The per-lane stack (prefix product, choice, range end, previous cut value,
// prefix rank) lives in LDS as [level][lane]; cut values live in registers as
// packed bytes.  A lane's leaves are accumulated with a compensated (TwoSum)
// complex sum, multiplied by the frontier amplitude and written back in place
// of it; the per-pattern total is formed by the reduction kernel in a fixed
// order, so results do not depend on which lane took which entry.
#include "lofp_device.h"

namespace lofp {

template <int NW>
struct PackedCuts {
    uint32_t w[NW];
    __device__ __forceinline__ int get(int idx) const
    {
        uint32_t s = w[0];
#pragma unroll
        for (int q = 1; q < NW; ++q) s = ((idx >> 2) == q) ? w[q] : s;
        return (int)((s >> ((idx & 3) * 8)) & 0xffu);
    }
    __device__ __forceinline__ void set(int idx, int val)
    {
        const int sh = (idx & 3) * 8;
#pragma unroll
        for (int q = 0; q < NW; ++q)
            if ((idx >> 2) == q) w[q] = (w[q] & ~(0xffu << sh)) | ((uint32_t)val << sh);
    }
};

template <int NW, bool TAB_LDS, bool FP32>
__global__ __launch_bounds__(64) void k_dfs(DfsArgs g)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *tab_s = reinterpret_cast<double2 *>(smem);
    int4 *lev = reinterpret_cast<int4 *>(tab_s + (TAB_LDS ? g.tab_len : 0));
    double2 *stP = reinterpret_cast<double2 *>(lev + g.levels);
    int2 *stM = reinterpret_cast<int2 *>(stP + g.levels * blockDim.x);
    const int tid = threadIdx.x, bd = blockDim.x;

    if (TAB_LDS)
        for (int i = tid; i < g.tab_len; i += bd) tab_s[i] = g.tab[i];
    for (int i = tid; i < g.levels; i += bd) lev[i] = g.level_info[i];
    __syncthreads();
    const double2 *tab = TAB_LDS ? tab_s : g.tab;

    const int nc = g.m - 1, W = table_cols(g.n), span = (g.D + 1) * nc;
    const int last = g.levels - 1;

    PackedCuts<NW> A;
    int64_t k = 0;
    const int16_t *plo = nullptr, *phi = nullptr;
    const int32_t *Eb = nullptr;
    const double2 *Bp = nullptr;
    int d = 0, v = 0, vhi = -1, old = 0, prev = 0, N = 0, x1 = 0, a = 0, tb = 0, rank = 0;
    double2 P = make_double2(1.0, 0.0);
    float2 Pf = make_float2(1.f, 0.f);
    CSum sr{0.0, 0.0}, si{0.0, 0.0};
    unsigned long long leaves = 0, edges = 0;
    bool need = true;

    auto init_level = [&]() {
        const int4 L = lev[d];
        a = L.x;
        tb = L.z;
        const int t = L.y + 1;
        prev = a > 0 ? A.get(a - 1) : 0;
        const int next = a + 1 < nc ? A.get(a + 1) : g.n;
        old = A.get(a);
        x1 = old - prev;
        N = next - prev;
        const int Lo = plo[t * nc + a], Hi = phi[t * nc + a];
        v = Lo > prev ? Lo : prev;
        vhi = Hi < next ? Hi : next;
    };

    while (true) {
        if (need) {
            const unsigned long long kk = atomicAdd(g.work_counter, 1ull);
            if (kk >= (unsigned long long)g.total) break;
            k = (int64_t)kk;
            const int p = find_pattern(g.off_front, g.B, k);
            const int64_t i = k - g.off_front[p];
            plo = g.lo + (int64_t)p * span;
            phi = g.hi + (int64_t)p * span;
            Eb = g.E_back + (int64_t)p * nc * W;
            Bp = g.back + g.off_back[p];
            const int32_t *Cf = g.C_front + (int64_t)p * nc * W;
            // unrank the frontier configuration into packed cut values
            int64_t rem = i;
            int pv = 0;
            rank = 0;
#pragma unroll
            for (int q = 0; q < NW; ++q) A.w[q] = 0;
#pragma unroll
            for (int r = 0; r < 4 * NW; ++r) {
                if (r < nc) {
                    const int t = g.st_front[r];
                    const int Lr = plo[t * nc + r], Hr = phi[t * nc + r];
                    const int32_t *Cr = Cf + r * W;
                    const int64_t base = Cr[pv];
                    int vv = pv > Lr ? pv : Lr;
                    while (vv < Hr && (int64_t)Cr[vv + 1] - base <= rem) ++vv;
                    rem -= (int64_t)Cr[vv] - base;
                    pv = vv;
                    A.w[r >> 2] |= (uint32_t)vv << ((r & 3) * 8);
                    rank += Eb[r * W + vv];
                }
            }
            d = 0;
            P = make_double2(1.0, 0.0);
            Pf = make_float2(1.f, 0.f);
            sr = CSum{0.0, 0.0};
            si = CSum{0.0, 0.0};
            init_level();
            need = false;
        }
        if (v > vhi) {
            if (d == 0) {
                const double2 f = g.front[k];
                const double2 s = make_double2(sr.s + sr.c, si.s + si.c);
                g.front[k] = cmul(f, s);
                need = true;
                continue;
            }
            A.set(a, old);
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
            prev = a > 0 ? A.get(a - 1) : 0;
            const int next = a + 1 < nc ? A.get(a + 1) : g.n;
            x1 = old - prev;
            N = next - prev;
            continue;
        }
        const double2 w = tab[tb + sector_offset(N) + x1 * (N + 1) + (v - prev)];
        const int rn = rank + Eb[a * W + v] - Eb[a * W + old];
        ++edges;
        if (FP32) {
            const float2 wf = make_float2((float)w.x, (float)w.y);
            const float2 Pn = make_float2(Pf.x * wf.x - Pf.y * wf.y, Pf.x * wf.y + Pf.y * wf.x);
            if (d == last) {
                const double2 b = Bp[rn];
                const double2 c = cmul(make_double2((double)Pn.x, (double)Pn.y), b);
                csum_add(sr, c.x);
                csum_add(si, c.y);
                ++leaves;
                ++v;
                continue;
            }
            stP[d * bd + tid] = make_double2((double)Pf.x, (double)Pf.y);
            stM[d * bd + tid] = make_int2(v | (vhi << 8) | (old << 16), rank);
            A.set(a, v);
            ++d;
            Pf = Pn;
        } else {
            const double2 Pn = cmul(P, w);
            if (d == last) {
                const double2 c = cmul(Pn, Bp[rn]);
                csum_add(sr, c.x);
                csum_add(si, c.y);
                ++leaves;
                ++v;
                continue;
            }
            stP[d * bd + tid] = P;
            stM[d * bd + tid] = make_int2(v | (vhi << 8) | (old << 16), rank);
            A.set(a, v);
            ++d;
            P = Pn;
        }
        rank = rn;
        init_level();
    }
    atomicAdd(g.stat_leaves, leaves);
    atomicAdd(g.stat_edges, edges);
}

template <bool TAB_LDS, bool FP32>
static hipError_t launch_dfs_nw(const DfsArgs &a, int grid, int block, size_t lds, hipStream_t stream)
{
    const int nc = a.m - 1;
    if (nc <= 8) hipLaunchKernelGGL((k_dfs<2, TAB_LDS, FP32>), dim3(grid), dim3(block), lds, stream, a);
    else if (nc <= 16) hipLaunchKernelGGL((k_dfs<4, TAB_LDS, FP32>), dim3(grid), dim3(block), lds, stream, a);
    else if (nc <= 24) hipLaunchKernelGGL((k_dfs<6, TAB_LDS, FP32>), dim3(grid), dim3(block), lds, stream, a);
    else hipLaunchKernelGGL((k_dfs<8, TAB_LDS, FP32>), dim3(grid), dim3(block), lds, stream, a);
    return hipGetLastError();
}

hipError_t launch_dfs(const DfsArgs &a, int grid, int block, hipStream_t stream)
{
    if (a.total == 0 || a.levels == 0) return hipSuccess;
    const size_t stack = (size_t)a.levels * block * (sizeof(double2) + sizeof(int2));
    const size_t meta = (size_t)a.levels * sizeof(int4);
    const size_t tabb = (size_t)a.tab_len * sizeof(double2);
    const bool lds_tab = tabb + meta + stack <= 64 * 1024;
    const size_t lds = (lds_tab ? tabb : 0) + meta + stack;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    if (lds_tab) {
        if (a.fp32_products) return launch_dfs_nw<true, true>(a, grid, block, lds, stream);
        return launch_dfs_nw<true, false>(a, grid, block, lds, stream);
    }
    if (a.fp32_products) return launch_dfs_nw<false, true>(a, grid, block, lds, stream);
    return launch_dfs_nw<false, false>(a, grid, block, lds, stream);
}

}  // namespace lofp
