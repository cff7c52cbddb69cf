// contract.hip -- mode-axis contraction of the path sum (Sec. II.C).
//
// The paper cuts the circuit into horizontal contraction blocks and carries,
// from one block to the next, the photon numbers of the waveguides crossing
// the boundary together with their summed amplitudes.  Here the boundary
// between modes r and r+1 is the cut r, and what crosses it over the whole
// circuit is the sequence of its values A_t(r): it changes only at the beam
// splitters on that cut, so its history is a short tuple of "versions" (the
// first fixed by S, the last by T; in a brickwork one version per block of
// two layers).  A valid path is one choice of every free version, and its
// weight is the product over splitters of W_g(x1, N, y1), each reading four
// versions: cut r before and after the splitter and cuts r-1 and r+1 at that
// time (W = 0 outside 0 <= x1, y1 <= N, which also enforces the order between
// neighbouring cuts).
//
// The sum over all versions is contracted one splitter at a time, cut by cut
// from the top (the order of the paper's blocks): a dense state holds the
// partial sum as a function of the versions that are still needed; each step
// introduces the versions its splitter touches for the first time, multiplies
// by the splitter's transition amplitude, and sums out versions that no later
// splitter reads.  The host turns the circuit into this step program once
// (which versions are live, where each one sits); per pattern only the value
// ranges (from that pattern's cut bounds) differ.
//
// One 256-thread block per pattern; the two state buffers live in LDS when
// they fit, else in a per-pattern global workspace.  Each step is one pass
// over the new state, each entry gathered in a fixed order; the final sum is
// compensated and combined in a fixed order.  With unit weights the same
// program counts the valid paths.
#include <algorithm>
#include <utility>

#include "lofp_device.h"

namespace lofp {

// A job whose state does not fit its buffers stops (whole block, uniform
// condition): the launch's overflow flag, the job's own flag and a NaN in
// its amplitude record it.
__device__ __forceinline__ void job_overflow(const ContractJob &g, int32_t *overflow)
{
    if (threadIdx.x != 0) return;
    atomicOr(overflow, 1);
    if (g.ovf) *g.ovf = 1;
    if (g.out) *g.out = nan2();
}

// Per-step layout, built once per job from the step program and the job's
// intervals (all values uniform over the block).  New entry e decodes into
// digits d_q = (e / nstr[q]) mod rad_q; the old entry it reads sits at
// sum_q d_q * mstr[q] + i0 * sstr0 + i1 * sstr1 over the summed versions.
// Per digit q: dig[q] = {nstr, mstr, magic, shift} and ninv[q] = 1 / nstr, where
// e / nstr == (e * magic) >> shift exactly for every entry index e < 2^22
// (division by an invariant integer, Granlund and Montgomery: with
// shift = 31 + ceil(log2 nstr) and magic = ceil(2^shift / nstr) the error of
// e * magic / 2^shift stays below 2^-9 / nstr).
// The splitter's photon numbers x1 (mode r in), y1 (mode r out) and N (both
// modes) are differences of its four cut references, so each is an affine
// function of the entry's first four digits and of the summed versions i0,
// i1: Q = kq + sum_j wq[j] d_j + cq0 i0 + cq1 i1 for Q in (x1, y1, N), with
// weights and coefficients in {-1, 0, 1} (q = x, y, n below).
struct StepDesc {
    int new_size, n_new, gate;
    int srad0, srad1, sstr0, sstr1;
    int kx, ky, kn;
    int cx0, cy0, cn0, cx1, cy1, cn1;
    int4 wx, wy, wn;
    int4 dig[kMaxActive];
    float ninv[kMaxActive];
};

__device__ __forceinline__ int magic_div(int e, int4 g)
{
    return (int)(((unsigned long long)(unsigned)e * (unsigned)g.z) >> g.w);
}
constexpr int kDescChunk = 16;   // step layouts built per pass

// Step layouts of up to kDescChunk steps, sixteen lanes per step (lane q owns
// digit q: its strides by prefix products over the lanes, its magic
// multiplier); the step's own fields are written by the group's first lane.
// MAGIC: also the magic multipliers (wide blocks decode with them).
template <bool MAGIC, int BS>
__device__ void build_descs(const ContractStep *steps, int nk, const int *vlo, const int *vrad, const int *spre,
                            const int *tpre, int n, StepDesc *descs)
{
    static_assert(kMaxActive == 16, "one lane per digit in groups of 16");
    const int q = threadIdx.x & 15;
    for (int k = threadIdx.x >> 4; k < nk; k += BS / 16) {
        const ContractStep &st = steps[k];
        StepDesc &d = descs[k];
        const int n_new = st.n_new, n_old = st.n_old;
        // stride of old digit q: product of the old radii before it
        const int ro = q < n_old ? vrad[st.old_vars[q]] : 1;
        int oin = ro;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const int y = __shfl_up(oin, o, 16);
            if (q >= o) oin *= y;
        }
        int ostr = __shfl_up(oin, 1, 16);
        if (q == 0) ostr = 1;
        // stride of new digit q (saturating: 2^30 marks a state too large)
        const long long rn = q < n_new ? vrad[st.new_vars[q]] : 1;
        long long nin = rn;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const long long y = __shfl_up(nin, o, 16);
            if (q >= o) nin = nin * y < (1LL << 31) ? nin * y : (1LL << 31);
        }
        long long nex = __shfl_up(nin, 1, 16);
        if (q == 0) nex = 1;
        const int nsi = nex < (1 << 30) ? (int)nex : (1 << 30);
        const int src = q < n_new ? st.new_to_old[q] : -1;
        const int ms_src = __shfl(ostr, src >= 0 ? src : 0, 16);
        const int ms = src >= 0 ? ms_src : 0;
        // magic = ceil(2^sh / nsi), only where entries get decoded: a stride of
        // 0 (an empty interval: no entries) or above 2^22 (a state too large to
        // run) never divides.  A double quotient, then exact integer fix-ups;
        // below 2^53 the quotient is off by at most one, so each runs at most
        // once.
        int sh = 0;
        unsigned long long mg = 0;
        if (MAGIC && nsi >= 1 && nsi <= (1 << 22)) {
            const int l = nsi > 1 ? 32 - __clz(nsi - 1) : 0;   // ceil(log2 nsi)
            sh = 31 + l;
            const unsigned long long two_sh = 1ULL << sh, dn = (unsigned long long)nsi;
            mg = (unsigned long long)((double)two_sh / (double)nsi);
            if (mg * dn < two_sh) ++mg;
            if (mg > 1 && (mg - 1) * dn >= two_sh) --mg;
        }
        d.dig[q] = make_int4(nsi, ms, (int)(unsigned)mg, sh);
        d.ninv[q] = 1.0f / (float)nsi;
        // old strides of the summed versions
        const int so0 = st.n_sum > 0 ? st.sum_to_old[0] : -1, so1 = st.n_sum > 1 ? st.sum_to_old[1] : -1;
        const int ss0 = __shfl(ostr, so0 >= 0 ? so0 : 0, 16), ss1 = __shfl(ostr, so1 >= 0 ? so1 : 0, 16);
        const long long ntot = __shfl(nin, 15, 16);
        if (q != 0) continue;
        d.new_size = ntot < (1 << 30) ? (int)ntot : (1 << 30);
        d.n_new = n_new;
        d.gate = st.gate;
        d.srad0 = 1; d.srad1 = 1; d.sstr0 = 0; d.sstr1 = 0;
        int slo[2] = {0, 0};
        if (st.n_sum > 0) {
            const int v = st.sum_vars[0];
            d.srad0 = vrad[v]; slo[0] = vlo[v]; d.sstr0 = so0 >= 0 ? ss0 : 0;
        }
        if (st.n_sum > 1) {
            const int v = st.sum_vars[1];
            d.srad1 = vrad[v]; slo[1] = vlo[v]; d.sstr1 = so1 >= 0 ? ss1 : 0;
        }
        // each reference as k + (digit j) + c0 i0 + c1 i1
        int K[4], J[4], C0[4], C1[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int kind = st.ref_kind[k], arg = st.ref_arg[k];
            J[k] = -1; C0[k] = 0; C1[k] = 0;
            if (kind == CREF_NEW) {
                K[k] = vlo[st.new_vars[arg]];
                J[k] = arg;
            } else if (kind == CREF_SUM) {
                K[k] = slo[arg & 1];
                C0[k] = arg == 0;
                C1[k] = arg == 1;
            } else {
                K[k] = kind == CREF_ZERO ? 0 : kind == CREF_N ? n : kind == CREF_SPRE ? spre[arg] : tpre[arg];
            }
        }
        // x1 = before - below, y1 = after - below, N = above - below
        d.kx = K[0] - K[2]; d.ky = K[1] - K[2]; d.kn = K[3] - K[2];
        d.cx0 = C0[0] - C0[2]; d.cy0 = C0[1] - C0[2]; d.cn0 = C0[3] - C0[2];
        d.cx1 = C1[0] - C1[2]; d.cy1 = C1[1] - C1[2]; d.cn1 = C1[3] - C1[2];
        int w[3][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int below = J[2] == j;
            w[0][j] = (J[0] == j) - below;
            w[1][j] = (J[1] == j) - below;
            w[2][j] = (J[3] == j) - below;
        }
        d.wx = make_int4(w[0][0], w[0][1], w[0][2], w[0][3]);
        d.wy = make_int4(w[1][0], w[1][1], w[1][2], w[1][3]);
        d.wn = make_int4(w[2][0], w[2][1], w[2][2], w[2][3]);
    }
}

// Step layout of one step by one thread (small blocks, where sixteen lanes
// per step would take several passes).  MAGIC: also the magic multipliers.
template <bool MAGIC>
__device__ inline void build_desc(const ContractStep &st, const int *vlo, const int *vrad, const int *spre,
                                  const int *tpre, int n, StepDesc &d)
{
    const int n_new = st.n_new, n_old = st.n_old;
    int ostr[kMaxActive];
    {
        int os = 1;
#pragma unroll
        for (int q = 0; q < kMaxActive; ++q) {
            ostr[q] = os;
            if (q < n_old) os *= vrad[st.old_vars[q]];
        }
    }
    long long ns = 1;
#pragma unroll
    for (int q = 0; q < kMaxActive; ++q) {
        int ms = 0;
        if (q < n_new) {
            const int v = st.new_vars[q], src = st.new_to_old[q];
#pragma unroll
            for (int q2 = 0; q2 < kMaxActive; ++q2) ms = (q2 == src) ? ostr[q2] : ms;
        }
        const int nsi = ns < (1 << 30) ? (int)ns : (1 << 30);
        // magic = ceil(2^sh / nsi), only where entries get decoded: a stride of
        // 0 (an empty interval: no entries) or above 2^22 (a state too large to
        // run) never divides.  A double quotient, then exact integer fix-ups;
        // below 2^53 the quotient is off by at most one, so each loop runs at
        // most once.
        int sh = 0;
        unsigned long long mg = 0;
        if (MAGIC && nsi >= 1 && nsi <= (1 << 22)) {
            const int l = nsi > 1 ? 32 - __clz(nsi - 1) : 0;   // ceil(log2 nsi)
            sh = 31 + l;
            const unsigned long long two_sh = 1ULL << sh, dn = (unsigned long long)nsi;
            mg = (unsigned long long)((double)two_sh / (double)nsi);
            if (mg * dn < two_sh) ++mg;
            if (mg > 1 && (mg - 1) * dn >= two_sh) --mg;
        }
        d.dig[q] = make_int4(nsi, ms, (int)(unsigned)mg, sh);
        d.ninv[q] = 1.0f / (float)nsi;
        if (q < n_new) ns *= vrad[st.new_vars[q]];
    }
    d.new_size = ns < (1 << 30) ? (int)ns : (1 << 30);
    d.n_new = n_new;
    d.gate = st.gate;
    d.srad0 = 1; d.srad1 = 1; d.sstr0 = 0; d.sstr1 = 0;
    int slo[2] = {0, 0};
    if (st.n_sum > 0) {
        const int v = st.sum_vars[0], src = st.sum_to_old[0];
        int ss = 0;
#pragma unroll
        for (int q2 = 0; q2 < kMaxActive; ++q2) ss = (q2 == src) ? ostr[q2] : ss;
        d.srad0 = vrad[v]; slo[0] = vlo[v]; d.sstr0 = ss;
    }
    if (st.n_sum > 1) {
        const int v = st.sum_vars[1], src = st.sum_to_old[1];
        int ss = 0;
#pragma unroll
        for (int q2 = 0; q2 < kMaxActive; ++q2) ss = (q2 == src) ? ostr[q2] : ss;
        d.srad1 = vrad[v]; slo[1] = vlo[v]; d.sstr1 = ss;
    }
    // each reference as k + (digit j) + c0 i0 + c1 i1
    int K[4], J[4], C0[4], C1[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int kind = st.ref_kind[k], arg = st.ref_arg[k];
        J[k] = -1; C0[k] = 0; C1[k] = 0;
        if (kind == CREF_NEW) {
            K[k] = vlo[st.new_vars[arg]];
            J[k] = arg;
        } else if (kind == CREF_SUM) {
            K[k] = slo[arg & 1];
            C0[k] = arg == 0;
            C1[k] = arg == 1;
        } else {
            K[k] = kind == CREF_ZERO ? 0 : kind == CREF_N ? n : kind == CREF_SPRE ? spre[arg] : tpre[arg];
        }
    }
    // x1 = before - below, y1 = after - below, N = above - below
    d.kx = K[0] - K[2]; d.ky = K[1] - K[2]; d.kn = K[3] - K[2];
    d.cx0 = C0[0] - C0[2]; d.cy0 = C0[1] - C0[2]; d.cn0 = C0[3] - C0[2];
    d.cx1 = C1[0] - C1[2]; d.cy1 = C1[1] - C1[2]; d.cn1 = C1[3] - C1[2];
    int w[3][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int below = J[2] == j;
        w[0][j] = (J[0] == j) - below;
        w[1][j] = (J[1] == j) - below;
        w[2][j] = (J[3] == j) - below;
    }
    d.wx = make_int4(w[0][0], w[0][1], w[0][2], w[0][3]);
    d.wy = make_int4(w[1][0], w[1][1], w[1][2], w[1][3]);
    d.wn = make_int4(w[2][0], w[2][1], w[2][2], w[2][3]);
}

// Entries of a new state for one step: each entry gathers its summed
// versions in a fixed order (i1 outer, i0 inner), the same trip counts in
// every lane.  Loads and products carry no branch, so the visits of an entry
// overlap: a visit without a transition (not 0 <= x1, y1 <= N) reads the gate
// table's zero slot and adds an exact zero.  STATS: also count the
// transitions with a nonzero source (statistics only).
//
// Decoding an entry into its digits: small blocks keep the step's strides in
// registers (an unrolled loop, float-reciprocal quotients); wide blocks, which
// run more waves per SIMD and so have fewer registers per lane, read each
// digit's stride and magic multiplier from the step layout in LDS, two
// digits per loop pass so their reads overlap.
template <bool COUNT, bool F32, int BS, bool STATS>
__device__ __forceinline__ void step_entries(const StepDesc &d, const double2 *__restrict__ bufA,
                                             double2 *__restrict__ bufB, const gdouble *__restrict__ W,
                                             unsigned zslot, unsigned long long &trans)
{
    constexpr bool kRolled = BS >= 512;
    const int n_new = d.n_new, new_size = d.new_size;
    int nstr[kRolled ? 1 : kMaxActive], mstr[kRolled ? 1 : kMaxActive];
    float ninv[kRolled ? 1 : kMaxActive];
    if (!kRolled) {
#pragma unroll
        for (int q = 0; q < (kRolled ? 1 : kMaxActive); ++q) {
            nstr[q] = d.dig[q].x;
            mstr[q] = d.dig[q].y;
            ninv[q] = d.ninv[q];
        }
    }
    const int srad0 = d.srad0, srad1 = d.srad1, sstr0 = d.sstr0, sstr1 = d.sstr1;
    const int cx0 = d.cx0, cy0 = d.cy0, cn0 = d.cn0, cx1 = d.cx1, cy1 = d.cy1, cn1 = d.cn1;
    const int4 wx = d.wx, wy = d.wy, wn = d.wn;
    for (int e = threadIdx.x; e < new_size; e += BS) {
        int rem = e, base_old = 0;
        int d0 = 0, d1 = 0, d2 = 0, d3 = 0;
        if (kRolled) {
#pragma unroll 2
            for (int q = n_new - 1; q >= 0; --q) {
                const int4 g = d.dig[q];
                const int dq = magic_div(rem, g);
                rem -= dq * g.x;
                base_old += dq * g.y;
                d0 = q == 0 ? dq : d0;
                d1 = q == 1 ? dq : d1;
                d2 = q == 2 ? dq : d2;
                d3 = q == 3 ? dq : d3;
            }
        } else {
#pragma unroll
            for (int q = (kRolled ? 1 : kMaxActive) - 1; q >= 0; --q) {
                if (q < n_new) {
                    const int dq = qdiv(rem, nstr[q], ninv[q]);
                    rem -= dq * nstr[q];
                    base_old += dq * mstr[q];
                    if (q == 0) d0 = dq;
                    if (q == 1) d1 = dq;
                    if (q == 2) d2 = dq;
                    if (q == 3) d3 = dq;
                }
            }
        }
        // the splitter's photon numbers at i0 = i1 = 0
        const int bx = d.kx + wx.x * d0 + wx.y * d1 + wx.z * d2 + wx.w * d3;
        const int by = d.ky + wy.x * d0 + wy.y * d1 + wy.z * d2 + wy.w * d3;
        const int bn = d.kn + wn.x * d0 + wn.y * d1 + wn.z * d2 + wn.w * d3;
        double2 acc = make_double2(0.0, 0.0);
        // one transition: acc += prev * W[wi] (an invalid one reads the zero slot)
        auto visit = [&](const double2 prev, bool ok, unsigned wi) {
            if (STATS && ok && (prev.x != 0.0 || prev.y != 0.0)) ++trans;
            if (COUNT && F32) {
                // absolute form: states hold sums of |path weight|, each
                // transition weighs |Re W| + |Im W| >= |W|
                const unsigned wo = 2u * (ok ? wi : zslot);
                acc.x += prev.x * (fabs(W[wo]) + fabs(W[wo + 1]));
            } else if (COUNT) {
                acc.x += ok ? prev.x : 0.0;
            } else {
                const unsigned wo = 2u * (ok ? wi : zslot);
                const double2 w = make_double2(W[wo], W[wo + 1]);
                if (F32) {
                    const float px = (float)prev.x, py = (float)prev.y, wx_ = (float)w.x, wy_ = (float)w.y;
                    acc.x += (double)(px * wx_ - py * wy_);
                    acc.y += (double)(px * wy_ + py * wx_);
                } else {
                    acc = cfma(prev, w, acc);
                }
            }
        };
        for (int i1 = 0; i1 < srad1; ++i1) {
            const int gx = bx + cx1 * i1, gy = by + cy1 * i1, gn = bn + cn1 * i1;
            const int ob = base_old + i1 * sstr1;
            // the splitter's photon numbers and the table offset of sector N,
            // sum_{k<N} (k+1)^2 = N(N+1)(2N+1)/6, stepped along i0 (the
            // polynomial is an integer for every N, so the recurrence
            // off(N+1) = off(N) + (N+1)^2 also holds through negative N,
            // where the visit reads the zero slot)
            int N = gn, x1 = gx, y1 = gy;
            int off = N * (N + 1) * (2 * N + 1) / 6;
#pragma unroll 2
            for (int i0 = 0; i0 < srad0; ++i0) {
                const double2 prev = bufA[ob + i0 * sstr0];
                const bool ok = (x1 < y1 ? x1 : y1) >= 0 && (x1 > y1 ? x1 : y1) <= N;
                visit(prev, ok, (unsigned)(off + x1 * (N + 1) + y1));
                const int Nn = N + cn0;
                off += cn0 > 0 ? Nn * Nn : (cn0 < 0 ? -(N * N) : 0);
                N = Nn; x1 += cx0; y1 += cy0;
            }
        }
        bufB[e] = acc;
    }
}

// LDS of one job: [vlo | vrad | spre | tpre | scratch int] [descriptors]
// [state buffers (2), when in LDS]
__host__ __device__ inline size_t job_lds_head(int nvars, int nc)
{
    size_t off = (size_t)(2 * nvars + 2 * nc + 4) * sizeof(int);
    off = (off + 15) & ~(size_t)15;
    off += (size_t)kDescChunk * sizeof(StepDesc);
    off = (off + 15) & ~(size_t)15;
    return off;
}

// Intervals of the job's versions and prefix sums of S and T into LDS.
// Returns false (after writing a zero amplitude) when the job has no path.
template <int BS>
__device__ bool contract_setup(const ContractJob &g, unsigned char *smem)
{
    if (*g.infeasible) {
        if (threadIdx.x == 0 && g.out) *g.out = make_double2(0.0, 0.0);
        return false;
    }
    const int nc = g.m - 1;
    int *vlo = reinterpret_cast<int *>(smem);
    int *vrad = vlo + g.nvars;
    int *spre = vrad + g.nvars;
    int *tpre = spre + nc;
    for (int r = threadIdx.x; r < nc; r += BS) {
        int s = 0, t = 0;
        for (int i = 0; i <= r; ++i) { s += g.S[i]; t += g.T[i]; }
        spre[r] = s;
        tpre[r] = t;
    }
    for (int v = threadIdx.x; v < g.nvars; v += BS) {
        const int t = g.var_time[v], r = g.var_cut[v];
        const int L = g.lo[t * nc + r], H = g.hi[t * nc + r];
        vlo[v] = L;
        vrad[v] = H - L + 1;
    }
    __syncthreads();
    return true;
}

// Largest state of the job's program (after contract_setup), by threads over steps.
template <int BS>
__device__ int job_max_state(const ContractJob &g, unsigned char *smem)
{
    const int nc = g.m - 1;
    const int *vrad = reinterpret_cast<const int *>(smem) + g.nvars;
    int *red = const_cast<int *>(vrad) + g.nvars + 2 * nc;
    if (threadIdx.x == 0) *red = 1;
    __syncthreads();
    int best = 1;
    for (int si = threadIdx.x; si < g.nsteps; si += BS) {
        const ContractStep &st = g.steps[si];
        long long ns = 1;
        for (int q = 0; q < st.n_new; ++q) ns *= vrad[st.new_vars[q]];
        const int s = ns > (1 << 22) ? (1 << 22) + 1 : (int)ns;
        best = s > best ? s : best;
    }
    atomicMax(red, best);
    __syncthreads();
    const int r = *red;
    __syncthreads();
    return r;
}

// The contraction of one pattern by one block (after contract_setup).  F32:
// each transition product prev * W is formed in FP32 (the path-product
// precision of the FP32 form); states and sums stay FP64.  STATS: count the
// transitions with a nonzero source into *stat_transitions.
template <bool COUNT, bool F32, bool LDS_STATE, int BS, bool STATS>
__device__ void contract_run(const ContractJob &g, unsigned char *smem, unsigned long long *stat_transitions,
                             int32_t *overflow, unsigned char *stage_lds = nullptr)
{
    const int nc = g.m - 1;
    const int *vlo = reinterpret_cast<const int *>(smem);
    const int *vrad = vlo + g.nvars;
    const int *spre = vrad + g.nvars;
    const int *tpre = spre + nc;
    size_t off = (size_t)(2 * g.nvars + 2 * nc + 4) * sizeof(int);
    off = (off + 15) & ~(size_t)15;
    StepDesc *desc = reinterpret_cast<StepDesc *>(smem + off);
    double2 *bufA, *bufB;
    if (!LDS_STATE && g.ws == nullptr) {
        // no global workspace was planned for this job
        job_overflow(g, overflow);
        return;
    }
    if (LDS_STATE) bufA = reinterpret_cast<double2 *>(smem + job_lds_head(g.nvars, nc));
    else bufA = g.ws;
    bufB = bufA + g.max_states;
    if (threadIdx.x == 0) bufA[0] = make_double2(1.0, 0.0);
    unsigned long long trans = 0;
    int cur_size = 1;
    for (int si = 0; si < g.nsteps; ++si) {
        const int slot = si % kDescChunk;
        if (slot == 0) {
            // layouts of the next steps, from the steps copied into LDS by
            // the whole block (the next state buffer is free until the step
            // writes it; a job whose state is in global memory gets an LDS
            // area from its caller)
            const int nk = g.nsteps - si < kDescChunk ? g.nsteps - si : kDescChunk;
            const ContractStep *src = g.steps + si;
            unsigned char *stg = LDS_STATE ? reinterpret_cast<unsigned char *>(bufB) : stage_lds;
            if (stg && (!LDS_STATE || (size_t)g.max_states * sizeof(double2) >= kDescChunk * sizeof(ContractStep))) {
                const int nw = nk * (int)(sizeof(ContractStep) / sizeof(int));
                const int *s4 = reinterpret_cast<const int *>(src);
                int *d4 = reinterpret_cast<int *>(stg);
                for (int i = threadIdx.x; i < nw; i += BS) d4[i] = s4[i];
                __syncthreads();
                src = reinterpret_cast<const ContractStep *>(stg);
            }
            if (BS >= 256) {
                build_descs<(BS >= 512), BS>(src, nk, vlo, vrad, spre, tpre, g.n, desc);
            } else {
                for (int k = threadIdx.x; k < nk; k += BS)
                    build_desc<(BS >= 512)>(src[k], vlo, vrad, spre, tpre, g.n, desc[k]);
            }
            __syncthreads();
        }
        const StepDesc &d = desc[slot];
        const int new_size = d.new_size;
        if (new_size > g.max_states) {
            job_overflow(g, overflow);
            return;
        }
        step_entries<COUNT, F32, BS, STATS>(d, bufA, bufB, (const gdouble *)(g.table + (int64_t)d.gate * g.tab_stride),
                                            (unsigned)(g.tab_stride - 1), trans);
        __syncthreads();
        double2 *t = bufA; bufA = bufB; bufB = t;
        cur_size = new_size;
    }
    if (g.state_out) {
        // half of a split contraction: hand the state over instead of summing it
        if (cur_size > g.state_cap) {
            job_overflow(g, overflow);
            return;
        }
        if (!g.out_remap || g.nsteps == 0) {
            for (int i = threadIdx.x; i < cur_size; i += BS) g.state_out[i] = bufA[i];
        } else {
            // write in the order out_pos gives (mixed radix over the same
            // radii); the step layouts' LDS is free by now
            int *s_rad = reinterpret_cast<int *>(desc), *s_ostr = s_rad + kMaxActive;
            const ContractStep &last = g.steps[g.nsteps - 1];
            const int nv = last.n_new;
            if (threadIdx.x == 0) {
                for (int q = 0; q < nv; ++q) s_rad[q] = vrad[last.new_vars[q]];
                for (int q = 0; q < nv; ++q) {
                    const int pq = (int)(g.out_pos >> (4 * q)) & 15;
                    int st = 1;
                    for (int q2 = 0; q2 < nv; ++q2)
                        if (((int)(g.out_pos >> (4 * q2)) & 15) < pq) st *= s_rad[q2];
                    s_ostr[q] = st;
                }
            }
            __syncthreads();
            for (int i = threadIdx.x; i < cur_size; i += BS) {
                int rem = i, o = 0;
                for (int q = 0; q < nv; ++q) {
                    const int r = s_rad[q];
                    const int d = rem % r;
                    rem /= r;
                    o += d * s_ostr[q];
                }
                g.state_out[o] = bufA[i];
            }
        }
        if (STATS) atomicAdd(stat_transitions, trans);
        return;
    }
    // amplitude = sum of the final state (a single entry once every version is summed)
    CSum sr{0.0, 0.0}, si{0.0, 0.0};
    for (int i = threadIdx.x; i < cur_size; i += BS) {
        const double2 x = bufA[i];
        csum_add(sr, x.x);
        csum_add(si, x.y);
    }
#pragma unroll
    for (int off2 = 32; off2 >= 1; off2 >>= 1) {
        CSum b{__shfl_xor(sr.s, off2, 64), __shfl_xor(sr.c, off2, 64)};
        CSum c{__shfl_xor(si.s, off2, 64), __shfl_xor(si.c, off2, 64)};
        if (threadIdx.x & off2) { CSum t = sr; sr = b; b = t; t = si; si = c; c = t; }
        csum_merge(sr, b);
        csum_merge(si, c);
    }
    __shared__ CSum part[2][BS / 64];
    if ((threadIdx.x & 63) == 0) { part[0][threadIdx.x >> 6] = sr; part[1][threadIdx.x >> 6] = si; }
    __syncthreads();
    if (threadIdx.x == 0) {
        CSum a = part[0][0], b = part[1][0];
        for (int w = 1; w < BS / 64; ++w) { csum_merge(a, part[0][w]); csum_merge(b, part[1][w]); }
        *g.out = make_double2(a.s + a.c, b.s + b.c);
    }
    if (STATS) atomicAdd(stat_transitions, trans);
}

// The contraction of pattern p of a single-circuit launch.
template <bool COUNT, bool F32, bool LDS_STATE, int BS, bool STATS>
__device__ void contract_pattern(const ContractArgs &g, int p, unsigned char *smem)
{
    const int nc = g.m - 1, span = (g.D + 1) * nc;
    ContractJob j;
    j.m = g.m; j.n = g.n; j.D = g.D; j.nvars = g.nvars; j.nsteps = g.nsteps;
    j.tab_stride = g.tab_stride; j.max_states = g.max_states; j.fp32 = g.fp32;
    j.steps = g.steps; j.var_cut = g.var_cut; j.var_time = g.var_time; j.table = g.table;
    j.S = g.S; j.T = g.T + (int64_t)p * g.m;
    j.lo = g.lo + (int64_t)p * span; j.hi = g.hi + (int64_t)p * span;
    j.infeasible = g.infeasible + p;
    j.out = g.out + p;
    j.ws = LDS_STATE ? nullptr : g.ws + (int64_t)p * 2 * g.max_states;
    j.state_out = nullptr;
    j.state_cap = 0;
    j.stats = g.stats;
    j.ovf = nullptr;
    if (!contract_setup<BS>(j, smem)) return;
    if (!LDS_STATE && g.lds_states > 0) {
        // this pattern's own largest state decides: LDS when it fits, else
        // its workspace slice
        if (job_max_state<BS>(j, smem) <= g.lds_states) {
            j.max_states = g.lds_states;
            contract_run<COUNT, F32, true, BS, STATS>(j, smem, g.stat_transitions, g.overflow);
        } else {
            contract_run<COUNT, F32, false, BS, STATS>(j, smem, g.stat_transitions, g.overflow);
        }
        return;
    }
    contract_run<COUNT, F32, LDS_STATE, BS, STATS>(j, smem, g.stat_transitions, g.overflow);
}

// Single circuit, one block per pattern.
template <bool COUNT, bool F32, bool LDS_STATE, int BS, bool STATS>
__global__ __launch_bounds__(BS) void k_contract(ContractArgs g)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if (g.skip && *g.skip) return;   // the batch went to the split contraction
    contract_pattern<COUNT, F32, LDS_STATE, BS, STATS>(g, (int)blockIdx.x, smem);
}

// One job of a multi-job launch (job jb; `slice` picks its workspace slice).
template <bool F32, bool LDS_STATE, int BS, bool STATS, bool ABS>
__device__ void multi_job(const ContractJob *__restrict__ jobs, int jb, int slice,
                          unsigned long long *stat_transitions, int32_t *overflow, const MultiOverride &ov,
                          unsigned char *smem)
{
    ContractJob j = jobs[jb];
    if (ov.max_states > 0) {
        j.max_states = ov.max_states;
        j.ws = ov.ws_base ? ov.ws_base + (int64_t)slice * 2 * ov.max_states : nullptr;
        if (ov.state_base) {
            j.state_out = ov.state_base + (int64_t)jb * ov.state_cap;
            j.state_cap = ov.state_cap;
        }
    }
    if (!contract_setup<BS>(j, smem)) return;
    if (ov.lds_states > 0) {
        // per-job choice: the state in LDS when this job's largest state fits
        if (job_max_state<BS>(j, smem) <= ov.lds_states) {
            j.max_states = ov.lds_states;
            contract_run<ABS, F32 || ABS, true, BS, STATS>(j, smem, stat_transitions, overflow);
        } else {
            // the LDS its state would have used stages the step programs
            unsigned char *stg = (size_t)ov.lds_states * 2 * sizeof(double2) >= kDescChunk * sizeof(ContractStep)
                                     ? smem + job_lds_head(j.nvars, j.m - 1) : nullptr;
            contract_run<ABS, F32 || ABS, false, BS, STATS>(j, smem, stat_transitions, overflow, stg);
        }
        return;
    }
    contract_run<ABS, F32 || ABS, LDS_STATE, BS, STATS>(j, smem, stat_transitions, overflow);
}

// Many circuits, one block per job (in the order ov.order gives: the
// largest jobs first, so that every CU starts one of them); or, with
// ov.next set, a grid of the blocks that can be resident: block b takes job
// b and then further jobs from that counter, in the same order, until
// *ov.njobs are taken, each block using workspace slice blockIdx.x.
// Waves per SIMD a multi-job block size is compiled for: 512-thread blocks
// run three jobs (24 waves) per CU.
template <int BS> constexpr int multi_waves_per_simd() { return BS >= 512 ? 6 : 1; }

// ABS: the absolute form (sum over paths of the product of |Re W| + |Im W|),
// which bounds the rounding error of the FP32-product form.
template <bool F32, bool LDS_STATE, int BS, bool STATS, bool ABS>
__global__ __launch_bounds__(BS, multi_waves_per_simd<BS>()) void k_contract_multi(const ContractJob *__restrict__ jobs,
                                                       unsigned long long *stat_transitions, int32_t *overflow,
                                                       MultiOverride ov)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if (ov.next) {
        // block b takes job b, then jobs gridDim.x, gridDim.x + 1, ... from
        // the counter: no atomic for the first round, and a block past the
        // job count returns at once
        __shared__ int s_k;
        const int nj = *ov.njobs;
        int k = (int)blockIdx.x;
        for (;;) {
            if (k >= nj) return;   // every block ends here once the jobs are taken
            multi_job<F32, LDS_STATE, BS, STATS, ABS>(jobs, ov.order ? ov.order[k] : k, (int)blockIdx.x,
                                                      stat_transitions, overflow, ov, smem);
            __syncthreads();   // the job is done with LDS and s_k
            if (threadIdx.x == 0) s_k = (int)gridDim.x + atomicAdd(ov.next, 1);
            __syncthreads();
            k = s_k;
        }
    }
    if (ov.njobs && (int)blockIdx.x >= *ov.njobs) return;
    const int jb = ov.order ? ov.order[blockIdx.x] : (int)blockIdx.x;
    multi_job<F32, LDS_STATE, BS, STATS, ABS>(jobs, jb, jb, stat_transitions, overflow, ov, smem);
}

// Largest state of each job's program under its intervals.
__global__ void k_multi_sizes(int count, const ContractJob *__restrict__ jobs, int *mx)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const ContractJob j = jobs[i];
    if (*j.infeasible) return;
    const int nc = j.m - 1;
    long long best = 1;
    for (int si = 0; si < j.nsteps; ++si) {
        const ContractStep &st = j.steps[si];
        long long ns = 1;
        for (int q = 0; q < st.n_new; ++q) {
            const int v = st.new_vars[q];
            const int t = j.var_time[v], r = j.var_cut[v];
            const long long rad = j.hi[t * nc + r] - j.lo[t * nc + r] + 1;
            ns *= rad > 0 ? rad : 0;
        }
        if (ns > best) best = ns;
    }
    atomicMax(mx, best > (1 << 22) ? (1 << 22) + 1 : (int)best);
}

hipError_t launch_multi_sizes(int count, const ContractJob *jobs, int *mx, hipStream_t stream)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_multi_sizes, dim3((count + 63) / 64), dim3(64), 0, stream, count, jobs, mx);
    return hipGetLastError();
}

// Largest state of the step program for each pattern (one thread per pattern).
__global__ void k_contract_sizes(ContractArgs g, int *max_size)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= g.B || g.infeasible[p]) return;
    const int nc = g.m - 1, span = (g.D + 1) * nc;
    const int16_t *lo = g.lo + (int64_t)p * span, *hi = g.hi + (int64_t)p * span;
    long long mx = 1;
    for (int si = 0; si < g.nsteps; ++si) {
        const ContractStep &st = g.steps[si];
        long long ns = 1;
        for (int q = 0; q < st.n_new; ++q) {
            const int v = st.new_vars[q];
            const int t = g.var_time[v], r = g.var_cut[v];
            ns *= (long long)(hi[t * nc + r] - lo[t * nc + r] + 1);
        }
        if (ns > mx) mx = ns;
    }
    atomicMax(max_size, mx > (1 << 22) ? (1 << 22) + 1 : (int)mx);
}

hipError_t launch_contract_sizes(const ContractArgs &a, int *max_size, hipStream_t stream)
{
    if (a.B == 0) return hipSuccess;
    hipLaunchKernelGGL(k_contract_sizes, dim3((a.B + 63) / 64), dim3(64), 0, stream, a, max_size);
    return hipGetLastError();
}

int contract_multi_resident_blocks(size_t lds_bytes, int max_states)
{
    int dev = 0, cus = 0, lds_cu = 0, thr_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        lds_cu <= 0)
        lds_cu = 160 * 1024;
    if (hipDeviceGetAttribute(&thr_cu, hipDeviceAttributeMaxThreadsPerMultiProcessor, dev) != hipSuccess ||
        thr_cu <= 0)
        thr_cu = 2048;
    const bool wide = contract_block_size(max_states) != 64;
    const int bs = wide ? 512 : 64;
    // blocks per CU: by LDS, by waves (the launch bound of a 512-thread
    // block allows six waves per SIMD, four SIMDs per CU), by threads
    int per_cu = lds_bytes > 0 ? (int)((size_t)lds_cu / lds_bytes) : thr_cu / bs;
    per_cu = std::min(per_cu, thr_cu / bs);
    if (wide) per_cu = std::min(per_cu, 4 * multi_waves_per_simd<512>() / (512 / 64));
    return cus * std::max(per_cu, 1);
}

__global__ void k_fill_i32(int32_t *p, size_t n, int32_t v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_fill_i32(int32_t *p, size_t n, int32_t v, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

size_t contract_job_lds_bytes(int nvars, int m, int max_states, bool state_in_lds)
{
    size_t off = job_lds_head(nvars, m - 1);
    return off + (state_in_lds ? (size_t)2 * max_states * sizeof(double2) : 0);
}

size_t max_lds_per_block()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        return 64 * 1024;
    return (size_t)v;
}

size_t contract_lds_bytes(const ContractArgs &a, bool state_in_lds)
{
    return contract_job_lds_bytes(a.nvars, a.m, a.max_states, state_in_lds);
}

template <bool COUNT, bool F32, bool LDS_STATE>
static void launch_contract_t(const ContractArgs &a, size_t dyn, hipStream_t stream)
{
    const bool wide = a.block ? a.block != 64 : contract_block_size(a.max_states) != 64;
    if (a.stats) {
        if (wide) hipLaunchKernelGGL((k_contract<COUNT, F32, LDS_STATE, 256, true>), dim3(a.B), dim3(256), dyn, stream, a);
        else hipLaunchKernelGGL((k_contract<COUNT, F32, LDS_STATE, 64, true>), dim3(a.B), dim3(64), dyn, stream, a);
    } else {
        if (wide) hipLaunchKernelGGL((k_contract<COUNT, F32, LDS_STATE, 256, false>), dim3(a.B), dim3(256), dyn, stream, a);
        else hipLaunchKernelGGL((k_contract<COUNT, F32, LDS_STATE, 64, false>), dim3(a.B), dim3(64), dyn, stream, a);
    }
}

hipError_t launch_contract(const ContractArgs &a, hipStream_t stream)
{
    if (a.B == 0) return hipSuccess;
    const bool in_lds = a.ws == nullptr;
    size_t dyn = contract_lds_bytes(a, in_lds);
    if (!in_lds && a.lds_states > 0)   // per-pattern choice: room for LDS states too
        dyn = contract_job_lds_bytes(a.nvars, a.m, a.lds_states, true);
    if (dyn > 64 * 1024) return hipErrorInvalidValue;
    if (a.count_only) {
        if (in_lds) launch_contract_t<true, false, true>(a, dyn, stream);
        else launch_contract_t<true, false, false>(a, dyn, stream);
    } else if (a.fp32) {
        if (in_lds) launch_contract_t<false, true, true>(a, dyn, stream);
        else launch_contract_t<false, true, false>(a, dyn, stream);
    } else {
        if (in_lds) launch_contract_t<false, false, true>(a, dyn, stream);
        else launch_contract_t<false, false, false>(a, dyn, stream);
    }
    return hipGetLastError();
}

template <bool F32, bool LDS_STATE>
static void launch_multi_t(int count, const ContractJob *jobs, size_t dyn, int max_states,
                           unsigned long long *st, int32_t *ov, MultiOverride o, bool stats, bool abs,
                           hipStream_t stream)
{
    // many small jobs: one wave each; larger jobs: 512 threads, so a step's
    // entries spread thin and the three jobs sharing a CU hide each other's
    // latencies
    const bool wide = contract_block_size(max_states) != 64;
    const dim3 g(count);
    if (abs) {
        if (wide) hipLaunchKernelGGL((k_contract_multi<true, LDS_STATE, 512, false, true>), g, dim3(512), dyn, stream, jobs, st, ov, o);
        else hipLaunchKernelGGL((k_contract_multi<true, LDS_STATE, 64, false, true>), g, dim3(64), dyn, stream, jobs, st, ov, o);
    } else if (stats) {
        if (wide) hipLaunchKernelGGL((k_contract_multi<F32, LDS_STATE, 512, true, false>), g, dim3(512), dyn, stream, jobs, st, ov, o);
        else hipLaunchKernelGGL((k_contract_multi<F32, LDS_STATE, 64, true, false>), g, dim3(64), dyn, stream, jobs, st, ov, o);
    } else {
        if (wide) hipLaunchKernelGGL((k_contract_multi<F32, LDS_STATE, 512, false, false>), g, dim3(512), dyn, stream, jobs, st, ov, o);
        else hipLaunchKernelGGL((k_contract_multi<F32, LDS_STATE, 64, false, false>), g, dim3(64), dyn, stream, jobs, st, ov, o);
    }
}

hipError_t launch_contract_multi(int count, const ContractJob *jobs, size_t lds_bytes, int max_states,
                                 bool state_in_lds, bool fp32, unsigned long long *stat_transitions,
                                 int32_t *overflow, hipStream_t stream, MultiOverride o, bool stats, bool abs)
{
    if (count == 0) return hipSuccess;
    if (lds_bytes > max_lds_per_block()) return hipErrorInvalidValue;
    unsigned long long *st = stat_transitions;
    if (fp32) {
        if (state_in_lds) launch_multi_t<true, true>(count, jobs, lds_bytes, max_states, st, overflow, o, stats, abs, stream);
        else launch_multi_t<true, false>(count, jobs, lds_bytes, max_states, st, overflow, o, stats, abs, stream);
    } else {
        if (state_in_lds) launch_multi_t<false, true>(count, jobs, lds_bytes, max_states, st, overflow, o, stats, abs, stream);
        else launch_multi_t<false, false>(count, jobs, lds_bytes, max_states, st, overflow, o, stats, abs, stream);
    }
    return hipGetLastError();
}

}  // namespace lofp
