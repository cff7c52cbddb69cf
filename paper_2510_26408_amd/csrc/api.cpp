// api.cpp -- host side of the C-ABI (include/lofp.h): circuit ingest and
// validation, light-cone tables, planning of the frontier cut, device
// workspace, and the order of kernel launches for one batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <array>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "host_internal.h"

using namespace lofp;

namespace lofp {
namespace host {

namespace {
thread_local std::string g_err;
}

lofp_status fail(lofp_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

void clear_error() { g_err.clear(); }
const char *last_error() { return g_err.c_str(); }

}  // namespace host
}  // namespace lofp

namespace lofp {
namespace host {

// -------------------------------------------------------------- light cones
// Reach intervals: a photon in mode s can be in modes [lo, hi] after some
// layers; one more layer widens the interval by the pairs that straddle its
// ends (Sec. II.B, Fig. light_cones).
void reach_step(const lofp_circuit_s &c, int layer, int &lo, int &hi)
{
    const int nl = (lo > 0 && c.cut_gate[layer * c.nc + lo - 1]) ? lo - 1 : lo;
    const int nh = (hi < c.m - 1 && c.cut_gate[layer * c.nc + hi]) ? hi + 1 : hi;
    lo = nl;
    hi = nh;
}

void build_reach(lofp_circuit_s &c)
{
    const int m = c.m, D = c.D;
    c.fr_lo.assign((D + 1) * m, 0);
    c.fr_hi.assign((D + 1) * m, 0);
    c.br_lo.assign((D + 1) * m, 0);
    c.br_hi.assign((D + 1) * m, 0);
    for (int s = 0; s < m; ++s) {
        int lo = s, hi = s;
        c.fr_lo[s] = (int8_t)lo;
        c.fr_hi[s] = (int8_t)hi;
        for (int t = 0; t < D; ++t) {
            reach_step(c, t, lo, hi);
            c.fr_lo[(t + 1) * m + s] = (int8_t)lo;
            c.fr_hi[(t + 1) * m + s] = (int8_t)hi;
        }
        lo = hi = s;
        c.br_lo[D * m + s] = (int8_t)lo;
        c.br_hi[D * m + s] = (int8_t)hi;
        for (int t = D - 1; t >= 0; --t) {
            reach_step(c, t, lo, hi);
            c.br_lo[t * m + s] = (int8_t)lo;
            c.br_hi[t * m + s] = (int8_t)hi;
        }
    }
}

void build_stage_maps(lofp_circuit_s &c)
{
    const int nc = c.nc;
    c.stage_time.assign((size_t)(c.G + 1) * nc, 0);
    for (int s = 0; s <= c.G; ++s) {
        for (int r = 0; r < nc; ++r) {
            int t;
            if (s == c.G) {
                t = c.D;
            } else {
                const int l = c.gate_layer[s];
                t = l;
                const int gid = c.gate_at[l * nc + r];
                if (gid >= 0 && gid < s) t = l + 1;
            }
            c.stage_time[(size_t)s * nc + r] = (uint8_t)t;
        }
    }
    c.cut_ngates.assign(nc, 0);
    c.cut_gates.assign((size_t)nc * std::max(c.D, 1), -1);
    for (int g = 0; g < c.G; ++g) {
        const int r = c.gate_cut[g];
        c.cut_gates[(size_t)r * std::max(c.D, 1) + c.cut_ngates[r]] = g;
        c.cut_ngates[r]++;
    }
    c.ver_at.assign((size_t)(c.D + 1) * nc, 0);
    for (int t = 1; t <= c.D; ++t)
        for (int r = 0; r < nc; ++r)
            c.ver_at[(size_t)t * nc + r] = c.ver_at[(size_t)(t - 1) * nc + r] + (c.cut_gate[(t - 1) * nc + r] ? 1 : 0);
}

lofp_status check_S(const lofp_circuit_s &c, const int32_t *S, int &n)
{
    if (!S) return fail(LOFP_EINVAL, "S is null");
    n = 0;
    for (int i = 0; i < c.m; ++i) {
        if (S[i] < 0) return fail(LOFP_EINVAL, "negative occupation in S");
        n += S[i];
    }
    if (n > kMaxPhotons) return fail(LOFP_ENOTSUP, "more than 64 photons");
    return LOFP_OK;
}

// Host S-only bounds: light cone of S and conservation, T unknown.
void s_only_bounds(const lofp_circuit_s &c, const int32_t *S, int n, std::vector<int16_t> &lo,
                   std::vector<int16_t> &hi)
{
    const int m = c.m, nc = c.nc, D = c.D;
    lo.assign((size_t)(D + 1) * nc, 0);
    hi.assign((size_t)(D + 1) * nc, (int16_t)n);
    for (int t = 0; t <= D; ++t)
        for (int r = 0; r < nc; ++r) {
            int ls = 0, hs = 0;
            for (int s = 0; s < m; ++s) {
                if (c.fr_hi[t * m + s] <= r) ls += S[s];
                if (c.fr_lo[t * m + s] <= r) hs += S[s];
            }
            lo[(size_t)t * nc + r] = (int16_t)ls;
            hi[(size_t)t * nc + r] = (int16_t)hs;
        }
    (void)propagate_bounds(m, D, n, c.cut_gate.data(), lo.data(), hi.data());
}

void s_only_cached(lofp_circuit_s &c, const int32_t *S, int n)
{
    if (!c.sb_S.empty() && std::equal(c.sb_S.begin(), c.sb_S.end(), S)) return;
    c.sb_S.assign(S, S + c.m);
    s_only_bounds(c, S, n, c.sb_lo, c.sb_hi);
    c.sb_prog = -1;
    c.sb_split.clear();
}

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Appends one array to the staging bytes at a 256-byte boundary and points
// the DevBuf view at its device copy.
template <class T>
void stage(std::vector<unsigned char> &h, size_t base, char *dev, const std::vector<T> &v, DevBuf &view)
{
    const size_t off = align256(h.size());
    const size_t bytes = v.size() * sizeof(T);
    h.resize(off + std::max<size_t>(bytes, 16), 0);
    if (bytes) std::memcpy(h.data() + off, v.data(), bytes);
    set_view(view, dev + base + off, std::max<size_t>(bytes, 16));
}

}  // namespace

// Device side of circuits: constants, the contraction program (when built)
// and the transition tables for n photons.  Everything the listed circuits
// still lack goes into one pooled block, filled by one copy and one
// table-build launch; the circuits share the block.
lofp_status init_circuits(const std::vector<std::pair<lofp_circuit_s *, int>> &list, hipStream_t s)
{
    struct Part {
        lofp_circuit_s *c;
        int n;
        bool consts, prog, table;
        int nt, stride;
        size_t tab_off;
    };
    std::vector<Part> parts;
    size_t tab_bytes = 0;
    for (const auto &e : list) {
        lofp_circuit_s *c = e.first;
        Part P{c, e.second, !c->dev_ready, !c->prog_on_device && c->prog_built && c->prog_error.empty(),
               c->n_tab < e.second, 0, 0, 0};
        bool dup = false;
        for (Part &q : parts)
            if (q.c == c) { q.n = std::max(q.n, P.n); q.table = q.c->n_tab < q.n; dup = true; }
        if (dup) continue;
        if (P.consts || P.prog || P.table) parts.push_back(P);
    }
    if (parts.empty()) return LOFP_OK;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    for (Part &P : parts) {
        if (!P.table) continue;
        P.nt = std::max(P.n, 4);
        P.stride = sector_offset(P.nt + 1) + 1;   // sectors N = 0..nt, then a zero slot
        P.tab_off = tab_bytes;
        tab_bytes += align256((size_t)std::max(P.c->G, 1) * P.stride * sizeof(double2));
    }
    // first pass: sizes (the staging layout is deterministic, so build it
    // once to learn the size, then with the device base)
    auto fill = [&](std::vector<unsigned char> &h, char *dev_base) {
        h.clear();
        for (Part &P : parts) {
            lofp_circuit_s &c = *P.c;
            if (P.consts) {
                std::vector<double> th(c.G), ph(c.G);
                for (int g = 0; g < c.G; ++g) { th[g] = c.gates[g].theta; ph[g] = c.gates[g].phi; }
                // exact mode swaps of compiled distant pairs: theta NaN marks
                // them for the table kernel, phi carries the sign of sin theta
                for (int g = 0; g < c.G; ++g)
                    if (c.gate_swap[g]) { th[g] = std::nan(""); ph[g] = c.gate_swap[g] == 1 ? -1.0 : 1.0; }
                stage(h, 0, dev_base, th, c.d_theta);
                stage(h, 0, dev_base, ph, c.d_phi);
                stage(h, 0, dev_base, c.fr_lo, c.d_fr_lo);
                stage(h, 0, dev_base, c.fr_hi, c.d_fr_hi);
                stage(h, 0, dev_base, c.br_lo, c.d_br_lo);
                stage(h, 0, dev_base, c.br_hi, c.d_br_hi);
                stage(h, 0, dev_base, c.cut_gate, c.d_cut_gate);
                stage(h, 0, dev_base, c.stage_time, c.d_stage_time);
                stage(h, 0, dev_base, c.gate_cut, c.d_gate_cut);
                stage(h, 0, dev_base, c.gate_layer, c.d_gate_layer);
                stage(h, 0, dev_base, c.cut_ngates, c.d_cut_ngates);
                stage(h, 0, dev_base, c.cut_gates, c.d_cut_gates);
                stage(h, 0, dev_base, c.ver_at, c.d_ver_at);
                stage(h, 0, dev_base, std::vector<unsigned long long>(16, 0), c.d_counters);
            }
            if (P.prog) {
                stage(h, 0, dev_base, c.var_cut, c.d_var_cut);
                stage(h, 0, dev_base, c.var_time, c.d_var_time);
                stage(h, 0, dev_base, c.steps, c.d_steps);
            }
        }
    };
    std::vector<unsigned char> h;
    fill(h, nullptr);
    const size_t jobs_off = align256(h.size());
    int njobs = 0;
    for (const Part &P : parts) njobs += P.table ? 1 : 0;
    const size_t const_bytes = jobs_off + align256((size_t)std::max(njobs, 1) * sizeof(TableJob));
    auto blk = std::make_shared<SharedBlock>();
    blk->bytes = const_bytes + tab_bytes;
    blk->device = dev;
    blk->p = pool_alloc(blk->bytes, dev);
    if (!blk->p) return fail(LOFP_ENOMEM, "device memory for circuit set-up");
    char *base = static_cast<char *>(blk->p);
    fill(h, base);
    std::vector<TableJob> jobs;
    int max_gates = 0;
    for (Part &P : parts) {
        lofp_circuit_s &c = *P.c;
        if (P.table) {
            TableJob J;
            J.G = c.G; J.n_tab = P.nt; J.stride = P.stride;
            J.theta = c.d_theta.as<double>(); J.phi = c.d_phi.as<double>();
            const size_t tb = (size_t)std::max(c.G, 1) * P.stride * sizeof(double2);
            set_view(c.d_table, base + const_bytes + P.tab_off, tb);
            J.table = c.d_table.as<double2>();
            jobs.push_back(J);
            max_gates = std::max(max_gates, c.G);
        }
    }
    h.resize(const_bytes, 0);
    if (!jobs.empty()) std::memcpy(h.data() + jobs_off, jobs.data(), jobs.size() * sizeof(TableJob));
    HIPCHK(hipMemcpyAsync(base, h.data(), const_bytes, hipMemcpyHostToDevice, s));
    HIPCHK(launch_build_tables_multi((int)jobs.size(), reinterpret_cast<const TableJob *>(base + jobs_off),
                                     max_gates, s));
    for (Part &P : parts) {
        lofp_circuit_s &c = *P.c;
        c.blocks.push_back(blk);
        if (P.consts) c.dev_ready = true;
        if (P.prog) c.prog_on_device = true;
        if (P.table) { c.n_tab = P.nt; c.tab_stride = P.stride; }
        c.pending_init = true;
    }
    return LOFP_OK;
}

lofp_status device_init(lofp_circuit_s &c, int n, hipStream_t s)
{
    return init_circuits({{&c, n}}, s);
}

lofp_status run_bounds(lofp_circuit_s &c, int B, int n, const int32_t *T_dev, hipStream_t s)
{
    const size_t span = (size_t)(c.D + 1) * c.nc;
    HIPCHK(ensure(c.d_lo, (size_t)B * span * sizeof(int16_t)));
    HIPCHK(ensure(c.d_hi, (size_t)B * span * sizeof(int16_t)));
    HIPCHK(ensure(c.d_inf, (size_t)B * sizeof(int32_t)));
    HIPCHK(launch_bounds(B, c.m, c.D, n, c.d_S.as<int32_t>(), T_dev, c.d_fr_lo.as<int8_t>(),
                         c.d_fr_hi.as<int8_t>(), c.d_br_lo.as<int8_t>(), c.d_br_hi.as<int8_t>(),
                         c.d_cut_gate.as<uint8_t>(), c.d_lo.as<int16_t>(), c.d_hi.as<int16_t>(),
                         c.d_inf.as<int32_t>(), s));
    return LOFP_OK;
}

// Contraction programs.  Every free version of a cut (the cut's value between
// two of its splitters) is a variable; every splitter is a factor reading four
// versions (cut r before and after it, cuts r-1 and r+1 at its time).  A
// schedule takes the factors in a given order: a step introduces the
// variables its factor reads for the first time and sums out those no later
// factor (and no external consumer) reads.  The live list after a step
// starts with the step's own still-live references so the kernel finds them
// at fixed positions.
void build_factors(lofp_circuit_s &c)
{
    const int nc = c.nc, Dm = std::max(c.D, 1);
    c.var_of.assign(nc, {});
    c.var_cut.clear();
    c.var_time.clear();
    for (int r = 0; r < nc; ++r) {
        const int k = c.cut_ngates[r];
        c.var_of[r].assign(k + 1, -1);
        for (int v = 1; v < k; ++v) {
            c.var_of[r][v] = (int)c.var_cut.size();
            c.var_cut.push_back(r);
            c.var_time.push_back(c.gate_layer[c.cut_gates[(size_t)r * Dm + v - 1]] + 1);
        }
    }
    c.nvars = (int)c.var_cut.size();
    auto version_ref = [&](int r, int v) -> FRef {
        if (r < 0) return {CREF_ZERO, 0};
        if (r >= nc) return {CREF_N, 0};
        if (v == 0) return {CREF_SPRE, r};
        if (v == c.cut_ngates[r]) return {CREF_TPRE, r};
        return {-1, c.var_of[r][v]};
    };
    c.fac.clear();
    c.fgate.clear();
    c.fcut.clear();
    for (int r = 0; r < nc; ++r) {
        const int k = c.cut_ngates[r];
        for (int j = 1; j <= k; ++j) {
            const int g = c.cut_gates[(size_t)r * Dm + j - 1];
            const int l = c.gate_layer[g];
            std::array<FRef, 4> f;
            f[0] = version_ref(r, j - 1);
            f[1] = version_ref(r, j);
            f[2] = r > 0 ? version_ref(r - 1, c.ver_at[(size_t)l * nc + r - 1]) : FRef{CREF_ZERO, 0};
            f[3] = r + 1 < nc ? version_ref(r + 1, c.ver_at[(size_t)l * nc + r + 1]) : FRef{CREF_N, 0};
            c.fac.push_back(f);
            c.fgate.push_back(g);
            c.fcut.push_back(r);
        }
    }
}

Schedule schedule_factors(const lofp_circuit_s &c, const std::vector<int> &order, const std::vector<char> &external)
{
    Schedule sc;
    if (c.nvars > kMaxContractVars) { sc.error = "too many free cut versions for the contraction"; return sc; }
    std::vector<int> last_use(c.nvars, -1);
    for (size_t f = 0; f < order.size(); ++f)
        for (const FRef &x : c.fac[order[f]])
            if (x.kind < 0) last_use[x.arg] = (int)f;
    for (int v = 0; v < c.nvars; ++v)
        if (!external.empty() && external[v]) last_use[v] = (int)order.size();  // never summed here
    // live versions in layout order, and each version's position in the
    // current (old) and next (new) layouts (-1: not there)
    int act[kMaxActive], n_act = 0;
    std::vector<int> pos_old(c.nvars, -1), pos_new(c.nvars, -1);
    sc.steps.reserve(order.size());
    for (size_t f = 0; f < order.size(); ++f) {
        const std::array<FRef, 4> &fr = c.fac[order[f]];
        ContractStep st;
        std::memset(&st, 0, sizeof(st));
        st.gate = c.fgate[order[f]];
        // the splitter's free versions (distinct, in reference order)
        int F[4], nF = 0;
        for (const FRef &x : fr) {
            if (x.kind >= 0) continue;
            bool seen = false;
            for (int i = 0; i < nF; ++i) seen |= F[i] == x.arg;
            if (!seen) F[nF++] = x.arg;
        }
        int nl[kMaxActive], n_nl = 0, n_sum = 0;
        bool too_many = false;
        for (int i = 0; i < nF; ++i) {
            const int v = F[i];
            if (last_use[v] == (int)f) {
                if (n_sum == 2) { too_many = true; break; }
                st.sum_vars[n_sum++] = v;
            } else {
                if (n_nl == kMaxActive) { too_many = true; break; }
                nl[n_nl++] = v;
            }
        }
        for (int q = 0; q < n_act && !too_many; ++q) {
            const int v = act[q];
            bool inF = false;
            for (int i = 0; i < nF; ++i) inF |= F[i] == v;
            if (inF) continue;
            if (n_nl == kMaxActive) { too_many = true; break; }
            nl[n_nl++] = v;
        }
        if (too_many) {
            sc.error = "contraction state has too many live cut versions";
            return sc;
        }
        st.n_new = n_nl;
        st.n_old = n_act;
        st.n_sum = n_sum;
        for (int q = 0; q < n_act; ++q) st.old_vars[q] = act[q];
        for (int q = 0; q < n_nl; ++q) {
            st.new_vars[q] = nl[q];
            st.new_to_old[q] = pos_old[nl[q]];
            pos_new[nl[q]] = q;
        }
        for (int q = 0; q < n_sum; ++q) st.sum_to_old[q] = pos_old[st.sum_vars[q]];
        for (int k = 0; k < 4; ++k) {
            const FRef &x = fr[k];
            if (x.kind >= 0) {
                st.ref_kind[k] = x.kind;
                st.ref_arg[k] = x.arg;
            } else if (n_sum > 0 && st.sum_vars[0] == x.arg) {
                st.ref_kind[k] = CREF_SUM;
                st.ref_arg[k] = 0;
            } else if (n_sum > 1 && st.sum_vars[1] == x.arg) {
                st.ref_kind[k] = CREF_SUM;
                st.ref_arg[k] = 1;
            } else {
                st.ref_kind[k] = CREF_NEW;
                st.ref_arg[k] = pos_new[x.arg];
            }
        }
        sc.steps.push_back(st);
        // the new layout becomes the old one
        for (int q = 0; q < n_act; ++q) pos_old[act[q]] = -1;
        for (int q = 0; q < n_sum; ++q) pos_old[st.sum_vars[q]] = -1;
        for (int q = 0; q < n_nl; ++q) {
            act[q] = nl[q];
            pos_old[nl[q]] = q;
            pos_new[nl[q]] = -1;
        }
        n_act = n_nl;
    }
    sc.live_out.assign(act, act + n_act);
    return sc;
}

void build_program(lofp_circuit_s &c)
{
    c.prog_built = true;
    c.prog_error.clear();
    build_factors(c);
    std::vector<int> order(c.fac.size());
    for (size_t f = 0; f < order.size(); ++f) order[f] = (int)f;
    Schedule sc = schedule_factors(c, order, {});
    if (sc.error.empty() && !sc.live_out.empty()) sc.error = "contraction program left live versions";
    c.prog_error = sc.error;
    c.steps = sc.steps;
}

// Split programs: the factors of cuts 0..rs from the top, and those of cuts
// m-2..rs+1 from the bottom, each keeping live the versions the other half
// reads.  Both halves end with the same live versions (those of cuts rs and
// rs+1 that cross the split).
SplitProgram *get_split(lofp_circuit_s &c, int rs)
{
    auto it = c.splits.find(rs);
    if (it != c.splits.end()) return it->second.get();
    auto sp = std::make_unique<SplitProgram>();
    sp->rs = rs;
    std::vector<int> top, bot;
    std::vector<char> ref_top(c.nvars, 0), ref_bot(c.nvars, 0);
    for (size_t f = 0; f < c.fac.size(); ++f) {
        const bool is_top = c.fcut[f] <= rs;
        if (is_top) top.push_back((int)f);
        for (const FRef &x : c.fac[f])
            if (x.kind < 0) (is_top ? ref_top : ref_bot)[x.arg] = 1;
    }
    // bottom half: cuts from the last upwards, each cut's splitters in time order
    for (int r = c.nc - 1; r > rs; --r)
        for (size_t f = 0; f < c.fac.size(); ++f)
            if (c.fcut[f] == r) bot.push_back((int)f);
    sp->top = schedule_factors(c, top, ref_bot);
    sp->bot = schedule_factors(c, bot, ref_top);
    if (sp->top.error.empty() && sp->bot.error.empty()) {
        std::vector<int> a = sp->top.live_out, b = sp->bot.live_out;
        std::sort(a.begin(), a.end());
        std::sort(b.begin(), b.end());
        if (a != b) sp->top.error = "split halves disagree on the crossing versions";
        if ((int)sp->top.live_out.size() > kMaxActive) sp->top.error = "too many crossing versions";
    }
    SplitProgram *raw = sp.get();
    c.splits[rs] = std::move(sp);
    return raw;
}

// Largest contraction state of a step list under the given per-time bounds.
int64_t steps_state_bound(const lofp_circuit_s &c, const std::vector<ContractStep> &steps,
                          const std::vector<int16_t> &lo, const std::vector<int16_t> &hi)
{
    int64_t mx = 1;
    for (const ContractStep &st : steps) {
        int64_t ns = 1;
        for (int q = 0; q < st.n_new; ++q) {
            const int v = st.new_vars[q];
            const size_t i = (size_t)c.var_time[v] * c.nc + c.var_cut[v];
            ns *= std::max(1, hi[i] - lo[i] + 1);
            if (ns > (1LL << 40)) return ns;
        }
        mx = std::max(mx, ns);
    }
    return mx;
}

// Largest contraction state of the full program under the given per-time bounds.
int64_t program_state_bound(const lofp_circuit_s &c, const std::vector<int16_t> &lo, const std::vector<int16_t> &hi)
{
    int64_t mx = 1;
    for (const ContractStep &st : c.steps) {
        int64_t ns = 1;
        for (int q = 0; q < st.n_new; ++q) {
            const int v = st.new_vars[q];
            const size_t i = (size_t)c.var_time[v] * c.nc + c.var_cut[v];
            ns *= std::max(1, hi[i] - lo[i] + 1);
            if (ns > (1LL << 40)) return ns;
        }
        mx = std::max(mx, ns);
    }
    return mx;
}

lofp_status prepare_program(lofp_circuit_s &c, hipStream_t s)
{
    if (!c.prog_built) build_program(c);
    if (!c.prog_error.empty()) return fail(LOFP_ENOTSUP, c.prog_error);
    if (!c.prog_on_device) {
        HIPCHK(upload(c.d_var_cut, c.var_cut, s));
        HIPCHK(upload(c.d_var_time, c.var_time, s));
        HIPCHK(upload(c.d_steps, c.steps, s));
        c.prog_on_device = true;
        c.pending_init = true;
    }
    return LOFP_OK;
}

lofp_status ready_on_stream(lofp_circuit_s &c, hipStream_t s)
{
    if (c.pending_init) {
        if (!c.ready_ev) HIPCHK(hipEventCreateWithFlags(&c.ready_ev, hipEventDisableTiming));
        HIPCHK(hipEventRecord(c.ready_ev, s));
        c.ready_stream = s;
        c.pending_init = false;
    } else if (c.ready_ev && c.ready_stream != s) {
        HIPCHK(hipStreamWaitEvent(s, c.ready_ev, 0));
    }
    return LOFP_OK;
}

lofp_status run_contract_split(lofp_circuit_s &c, const int32_t *S, int n, int B, const int32_t *T_dev,
                               lofp_c128 *out_dev, int fp32, hipStream_t s, lofp_stats *st, bool count_work,
                               int state_limit, const SplitCfg &cfg, Timer &tm, bool &used, bool &bounds_done);

// The default split: the middle cut, 52 KiB of LDS per job (three jobs per
// CU), batches of 256 to 1024 patterns split without shared halves.  A
// circuit of at least kSplitChainGates splitters also splits batches below
// 256: a job's time is its chain of one-splitter steps (1.5-2 us each,
// nearly whatever the state size), so two half-length jobs in parallel and a
// join finish sooner than one job per pattern (one pattern of a 16-mode,
// 8-photon, depth-8 circuit: 0.18 -> 0.13 ms).  Shorter circuits keep one job per pattern: there the grouping
// and join kernels cost more than the shorter chain saves.
constexpr int kSplitChainGates = 40;

SplitCfg default_split_cfg(const lofp_circuit_s &c)
{
    SplitCfg k;
    k.rs = (c.nc - 1) / 2;
    if (c.G >= kSplitChainGates) k.small_min = 1;
    return k;
}

lofp_status run_contract_split_dev(lofp_circuit_s &c, const int32_t *S, int n, int B, const int32_t *T_dev,
                                   lofp_c128 *out_dev, int fp32, hipStream_t s, lofp_stats *st, bool count_work,
                                   int state_limit, const SplitCfg &cfg, Timer &tm, bool &used);

// state_limit > 0: no state buffer holds more entries (a result whose state
// would is NaN; ENOMEM when statistics are read back).
lofp_status run_contract(lofp_circuit_s &c, const int32_t *S, int n, int B, const int32_t *T_dev,
                         lofp_c128 *out_dev, int count_only, int fp32, hipStream_t s, lofp_stats *st,
                         bool count_work, int state_limit, Timer &tm, bool allow_split = true,
                         const SplitCfg *cfg_in = nullptr)
{
    lofp_status rc = prepare_program(c, s);
    if (rc != LOFP_OK) return rc;
    rc = ready_on_stream(c, s);
    if (rc != LOFP_OK) return rc;
    bool bounds_done = false;
    const SplitCfg cfg = cfg_in ? *cfg_in : default_split_cfg(c);
    if (!count_only && allow_split && B >= std::min(64, cfg.small_min) && cfg.mode != SplitCfg::kPerPattern) {
        bool used = false;
        if (cfg.mode == SplitCfg::kDevice) {
            rc = run_contract_split_dev(c, S, n, B, T_dev, out_dev, fp32, s, st, count_work, state_limit, cfg, tm, used);
            if (rc != LOFP_OK || used) return rc;
        }
        rc = run_contract_split(c, S, n, B, T_dev, out_dev, fp32, s, st, count_work, state_limit, cfg, tm, used,
                                bounds_done);
        if (rc != LOFP_OK || used) return rc;
    }
    if (!bounds_done) {
        tm.mark();
        rc = run_bounds(c, B, n, T_dev, s);
        if (rc != LOFP_OK) return rc;
    }
    unsigned long long *ctr = c.d_counters.as<unsigned long long>();
    HIPCHK(launch_fill_i32(reinterpret_cast<int32_t *>(ctr), 16, 0, s));   // a kernel: the call may be captured
    ContractArgs a{};
    a.B = B; a.m = c.m; a.n = n; a.D = c.D;
    a.S = c.d_S.as<int32_t>();
    a.T = T_dev;
    a.lo = c.d_lo.as<int16_t>(); a.hi = c.d_hi.as<int16_t>();
    a.infeasible = c.d_inf.as<int32_t>();
    a.nvars = c.nvars;
    a.var_cut = c.d_var_cut.as<int32_t>();
    a.var_time = c.d_var_time.as<int32_t>();
    a.nsteps = (int)c.steps.size();
    a.steps = c.d_steps.as<ContractStep>();
    a.table = c.d_table.as<double2>(); a.tab_stride = c.tab_stride;
    a.out = reinterpret_cast<double2 *>(out_dev);
    a.count_only = count_only;
    a.fp32 = fp32;
    a.stat_transitions = ctr + 3;
    a.overflow = reinterpret_cast<int32_t *>(ctr + 4);
    a.stats = st != nullptr && count_work;
    // state size: the S-side bound holds for every pattern; only when it is too
    // large for LDS ask the device for this batch's exact maximum
    s_only_cached(c, S, n);
    if (c.sb_prog < 0) c.sb_prog = program_state_bound(c, c.sb_lo, c.sb_hi);
    const int64_t max_states = c.sb_prog;
    a.max_states = (int)std::min<int64_t>(max_states, 1 << 22);
    a.ws = nullptr;
    if (max_states <= (1 << 22) && contract_lds_bytes(a, true) > 64 * 1024 &&
        (size_t)B * 2 * a.max_states * sizeof(double2) <= ((size_t)1 << 30)) {
        // a workspace sized by the S-side bound (no read-back)
        HIPCHK(ensure(c.d_ws, (size_t)B * 2 * a.max_states * sizeof(double2)));
        a.ws = c.d_ws.as<double2>();
        a.lds_states = contract_lds_room(a.nvars, a.m);   // patterns whose own state fits keep it in LDS
    } else if (max_states > (1 << 22) || contract_lds_bytes(a, true) > 64 * 1024) {
        int *d_max = reinterpret_cast<int32_t *>(ctr + 5);
        HIPCHK(launch_contract_sizes(a, d_max, s));
        int mx = 0;
        HIPCHK(hipMemcpyAsync(&mx, d_max, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (mx > (1 << 22)) return fail(LOFP_ENOMEM, "contraction state exceeds 2^22 entries");
        a.max_states = std::max(mx, 1);
        if (contract_lds_bytes(a, true) > 64 * 1024) {
            HIPCHK(ensure(c.d_ws, (size_t)B * 2 * a.max_states * sizeof(double2)));
            a.ws = c.d_ws.as<double2>();
            a.lds_states = contract_lds_room(a.nvars, a.m);
        }
    }
    if (state_limit > 0 && a.max_states > state_limit) a.max_states = state_limit;
    if (a.lds_states > a.max_states) a.lds_states = a.max_states;   // the limit holds in LDS too
    tm.mark();
    HIPCHK(launch_contract(a, s));
    tm.mark();
    if (st) {
        unsigned long long h[8];
        HIPCHK(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (h[4]) return fail(LOFP_ENOMEM, "contraction workspace overflow");
        st->transitions = (int64_t)h[3];
        st->max_state = a.max_states;
    }
    return LOFP_OK;
}

// Split contraction for a batch sharing S (Sec. II.C, both ends at once): the
// top half of the contraction depends on T only through T's modes 0..rs+1, the
// bottom half only through modes rs+1..m-1, so each distinct top (bottom) part
// is contracted once and every pattern is finished by a dot product of its two
// halves over the crossing versions.  The grouping runs on the device; the
// host reads back the key claim counts (one synchronisation) to size the
// launch.

lofp_status run_contract_split(lofp_circuit_s &c, const int32_t *S, int n, int B, const int32_t *T_dev,
                               lofp_c128 *out_dev, int fp32, hipStream_t s, lofp_stats *st, bool count_work,
                               int state_limit, const SplitCfg &cfg, Timer &tm, bool &used, bool &bounds_done)
{
    used = false;
    bounds_done = false;
    const int m = c.m, nc = c.nc, span = (c.D + 1) * nc;
    if (nc < 4 || c.D < 2) return LOFP_OK;
    const int rs = cfg.rs;
    if (rs < 0 || rs > nc - 2) return LOFP_OK;
    SplitProgram *sp = get_split(c, rs);
    if (!sp->top.error.empty() || !sp->bot.error.empty()) return LOFP_OK;
    if (!sp->on_device) {
        HIPCHK(upload(sp->d_top, sp->top.steps, s));
        HIPCHK(upload(sp->d_bot, sp->bot.steps, s));
        sp->on_device = true;
    }
    if (!c.h_pin) HIPCHK(hipHostMalloc((void **)&c.h_pin, 1024, hipHostMallocDefault));
    tm.mark();
    lofp_status rc = run_bounds(c, B, n, T_dev, s);
    if (rc != LOFP_OK) return rc;
    bounds_done = true;
    // group the patterns by their two halves of T
    int cap = 1;
    while (cap < 4 * B) cap <<= 1;   // load factor <= 1/4: short probe runs
    // the table, slot keys and hulls keep the layout of the largest capacity
    // seen on this circuit (key_layout.h), so a smaller batch only touches
    // rows that earlier calls left empty
    const KeyLayoutPlan kl = plan_key_layout(c.klay, cap, span);
    HIPCHK(ensure(c.d_ktab, kl.table_bytes));
    HIPCHK(ensure(c.d_kslot, (size_t)2 * B * sizeof(int)));
    HIPCHK(ensure(c.d_kof, kl.slot_key_bytes));
    HIPCHK(ensure(c.d_krep, (size_t)2 * kKeySubs * B * sizeof(int)));
    HIPCHK(ensure(c.d_kcnt, (2 * kKeySubs + 8) * sizeof(int)));   // as the device-decided form lays it out
    HIPCHK(ensure(c.d_khull, kl.hull_bytes));
    HIPCHK(ensure(c.d_klohi, (size_t)2 * 2 * B * span * sizeof(int16_t)));
    KeyArgs ka{};
    ka.B = B; ka.m = m; ka.n = n; ka.rs = rs; ka.cap = cap; ka.span = span; ka.stride = kl.stride;
    ka.T = T_dev;
    ka.lo = c.d_lo.as<int16_t>(); ka.hi = c.d_hi.as<int16_t>();
    ka.infeasible = c.d_inf.as<int32_t>();
    ka.table = c.d_ktab.as<unsigned long long>(); ka.slot = c.d_kslot.as<int>();
    ka.slot_key = c.d_kof.as<int>(); ka.key_slot = c.d_krep.as<int>(); ka.count = c.d_kcnt.as<int>();
    ka.hlo = c.d_khull.as<int>(); ka.hhi = ka.hlo + key_hull_hi_offset(kl.stride, span);
    ka.klo = c.d_klohi.as<int16_t>(); ka.khi = ka.klo + (size_t)2 * B * span;
    ka.counters = c.d_counters.as<unsigned long long>();
    HIPCHK(ensure(c.d_korder, (size_t)2 * 2 * B * sizeof(int)));
    ka.job_bucket = c.d_korder.as<int>();
    ka.order = ka.job_bucket + 2 * B;
    // the table, the slot hulls and the counts are left empty by the jobs
    // (or reset) kernel of each call; they are cleared here only when laid
    // out anew or when a previous call stopped before that kernel
    if (kl.clear) {
        const size_t rows = (size_t)2 * kl.stride;
        HIPCHK(hipMemsetAsync(ka.table, 0xFF, rows * sizeof(unsigned long long), s));
        HIPCHK(hipMemsetAsync(ka.hlo, 0x7F, rows * span * sizeof(int), s));
        HIPCHK(hipMemsetAsync(ka.hhi, 0xFF, rows * span * sizeof(int), s));
        HIPCHK(hipMemsetAsync(ka.count, 0, 2 * kKeySubs * sizeof(int), s));
    }
    c.klay.clean = false;
    HIPCHK(launch_keys(ka, s));
    HIPCHK(hipMemcpyAsync(c.h_pin, c.d_kcnt.p, 2 * kKeySubs * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int ntop = 0, nbot = 0;
    for (int i = 0; i < kKeySubs; ++i) { ntop += c.h_pin[i]; nbot += c.h_pin[kKeySubs + i]; }
    // Split when the halves are shared (at most 3/4 as many halves as
    // patterns), or when the batch is small enough that one job per pattern
    // would leave most of the GPU idle (up to four 64-lane jobs per CU): the
    // two halves then run side by side at half the steps each.
    const bool shared = (int64_t)(ntop + nbot) * 4 <= (int64_t)B * 3;
    const bool small = B >= cfg.small_min && B <= cfg.small_max;
    if (!shared && !small) {
        // little sharing: contract per pattern (the bounds are in place)
        HIPCHK(launch_key_reset(ka, ntop, nbot, s));
        HIPCHK(hipMemsetAsync(ka.count, 0, 2 * kKeySubs * sizeof(int), s));
        c.klay.clean = true;
        return LOFP_OK;
    }
    used = true;
    // state capacity from the S-side intervals (they contain every key's
    // hull); the device is asked only when that bound is too large
    s_only_cached(c, S, n);
    auto sit = c.sb_split.find(rs);
    if (sit == c.sb_split.end())
        sit = c.sb_split.emplace(rs, std::max(steps_state_bound(c, sp->top.steps, c.sb_lo, c.sb_hi),
                                              steps_state_bound(c, sp->bot.steps, c.sb_lo, c.sb_hi))).first;
    const int64_t cap_s = sit->second;
    const int nj = ntop + nbot;
    ContractJob tj{};
    tj.m = m; tj.n = n; tj.D = c.D; tj.nvars = c.nvars; tj.tab_stride = c.tab_stride; tj.fp32 = fp32;
    tj.var_cut = c.d_var_cut.as<int32_t>(); tj.var_time = c.d_var_time.as<int32_t>();
    tj.table = c.d_table.as<double2>(); tj.S = c.d_S.as<int32_t>();
    tj.stats = st != nullptr && count_work;
    ContractJob bj = tj;
    tj.nsteps = (int)sp->top.steps.size(); tj.steps = sp->d_top.as<ContractStep>();
    bj.nsteps = (int)sp->bot.steps.size(); bj.steps = sp->d_bot.as<ContractStep>();
    // the bottom states are written in the top state's variable order
    {
        const std::vector<int> &tl = sp->top.live_out, &bl = sp->bot.live_out;
        bj.out_remap = 1;
        bj.out_pos = 0;
        for (size_t q2 = 0; q2 < bl.size(); ++q2)
            bj.out_pos |= (uint64_t)(std::find(tl.begin(), tl.end(), bl[q2]) - tl.begin()) << (4 * q2);
    }
    HIPCHK(ensure(c.d_jobs, (size_t)std::max(nj, 1) * sizeof(ContractJob)));
    HIPCHK(ensure(c.d_kinf, (size_t)2 * std::max(nj, 1) * sizeof(int32_t)));   // per job: no path, overflow
    HIPCHK(launch_key_jobs(ka, ntop, nbot, tj, bj, c.d_jobs.as<ContractJob>(), c.d_kinf.as<int32_t>(), s));
    c.klay.clean = true;
    unsigned long long *ctr = c.d_counters.as<unsigned long long>();   // zeroed by k_key_jobs
    int mx;
    if (cap_s <= (1 << 20)) {
        mx = (int)std::max<int64_t>(cap_s, 1);
    } else {
        int *d_max = reinterpret_cast<int *>(ctr + 5);
        HIPCHK(launch_multi_sizes(nj, c.d_jobs.as<ContractJob>(), d_max, s));
        HIPCHK(hipMemcpyAsync(c.h_pin + 2 * kKeySubs, d_max, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        mx = c.h_pin[2 * kKeySubs];
        if (mx > (1 << 22)) return fail(LOFP_ENOMEM, "contraction state exceeds 2^22 entries");
        mx = std::max(mx, 1);
    }
    if (state_limit > 0 && mx > state_limit) mx = state_limit;
    // LDS budget of a job (a few jobs per CU), of which what the descriptors
    // and interval arrays leave holds the two state buffers; a job whose own
    // largest state does not fit keeps them in its workspace slice
    const size_t lds_job = std::min<size_t>(max_lds_per_block(), (size_t)cfg.lds_kb * 1024);
    const size_t lds_fixed = contract_job_lds_bytes(c.nvars, m, 0, true);
    const int64_t room = lds_job > lds_fixed ? (int64_t)((lds_job - lds_fixed) / (2 * sizeof(double2))) : 0;
    const int lds_states = (int)std::min<int64_t>(mx, room);
    MultiOverride ov{mx, nullptr, nullptr, mx, lds_states, ka.order};
    if (lds_states < mx) {
        HIPCHK(ensure(c.d_ws, (size_t)nj * 2 * mx * sizeof(double2)));
        ov.ws_base = c.d_ws.as<double2>();
    }
    HIPCHK(ensure(c.d_kstate, (size_t)std::max(nj, 1) * mx * sizeof(double2)));
    ov.state_base = c.d_kstate.as<double2>();
    tm.mark();
    const bool any_lds = lds_states > 0;
    HIPCHK(launch_contract_multi(nj, c.d_jobs.as<ContractJob>(),
                                 contract_job_lds_bytes(c.nvars, m, any_lds ? lds_states : 0, any_lds),
                                 any_lds ? lds_states : mx, any_lds, fp32 != 0, ctr + 3,
                                 reinterpret_cast<int32_t *>(ctr + 4), s, ov, st != nullptr && count_work));
    tm.mark();
    JoinArgs ja{};
    ja.B = B; ja.m = m; ja.n = n; ja.D = c.D;
    ja.lo = c.d_lo.as<int16_t>(); ja.hi = c.d_hi.as<int16_t>();
    ja.infeasible = c.d_inf.as<int32_t>();
    ja.slot = ka.slot; ja.slot_key = ka.slot_key; ja.stride = kl.stride;
    ja.tlo = ka.klo; ja.thi = ka.khi;
    ja.blo = ka.klo + (size_t)B * span; ja.bhi = ka.khi + (size_t)B * span;
    ja.nshared = (int)sp->top.live_out.size();
    for (int q = 0; q < ja.nshared; ++q) {
        const int v = sp->top.live_out[q];
        ja.cidx[q] = c.var_time[v] * nc + c.var_cut[v];
    }
    ja.top_state = c.d_kstate.as<double2>();
    ja.bot_state = c.d_kstate.as<double2>() + (size_t)ntop * mx;
    ja.state_cap = mx;
    ja.top_ovf = c.d_kinf.as<int32_t>() + nj;
    ja.bot_ovf = ja.top_ovf + ntop;
    ja.out = reinterpret_cast<double2 *>(out_dev);
    HIPCHK(launch_join(ja, s));
    tm.mark();
    if (st) {
        unsigned long long h[8];
        HIPCHK(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (h[4]) return fail(LOFP_ENOMEM, "contraction workspace overflow");
        st->transitions = (int64_t)h[3];
        st->max_state = mx;
        st->split_cut = rs;
        st->lds_kb = cfg.lds_kb;
        st->split_top_keys = ntop;
        st->split_bottom_keys = nbot;
    }
    return LOFP_OK;
}

// The split contraction with every launch sized for the worst case and the
// split decided on the device (launch_key_jobs_dev): no host read-back and no
// memset, so the call can be captured in a graph.  Sizes come from the
// S-side intervals only (they contain every pattern's).  The per-pattern
// contraction is launched too and runs only when the device did not split.
// Leaves used = false, with nothing enqueued, where those sizes are too
// large (the host-sized form then runs).
lofp_status run_contract_split_dev(lofp_circuit_s &c, const int32_t *S, int n, int B, const int32_t *T_dev,
                                   lofp_c128 *out_dev, int fp32, hipStream_t s, lofp_stats *st, bool count_work,
                                   int state_limit, const SplitCfg &cfg, Timer &tm, bool &used)
{
    used = false;
    const int m = c.m, nc = c.nc, span = (c.D + 1) * nc;
    if (nc < 4 || c.D < 2) return LOFP_OK;
    const int rs = cfg.rs;
    if (rs < 0 || rs > nc - 2) return LOFP_OK;
    SplitProgram *sp = get_split(c, rs);
    if (!sp->top.error.empty() || !sp->bot.error.empty()) return LOFP_OK;
    s_only_cached(c, S, n);
    auto sit = c.sb_split.find(rs);
    if (sit == c.sb_split.end())
        sit = c.sb_split.emplace(rs, std::max(steps_state_bound(c, sp->top.steps, c.sb_lo, c.sb_hi),
                                              steps_state_bound(c, sp->bot.steps, c.sb_lo, c.sb_hi))).first;
    const int64_t cap_s = sit->second;
    if (cap_s > (1 << 20)) return LOFP_OK;
    if (c.sb_prog < 0) c.sb_prog = program_state_bound(c, c.sb_lo, c.sb_hi);
    if (c.sb_prog > (1 << 22)) return LOFP_OK;
    // the final state of a half: its crossing versions over their S-side ranges
    int64_t fin = 1;
    for (int v : sp->top.live_out) {
        const size_t i = (size_t)c.var_time[v] * nc + c.var_cut[v];
        fin *= std::max(1, c.sb_hi[i] - c.sb_lo[i] + 1);
    }
    int mx = (int)std::max<int64_t>(cap_s, 1);
    int fin_cap = (int)std::max<int64_t>(std::min<int64_t>(fin, cap_s), 1);
    int pp_states = (int)std::max<int64_t>(c.sb_prog, 1);
    if (state_limit > 0) {
        mx = std::min(mx, state_limit);
        fin_cap = std::min(fin_cap, state_limit);
        pp_states = std::min(pp_states, state_limit);
    }
    // the per-pattern contraction (runs only if the device does not split;
    // a configuration that splits every batch never runs it, so it is not
    // launched: its B blocks would only return)
    const bool always_split = cfg.small_min <= 1 && cfg.small_max == std::numeric_limits<int>::max();
    ContractArgs pa{};
    pa.B = B; pa.m = m; pa.n = n; pa.D = c.D;
    pa.nvars = c.nvars;
    pa.max_states = pp_states;
    const bool pp_lds = contract_lds_bytes(pa, true) <= 64 * 1024;
    const size_t pp_ws = pp_lds || always_split ? 0 : (size_t)B * 2 * pp_states * sizeof(double2);
    if (pp_ws > ((size_t)1 << 30)) return LOFP_OK;
    used = true;
    if (!sp->on_device) {
        HIPCHK(upload(sp->d_top, sp->top.steps, s));
        HIPCHK(upload(sp->d_bot, sp->bot.steps, s));
        sp->on_device = true;
    }
    tm.mark();
    lofp_status rc = run_bounds(c, B, n, T_dev, s);
    if (rc != LOFP_OK) return rc;
    int cap = 1;
    while (cap < 4 * B) cap <<= 1;
    const KeyLayoutPlan kl = plan_key_layout(c.klay, cap, span);
    HIPCHK(ensure(c.d_ktab, kl.table_bytes));
    HIPCHK(ensure(c.d_kslot, (size_t)2 * B * sizeof(int)));
    HIPCHK(ensure(c.d_kof, kl.slot_key_bytes));
    HIPCHK(ensure(c.d_krep, (size_t)2 * kKeySubs * B * sizeof(int)));
    HIPCHK(ensure(c.d_kcnt, (2 * kKeySubs + 8) * sizeof(int)));   // claim counts, then the decision words
    HIPCHK(ensure(c.d_khull, kl.hull_bytes));
    HIPCHK(ensure(c.d_klohi, (size_t)2 * 2 * B * span * sizeof(int16_t)));
    HIPCHK(ensure(c.d_korder, (size_t)2 * 2 * B * sizeof(int)));
    HIPCHK(ensure(c.d_jobs, (size_t)2 * B * sizeof(ContractJob)));
    HIPCHK(ensure(c.d_kinf, (size_t)4 * B * sizeof(int32_t)));
    HIPCHK(ensure(c.d_kstate, (size_t)2 * B * fin_cap * sizeof(double2)));
    KeyArgs ka{};
    ka.B = B; ka.m = m; ka.n = n; ka.rs = rs; ka.cap = cap; ka.span = span; ka.stride = kl.stride;
    ka.T = T_dev;
    ka.lo = c.d_lo.as<int16_t>(); ka.hi = c.d_hi.as<int16_t>();
    ka.infeasible = c.d_inf.as<int32_t>();
    ka.table = c.d_ktab.as<unsigned long long>(); ka.slot = c.d_kslot.as<int>();
    ka.slot_key = c.d_kof.as<int>(); ka.key_slot = c.d_krep.as<int>(); ka.count = c.d_kcnt.as<int>();
    ka.hlo = c.d_khull.as<int>(); ka.hhi = ka.hlo + key_hull_hi_offset(kl.stride, span);
    ka.klo = c.d_klohi.as<int16_t>(); ka.khi = ka.klo + (size_t)2 * B * span;
    ka.counters = c.d_counters.as<unsigned long long>();
    ka.job_bucket = c.d_korder.as<int>();
    ka.order = ka.job_bucket + 2 * B;
    ka.ctl = ka.count + 2 * kKeySubs;
    ka.small_min = cfg.small_min;
    ka.small_max = cfg.small_max;
    if (kl.clear) {
        // fill kernels rather than memsets (the call may be captured)
        const size_t rows = (size_t)2 * kl.stride;
        HIPCHK(launch_fill_i32(reinterpret_cast<int32_t *>(ka.table), rows * 2, -1, s));
        HIPCHK(launch_fill_i32(ka.hlo, rows * span, kHullEmptyLo, s));
        HIPCHK(launch_fill_i32(ka.hhi, rows * span, kHullEmptyHi, s));
        HIPCHK(launch_fill_i32(ka.count, 2 * kKeySubs, 0, s));
    }
    c.klay.clean = false;
    HIPCHK(launch_keys(ka, s));
    ContractJob tj{};
    tj.m = m; tj.n = n; tj.D = c.D; tj.nvars = c.nvars; tj.tab_stride = c.tab_stride; tj.fp32 = fp32;
    tj.var_cut = c.d_var_cut.as<int32_t>(); tj.var_time = c.d_var_time.as<int32_t>();
    tj.table = c.d_table.as<double2>(); tj.S = c.d_S.as<int32_t>();
    tj.stats = st != nullptr && count_work;
    ContractJob bj = tj;
    tj.nsteps = (int)sp->top.steps.size(); tj.steps = sp->d_top.as<ContractStep>();
    bj.nsteps = (int)sp->bot.steps.size(); bj.steps = sp->d_bot.as<ContractStep>();
    {
        const std::vector<int> &tl = sp->top.live_out, &bl = sp->bot.live_out;
        bj.out_remap = 1;
        bj.out_pos = 0;
        for (size_t q2 = 0; q2 < bl.size(); ++q2)
            bj.out_pos |= (uint64_t)(std::find(tl.begin(), tl.end(), bl[q2]) - tl.begin()) << (4 * q2);
    }
    HIPCHK(launch_key_jobs_dev(ka, tj, bj, c.d_jobs.as<ContractJob>(), c.d_kinf.as<int32_t>(),
                               c.d_kstate.as<double2>(), fin_cap, s));
    c.klay.clean = true;
    unsigned long long *ctr = c.d_counters.as<unsigned long long>();   // zeroed by the jobs kernel
    const size_t lds_job = std::min<size_t>(max_lds_per_block(), (size_t)cfg.lds_kb * 1024);
    const size_t lds_fixed = contract_job_lds_bytes(c.nvars, m, 0, true);
    const int64_t room = lds_job > lds_fixed ? (int64_t)((lds_job - lds_fixed) / (2 * sizeof(double2))) : 0;
    const int lds_states = (int)std::min<int64_t>(mx, room);
    const bool any_lds = lds_states > 0;
    const size_t lds_bytes = contract_job_lds_bytes(c.nvars, m, any_lds ? lds_states : 0, any_lds);
    // a grid of the blocks that can be resident, taking the jobs, largest
    // first, from a counter: no block waits for a job that does not exist,
    // and each block keeps one workspace slice for the jobs whose state does
    // not fit LDS
    const int grid =
        std::max(1, std::min(2 * B, contract_multi_resident_blocks(lds_bytes, any_lds ? lds_states : mx)));
    MultiOverride ov{mx, nullptr, nullptr, fin_cap, lds_states, ka.order};
    ov.njobs = ka.ctl + 1;
    ov.next = ka.ctl + 4;
    if (lds_states < mx) {
        HIPCHK(ensure(c.d_ws, (size_t)grid * 2 * mx * sizeof(double2)));
        ov.ws_base = c.d_ws.as<double2>();
    }
    tm.mark();
    HIPCHK(launch_contract_multi(grid, c.d_jobs.as<ContractJob>(), lds_bytes, any_lds ? lds_states : mx, any_lds,
                                 fp32 != 0, ctr + 3, reinterpret_cast<int32_t *>(ctr + 4), s, ov,
                                 st != nullptr && count_work));
    pa.S = c.d_S.as<int32_t>();
    pa.T = T_dev;
    pa.lo = c.d_lo.as<int16_t>(); pa.hi = c.d_hi.as<int16_t>();
    pa.infeasible = c.d_inf.as<int32_t>();
    pa.var_cut = c.d_var_cut.as<int32_t>();
    pa.var_time = c.d_var_time.as<int32_t>();
    pa.nsteps = (int)c.steps.size();
    pa.steps = c.d_steps.as<ContractStep>();
    pa.table = c.d_table.as<double2>(); pa.tab_stride = c.tab_stride;
    pa.out = reinterpret_cast<double2 *>(out_dev);
    pa.fp32 = fp32;
    pa.stat_transitions = ctr + 3;
    pa.overflow = reinterpret_cast<int32_t *>(ctr + 4);
    pa.stats = st != nullptr && count_work;
    pa.skip = ka.ctl;
    if (!always_split) {
        if (!pp_lds) {
            HIPCHK(ensure(c.d_ws2, pp_ws));
            pa.ws = c.d_ws2.as<double2>();
            pa.lds_states = std::min(contract_lds_room(pa.nvars, pa.m), pp_states);
        }
        HIPCHK(launch_contract(pa, s));
    }
    tm.mark();
    JoinArgs ja{};
    ja.B = B; ja.m = m; ja.n = n; ja.D = c.D;
    ja.lo = c.d_lo.as<int16_t>(); ja.hi = c.d_hi.as<int16_t>();
    ja.infeasible = c.d_inf.as<int32_t>();
    ja.slot = ka.slot; ja.slot_key = ka.slot_key; ja.stride = kl.stride;
    ja.tlo = ka.klo; ja.thi = ka.khi;
    ja.blo = ka.klo + (size_t)B * span; ja.bhi = ka.khi + (size_t)B * span;
    ja.nshared = (int)sp->top.live_out.size();
    for (int q = 0; q < ja.nshared; ++q) {
        const int v = sp->top.live_out[q];
        ja.cidx[q] = c.var_time[v] * nc + c.var_cut[v];
    }
    ja.top_state = c.d_kstate.as<double2>();
    ja.bot_state = ja.top_state + (size_t)B * fin_cap;
    ja.state_cap = fin_cap;
    ja.top_ovf = c.d_kinf.as<int32_t>() + 2 * (size_t)B;
    ja.bot_ovf = ja.top_ovf + B;
    ja.split_flag = ka.ctl;
    ja.out = reinterpret_cast<double2 *>(out_dev);
    HIPCHK(launch_join(ja, s));
    tm.mark();
    if (st) {
        unsigned long long h[8];
        int ctl[4];
        HIPCHK(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(ctl, ka.ctl, sizeof(ctl), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (h[4]) return fail(LOFP_ENOMEM, "contraction workspace overflow");
        st->transitions = (int64_t)h[3];
        st->max_state = ctl[0] ? mx : pp_states;
        st->split_cut = ctl[0] ? rs : 0;
        st->lds_kb = ctl[0] ? cfg.lds_kb : 0;
        st->split_top_keys = ctl[0] ? ctl[2] : 0;
        st->split_bottom_keys = ctl[0] ? ctl[3] : 0;
    }
    return LOFP_OK;
}

// The tuner: times each candidate way of contracting a batch sharing S (the
// split cut one either side of the middle, 40 / 52 / 64 KiB of LDS per
// split job, or one job per pattern) on the caller's data, three timed calls
// after one untimed, and returns the one with the smallest median.  Every
// candidate computes the same amplitudes (in another order of summation).
lofp_status tune_contract(lofp_circuit_s &c, const int32_t *S, int n, int B, const int32_t *T_dev, lofp_c128 *out_dev,
                          int fp32, int state_limit, hipStream_t s, SplitCfg &best)
{
    std::vector<SplitCfg> cand;
    const SplitCfg d = default_split_cfg(c);
    for (int drs : {0, -1, 1})
        for (int kb : {52, 40, 64}) {
            SplitCfg k = d;
            k.rs = d.rs + drs;
            k.lds_kb = kb;
            if (k.rs < 0 || k.rs > c.nc - 2) continue;
            cand.push_back(k);
            // the same, split whatever the sharing: no per-pattern launch
            k.small_min = 1;
            k.small_max = std::numeric_limits<int>::max();
            cand.push_back(k);
        }
    if (B < d.small_max && B < 256) {
        // a small batch: split or not, whatever the circuit's default
        for (int drs : {0, -1, 1}) {
            SplitCfg k = d;
            k.rs = d.rs + drs;
            k.small_min = d.small_min == 1 ? 256 : 1;
            if (k.rs >= 0 && k.rs <= c.nc - 2) cand.push_back(k);
        }
    }
    SplitCfg pp = d;
    pp.mode = SplitCfg::kPerPattern;
    cand.push_back(pp);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) { (void)hipEventDestroy(e0); return fail(LOFP_EDEVICE, hipGetErrorString(he)); }
    double best_ms = 1e300;
    lofp_status rc = LOFP_OK;
    for (const SplitCfg &k : cand) {
        Timer off;
        rc = run_contract(c, S, n, B, T_dev, out_dev, 0, fp32, s, nullptr, false, state_limit, off, true, &k);
        if (rc != LOFP_OK) break;
        float t[3];
        for (int r = 0; r < 3 && rc == LOFP_OK; ++r) {
            he = hipEventRecord(e0, s);
            if (he == hipSuccess) rc = run_contract(c, S, n, B, T_dev, out_dev, 0, fp32, s, nullptr, false, state_limit,
                                                    off, true, &k);
            if (rc != LOFP_OK) break;
            if (he == hipSuccess) he = hipEventRecord(e1, s);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            if (he == hipSuccess) he = hipEventElapsedTime(&t[r], e0, e1);
            if (he != hipSuccess) rc = fail(LOFP_EDEVICE, hipGetErrorString(he));
        }
        if (rc != LOFP_OK) break;
        std::sort(t, t + 3);
        if (t[1] < best_ms) { best_ms = t[1]; best = k; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

lofp_status run_pathsum(lofp_circuit_s &c, const int32_t *S, int n, int B, const int32_t *T_dev,
                        lofp_c128 *out_dev, const lofp_opts &o, hipStream_t s, lofp_stats *st, Timer &tm)
{
    const int D = c.D, G = c.G, nc = c.nc;
    // ---- plan the cut: backward frontier over the last two layers (their
    // path is unique given the configuration before them, Eq. (10)), forward
    // frontier one layer earlier; the layers in between are enumerated
    int bl = o.bwd_layer, fl = o.fwd_layer;
    if (bl < 0) bl = std::min(D, std::max({0, D - 2, fl}));
    if (bl < 0 || bl > D) return fail(LOFP_EINVAL, "need 0 <= bwd_layer <= depth");
    if (fl > bl) return fail(LOFP_EINVAL, "need fwd_layer <= bwd_layer");
    const bool auto_fwd = fl < 0;
    const int sb = c.layer_start[bl];
    // stage slots: with an automatic forward cut every stage up to the
    // backward frontier is counted first, so the cut can be chosen from the
    // exact frontier sizes
    std::vector<int32_t> slot_stage;
    std::vector<int> slot_of(G + 1, -1);
    const int s_last_fwd = auto_fwd ? sb : c.layer_start[fl];
    for (int st_ = 0; st_ <= s_last_fwd; ++st_) { slot_of[st_] = (int)slot_stage.size(); slot_stage.push_back(st_); }
    for (int st_ = sb; st_ <= G; ++st_)
        if (slot_of[st_] < 0) { slot_of[st_] = (int)slot_stage.size(); slot_stage.push_back(st_); }
    const int nslots = (int)slot_stage.size();
    const size_t tsz = (size_t)nc * table_cols(n);

    tm.mark();  // 0
    lofp_status rc = run_bounds(c, B, n, T_dev, s);
    if (rc != LOFP_OK) return rc;
    HIPCHK(upload(c.d_slot_stage, slot_stage, s));
    HIPCHK(ensure(c.d_C, (size_t)nslots * B * tsz * sizeof(int32_t)));
    HIPCHK(ensure(c.d_E, (size_t)nslots * B * tsz * sizeof(int32_t)));
    HIPCHK(ensure(c.d_count, ((size_t)nslots * B + 1) * sizeof(int32_t)));
    int32_t *overflow = c.d_count.as<int32_t>() + (size_t)nslots * B;
    HIPCHK(hipMemsetAsync(overflow, 0, sizeof(int32_t), s));
    HIPCHK(launch_stage_tables(B, c.m, D, n, nslots, c.d_slot_stage.as<int32_t>(), c.d_stage_time.as<uint8_t>(),
                               c.d_lo.as<int16_t>(), c.d_hi.as<int16_t>(), c.d_inf.as<int32_t>(),
                               c.d_C.as<int32_t>(), c.d_E.as<int32_t>(), c.d_count.as<int32_t>(), overflow, s));
    std::vector<int32_t> cnt((size_t)nslots * B + 1);
    HIPCHK(hipMemcpyAsync(cnt.data(), c.d_count.p, cnt.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    // per-slot totals (a count of -1 marks a state space beyond 2^31)
    std::vector<int64_t> tot(nslots, 0);
    std::vector<char> over(nslots, 0);
    for (int k = 0; k < nslots; ++k)
        for (int p = 0; p < B; ++p) {
            const int32_t v = cnt[(size_t)k * B + p];
            if (v < 0) over[k] = 1; else tot[k] += v;
        }
    if (auto_fwd) {
        // Schroedinger-Feynman trade-off: merge forward as far as the frontier
        // fits the memory budget; the layers left between the frontiers are
        // enumerated depth-first (at most kMaxDfsGates splitters, for the
        // LDS stack)
        size_t budget = (size_t)std::max(o.frontier_budget_kb, 0) << 10;
        if (budget == 0) {
            size_t fr = 0, total = 0;
            budget = hipMemGetInfo(&fr, &total) == hipSuccess ? fr / 4 : ((size_t)8 << 30);
        }
        fl = -1;
        for (int cand = bl; cand >= 0; --cand) {
            const int sf_c = c.layer_start[cand];
            if (sb - sf_c > kMaxDfsGates) break;
            bool ok = true;
            int64_t mx = 0;
            for (int st_ = 0; st_ <= sf_c && ok; ++st_) {
                const int k = slot_of[st_];
                if (over[k]) ok = false;
                mx = std::max(mx, tot[k]);
            }
            if (ok && (size_t)mx * 2 * sizeof(double2) <= budget) { fl = cand; break; }
        }
        if (fl < 0) return fail(LOFP_ENOMEM, "no forward frontier fits the memory budget within the depth-first limit");
    }
    const int sf = c.layer_start[fl];
    for (int st_ = 0; st_ <= sf; ++st_)
        if (over[slot_of[st_]]) return fail(LOFP_ENOMEM, "a frontier state space exceeds 2^31 states");
    for (int st_ = sb; st_ <= G; ++st_)
        if (over[slot_of[st_]]) return fail(LOFP_ENOMEM, "a frontier state space exceeds 2^31 states");
    std::vector<int64_t> off((size_t)nslots * (B + 1));
    std::vector<int32_t> coff((size_t)nslots * (B + 1));   // chunk offsets (kGateChunk)
    std::vector<int32_t> nch(nslots);
    static_assert(kGateChunk == kDfsChunk, "one chunk size for frontier and depth-first kernels");
    for (int k = 0; k < nslots; ++k) {
        int64_t acc = 0, ca = 0;
        for (int p = 0; p < B; ++p) {
            const int64_t v = std::max<int32_t>(0, cnt[(size_t)k * B + p]);
            off[(size_t)k * (B + 1) + p] = acc;
            coff[(size_t)k * (B + 1) + p] = (int32_t)std::min<int64_t>(ca, 0x7fffffff);
            acc += v;
            ca += (v + kGateChunk - 1) / kGateChunk;
        }
        off[(size_t)k * (B + 1) + B] = acc;
        coff[(size_t)k * (B + 1) + B] = (int32_t)std::min<int64_t>(ca, 0x7fffffff);
        nch[k] = (int32_t)std::min<int64_t>(ca, 0x7fffffff);
    }
    // per-XCD chunk lists: patterns x, x+8, x+16, ... for XCD x
    const int nbx = (B + kXcds - 1) / kXcds;
    std::vector<int32_t> xoff((size_t)nslots * kXcds * (nbx + 1));
    std::vector<int32_t> xgrid(nslots);
    for (int k = 0; k < nslots; ++k) {
        int longest = 0;
        for (int x = 0; x < kXcds; ++x) {
            int32_t *xo = xoff.data() + ((size_t)k * kXcds + x) * (nbx + 1);
            int64_t acc = 0;
            for (int i = 0; i < nbx; ++i) {
                xo[i] = (int32_t)acc;
                const int p = x + kXcds * i;
                if (p < B) acc += (std::max<int32_t>(0, cnt[(size_t)k * B + p]) + kGateChunk - 1) / kGateChunk;
            }
            xo[nbx] = (int32_t)std::min<int64_t>(acc, 0x7fffffff);
            longest = std::max(longest, xo[nbx]);
        }
        xgrid[k] = (int)std::min<int64_t>((int64_t)longest * kXcds, 0x7fffffff);
    }
    HIPCHK(upload(c.d_off, off, s));
    HIPCHK(upload(c.d_coff, xoff, s));
    (void)coff;
    const int64_t *d_off = c.d_off.as<int64_t>();
    auto xoffp = [&](int stage) { return c.d_coff.as<int32_t>() + (size_t)slot_of[stage] * kXcds * (nbx + 1); };
    auto gridp = [&](int stage) { return xgrid[slot_of[stage]]; };
    auto offp = [&](int stage) { return d_off + (size_t)slot_of[stage] * (B + 1); };
    auto Cp = [&](int stage) { return c.d_C.as<int32_t>() + (size_t)slot_of[stage] * B * tsz; };
    auto Ep = [&](int stage) { return c.d_E.as<int32_t>() + (size_t)slot_of[stage] * B * tsz; };
    auto totp = [&](int stage) { return tot[slot_of[stage]]; };
    int64_t fmax = 0, bmax = 0, bfs_states = 0;
    for (int st_ = 0; st_ <= sf; ++st_) { fmax = std::max(fmax, totp(st_)); bfs_states += totp(st_); }
    for (int st_ = sb; st_ <= G; ++st_) { bmax = std::max(bmax, totp(st_)); bfs_states += totp(st_); }
    HIPCHK(ensure(c.d_fa, (size_t)fmax * sizeof(double2)));
    HIPCHK(ensure(c.d_fb, (size_t)fmax * sizeof(double2)));
    HIPCHK(ensure(c.d_ba, (size_t)bmax * sizeof(double2)));
    HIPCHK(ensure(c.d_bb, (size_t)bmax * sizeof(double2)));
    tm.mark();  // 1

    // ---- forward frontier: S expanded through gates 0..sf-1
    double2 *F = c.d_fa.as<double2>(), *Fn = c.d_fb.as<double2>();
    HIPCHK(launch_seed(B, offp(0), F, s));
    const size_t span = (size_t)(D + 1) * nc;
    for (int g = 0; g < sf; ++g) {
        GateArgs a{};
        a.B = B; a.m = c.m; a.n = n; a.D = D; a.cut = c.gate_cut[g];
        a.st_tgt = c.d_stage_time.as<uint8_t>() + (size_t)(g + 1) * nc;
        a.st_src = c.d_stage_time.as<uint8_t>() + (size_t)g * nc;
        a.lo = c.d_lo.as<int16_t>(); a.hi = c.d_hi.as<int16_t>();
        a.C_tgt = Cp(g + 1); a.E_src = Ep(g);
        a.off_tgt = offp(g + 1); a.off_src = offp(g);
        a.W = c.d_table.as<double2>() + (size_t)g * c.tab_stride;
        a.src = F; a.dst = Fn; a.total_tgt = totp(g + 1);
        a.xoff = xoffp(g + 1); a.nbx = nbx; a.grid = gridp(g + 1);
        HIPCHK(launch_gate(a, true, s));
        std::swap(F, Fn);
    }
    tm.mark();  // 2
    // ---- backward frontier: T expanded back through gates G-1..sb
    double2 *Bv = c.d_ba.as<double2>(), *Bn = c.d_bb.as<double2>();
    HIPCHK(launch_seed(B, offp(G), Bv, s));
    for (int g = G - 1; g >= sb; --g) {
        GateArgs a{};
        a.B = B; a.m = c.m; a.n = n; a.D = D; a.cut = c.gate_cut[g];
        a.st_tgt = c.d_stage_time.as<uint8_t>() + (size_t)g * nc;
        a.st_src = c.d_stage_time.as<uint8_t>() + (size_t)(g + 1) * nc;
        a.lo = c.d_lo.as<int16_t>(); a.hi = c.d_hi.as<int16_t>();
        a.C_tgt = Cp(g); a.E_src = Ep(g + 1);
        a.off_tgt = offp(g); a.off_src = offp(g + 1);
        a.W = c.d_table.as<double2>() + (size_t)g * c.tab_stride;
        a.src = Bv; a.dst = Bn; a.total_tgt = totp(g);
        a.xoff = xoffp(g); a.nbx = nbx; a.grid = gridp(g);
        HIPCHK(launch_gate(a, false, s));
        std::swap(Bv, Bn);
    }
    tm.mark();  // 3
    (void)span;
    unsigned long long *ctr = c.d_counters.as<unsigned long long>();
    HIPCHK(hipMemsetAsync(ctr, 0, 16 * sizeof(unsigned long long), s));
    const int levels = sb - sf;
    if (levels > 0 && totp(sf) > 0) {
        // compact image of the middle gates' tables: sectors up to the largest
        // photon number the S-side light cone allows at each gate
        std::vector<int16_t> slo, shi;
        s_only_bounds(c, S, n, slo, shi);
        std::vector<int4> info(levels);
        std::vector<int> nmax(levels);
        int tab_len = 0;
        for (int d = 0; d < levels; ++d) {
            const int g = sf + d, a = c.gate_cut[g], l = c.gate_layer[g];
            const int up = a + 1 < nc ? shi[(size_t)l * nc + a + 1] : n;
            const int dn = a > 0 ? slo[(size_t)l * nc + a - 1] : 0;
            nmax[d] = std::max(0, std::min(n, up - dn));
            info[d] = make_int4(a, l, tab_len, 0);
            tab_len += sector_offset(nmax[d] + 1);
        }
        HIPCHK(upload(c.d_levels, info, s));
        HIPCHK(ensure(c.d_tab_mid, (size_t)std::max(tab_len, 1) * sizeof(double2)));
        for (int d = 0; d < levels; ++d)
            HIPCHK(hipMemcpyAsync(c.d_tab_mid.as<double2>() + info[d].z,
                                  c.d_table.as<double2>() + (size_t)(sf + d) * c.tab_stride,
                                  (size_t)sector_offset(nmax[d] + 1) * sizeof(double2), hipMemcpyDeviceToDevice, s));
        const int words = nc <= 8 ? 2 : nc <= 16 ? 4 : nc <= 24 ? 6 : 8;
        HIPCHK(ensure(c.d_cfg, (size_t)totp(sf) * words * sizeof(uint32_t)));
        HIPCHK(ensure(c.d_rankb, (size_t)totp(sf) * sizeof(int32_t)));
        AnnotateArgs an{};
        an.B = B; an.m = c.m; an.n = n; an.D = D;
        an.st_front = c.d_stage_time.as<uint8_t>() + (size_t)sf * nc;
        an.lo = c.d_lo.as<int16_t>(); an.hi = c.d_hi.as<int16_t>();
        an.C_front = Cp(sf); an.E_back = Ep(sb);
        an.off_front = offp(sf);
        an.xoff = xoffp(sf); an.nbx = nbx; an.nchunks = gridp(sf);
        an.cfg_words = words;
        an.cfg = c.d_cfg.as<uint32_t>();
        an.rank_back = c.d_rankb.as<int32_t>();
        HIPCHK(launch_annotate(an, s));
        DfsArgs a{};
        a.B = B; a.m = c.m; a.n = n; a.D = D;
        a.levels = levels;
        a.level_info = c.d_levels.as<int4>();
        a.tab = c.d_tab_mid.as<double2>();
        a.tab_len = tab_len;
        a.lo = c.d_lo.as<int16_t>(); a.hi = c.d_hi.as<int16_t>();
        a.E_back = Ep(sb);
        a.cfg = c.d_cfg.as<uint32_t>();
        a.rank_back = c.d_rankb.as<int32_t>();
        a.cfg_words = words;
        a.off_front = offp(sf); a.off_back = offp(sb);
        a.front = F; a.back = Bv;
        a.total = totp(sf);
        a.xoff = xoffp(sf);
        a.nbx = nbx;
        a.work_counter = ctr + 8;
        a.stat_leaves = ctr + 1;
        a.stat_edges = ctr + 2;
        a.fp32_products = o.precision == LOFP_PREC_FP32;
        const size_t lds = dfs_lds_bytes(a);
        if (lds > 64 * 1024)
            return fail(LOFP_ENOTSUP, "too many beam splitters between the frontiers for the LDS stack; "
                                      "move the forward frontier later");
        int dev = 0, ncu = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
                ncu = prop.multiProcessorCount;
        }
        const int occ = dfs_blocks_per_cu(a);
        const int per_cu = occ > 0 ? occ : (int)std::max<size_t>(1, std::min<size_t>(8, (160 * 1024) / std::max<size_t>(lds, 1)));
        const int64_t grid = std::min<int64_t>((int64_t)ncu * per_cu, std::max(gridp(sf), 1));
        tm.mark();  // 4
        HIPCHK(launch_dfs(a, (int)std::max<int64_t>(grid, 1), s));
        tm.mark();  // 5
        HIPCHK(launch_reduce(B, offp(sf), F, nullptr, reinterpret_cast<double2 *>(out_dev), s));
    } else {
        tm.mark();  // 4
        tm.mark();  // 5
        if (sf == sb)
            HIPCHK(launch_reduce(B, offp(sf), F, Bv, reinterpret_cast<double2 *>(out_dev), s));
        else
            HIPCHK(launch_reduce(B, offp(sf), F, nullptr, reinterpret_cast<double2 *>(out_dev), s));
    }
    tm.mark();  // 6
    if (st) {
        st->fwd_layer = fl;
        st->bwd_layer = bl;
        st->dfs_levels = levels;
        st->frontier_states = totp(sf);
        st->backward_states = totp(sb);
        st->bfs_states = bfs_states;
        unsigned long long h[8];
        HIPCHK(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        st->dfs_leaves = (int64_t)h[1];
        st->dfs_edges = (int64_t)h[2];
        if (tm.on) {
            st->ms_plan = tm.ms(0, 1);
            st->ms_forward = tm.ms(1, 2);
            st->ms_backward = tm.ms(2, 3);
            st->ms_dfs = tm.ms(4, 5);
            st->ms_reduce = tm.ms(5, 6);
        }
    }
    return LOFP_OK;
}

lofp_status clone_circuit(const lofp_circuit_s &c, lofp_circuit_s **out)
{
    std::vector<int32_t> lens(std::max(c.D, 1), 0);
    for (int l = 0; l < c.D; ++l) lens[l] = c.layer_start[l + 1] - c.layer_start[l];
    lofp_circuit k = nullptr;
    lofp_status rc = lofp_circuit_create(c.m, c.D, lens.data(), c.gates.empty() ? nullptr : c.gates.data(), &k);
    if (rc != LOFP_OK) return rc;
    // the compiled layers hold adjacent pairs only, so the gate order is c's
    k->gate_swap = c.gate_swap;
    k->user_gate = c.user_gate;
    k->user_depth = c.user_depth;
    k->compiled = c.compiled;
    k->tuned = c.tuned;
    *out = k;
    return LOFP_OK;
}

}  // namespace host
}  // namespace lofp

using namespace lofp::host;

// ===================================================================== C-ABI
extern "C" {

const char *lofp_last_error(void) { return lofp::host::last_error(); }

const char *lofp_version(void) { return "lofp-mi355x 0.1 (gfx950)"; }

lofp_status lofp_circuit_create(int32_t m, int32_t n_layers, const int32_t *layer_len, const lofp_bs *bs,
                                lofp_circuit *out)
{
    if (!out) return fail(LOFP_EINVAL, "out is null");
    if (m < 2) return fail(LOFP_EINVAL, "need at least 2 modes");
    if (m > kMaxModes) return fail(LOFP_ENOTSUP, "more than 32 modes");
    if (n_layers < 0 || n_layers > 250) return fail(LOFP_EINVAL, "bad layer count");
    if (n_layers > 0 && !layer_len) return fail(LOFP_EINVAL, "layer_len is null");
    int total = 0;
    for (int l = 0; l < n_layers; ++l) {
        if (layer_len[l] < 0) return fail(LOFP_EINVAL, "negative layer length");
        total += layer_len[l];
    }
    if (total > 0 && !bs) return fail(LOFP_EINVAL, "bs is null");
    // Check the layers, then compile them to adjacent pairs.  A splitter on
    // distant modes (a, b) (Sec. II.A allows distant connections) becomes
    // the exact product P^-1 BS(a, a+1) P, where P moves mode b next to a by
    // exact swaps [[0, 1], [-1, 0]] (theta = -pi/2, phi = 0) on (b-1, b),
    // ..., (a+1, a+2) (each maps mode k+1 to +k and mode k to -(k+1)) and
    // P^-1 is the chain of their inverses (theta = pi/2, phi = 0) in reverse
    // order: on single-photon states it maps mode a to U11 a + U21 b and
    // mode b to U12 a + U22 b and fixes every other mode, so every Fock
    // amplitude is that of the original splitter.  The swaps' tables are
    // built with cos theta = 0 exactly (a permutation with signs), so they
    // add no path of nonzero weight.  The adjacent splitters of a layer stay
    // one layer; each distant one adds its own layers after them (splitters
    // of one layer commute).
    std::vector<std::vector<lofp_bs>> ilayers;
    std::vector<std::vector<uint8_t>> iswap;   // per internal splitter: 0, or 1 / 2 for a swap / its inverse
    std::vector<int> user_gate;   // internal gate of each user splitter, in application order
    bool compiled = false;
    int k = 0;
    for (int l = 0; l < n_layers; ++l) {
        std::vector<lofp_bs> layer(bs + k, bs + k + layer_len[l]);
        k += layer_len[l];
        std::vector<int> used(m, 0);
        for (const auto &b : layer) {
            if (b.a < 0 || b.b < 0 || b.a >= m || b.b >= m || b.a >= b.b)
                return fail(LOFP_EINVAL, "beam splitter modes out of range or a >= b");
            if (used[b.a] || used[b.b]) return fail(LOFP_EINVAL, "mode used twice in one layer");
            used[b.a] = used[b.b] = 1;
        }
        std::vector<lofp_bs> adj;
        std::vector<std::pair<int, lofp_bs>> far;   // (position in the layer, splitter)
        for (size_t i = 0; i < layer.size(); ++i) {
            if (layer[i].b == layer[i].a + 1) adj.push_back(layer[i]);
            else far.emplace_back((int)i, layer[i]);
        }
        std::stable_sort(adj.begin(), adj.end(), [](const lofp_bs &x, const lofp_bs &y) { return x.a < y.a; });
        // user gate order inside a layer is by upper mode, as the internal layer stores it
        std::vector<lofp_bs> order = layer;
        std::stable_sort(order.begin(), order.end(), [](const lofp_bs &x, const lofp_bs &y) { return x.a < y.a; });
        int first = 0;
        for (const auto &L : ilayers) first += (int)L.size();
        std::map<int, int> gate_of_a;   // upper mode -> internal gate id
        if (!adj.empty() || far.empty()) {
            for (size_t i = 0; i < adj.size(); ++i) gate_of_a[adj[i].a] = first + (int)i;
            first += (int)adj.size();
            ilayers.push_back(adj);
            iswap.push_back(std::vector<uint8_t>(adj.size(), 0));
        }
        std::stable_sort(far.begin(), far.end(),
                         [](const std::pair<int, lofp_bs> &x, const std::pair<int, lofp_bs> &y) { return x.second.a < y.second.a; });
        for (const auto &fb : far) {
            compiled = true;
            const lofp_bs &b = fb.second;
            const double half_pi = 1.5707963267948966;
            for (int q = b.b - 1; q >= b.a + 1; --q) {
                ilayers.push_back({lofp_bs{q, q + 1, -half_pi, 0.0}});
                iswap.push_back({1});
                ++first;
            }
            ilayers.push_back({lofp_bs{b.a, b.a + 1, b.theta, b.phi}});
            iswap.push_back({0});
            gate_of_a[b.a] = first++;
            for (int q = b.a + 1; q <= b.b - 1; ++q) {
                ilayers.push_back({lofp_bs{q, q + 1, half_pi, 0.0}});
                iswap.push_back({2});
                ++first;
            }
        }
        for (const auto &b : order) user_gate.push_back(gate_of_a[b.a]);
    }
    if (ilayers.size() > 250) return fail(LOFP_ENOTSUP, "more than 250 layers after compiling distant pairs");
    const int D = (int)ilayers.size();
    auto *c = new lofp_circuit_s();
    c->m = m;
    c->D = D;
    c->nc = m - 1;
    c->user_depth = n_layers;
    c->compiled = compiled;
    c->user_gate = user_gate;
    c->cut_gate.assign((size_t)std::max(D, 1) * c->nc, 0);
    c->gate_at.assign((size_t)std::max(D, 1) * c->nc, -1);
    c->layer_start.assign(D + 1, 0);
    for (int l = 0; l < D; ++l) {
        c->layer_start[l] = (int)c->gates.size();
        for (size_t i = 0; i < ilayers[l].size(); ++i) {
            const lofp_bs &b = ilayers[l][i];
            const int g = (int)c->gates.size();
            c->gates.push_back(b);
            c->gate_swap.push_back(iswap[l][i]);
            c->gate_cut.push_back(b.a);
            c->gate_layer.push_back(l);
            c->cut_gate[(size_t)l * c->nc + b.a] = 1;
            c->gate_at[(size_t)l * c->nc + b.a] = g;
        }
    }
    c->G = (int)c->gates.size();
    c->layer_start[D] = c->G;
    build_reach(*c);
    build_stage_maps(*c);
    *out = c;
    return LOFP_OK;
}

lofp_status lofp_circuit_compiled(lofp_circuit c, int32_t *n_layers, int32_t *layer_len, lofp_bs *bs,
                                  int32_t capacity)
{
    if (!c || !n_layers) return fail(LOFP_EINVAL, "null argument");
    *n_layers = c->D;
    if (!layer_len && !bs) return LOFP_OK;
    if (!layer_len || !bs) return fail(LOFP_EINVAL, "layer_len and bs go together");
    if (capacity < c->G) return fail(LOFP_EINVAL, "bs holds fewer than the compiled splitters");
    for (int l = 0; l < c->D; ++l) layer_len[l] = c->layer_start[l + 1] - c->layer_start[l];
    for (int g = 0; g < c->G; ++g) bs[g] = c->gates[g];
    return LOFP_OK;
}

lofp_status lofp_circuit_destroy(lofp_circuit c)
{
    if (!c) return fail(LOFP_EINVAL, "null circuit");
    DevBuf *bufs[] = {&c->d_table, &c->d_theta, &c->d_phi, &c->d_fr_lo, &c->d_fr_hi, &c->d_br_lo, &c->d_br_hi,
                      &c->d_cut_gate, &c->d_stage_time, &c->d_gate_cut, &c->d_gate_layer, &c->d_cut_ngates,
                      &c->d_cut_gates, &c->d_ver_at, &c->d_var_cut, &c->d_var_time, &c->d_steps, &c->d_S, &c->d_lo, &c->d_hi, &c->d_inf, &c->d_C, &c->d_E,
                      &c->d_count, &c->d_slot_stage, &c->d_off, &c->d_coff, &c->d_fa, &c->d_fb, &c->d_ba, &c->d_bb,
                      &c->d_levels, &c->d_tab_mid, &c->d_counters, &c->d_T, &c->d_out, &c->d_ws,
                      &c->d_cfg, &c->d_rankb, &c->d_ktab, &c->d_kslot, &c->d_kof, &c->d_krep, &c->d_kcnt,
                      &c->d_khull, &c->d_klohi, &c->d_kinf, &c->d_jobs, &c->d_kstate, &c->d_korder, &c->d_ws2};
    // pooled blocks are reused at once, so no work of this circuit may be left
    if (c->dev_ready || !c->blocks.empty()) (void)hipDeviceSynchronize();
    for (DevBuf *b : bufs) release(*b);
    if (c->h_pin) (void)hipHostFree(c->h_pin);
    if (c->ready_ev) (void)hipEventDestroy(c->ready_ev);
    if (c->last_ev) (void)hipEventDestroy(c->last_ev);
    delete c;
    return LOFP_OK;
}

lofp_status lofp_light_cone(lofp_circuit c, int32_t layer, int32_t mode, int32_t *past_lo, int32_t *past_hi,
                            int32_t *fut_lo, int32_t *fut_hi)
{
    if (!c || !past_lo || !past_hi || !fut_lo || !fut_hi) return fail(LOFP_EINVAL, "null argument");
    if (c->compiled) return fail(LOFP_ENOTSUP, "host queries of layers and cuts describe circuits of adjacent pairs only");
    if (layer < 0 || layer > c->D || mode < 0 || mode >= c->m) return fail(LOFP_EINVAL, "bad layer or mode");
    int lo = mode, hi = mode;
    for (int t = layer - 1; t >= 0; --t) reach_step(*c, t, lo, hi);
    *past_lo = lo;
    *past_hi = hi;
    lo = hi = mode;
    for (int t = layer; t < c->D; ++t) reach_step(*c, t, lo, hi);
    *fut_lo = lo;
    *fut_hi = hi;
    return LOFP_OK;
}

lofp_status lofp_bounds(lofp_circuit c, const int32_t *S, const int32_t *T, int32_t *lo, int32_t *hi,
                        int32_t *feasible)
{
    if (!c || !T || !lo || !hi || !feasible) return fail(LOFP_EINVAL, "null argument");
    if (c->compiled) return fail(LOFP_ENOTSUP, "host queries of layers and cuts describe circuits of adjacent pairs only");
    int n = 0;
    lofp_status rc = check_S(*c, S, n);
    if (rc != LOFP_OK) return rc;
    const size_t span = (size_t)(c->D + 1) * c->nc;
    std::vector<int16_t> L(span), H(span);
    int nT = 0;
    for (int i = 0; i < c->m; ++i) {
        if (T[i] < 0) return fail(LOFP_EINVAL, "negative occupation in T");
        nT += T[i];
    }
    int infeasible = 1;
    if (nT == n) {
        light_cone_bounds(c->m, c->D, S, T, c->fr_lo.data(), c->fr_hi.data(), c->br_lo.data(), c->br_hi.data(),
                          L.data(), H.data());
        infeasible = propagate_bounds(c->m, c->D, n, c->cut_gate.data(), L.data(), H.data());
    } else {
        std::fill(L.begin(), L.end(), 1);
        std::fill(H.begin(), H.end(), 0);
    }
    for (size_t i = 0; i < span; ++i) { lo[i] = L[i]; hi[i] = H[i]; }
    *feasible = !infeasible;
    return LOFP_OK;
}

lofp_status lofp_bounds_batch(lofp_circuit c, const int32_t *S, int32_t batch, const int32_t *T, int32_t *lo,
                              int32_t *hi, int32_t *feasible)
{
    if (!c) return fail(LOFP_EINVAL, "null circuit");
    if (c->compiled) return fail(LOFP_ENOTSUP, "host queries of layers and cuts describe circuits of adjacent pairs only");
    if (batch < 0) return fail(LOFP_EINVAL, "negative batch");
    if (batch > 0 && (!T || !lo || !hi || !feasible)) return fail(LOFP_EINVAL, "null argument");
    int n = 0;
    lofp_status rc = check_S(*c, S, n);
    if (rc != LOFP_OK) return rc;
    if (batch == 0) return LOFP_OK;
    for (int64_t i = 0; i < (int64_t)batch * c->m; ++i)
        if (T[i] < 0) return fail(LOFP_EINVAL, "negative occupation in T");
    std::lock_guard<std::mutex> lk(c->mu);
    hipStream_t s = nullptr;
    rc = device_init(*c, n, s);
    if (rc != LOFP_OK) return rc;
    StreamUse use(*c, s);
    HIPCHK(use.begin());
    std::vector<int32_t> Sv(S, S + c->m);
    if (Sv != c->S_dev) {
        HIPCHK(upload(c->d_S, Sv, s));
        c->S_dev = Sv;
    }
    rc = ready_on_stream(*c, s);
    if (rc != LOFP_OK) return rc;
    const size_t span = (size_t)(c->D + 1) * c->nc;
    DevBuf dT;
    std::vector<int16_t> L((size_t)batch * span), H((size_t)batch * span);
    std::vector<int32_t> inf(batch);
    hipError_t e = ensure(dT, (size_t)batch * c->m * sizeof(int32_t));
    if (e == hipSuccess)
        e = hipMemcpyAsync(dT.p, T, (size_t)batch * c->m * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        rc = run_bounds(*c, batch, n, dT.as<int32_t>(), s);
        if (rc == LOFP_OK) {
            e = hipMemcpyAsync(L.data(), c->d_lo.p, L.size() * sizeof(int16_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(H.data(), c->d_hi.p, H.size() * sizeof(int16_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(inf.data(), c->d_inf.p, inf.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
    }
    release(dT);
    if (rc != LOFP_OK) return rc;
    if (e != hipSuccess) return fail(LOFP_EDEVICE, hipGetErrorString(e));
    for (size_t i = 0; i < L.size(); ++i) { lo[i] = L[i]; hi[i] = H[i]; }
    for (int p = 0; p < batch; ++p) feasible[p] = !inf[p];
    return LOFP_OK;
}

lofp_status lofp_bs_table(lofp_circuit c, int32_t gate, int32_t N, lofp_c128 *out)
{
    if (!c || !out) return fail(LOFP_EINVAL, "null argument");
    if (gate < 0 || gate >= (int32_t)c->user_gate.size() || N < 0 || N > kMaxPhotons)
        return fail(LOFP_EINVAL, "bad gate or N");
    gate = c->user_gate[gate];
    std::lock_guard<std::mutex> lk(c->mu);
    hipStream_t s = nullptr;
    lofp_status rc = device_init(*c, N, s);
    if (rc != LOFP_OK) return rc;
    HIPCHK(hipMemcpyAsync(out, c->d_table.as<double2>() + (size_t)gate * c->tab_stride + sector_offset(N),
                          (size_t)(N + 1) * (N + 1) * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return LOFP_OK;
}

// Largest batch one pass takes; larger batches run in passes of this size.
// It bounds the per-call workspace of the split contraction, whose grouping
// keeps a hash slot and a hull row of 2 x span ints per four patterns of the
// batch (about 280 MiB at this size on the 16-mode, depth-8 workload).
constexpr int kMaxPass = 32768;

lofp_status lofp_amplitudes_device(lofp_circuit c, const int32_t *S, int32_t batch, const int32_t *T_dev,
                                   lofp_c128 *out_dev, const lofp_opts *opts, void *stream, lofp_stats *stats)
{
    if (!c) return fail(LOFP_EINVAL, "null circuit");
    if (batch < 0) return fail(LOFP_EINVAL, "negative batch");
    if (batch > 0 && (!T_dev || !out_dev)) return fail(LOFP_EINVAL, "null T or out");
    if (batch > kMaxPass) {
        lofp_stats tot{}, one{};
        for (int32_t off = 0; off < batch; off += kMaxPass) {
            const int32_t nb = batch - off < kMaxPass ? batch - off : kMaxPass;
            lofp_status rc = lofp_amplitudes_device(c, S, nb, T_dev + (int64_t)off * c->m, out_dev + off, opts,
                                                    stream, stats ? &one : nullptr);
            if (rc != LOFP_OK) return rc;
            if (!stats) continue;
            tot.fwd_layer = one.fwd_layer; tot.bwd_layer = one.bwd_layer; tot.dfs_levels = one.dfs_levels;
            tot.frontier_states += one.frontier_states; tot.backward_states += one.backward_states;
            tot.bfs_states += one.bfs_states; tot.dfs_leaves += one.dfs_leaves; tot.dfs_edges += one.dfs_edges;
            tot.transitions += one.transitions;
            tot.ms_plan += one.ms_plan; tot.ms_forward += one.ms_forward; tot.ms_backward += one.ms_backward;
            tot.ms_dfs += one.ms_dfs; tot.ms_reduce += one.ms_reduce; tot.ms_contract += one.ms_contract;
            tot.ms_total += one.ms_total;
            tot.method_used = one.method_used;
            tot.split_top_keys += one.split_top_keys; tot.split_bottom_keys += one.split_bottom_keys;
            tot.max_state = std::max(tot.max_state, one.max_state);
        }
        if (stats) { *stats = tot; stats->batch = batch; }
        return LOFP_OK;
    }
    int n = 0;
    lofp_status rc = check_S(*c, S, n);
    if (rc != LOFP_OK) return rc;
    lofp_opts o{};
    o.method = LOFP_METHOD_AUTO;
    o.precision = LOFP_PREC_FP64;
    o.fwd_layer = -1;
    o.bwd_layer = -1;
    if (opts) o = *opts;
    if (o.precision != LOFP_PREC_FP64 && o.precision != LOFP_PREC_FP32) return fail(LOFP_EINVAL, "bad precision");
    if (o.method < 0 || o.method > LOFP_METHOD_CONTRACT) return fail(LOFP_EINVAL, "bad method");
    if (o.split < LOFP_SPLIT_AUTO || o.split > LOFP_SPLIT_ALWAYS) return fail(LOFP_EINVAL, "bad split mode");
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->batch = batch;
    }
    if (batch == 0) return LOFP_OK;
    std::lock_guard<std::mutex> lk(c->mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = device_init(*c, n, s);
    if (rc != LOFP_OK) return rc;
    StreamUse use(*c, s);
    HIPCHK(use.begin());
    std::vector<int32_t> Sv(S, S + c->m);
    if (Sv != c->S_dev) {
        HIPCHK(upload(c->d_S, Sv, s));
        c->S_dev = Sv;
    }
    Timer tm;
    tm.on = o.record_timing != 0 && stats != nullptr;
    tm.s = s;
    tm.mark();
    int method = o.method;
    if (method == LOFP_METHOD_AUTO) {
        // the paper's choice for depth > 2: contract along the modes when the
        // contraction state is affordable, otherwise enumerate paths
        method = LOFP_METHOD_PATHSUM;
        if (prepare_program(*c, s) == LOFP_OK) {
            s_only_cached(*c, S, n);
            if (c->sb_prog < 0) c->sb_prog = program_state_bound(*c, c->sb_lo, c->sb_hi);
            if (c->sb_prog <= (1 << 20)) method = LOFP_METHOD_CONTRACT;
        }
        clear_error();
    }
    if (stats) stats->method_used = method;
    if (method == LOFP_METHOD_CONTRACT) {
        Timer inner;
        inner.on = tm.on;
        inner.s = s;
        const int fp32 = o.precision == LOFP_PREC_FP32;
        const SplitCfg *cfg = nullptr;
        SplitCfg fixed = default_split_cfg(*c);
        if (o.split == LOFP_SPLIT_NEVER) {
            fixed.mode = SplitCfg::kPerPattern;
            cfg = &fixed;
        } else if (o.split == LOFP_SPLIT_ALWAYS) {
            fixed.small_min = 1;
            fixed.small_max = std::numeric_limits<int>::max();
            cfg = &fixed;
        } else if (o.autotune) {
            // the tuned way for this S, batch size, precision and state limit
            const lofp_circuit_s::TuneKey key{Sv, {batch, fp32, o.state_limit}};
            auto it = c->tuned.find(key);
            if (it == c->tuned.end()) {
                SplitCfg best = default_split_cfg(*c);
                rc = tune_contract(*c, S, n, batch, T_dev, out_dev, fp32, o.state_limit, s, best);
                if (rc != LOFP_OK) return rc;
                it = c->tuned.emplace(key, best).first;
            }
            cfg = &it->second;
            if (stats) stats->tuned = 1;
        }
        rc = run_contract(*c, S, n, batch, T_dev, out_dev, 0, fp32, s, stats, o.count_work != 0, o.state_limit, inner,
                          true, cfg);
        if (rc == LOFP_OK && stats && tm.on) {
            // bounds (and key hulls), contraction kernel, join of split halves
            stats->ms_plan = inner.ms(0, 1);
            stats->ms_contract = inner.ms(1, 2);
            stats->ms_reduce = inner.ms(2, 3);
        }
    } else {
        Timer inner;
        inner.on = tm.on;
        inner.s = s;
        rc = ready_on_stream(*c, s);
        if (rc == LOFP_OK) rc = run_pathsum(*c, S, n, batch, T_dev, out_dev, o, s, stats, inner);
    }
    if (rc != LOFP_OK) return rc;
    tm.mark();
    if (tm.on) {
        HIPCHK(hipStreamSynchronize(s));
        stats->ms_total = tm.ms(0, 1);
    }
    return LOFP_OK;
}

lofp_status lofp_amplitudes(lofp_circuit c, const int32_t *S, int32_t batch, const int32_t *T, lofp_c128 *out,
                            const lofp_opts *opts, lofp_stats *stats)
{
    if (!c) return fail(LOFP_EINVAL, "null circuit");
    if (batch < 0) return fail(LOFP_EINVAL, "negative batch");
    if (batch > 0 && (!T || !out)) return fail(LOFP_EINVAL, "null T or out");
    if (batch == 0) {
        if (stats) { std::memset(stats, 0, sizeof(*stats)); }
        return LOFP_OK;
    }
    for (int64_t i = 0; i < (int64_t)batch * c->m; ++i)
        if (T[i] < 0) return fail(LOFP_EINVAL, "negative occupation in T");
    DevBuf dT, dO;
    hipStream_t s = nullptr;
    HIPCHK(ensure(dT, (size_t)batch * c->m * sizeof(int32_t)));
    HIPCHK(ensure(dO, (size_t)batch * sizeof(lofp_c128)));
    hipError_t e = hipMemcpyAsync(dT.p, T, (size_t)batch * c->m * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) { release(dT); release(dO); return fail(LOFP_EDEVICE, hipGetErrorString(e)); }
    lofp_status rc = lofp_amplitudes_device(c, S, batch, dT.as<int32_t>(), dO.as<lofp_c128>(), opts, s, stats);
    if (rc == LOFP_OK) {
        e = hipMemcpyAsync(out, dO.p, (size_t)batch * sizeof(lofp_c128), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = fail(LOFP_EDEVICE, hipGetErrorString(e));
    }
    release(dT);
    release(dO);
    return rc;
}

lofp_status lofp_amplitude(lofp_circuit c, const int32_t *S, const int32_t *T, lofp_c128 *out)
{
    return lofp_amplitudes(c, S, 1, T, out, nullptr, nullptr);
}

lofp_status lofp_path_counts(lofp_circuit c, const int32_t *S, int32_t batch, const int32_t *T, double *counts)
{
    if (!c) return fail(LOFP_EINVAL, "null circuit");
    if (c->compiled) return fail(LOFP_ENOTSUP, "path counts of circuits with distant pairs (the compiled circuit has more paths)");
    if (batch < 0) return fail(LOFP_EINVAL, "negative batch");
    if (batch > 0 && (!T || !counts)) return fail(LOFP_EINVAL, "null T or counts");
    if (batch == 0) return LOFP_OK;
    int n = 0;
    lofp_status rc = check_S(*c, S, n);
    if (rc != LOFP_OK) return rc;
    for (int64_t i = 0; i < (int64_t)batch * c->m; ++i)
        if (T[i] < 0) return fail(LOFP_EINVAL, "negative occupation in T");
    std::lock_guard<std::mutex> lk(c->mu);
    hipStream_t s = nullptr;
    rc = device_init(*c, n, s);
    if (rc != LOFP_OK) return rc;
    StreamUse use(*c, s);
    HIPCHK(use.begin());
    std::vector<int32_t> Sv(S, S + c->m);
    if (Sv != c->S_dev) {
        HIPCHK(upload(c->d_S, Sv, s));
        c->S_dev = Sv;
    }
    HIPCHK(ensure(c->d_T, (size_t)batch * c->m * sizeof(int32_t)));
    HIPCHK(ensure(c->d_out, (size_t)batch * sizeof(double2)));
    HIPCHK(hipMemcpyAsync(c->d_T.p, T, (size_t)batch * c->m * sizeof(int32_t), hipMemcpyHostToDevice, s));
    Timer tm;
    lofp_stats st{};
    rc = run_contract(*c, S, n, batch, c->d_T.as<int32_t>(), c->d_out.as<lofp_c128>(), 1, 0, s, &st, false, 0, tm);
    if (rc != LOFP_OK) return rc;
    std::vector<double2> h(batch);
    HIPCHK(hipMemcpyAsync(h.data(), c->d_out.p, (size_t)batch * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int p = 0; p < batch; ++p) counts[p] = h[p].x;
    return LOFP_OK;
}

lofp_status lofp_all_outputs(lofp_circuit c, const int32_t *S, int64_t capacity, int32_t *T_out, lofp_c128 *amp_out,
                             int64_t *count, const lofp_opts *opts)
{
    if (!c || !count) return fail(LOFP_EINVAL, "null circuit or count");
    int n = 0;
    lofp_status rc = check_S(*c, S, n);
    if (rc != LOFP_OK) return rc;
    // C(m+n-1, n) patterns, exact while it fits (capped at 2^31)
    const int m = c->m;
    double cnt = 1.0;
    for (int i = 1; i <= n; ++i) cnt = cnt * (double)(m - 1 + i) / (double)i;
    const int64_t total = (int64_t)std::llround(cnt);
    if (cnt > 2147483647.0) return fail(LOFP_ENOTSUP, "more than 2^31 output patterns");
    *count = total;
    if (!T_out && !amp_out) return LOFP_OK;
    if (!T_out || !amp_out) return fail(LOFP_EINVAL, "T_out and amp_out go together");
    if (capacity < total) return fail(LOFP_EINVAL, "capacity below the number of output patterns");
    // decreasing lexicographic order: from (n, 0, ..., 0) to (0, ..., 0, n);
    // the successor moves one photon from the last nonzero mode before the
    // end to the next mode and gathers every later photon there
    std::vector<int32_t> t(m, 0);
    t[0] = n;
    for (int64_t p = 0; p < total; ++p) {
        std::copy(t.begin(), t.end(), T_out + p * m);
        int i = m - 2;
        while (i >= 0 && t[i] == 0) --i;
        if (i < 0) break;
        int tail = 0;
        for (int j = i + 1; j < m; ++j) { tail += t[j]; t[j] = 0; }
        t[i] -= 1;
        t[i + 1] = tail + 1;
    }
    // amplitudes in passes on the default stream
    const int64_t pass = 32768;
    DevBuf dT, dO;
    HIPCHK(ensure(dT, (size_t)std::min(total, pass) * m * sizeof(int32_t)));
    HIPCHK(ensure(dO, (size_t)std::min(total, pass) * sizeof(lofp_c128)));
    hipStream_t s = nullptr;
    for (int64_t off = 0; off < total && rc == LOFP_OK; off += pass) {
        const int32_t nb = (int32_t)std::min(pass, total - off);
        hipError_t e = hipMemcpyAsync(dT.p, T_out + off * m, (size_t)nb * m * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) { rc = fail(LOFP_EDEVICE, hipGetErrorString(e)); break; }
        rc = lofp_amplitudes_device(c, S, nb, dT.as<int32_t>(), dO.as<lofp_c128>(), opts, s, nullptr);
        if (rc != LOFP_OK) break;
        e = hipMemcpyAsync(amp_out + off, dO.p, (size_t)nb * sizeof(lofp_c128), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = fail(LOFP_EDEVICE, hipGetErrorString(e));
    }
    release(dT);
    release(dO);
    return rc;
}

}  // extern "C"
