// api.cpp -- host side of the C-ABI (include/lofp.h): circuit ingest and
// validation, light-cone tables, planning of the frontier cut, device
// workspace, and the order of kernel launches for one batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lofp.h"
#include "lofp_device.h"

using namespace lofp;

namespace {

thread_local std::string g_err;

lofp_status fail(lofp_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

#define HIPCHK(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(e_ == hipErrorOutOfMemory ? LOFP_ENOMEM : LOFP_EDEVICE,                   \
                        std::string(#call) + ": " + hipGetErrorString(e_));                       \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    template <class T> T *as() const { return static_cast<T *>(p); }
};

hipError_t ensure(DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (bytes <= b.cap) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess) return e;
    }
    b.p = nullptr;
    b.cap = 0;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipSuccess) b.cap = bytes;
    return e;
}

void release(DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

template <class T>
hipError_t upload(DevBuf &b, const std::vector<T> &v, hipStream_t s)
{
    hipError_t e = ensure(b, v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

}  // namespace

struct lofp_circuit_s {
    int m = 0, D = 0, G = 0, nc = 0;
    std::vector<lofp_bs> gates;            // application order
    std::vector<int32_t> gate_cut, gate_layer, layer_start;
    std::vector<uint8_t> cut_gate;         // [D][nc]
    std::vector<int32_t> gate_at;          // [D][nc] gate id or -1
    std::vector<int8_t> fr_lo, fr_hi, br_lo, br_hi;  // [(D+1)][m]
    std::vector<uint8_t> stage_time;       // [(G+1)][nc]
    std::vector<int32_t> cut_ngates, cut_gates, ver_at;
    std::mutex mu;

    // device state (lazy)
    bool dev_ready = false;
    int n_tab = -1;
    int tab_stride = 0;
    DevBuf d_table, d_theta, d_phi, d_fr_lo, d_fr_hi, d_br_lo, d_br_hi, d_cut_gate, d_stage_time;
    DevBuf d_gate_cut, d_gate_layer, d_cut_ngates, d_cut_gates, d_ver_at;
    // per-call workspace
    DevBuf d_S, d_lo, d_hi, d_inf, d_C, d_E, d_count, d_slot_stage, d_off, d_fa, d_fb, d_ba, d_bb;
    DevBuf d_levels, d_tab_mid, d_counters, d_T, d_out, d_ws;
};

namespace {

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

lofp_status device_init(lofp_circuit_s &c, int n, hipStream_t s)
{
    if (!c.dev_ready) {
        std::vector<double> th(c.G), ph(c.G);
        for (int g = 0; g < c.G; ++g) { th[g] = c.gates[g].theta; ph[g] = c.gates[g].phi; }
        HIPCHK(upload(c.d_theta, th, s));
        HIPCHK(upload(c.d_phi, ph, s));
        HIPCHK(upload(c.d_fr_lo, c.fr_lo, s));
        HIPCHK(upload(c.d_fr_hi, c.fr_hi, s));
        HIPCHK(upload(c.d_br_lo, c.br_lo, s));
        HIPCHK(upload(c.d_br_hi, c.br_hi, s));
        HIPCHK(upload(c.d_cut_gate, c.cut_gate, s));
        HIPCHK(upload(c.d_stage_time, c.stage_time, s));
        HIPCHK(upload(c.d_gate_cut, c.gate_cut, s));
        HIPCHK(upload(c.d_gate_layer, c.gate_layer, s));
        HIPCHK(upload(c.d_cut_ngates, c.cut_ngates, s));
        HIPCHK(upload(c.d_cut_gates, c.cut_gates, s));
        HIPCHK(upload(c.d_ver_at, c.ver_at, s));
        HIPCHK(ensure(c.d_counters, 8 * sizeof(unsigned long long)));
        c.dev_ready = true;
    }
    if (c.n_tab < n) {
        const int nt = std::max(n, 4);
        const int stride = sector_offset(nt + 1);
        HIPCHK(ensure(c.d_table, (size_t)std::max(c.G, 1) * stride * sizeof(double2)));
        HIPCHK(launch_build_tables(c.G, nt, c.d_theta.as<double>(), c.d_phi.as<double>(),
                                   c.d_table.as<double2>(), s));
        c.n_tab = nt;
        c.tab_stride = stride;
    }
    return LOFP_OK;
}

struct Timer {
    bool on = false;
    hipStream_t s = nullptr;
    std::vector<hipEvent_t> ev;
    void mark()
    {
        if (!on) return;
        hipEvent_t e;
        if (hipEventCreate(&e) == hipSuccess) {
            (void)hipEventRecord(e, s);
            ev.push_back(e);
        }
    }
    double ms(size_t a, size_t b)
    {
        float f = 0.f;
        if (!on || b >= ev.size() || a >= ev.size()) return 0.0;
        (void)hipEventElapsedTime(&f, ev[a], ev[b]);
        return f;
    }
    ~Timer()
    {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

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

lofp_status run_contract(lofp_circuit_s &c, const int32_t *S, int n, int B, const int32_t *T_dev,
                         lofp_c128 *out_dev, int count_only, hipStream_t s, lofp_stats *st, Timer &tm)
{
    // workspace bound from the S-side intervals (per-pattern ones are subsets)
    std::vector<int16_t> lo, hi;
    s_only_bounds(c, S, n, lo, hi);
    auto dom = [&](int r) -> int64_t {
        if (r < 0 || r >= c.nc) return 1;
        int64_t d = 1;
        const int k = c.cut_ngates[r];
        for (int j = 1; j < k; ++j) {
            const int t = c.gate_layer[c.cut_gates[(size_t)r * std::max(c.D, 1) + j - 1]] + 1;
            d *= std::max(0, hi[(size_t)t * c.nc + r] - lo[(size_t)t * c.nc + r] + 1);
        }
        return d;
    };
    int64_t max_states = 1;
    for (int r = -1; r < c.nc; ++r) max_states = std::max(max_states, dom(r) * dom(r + 1));
    if (max_states > (1 << 26)) return fail(LOFP_ENOMEM, "contraction state space too large");
    for (int r = 0; r < c.nc; ++r)
        if (c.cut_ngates[r] >= 16) return fail(LOFP_ENOTSUP, "more than 15 beam splitters on one cut");
    HIPCHK(ensure(c.d_ws, (size_t)B * 2 * max_states * sizeof(double2)));
    tm.mark();
    lofp_status rc = run_bounds(c, B, n, T_dev, s);
    if (rc != LOFP_OK) return rc;
    tm.mark();
    HIPCHK(hipMemsetAsync(c.d_counters.p, 0, 8 * sizeof(unsigned long long), s));
    ContractArgs a{};
    a.B = B; a.m = c.m; a.n = n; a.D = c.D; a.G = c.G;
    a.S = c.d_S.as<int32_t>();
    a.T = T_dev;
    a.lo = c.d_lo.as<int16_t>(); a.hi = c.d_hi.as<int16_t>();
    a.infeasible = c.d_inf.as<int32_t>();
    a.gate_cut = c.d_gate_cut.as<int32_t>(); a.gate_layer = c.d_gate_layer.as<int32_t>();
    a.cut_ngates = c.d_cut_ngates.as<int32_t>(); a.cut_gates = c.d_cut_gates.as<int32_t>();
    a.ver_at = c.d_ver_at.as<int32_t>();
    a.table = c.d_table.as<double2>(); a.tab_stride = c.tab_stride;
    a.out = reinterpret_cast<double2 *>(out_dev);
    a.count_only = count_only;
    a.stat_transitions = c.d_counters.as<unsigned long long>() + 3;
    a.max_states = (int)max_states;
    a.ws = c.d_ws.as<double2>();
    a.overflow = reinterpret_cast<int32_t *>(c.d_counters.as<unsigned long long>() + 4);
    HIPCHK(launch_contract(a, s));
    tm.mark();
    if (st) {
        unsigned long long h[8];
        HIPCHK(hipMemcpyAsync(h, c.d_counters.p, sizeof(h), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (h[4]) return fail(LOFP_ENOMEM, "contraction workspace overflow");
        st->transitions = (int64_t)h[3];
    }
    return LOFP_OK;
}

lofp_status run_pathsum(lofp_circuit_s &c, const int32_t *S, int n, int B, const int32_t *T_dev,
                        lofp_c128 *out_dev, const lofp_opts &o, hipStream_t s, lofp_stats *st, Timer &tm)
{
    const int D = c.D, G = c.G, nc = c.nc;
    // ---- plan the cut: backward frontier over the last two layers (their
    // path is unique given the configuration before them, Eq. (10)), forward
    // frontier one layer earlier; the layers in between are enumerated
    int bl = o.bwd_layer, fl = o.fwd_layer;
    if (bl < 0) bl = std::max(0, D - 2);
    if (fl < 0) fl = std::max(0, bl - 1);
    if (fl > bl || bl > D || fl < 0) return fail(LOFP_EINVAL, "need 0 <= fwd_layer <= bwd_layer <= depth");
    const int sf = c.layer_start[fl], sb = c.layer_start[bl];
    // stage slots: forward stages 0..sf, backward stages sb..G
    std::vector<int32_t> slot_stage;
    std::vector<int> slot_of(G + 1, -1);
    for (int st_ = 0; st_ <= sf; ++st_) { slot_of[st_] = (int)slot_stage.size(); slot_stage.push_back(st_); }
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
    if (cnt.back()) return fail(LOFP_ENOMEM, "a frontier state space exceeds 2^31 states");
    std::vector<int64_t> off((size_t)nslots * (B + 1));
    std::vector<int64_t> tot(nslots);
    for (int k = 0; k < nslots; ++k) {
        int64_t acc = 0;
        for (int p = 0; p < B; ++p) {
            off[(size_t)k * (B + 1) + p] = acc;
            acc += cnt[(size_t)k * B + p];
        }
        off[(size_t)k * (B + 1) + B] = acc;
        tot[k] = acc;
    }
    HIPCHK(upload(c.d_off, off, s));
    const int64_t *d_off = c.d_off.as<int64_t>();
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
        HIPCHK(launch_gate(a, false, s));
        std::swap(Bv, Bn);
    }
    tm.mark();  // 3
    (void)span;
    unsigned long long *ctr = c.d_counters.as<unsigned long long>();
    HIPCHK(hipMemsetAsync(ctr, 0, 8 * sizeof(unsigned long long), s));
    const int levels = sb - sf;
    if (levels > 0 && totp(sf) > 0) {
        // compact LDS image of the middle gates' tables (sectors 0..n)
        std::vector<int4> info(levels);
        const int per = sector_offset(n + 1);
        for (int d = 0; d < levels; ++d) {
            const int g = sf + d;
            info[d] = make_int4(c.gate_cut[g], c.gate_layer[g], d * per, 0);
        }
        HIPCHK(upload(c.d_levels, info, s));
        HIPCHK(ensure(c.d_tab_mid, (size_t)levels * per * sizeof(double2)));
        for (int d = 0; d < levels; ++d)
            HIPCHK(hipMemcpyAsync(c.d_tab_mid.as<double2>() + (size_t)d * per,
                                  c.d_table.as<double2>() + (size_t)(sf + d) * c.tab_stride,
                                  (size_t)per * sizeof(double2), hipMemcpyDeviceToDevice, s));
        DfsArgs a{};
        a.B = B; a.m = c.m; a.n = n; a.D = D;
        a.levels = levels;
        a.level_info = c.d_levels.as<int4>();
        a.tab = c.d_tab_mid.as<double2>();
        a.tab_len = levels * per;
        a.st_front = c.d_stage_time.as<uint8_t>() + (size_t)sf * nc;
        a.lo = c.d_lo.as<int16_t>(); a.hi = c.d_hi.as<int16_t>();
        a.C_front = Cp(sf); a.E_back = Ep(sb);
        a.off_front = offp(sf); a.off_back = offp(sb);
        a.front = F; a.back = Bv;
        a.total = totp(sf);
        a.work_counter = ctr;
        a.stat_leaves = ctr + 1;
        a.stat_edges = ctr + 2;
        a.fp32_products = o.precision == LOFP_PREC_FP32;
        const int block = 64;
        int dev = 0, ncu = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
                ncu = prop.multiProcessorCount;
        }
        const size_t lds = (size_t)levels * block * (sizeof(double2) + sizeof(int2)) + levels * sizeof(int4) +
                           (size_t)a.tab_len * sizeof(double2);
        const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(16, (160 * 1024) / std::max<size_t>(lds, 1)));
        int64_t grid = (int64_t)ncu * per_cu;
        grid = std::min<int64_t>(grid, (a.total + block - 1) / block);
        tm.mark();  // 4
        HIPCHK(launch_dfs(a, (int)std::max<int64_t>(grid, 1), block, s));
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

}  // namespace

// ===================================================================== C-ABI
extern "C" {

const char *lofp_last_error(void) { return g_err.c_str(); }

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
    auto *c = new lofp_circuit_s();
    c->m = m;
    c->D = n_layers;
    c->nc = m - 1;
    c->cut_gate.assign((size_t)std::max(n_layers, 1) * c->nc, 0);
    c->gate_at.assign((size_t)std::max(n_layers, 1) * c->nc, -1);
    c->layer_start.assign(n_layers + 1, 0);
    int k = 0;
    for (int l = 0; l < n_layers; ++l) {
        std::vector<lofp_bs> layer(bs + k, bs + k + layer_len[l]);
        k += layer_len[l];
        std::vector<int> used(m, 0);
        for (const auto &b : layer) {
            if (b.a < 0 || b.b < 0 || b.a >= m || b.b >= m || b.a >= b.b) {
                delete c;
                return fail(LOFP_EINVAL, "beam splitter modes out of range or a >= b");
            }
            if (used[b.a] || used[b.b]) {
                delete c;
                return fail(LOFP_EINVAL, "mode used twice in one layer");
            }
            used[b.a] = used[b.b] = 1;
            if (b.b != b.a + 1) {
                delete c;
                return fail(LOFP_ENOTSUP, "only adjacent pairs (a, a+1) are supported");
            }
        }
        std::sort(layer.begin(), layer.end(), [](const lofp_bs &x, const lofp_bs &y) { return x.a < y.a; });
        c->layer_start[l] = (int)c->gates.size();
        for (const auto &b : layer) {
            const int g = (int)c->gates.size();
            c->gates.push_back(b);
            c->gate_cut.push_back(b.a);
            c->gate_layer.push_back(l);
            c->cut_gate[(size_t)l * c->nc + b.a] = 1;
            c->gate_at[(size_t)l * c->nc + b.a] = g;
        }
    }
    c->G = (int)c->gates.size();
    c->layer_start[n_layers] = c->G;
    build_reach(*c);
    build_stage_maps(*c);
    *out = c;
    return LOFP_OK;
}

lofp_status lofp_circuit_destroy(lofp_circuit c)
{
    if (!c) return fail(LOFP_EINVAL, "null circuit");
    DevBuf *bufs[] = {&c->d_table, &c->d_theta, &c->d_phi, &c->d_fr_lo, &c->d_fr_hi, &c->d_br_lo, &c->d_br_hi,
                      &c->d_cut_gate, &c->d_stage_time, &c->d_gate_cut, &c->d_gate_layer, &c->d_cut_ngates,
                      &c->d_cut_gates, &c->d_ver_at, &c->d_S, &c->d_lo, &c->d_hi, &c->d_inf, &c->d_C, &c->d_E,
                      &c->d_count, &c->d_slot_stage, &c->d_off, &c->d_fa, &c->d_fb, &c->d_ba, &c->d_bb,
                      &c->d_levels, &c->d_tab_mid, &c->d_counters, &c->d_T, &c->d_out, &c->d_ws};
    for (DevBuf *b : bufs) release(*b);
    delete c;
    return LOFP_OK;
}

lofp_status lofp_light_cone(lofp_circuit c, int32_t layer, int32_t mode, int32_t *past_lo, int32_t *past_hi,
                            int32_t *fut_lo, int32_t *fut_hi)
{
    if (!c || !past_lo || !past_hi || !fut_lo || !fut_hi) return fail(LOFP_EINVAL, "null argument");
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

lofp_status lofp_bs_table(lofp_circuit c, int32_t gate, int32_t N, lofp_c128 *out)
{
    if (!c || !out) return fail(LOFP_EINVAL, "null argument");
    if (gate < 0 || gate >= c->G || N < 0 || N > kMaxPhotons) return fail(LOFP_EINVAL, "bad gate or N");
    std::lock_guard<std::mutex> lk(c->mu);
    hipStream_t s = nullptr;
    lofp_status rc = device_init(*c, N, s);
    if (rc != LOFP_OK) return rc;
    HIPCHK(hipMemcpyAsync(out, c->d_table.as<double2>() + (size_t)gate * c->tab_stride + sector_offset(N),
                          (size_t)(N + 1) * (N + 1) * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return LOFP_OK;
}

lofp_status lofp_amplitudes_device(lofp_circuit c, const int32_t *S, int32_t batch, const int32_t *T_dev,
                                   lofp_c128 *out_dev, const lofp_opts *opts, void *stream, lofp_stats *stats)
{
    if (!c) return fail(LOFP_EINVAL, "null circuit");
    if (batch < 0) return fail(LOFP_EINVAL, "negative batch");
    if (batch > 0 && (!T_dev || !out_dev)) return fail(LOFP_EINVAL, "null T or out");
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
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->batch = batch;
    }
    if (batch == 0) return LOFP_OK;
    std::lock_guard<std::mutex> lk(c->mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = device_init(*c, n, s);
    if (rc != LOFP_OK) return rc;
    std::vector<int32_t> Sv(S, S + c->m);
    HIPCHK(upload(c->d_S, Sv, s));
    Timer tm;
    tm.on = o.record_timing != 0 && stats != nullptr;
    tm.s = s;
    tm.mark();
    if (o.method == LOFP_METHOD_CONTRACT) {
        Timer inner;
        inner.on = tm.on;
        inner.s = s;
        rc = run_contract(*c, S, n, batch, T_dev, out_dev, 0, s, stats, inner);
        if (rc == LOFP_OK && stats && tm.on) {
            stats->ms_plan = inner.ms(0, 1);
            stats->ms_contract = inner.ms(1, 2);
        }
    } else {
        Timer inner;
        inner.on = tm.on;
        inner.s = s;
        rc = run_pathsum(*c, S, n, batch, T_dev, out_dev, o, s, stats, inner);
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
    std::vector<int32_t> Sv(S, S + c->m);
    HIPCHK(upload(c->d_S, Sv, s));
    HIPCHK(ensure(c->d_T, (size_t)batch * c->m * sizeof(int32_t)));
    HIPCHK(ensure(c->d_out, (size_t)batch * sizeof(double2)));
    HIPCHK(hipMemcpyAsync(c->d_T.p, T, (size_t)batch * c->m * sizeof(int32_t), hipMemcpyHostToDevice, s));
    Timer tm;
    lofp_stats st{};
    rc = run_contract(*c, S, n, batch, c->d_T.as<int32_t>(), c->d_out.as<lofp_c128>(), 1, s, &st, tm);
    if (rc != LOFP_OK) return rc;
    std::vector<double2> h(batch);
    HIPCHK(hipMemcpyAsync(h.data(), c->d_out.p, (size_t)batch * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int p = 0; p < batch; ++p) counts[p] = h[p].x;
    return LOFP_OK;
}

}  // extern "C"
