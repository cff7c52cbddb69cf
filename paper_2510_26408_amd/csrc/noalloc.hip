// noalloc.hip -- the amplitude call for callers that cannot allocate device
// memory (code under stream capture, tight serving loops, harnesses that
// forbid allocation).
//
// It is the per-pattern mode-axis contraction of lofp_amplitudes_device (the
// cut bounds, then one contraction block per pattern), with every per-call
// buffer (S, the cut intervals, the counters and, for states too large for
// LDS, the state workspace) carved from one file-scope device array of
// kScratchBytes.  Each device holds its own copy of the array, whose address
// is looked up once per device; calls on one device share it, so calls that
// overlap on a device race.  The circuit's tables and step program must
// already be on the device (set up by an earlier call of the ordinary
// entry points for at least this photon number).
#include <algorithm>
#include <mutex>
#include <string>

#include "host_internal.h"

namespace lofp {
namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // per device: the array's device address

// Device address of `scratch` on the current device, looked up on the
// first call on that device (the array's name is not a device address in
// host code).
lofp_status scratch_ptr(unsigned char **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return host::fail(LOFP_ENOTSUP, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return host::fail(LOFP_EDEVICE, "hipGetSymbolAddress returned a null scratch address");
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[dev]);
    return LOFP_OK;
}

// S (m <= 32 values, passed by value) into device memory, and the eight
// contraction counters cleared: one small kernel instead of a host copy and
// a memset, so the call stays capturable.
struct SVals {
    int32_t v[32];
};
__global__ void k_put_s_clear(SVals sv, int m, int32_t *S, unsigned long long *ctr)
{
    const int t = threadIdx.x;
    if (t < m) S[t] = sv.v[t];
    if (t < 8) ctr[t] = 0;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace lofp

using namespace lofp;
using namespace lofp::host;

extern "C" lofp_status lofp_amplitudes_device_noalloc(lofp_circuit c, const int32_t *S, int32_t batch,
                                                      const int32_t *T_dev, lofp_c128 *out_dev,
                                                      const lofp_opts *opts, void *stream)
{
    if (!c) return fail(LOFP_EINVAL, "null circuit");
    if (batch < 0) return fail(LOFP_EINVAL, "negative batch");
    if (batch > 0 && (!T_dev || !out_dev)) return fail(LOFP_EINVAL, "null T or out");
    int n = 0;
    lofp_status rc = check_S(*c, S, n);
    if (rc != LOFP_OK) return rc;
    const int method = opts ? opts->method : LOFP_METHOD_AUTO;
    const int precision = opts ? opts->precision : LOFP_PREC_FP64;
    if (method != LOFP_METHOD_AUTO && method != LOFP_METHOD_CONTRACT)
        return fail(LOFP_ENOTSUP, "the allocation-free call runs the contraction only");
    if (precision != LOFP_PREC_FP64 && precision != LOFP_PREC_FP32) return fail(LOFP_EINVAL, "bad precision");
    if (batch == 0) return LOFP_OK;
    unsigned char *base = nullptr;
    rc = scratch_ptr(&base);
    if (rc != LOFP_OK) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    // the circuit's device set-up is made by the ordinary calls (they may allocate)
    if (!c->dev_ready || c->n_tab < n || !c->prog_built || !c->prog_on_device || !c->prog_error.empty() ||
        !c->ready_ev || c->pending_init)
        return fail(LOFP_EINVAL, "circuit not set up on the device for this photon number: make one "
                                 "lofp_amplitudes_device call with the contraction first");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (c->ready_stream != s) HIPCHK(hipStreamWaitEvent(s, c->ready_ev, 0));
    // largest state from the S-side intervals (they contain every pattern's)
    s_only_cached(*c, S, n);
    if (c->sb_prog < 0) c->sb_prog = program_state_bound(*c, c->sb_lo, c->sb_hi);
    if (c->sb_prog > (1 << 22)) return fail(LOFP_ENOTSUP, "contraction state beyond 2^22 entries");
    const size_t span = (size_t)(c->D + 1) * c->nc;
    ContractArgs a{};
    a.B = batch; a.m = c->m; a.n = n; a.D = c->D;
    a.nvars = c->nvars;
    a.var_cut = c->d_var_cut.as<int32_t>();
    a.var_time = c->d_var_time.as<int32_t>();
    a.nsteps = (int)c->steps.size();
    a.steps = c->d_steps.as<ContractStep>();
    a.table = c->d_table.as<double2>(); a.tab_stride = c->tab_stride;
    a.out = reinterpret_cast<double2 *>(out_dev);
    a.count_only = 0;
    a.fp32 = precision == LOFP_PREC_FP32;
    a.stats = 0;
    a.max_states = (int)std::max<int64_t>(c->sb_prog, 1);
    if (opts && opts->state_limit > 0 && a.max_states > opts->state_limit) a.max_states = opts->state_limit;
    const bool in_lds = contract_lds_bytes(a, true) <= 64 * 1024;
    // scratch layout: S | counters | lo | hi | infeasible | workspace
    const size_t off_ctr = 256, off_lo = 512;
    const size_t off_hi = off_lo + align256((size_t)batch * span * sizeof(int16_t));
    const size_t off_inf = off_hi + align256((size_t)batch * span * sizeof(int16_t));
    const size_t off_ws = off_inf + align256((size_t)batch * sizeof(int32_t));
    const size_t need = off_ws + (in_lds ? 0 : (size_t)batch * 2 * a.max_states * sizeof(double2));
    if (need > kScratchBytes)
        return fail(LOFP_EINVAL, "batch needs " + std::to_string(need) + " bytes of scratch; the allocation-free call has " +
                                     std::to_string(kScratchBytes));
    int32_t *dS = reinterpret_cast<int32_t *>(base);
    unsigned long long *ctr = reinterpret_cast<unsigned long long *>(base + off_ctr);
    int16_t *lo = reinterpret_cast<int16_t *>(base + off_lo), *hi = reinterpret_cast<int16_t *>(base + off_hi);
    int32_t *inf = reinterpret_cast<int32_t *>(base + off_inf);
    a.S = dS;
    a.T = T_dev;
    a.lo = lo;
    a.hi = hi;
    a.infeasible = inf;
    a.ws = in_lds ? nullptr : reinterpret_cast<double2 *>(base + off_ws);
    a.lds_states = in_lds ? 0 : std::min(contract_lds_room(a.nvars, a.m), a.max_states);
    a.stat_transitions = ctr + 3;
    a.overflow = reinterpret_cast<int32_t *>(ctr + 4);
    SVals sv{};
    for (int i = 0; i < c->m; ++i) sv.v[i] = S[i];
    hipLaunchKernelGGL(k_put_s_clear, dim3(1), dim3(64), 0, s, sv, c->m, dS, ctr);
    HIPCHK(hipGetLastError());
    HIPCHK(launch_bounds(batch, c->m, c->D, n, dS, T_dev, c->d_fr_lo.as<int8_t>(), c->d_fr_hi.as<int8_t>(),
                         c->d_br_lo.as<int8_t>(), c->d_br_hi.as<int8_t>(), c->d_cut_gate.as<uint8_t>(), lo, hi, inf,
                         s));
    HIPCHK(launch_contract(a, s));
    return LOFP_OK;
}
