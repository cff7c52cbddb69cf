// serve.cpp -- many circuits in one launch, and a serving loop built on it.
//
// A multi-circuit batch packs requests whose circuits may all differ (mode
// count, depth, angles) together with their S and T.  Each request becomes
// one job of one bounds launch and one contraction launch; the jobs carry
// pointers to their circuit's resident tables and step program.
//
// The server admits requests continuously: a worker thread takes whatever
// has arrived (up to max_batch, and while the admitted workspace stays under
// the memory budget), launches it as one batch on the next free stream, and
// goes on admitting while earlier batches run; several batches overlap on the
// device.  A request's latency runs from submit to the moment its batch's
// completion event is observed.  Each job's arithmetic depends only on its
// own request, so a result is bit-identical whether it ran alone or in a mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host_internal.h"

using namespace lofp;
using namespace lofp::host;

namespace {

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
    lofp_circuit c = nullptr;
    std::vector<int32_t> S, T;
    int n = 0;
    int64_t est = 1;        // contraction state bound (entries), from the S-side intervals
    uint64_t ticket = 0;
    double t_submit = 0;
    bool planned = false;
    bool fp64 = false;      // recomputed in FP64 (its FP32 bound was too loose)
    double abs_form = -1;   // absolute form from the FP32 pass (-1: none)
};

struct DoneRec {
    lofp_c128 amp;
    double latency_ms;      // < 0: the batch failed
    double err_bound;       // rounding bound of amp (NaN: not computed)
};

// Workspace bytes of one request (bounds + contraction state if global).
// Rounding bounds from the absolute form A_abs (the sum over paths of the
// products of |Re W| + |Im W|, which bounds the 1-norm of every exact state
// entry by the same sum over that entry's paths).  One step with relative
// error f per transition term turns an error E of each source entry (relative
// to its absolute-form value a) into at most (1 + f) E + f a, so after G
// splitters the error is at most ((1 + f)^G - 1) A_abs.  FP32 products: the
// source and the weight are each rounded to FP32 and the two products and the
// sum of each component round again (4 roundings, gamma_4 = 4u/(1 - 4u),
// u = 2^-24); their FP64 sum over the at most (n+1)^2 transitions into an
// entry adds (2k + 2) 2^-53.  FP64 (complex FMA chains): (2k + 2) 2^-53 alone.
// The final compensated sum adds 4 * 2^-53; the last factor covers the
// rounding of A_abs itself and of this formula.  Values in the FP32 normal
// range are assumed (an underflowing product adds an absolute 2^-149 or so).
double rounding_bound(int G, int n, double abs_form, bool fp32)
{
    const double k = (double)(n + 1) * (n + 1);
    const double u = 0x1p-24;
    const double f = (fp32 ? 4 * u / (1 - 4 * u) : 0.0) + (2 * k + 2) * 0x1p-53;
    const double grow = std::expm1((double)G * std::log1p(f)) + 4 * 0x1p-53;
    return grow * abs_form * (1 + 0x1p-30);
}

size_t req_bytes(const Req &r)
{
    const lofp_circuit_s &c = *r.c;
    return (size_t)(c.D + 1) * c.nc * 4 + 64 + (size_t)2 * r.est * sizeof(double2);
}

// Cheap validation of a request (the submitter's thread).
lofp_status check_request(Req &r)
{
    lofp_circuit_s &c = *r.c;
    if ((int)r.S.size() != c.m || (int)r.T.size() != c.m) return fail(LOFP_EINVAL, "S/T length");
    lofp_status rc = check_S(c, r.S.data(), r.n);
    if (rc != LOFP_OK) return rc;
    for (int v : r.T)
        if (v < 0) return fail(LOFP_EINVAL, "negative occupation in T");
    return LOFP_OK;
}

// Prepare a request on the host: the circuit's program and the contraction
// state bound from this request's exact intervals.
lofp_status plan_request(Req &r)
{
    lofp_status rc = check_request(r);
    if (rc != LOFP_OK) return rc;
    r.planned = true;
    lofp_circuit_s &c = *r.c;
    std::lock_guard<std::mutex> lk(c.mu);
    if (!c.prog_built) build_program(c);
    if (!c.prog_error.empty()) return fail(LOFP_ENOTSUP, c.prog_error);
    // exact per-request intervals (S and T are on the host here)
    const size_t span = (size_t)(c.D + 1) * c.nc;
    std::vector<int16_t> lo(span), hi(span);
    int nT = 0;
    for (int v : r.T) nT += v;
    if (nT != r.n) {
        r.est = 1;
        return LOFP_OK;
    }
    light_cone_bounds(c.m, c.D, r.S.data(), r.T.data(), c.fr_lo.data(), c.fr_hi.data(), c.br_lo.data(),
                      c.br_hi.data(), lo.data(), hi.data());
    if (propagate_bounds(c.m, c.D, r.n, c.cut_gate.data(), lo.data(), hi.data())) {
        r.est = 1;
        return LOFP_OK;
    }
    r.est = std::max<int64_t>(1, program_state_bound(c, lo, hi));
    if (r.est > (1 << 22)) return fail(LOFP_ENOMEM, "contraction state exceeds 2^22 entries");
    return LOFP_OK;
}

struct Batch {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    DevBuf d_ST, d_lohi, d_inf, d_out, d_bj, d_cj, d_ws, d_ctr, d_abs, d_cja;
    std::vector<ContractJob> cja;          // jobs of the absolute pass (outputs to d_abs)
    double *h_abs = nullptr;
    bool checked = false;                  // FP32 products with per-result bounds
    std::vector<BoundsJob> bj;
    std::vector<ContractJob> cj;
    lofp_c128 *h_out = nullptr;
    size_t h_cap = 0;
    std::vector<Req> reqs;
    size_t bytes = 0;
    bool busy = false;

    ~Batch()
    {
        DevBuf *b[] = {&d_ST, &d_lohi, &d_inf, &d_out, &d_bj, &d_cj, &d_ws, &d_ctr, &d_abs, &d_cja};
        for (DevBuf *x : b) release(*x);
        if (h_out) (void)hipHostFree(h_out);
        if (h_abs) (void)hipHostFree(h_abs);
        if (ev) (void)hipEventDestroy(ev);
    }
};

// Enqueue one multi-circuit batch on b.s (reqs already planned).  checked:
// FP32 products plus the absolute form of every request, from which each
// result's rounding bound follows (rounding_bound).
lofp_status launch_batch(Batch &b, int fp32, bool checked = false, Timer *tm = nullptr)
{
    b.checked = checked && fp32;
    const int count = (int)b.reqs.size();
    hipStream_t s = b.s;
    // circuits: resident tables and programs.  The batch's new circuits are
    // set up together (one pooled block, one copy, one table launch) on this
    // stream; later users on other streams wait for that set-up.  Circuit
    // locks are taken in address order.
    {
        std::vector<lofp_circuit_s *> cs;
        for (Req &r : b.reqs) cs.push_back(r.c);
        std::sort(cs.begin(), cs.end());
        cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
        std::vector<std::unique_lock<std::mutex>> locks;
        locks.reserve(cs.size());
        for (lofp_circuit_s *c : cs) locks.emplace_back(c->mu);
        std::vector<std::pair<lofp_circuit_s *, int>> need;
        need.reserve(b.reqs.size());
        for (Req &r : b.reqs) need.emplace_back(r.c, r.n);
        lofp_status rc = init_circuits(need, s);
        if (rc != LOFP_OK) return rc;
        for (lofp_circuit_s *c : cs) {
            rc = prepare_program(*c, s);
            if (rc != LOFP_OK) return rc;
            rc = ready_on_stream(*c, s);
            if (rc != LOFP_OK) return rc;
        }
    }
    // pack S, T and the per-request offsets
    std::vector<int32_t> ST;
    std::vector<size_t> st_off(count), lh_off(count);
    size_t lh = 0;
    int64_t max_est = 1;
    int max_vars = 0, max_m = 2;
    for (int i = 0; i < count; ++i) {
        const Req &r = b.reqs[i];
        st_off[i] = ST.size();
        ST.insert(ST.end(), r.S.begin(), r.S.end());
        ST.insert(ST.end(), r.T.begin(), r.T.end());
        lh_off[i] = lh;
        lh += (size_t)(r.c->D + 1) * r.c->nc;
        max_est = std::max(max_est, r.est);
        max_vars = std::max(max_vars, r.c->nvars);
        max_m = std::max(max_m, r.c->m);
    }
    HIPCHK(upload(b.d_ST, ST, s));
    HIPCHK(ensure(b.d_lohi, 2 * std::max<size_t>(lh, 1) * sizeof(int16_t)));
    HIPCHK(ensure(b.d_inf, count * sizeof(int32_t)));
    HIPCHK(ensure(b.d_out, count * sizeof(double2)));
    HIPCHK(ensure(b.d_ctr, 8 * sizeof(unsigned long long)));
    HIPCHK(hipMemsetAsync(b.d_ctr.p, 0, 8 * sizeof(unsigned long long), s));
    const bool in_lds = contract_job_lds_bytes(max_vars, max_m, (int)max_est, true) <= 64 * 1024;
    size_t ws_total = 0;
    if (!in_lds) {
        for (const Req &r : b.reqs) ws_total += (size_t)2 * r.est;
        HIPCHK(ensure(b.d_ws, ws_total * sizeof(double2)));
    }
    const int32_t *dST = b.d_ST.as<int32_t>();
    int16_t *dlo = b.d_lohi.as<int16_t>(), *dhi = dlo + lh;
    b.bj.resize(count);
    b.cj.resize(count);
    size_t ws_off = 0;
    int max_span = 1;
    for (int i = 0; i < count; ++i) {
        const Req &r = b.reqs[i];
        const lofp_circuit_s &c = *r.c;
        BoundsJob &J = b.bj[i];
        J.m = c.m; J.D = c.D; J.n = r.n;
        J.S = dST + st_off[i];
        J.T = dST + st_off[i] + c.m;
        J.fr_lo = c.d_fr_lo.as<int8_t>(); J.fr_hi = c.d_fr_hi.as<int8_t>();
        J.br_lo = c.d_br_lo.as<int8_t>(); J.br_hi = c.d_br_hi.as<int8_t>();
        J.cut_gate = c.d_cut_gate.as<uint8_t>();
        J.lo = dlo + lh_off[i];
        J.hi = dhi + lh_off[i];
        J.infeasible = b.d_inf.as<int32_t>() + i;
        ContractJob &K = b.cj[i];
        K.m = c.m; K.n = r.n; K.D = c.D; K.nvars = c.nvars; K.nsteps = (int)c.steps.size();
        K.tab_stride = c.tab_stride;
        K.max_states = in_lds ? (int)max_est : (int)r.est;
        K.fp32 = fp32;
        K.steps = c.d_steps.as<ContractStep>();
        K.var_cut = c.d_var_cut.as<int32_t>();
        K.var_time = c.d_var_time.as<int32_t>();
        K.table = c.d_table.as<double2>();
        K.S = J.S; K.T = J.T; K.lo = J.lo; K.hi = J.hi; K.infeasible = J.infeasible;
        K.out = b.d_out.as<double2>() + i;
        K.ws = in_lds ? nullptr : b.d_ws.as<double2>() + ws_off;
        K.state_out = nullptr;
        K.state_cap = 0;
        K.stats = 0;
        K.out_remap = 0;
        K.ovf = nullptr;
        ws_off += (size_t)2 * r.est;
        max_span = std::max(max_span, (c.D + 1) * (c.m - 1));
    }
    HIPCHK(upload(b.d_bj, b.bj, s));
    HIPCHK(upload(b.d_cj, b.cj, s));
    HIPCHK(launch_bounds_multi(count, b.d_bj.as<BoundsJob>(), max_span, s));
    const size_t lds = contract_job_lds_bytes(max_vars, max_m, (int)max_est, in_lds);
    unsigned long long *ctr = b.d_ctr.as<unsigned long long>();
    if (tm) tm->mark();
    HIPCHK(launch_contract_multi(count, b.d_cj.as<ContractJob>(), lds, (int)max_est, in_lds, fp32 != 0, ctr,
                                 reinterpret_cast<int32_t *>(ctr + 1), s));
    if (tm) tm->mark();
    if (b.checked) {
        // the absolute form: same jobs, FP64, outputs to d_abs
        HIPCHK(ensure(b.d_abs, count * sizeof(double2)));
        b.cja = b.cj;
        for (int i = 0; i < count; ++i) {
            b.cja[i].out = b.d_abs.as<double2>() + i;
            b.cja[i].fp32 = 0;
        }
        HIPCHK(upload(b.d_cja, b.cja, s));
        HIPCHK(launch_contract_multi(count, b.d_cja.as<ContractJob>(), lds, (int)max_est, in_lds, false, ctr,
                                     reinterpret_cast<int32_t *>(ctr + 1), s, MultiOverride{0, nullptr, nullptr, 0, 0, nullptr},
                                     false, true));
    }
    if (b.h_cap < (size_t)count) {
        if (b.h_out) (void)hipHostFree(b.h_out);
        if (b.h_abs) (void)hipHostFree(b.h_abs);
        b.h_out = nullptr;
        b.h_abs = nullptr;
        b.h_cap = 0;
        HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&b.h_out), std::max(count, 256) * sizeof(lofp_c128),
                             hipHostMallocDefault));
        HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&b.h_abs), std::max(count, 256) * sizeof(double) * 2,
                             hipHostMallocDefault));
        b.h_cap = std::max(count, 256);
    }
    HIPCHK(hipMemcpyAsync(b.h_out, b.d_out.p, count * sizeof(lofp_c128), hipMemcpyDeviceToHost, s));
    if (b.checked)
        HIPCHK(hipMemcpyAsync(b.h_abs, b.d_abs.p, count * 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    if (!b.ev) HIPCHK(hipEventCreateWithFlags(&b.ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(b.ev, s));
    return LOFP_OK;
}

}  // namespace

// ------------------------------------------------------------------ server
struct lofp_server_s {
    lofp_server_opts o{};
    std::mutex mu;
    std::condition_variable cv;            // results: completions
    std::condition_variable cv_plan;       // planners: submissions
    std::condition_variable cv_launch;     // launcher: planned requests
    std::deque<Req> queue;                 // submitted, not yet planned
    std::deque<Req> ready;                 // planned, waiting for a launch
    int planning = 0;                      // requests being planned now
    std::vector<std::thread> planners;
    std::unordered_map<uint64_t, DoneRec> done;
    int64_t fp64_fallbacks = 0;
    int64_t pathsum_fallbacks = 0;         // requests the contraction refused, summed by the path sum
    std::unordered_map<uint64_t, std::pair<lofp_status, std::string>> failed;   // ticket -> planning error
    std::vector<double> latencies;
    std::vector<std::unique_ptr<Batch>> batches;
    uint64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0, launches = 0, launched_reqs = 0;
    size_t inflight_bytes = 0;
    bool stop = false;
    std::string error;
    std::thread worker;
    int device = 0;
};

namespace {

void complete_batch(lofp_server_s &sv, Batch &b)
{
    const double t = now_ms();
    const double rtol = sv.o.fp32_rtol > 0 ? sv.o.fp32_rtol : 1e-6;
    std::lock_guard<std::mutex> lk(sv.mu);
    int64_t finished = 0;
    for (size_t i = 0; i < b.reqs.size(); ++i) {
        Req &r = b.reqs[i];
        const lofp_c128 a = b.h_out[i];
        double bound = std::nan("");
        if (b.checked) {
            r.abs_form = b.h_abs[2 * i];
            bound = rounding_bound(r.c->G, r.n, r.abs_form, true);
            if (bound > rtol * std::hypot(a.re, a.im)) {
                // the FP32 form cannot certify this result: recompute in FP64
                r.fp64 = true;
                sv.fp64_fallbacks++;
                sv.ready.push_front(std::move(r));
                continue;
            }
        } else if (r.fp64 && r.abs_form >= 0) {
            bound = rounding_bound(r.c->G, r.n, r.abs_form, false);
        }
        const double lat = t - r.t_submit;
        sv.done[r.ticket] = {a, lat, bound};
        sv.latencies.push_back(lat);
        ++finished;
    }
    sv.completed += finished;
    sv.inflight_bytes -= b.bytes;
    b.reqs.clear();
    b.busy = false;
    sv.cv.notify_all();
}

void worker_loop(lofp_server_s *sv)
{
    (void)hipSetDevice(sv->device);
    for (;;) {
        // completions first
        for (auto &bp : sv->batches) {
            Batch &b = *bp;
            if (b.busy && hipEventQuery(b.ev) == hipSuccess) complete_batch(*sv, b);
        }
        Batch *free_b = nullptr;
        for (auto &bp : sv->batches)
            if (!bp->busy) { free_b = bp.get(); break; }
        std::vector<Req> take;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->stop && sv->queue.empty() && sv->ready.empty() && sv->planning == 0) {
                bool any = false;
                for (auto &bp : sv->batches) any |= bp->busy;
                if (!any) return;
            }
            if (!free_b || sv->ready.empty()) {
                // nothing to launch: wait briefly for planned arrivals or completions
                sv->cv_launch.wait_for(lk, std::chrono::microseconds(20));
                continue;
            }
            // admission: planned arrivals so far, up to max_batch and the
            // memory budget (at least one request)
            size_t bytes = 0;
            const bool run_fp64 = sv->ready.front().fp64;   // a batch has one precision
            while (!sv->ready.empty() && (int)take.size() < sv->o.max_batch && sv->ready.front().fp64 == run_fp64) {
                const size_t rb = req_bytes(sv->ready.front());
                if (!take.empty() && sv->inflight_bytes + bytes + rb > (size_t)sv->o.memory_budget) break;
                bytes += rb;
                take.push_back(std::move(sv->ready.front()));
                sv->ready.pop_front();
            }
            sv->inflight_bytes += bytes;
            free_b->bytes = bytes;
        }
        free_b->reqs = std::move(take);
        free_b->busy = true;
        const bool fp32 = sv->o.precision == LOFP_PREC_FP32 && !free_b->reqs.front().fp64;
        lofp_status rc = launch_batch(*free_b, fp32, fp32);
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->launches++;
        sv->launched_reqs += (int64_t)free_b->reqs.size();
        if (rc != LOFP_OK) {
            sv->error = lofp_last_error();
            for (const Req &r : free_b->reqs) sv->done[r.ticket] = {lofp_c128{NAN, NAN}, -1.0, NAN};
            sv->completed += (int64_t)free_b->reqs.size();
            sv->inflight_bytes -= free_b->bytes;
            free_b->reqs.clear();
            free_b->busy = false;
            sv->cv.notify_all();
        }
    }
}

// Planner threads: requests are planned on the host (program, exact
// intervals, state bound) off the submitters' and the launcher's threads; a
// request that cannot run completes with its error.
// A request the contraction cannot take (its program or its state is too
// large) is summed by the path-sum form instead, on the planner thread's own
// stream, which overlaps the batches in flight.
struct PathsumLane {
    hipStream_t s = nullptr;
    DevBuf dT, dO;
    ~PathsumLane()
    {
        release(dT);
        release(dO);
        if (s) (void)hipStreamDestroy(s);
    }
    lofp_status run(const Req &r, lofp_c128 &out)
    {
        if (!s) HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        HIPCHK(ensure(dT, r.T.size() * sizeof(int32_t)));
        HIPCHK(ensure(dO, sizeof(lofp_c128)));
        HIPCHK(hipMemcpyAsync(dT.p, r.T.data(), r.T.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        lofp_opts o{};
        o.method = LOFP_METHOD_PATHSUM;
        o.fwd_layer = -1;
        o.bwd_layer = -1;
        lofp_status rc = lofp_amplitudes_device(r.c, r.S.data(), 1, dT.as<int32_t>(), dO.as<lofp_c128>(), &o, s, nullptr);
        if (rc != LOFP_OK) return rc;
        HIPCHK(hipMemcpyAsync(&out, dO.p, sizeof(lofp_c128), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return LOFP_OK;
    }
};

void planner_loop(lofp_server_s *sv)
{
    (void)hipSetDevice(sv->device);
    PathsumLane lane;
    for (;;) {
        Req r;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_plan.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
            if (sv->queue.empty()) return;   // stopping and nothing left
            r = std::move(sv->queue.front());
            sv->queue.pop_front();
            sv->planning++;
        }
        lofp_status rc = plan_request(r);
        lofp_c128 amp{0.0, 0.0};
        bool by_pathsum = false;
        if ((rc == LOFP_ENOTSUP || rc == LOFP_ENOMEM) && r.planned) {
            // a valid request the contraction refuses: the path sum instead
            rc = lane.run(r, amp);
            by_pathsum = rc == LOFP_OK;
        }
        const std::string err = rc == LOFP_OK ? std::string() : std::string(lofp_last_error());
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->planning--;
        if (by_pathsum) {
            const double lat = now_ms() - r.t_submit;
            sv->done[r.ticket] = {amp, lat, std::nan("")};
            sv->latencies.push_back(lat);
            sv->pathsum_fallbacks++;
            sv->completed++;
            sv->cv.notify_all();
        } else if (rc == LOFP_OK) {
            sv->ready.push_back(std::move(r));
        } else {
            sv->failed[r.ticket] = {rc, err};
            sv->completed++;
            sv->cv.notify_all();
        }
        sv->cv_launch.notify_one();
    }
}

}  // namespace

extern "C" {

lofp_status lofp_amplitudes_multi(int32_t count, const lofp_request *req, lofp_c128 *out, double *err_bound,
                                  const lofp_opts *opts, void *stream, lofp_stats *stats)
{
    if (count < 0) return fail(LOFP_EINVAL, "negative count");
    if (count > 0 && (!req || !out)) return fail(LOFP_EINVAL, "null requests or out");
    if (opts && opts->method == LOFP_METHOD_PATHSUM) return fail(LOFP_ENOTSUP, "multi-circuit batches use the contraction");
    if (stats) { std::memset(stats, 0, sizeof(*stats)); stats->batch = count; stats->method_used = LOFP_METHOD_CONTRACT; }
    if (count == 0) return LOFP_OK;
    const bool fp32 = opts && opts->precision == LOFP_PREC_FP32;
    const double rtol = opts && opts->fp32_rtol > 0 ? opts->fp32_rtol : 1e-6;
    Batch b;
    b.s = static_cast<hipStream_t>(stream);
    b.reqs.resize(count);
    for (int i = 0; i < count; ++i) {
        if (!req[i].circuit || !req[i].S || !req[i].T) return fail(LOFP_EINVAL, "null request field");
        Req &r = b.reqs[i];
        r.c = req[i].circuit;
        r.S.assign(req[i].S, req[i].S + r.c->m);
        r.T.assign(req[i].T, req[i].T + r.c->m);
        lofp_status rc = plan_request(r);
        if (rc != LOFP_OK) return rc;
    }
    Timer tm;
    tm.on = stats && opts && opts->record_timing;
    tm.s = b.s;
    tm.mark();
    lofp_status rc = launch_batch(b, fp32, fp32, &tm);
    if (rc != LOFP_OK) return rc;
    tm.mark();
    HIPCHK(hipStreamSynchronize(b.s));
    std::memcpy(out, b.h_out, count * sizeof(lofp_c128));
    {
        // the call has synchronised: an overflow (its results are NaN) is
        // reported whether or not statistics were asked for
        unsigned long long h[2];
        HIPCHK(hipMemcpy(h, b.d_ctr.p, sizeof(h), hipMemcpyDeviceToHost));
        if (h[1]) return fail(LOFP_ENOMEM, "contraction workspace overflow");
        if (stats) stats->transitions = (int64_t)h[0];
    }
    if (stats) {
        // the whole batch (copies, bounds, contraction), and the contraction kernel
        if (tm.on) { stats->ms_total = tm.ms(0, 3); stats->ms_contract = tm.ms(1, 2); }
    }
    for (int i = 0; i < count && err_bound; ++i) err_bound[i] = std::nan("");
    if (!fp32) return LOFP_OK;
    // bounds of the FP32 form; results it cannot certify are recomputed in FP64
    Batch f;
    f.s = b.s;
    std::vector<int> redo;
    for (int i = 0; i < count; ++i) {
        const double abs_form = b.h_abs[2 * i];
        const double bound = rounding_bound(b.reqs[i].c->G, b.reqs[i].n, abs_form, true);
        if (err_bound) err_bound[i] = bound;
        if (bound > rtol * std::hypot(out[i].re, out[i].im)) {
            redo.push_back(i);
            Req r = b.reqs[i];
            r.abs_form = abs_form;
            f.reqs.push_back(std::move(r));
        }
    }
    if (redo.empty()) return LOFP_OK;
    rc = launch_batch(f, 0, false);
    if (rc != LOFP_OK) return rc;
    HIPCHK(hipStreamSynchronize(f.s));
    for (size_t k = 0; k < redo.size(); ++k) {
        const int i = redo[k];
        out[i] = f.h_out[k];
        if (err_bound) err_bound[i] = rounding_bound(f.reqs[k].c->G, f.reqs[k].n, f.reqs[k].abs_form, false);
    }
    return LOFP_OK;
}

lofp_status lofp_server_create(const lofp_server_opts *o, lofp_server *out)
{
    if (!out) return fail(LOFP_EINVAL, "out is null");
    auto *sv = new lofp_server_s();
    sv->o.max_batch = 256;
    sv->o.streams = 2;
    sv->o.memory_budget = (int64_t)1 << 30;
    sv->o.precision = LOFP_PREC_FP64;
    if (o) {
        if (o->max_batch > 0) sv->o.max_batch = o->max_batch;
        if (o->streams > 0) sv->o.streams = std::min(o->streams, 8);
        if (o->memory_budget > 0) sv->o.memory_budget = o->memory_budget;
        sv->o.precision = o->precision;
        sv->o.fp32_rtol = o->fp32_rtol;
    }
    if (sv->o.precision != LOFP_PREC_FP64 && sv->o.precision != LOFP_PREC_FP32) {
        delete sv;
        return fail(LOFP_EINVAL, "bad precision");
    }
    (void)hipGetDevice(&sv->device);
    for (int i = 0; i < sv->o.streams; ++i) {
        auto b = std::make_unique<Batch>();
        hipError_t e = hipStreamCreateWithFlags(&b->s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete sv;
            return fail(LOFP_EDEVICE, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
        }
        sv->batches.push_back(std::move(b));
    }
    for (int i = 0; i < 2; ++i) sv->planners.emplace_back(planner_loop, sv);
    sv->worker = std::thread(worker_loop, sv);
    *out = sv;
    return LOFP_OK;
}

lofp_status lofp_server_submit(lofp_server sv, lofp_circuit c, const int32_t *S, const int32_t *T, uint64_t *ticket)
{
    if (!sv || !c || !S || !T || !ticket) return fail(LOFP_EINVAL, "null argument");
    Req r;
    r.c = c;
    r.S.assign(S, S + c->m);
    r.T.assign(T, T + c->m);
    lofp_status rc = check_request(r);   // planning happens on the worker
    if (rc != LOFP_OK) return rc;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return fail(LOFP_EINVAL, "server is stopping");
    r.ticket = sv->next_ticket++;
    r.t_submit = now_ms();
    *ticket = r.ticket;
    sv->queue.push_back(std::move(r));
    sv->submitted++;
    sv->cv_plan.notify_one();
    return LOFP_OK;
}

lofp_status lofp_server_result(lofp_server sv, uint64_t ticket, int32_t wait, lofp_c128 *out, double *latency_ms,
                               double *err_bound, int32_t *done)
{
    if (!sv || !done) return fail(LOFP_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    if (ticket == 0 || ticket >= sv->next_ticket) return fail(LOFP_EINVAL, "unknown ticket");
    for (;;) {
        auto fi = sv->failed.find(ticket);
        if (fi != sv->failed.end()) {
            const lofp_status st = fi->second.first;
            const std::string msg = fi->second.second;
            sv->failed.erase(fi);
            *done = 1;
            return fail(st, msg);
        }
        auto it = sv->done.find(ticket);
        if (it != sv->done.end()) {
            if (it->second.latency_ms < 0) {
                const std::string msg = sv->error;
                sv->done.erase(it);
                *done = 1;
                return fail(LOFP_EDEVICE, "request failed: " + msg);
            }
            if (out) *out = it->second.amp;
            if (latency_ms) *latency_ms = it->second.latency_ms;
            if (err_bound) *err_bound = it->second.err_bound;
            sv->done.erase(it);
            *done = 1;
            return LOFP_OK;
        }
        if (!wait) {
            *done = 0;
            return LOFP_OK;
        }
        sv->cv.wait(lk);
    }
}

lofp_status lofp_server_get_stats(lofp_server sv, lofp_server_stats *st)
{
    if (!sv || !st) return fail(LOFP_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    std::memset(st, 0, sizeof(*st));
    st->submitted = sv->submitted;
    st->completed = sv->completed;
    st->launches = sv->launches;
    st->mean_batch = sv->launches ? (double)sv->launched_reqs / (double)sv->launches : 0.0;
    st->fp64_fallbacks = sv->fp64_fallbacks;
    st->pathsum_fallbacks = sv->pathsum_fallbacks;
    if (!sv->latencies.empty()) {
        std::vector<double> v = sv->latencies;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) { return v[std::min(v.size() - 1, (size_t)(q * (v.size() - 1) + 0.5))]; };
        st->p50_ms = pct(0.50);
        st->p99_ms = pct(0.99);
        st->max_ms = v.back();
    }
    return LOFP_OK;
}

lofp_status lofp_server_destroy(lofp_server sv)
{
    if (!sv) return fail(LOFP_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv.notify_all();
        sv->cv_plan.notify_all();
        sv->cv_launch.notify_all();
    }
    for (auto &t : sv->planners)
        if (t.joinable()) t.join();
    if (sv->worker.joinable()) sv->worker.join();
    for (auto &b : sv->batches) {
        if (b->s) (void)hipStreamSynchronize(b->s);
    }
    for (auto &b : sv->batches) {
        hipStream_t s = b->s;
        b.reset();
        if (s) (void)hipStreamDestroy(s);
    }
    delete sv;
    return LOFP_OK;
}

}  // extern "C"
