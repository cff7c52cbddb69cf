// host_internal.h -- host-side internals shared by the C-ABI translation
// units (api.cpp, serve.cpp).  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "lofp.h"
#include "lofp_device.h"

namespace lofp {
namespace host {

lofp_status fail(lofp_status s, const std::string &msg);
void clear_error();
const char *last_error();

#define HIPCHK(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return ::lofp::host::fail(e_ == hipErrorOutOfMemory ? LOFP_ENOMEM : LOFP_EDEVICE,     \
                                      std::string(#call) + ": " + hipGetErrorString(e_));         \
    } while (0)

// A device buffer the owner allocates, or (view) a range of a block that
// someone else owns: a view is never freed through the DevBuf.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    bool view = false;
    template <class T> T *as() const { return static_cast<T *>(p); }
};

inline hipError_t ensure(DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (bytes <= b.cap) return hipSuccess;
    if (b.p && !b.view) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess) return e;
    }
    b.p = nullptr;
    b.cap = 0;
    b.view = false;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipSuccess) b.cap = bytes;
    return e;
}

inline void release(DevBuf &b)
{
    if (b.p && !b.view) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    b.view = false;
}

inline void set_view(DevBuf &b, void *p, size_t bytes)
{
    release(b);
    b.p = p;
    b.cap = bytes;
    b.view = true;
}

// Device memory pool for circuit set-up (csrc/pool.cpp): blocks come from
// 64 MiB slabs in power-of-two size classes and go back to per-class free
// lists, so creating many small circuits costs no hipMalloc each.  Slabs live
// until the process ends.
void *pool_alloc(size_t bytes, int device);
void pool_free(void *p, size_t bytes, int device);

// A pooled block shared by the circuits set up together; freed to the pool
// when the last of them is destroyed.
struct SharedBlock {
    void *p = nullptr;
    size_t bytes = 0;
    int device = 0;
    ~SharedBlock()
    {
        if (p) pool_free(p, bytes, device);
    }
};

template <class T>
hipError_t upload(DevBuf &b, const std::vector<T> &v, hipStream_t s)
{
    hipError_t e = ensure(b, v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// A factor reference: kind = CREF_* with arg = cut, or kind = -1 with arg =
// variable id.
struct FRef {
    int kind, arg;
};

struct Schedule {
    std::vector<lofp::ContractStep> steps;
    std::vector<int> live_out;   // live variables after the last step
    std::string error;
};

// How a batch sharing S is contracted (chosen by default or by the tuner).
struct SplitCfg {
    enum Mode { kDevice = 0, kHost = 1, kPerPattern = 2 };
    int mode = kDevice;   // device-decided split, host-sized split, or one job per pattern
    int rs = 0;           // split cut: the top half holds cuts 0..rs
    int lds_kb = 52;      // LDS of one job of the split contraction
    int small_min = 256;  // batch sizes split without shared halves
    int small_max = 1024;
};

struct SplitProgram {
    int rs = 0;
    Schedule top, bot;
    DevBuf d_top, d_bot;
    bool on_device = false;
    ~SplitProgram()
    {
        release(d_top);
        release(d_bot);
    }
};

}  // namespace host
}  // namespace lofp

struct lofp_circuit_s {
    using DevBuf = lofp::host::DevBuf;
    int m = 0, D = 0, G = 0, nc = 0;       // D, G: layers and splitters as compiled
    int user_depth = 0;                    // layers as given
    bool compiled = false;                 // distant pairs compiled to adjacent ones
    std::vector<int> user_gate;            // internal gate of each given splitter
    std::vector<uint8_t> gate_swap;        // per splitter: 0, 1 = exact swap
                                           // [[0,1],[-1,0]], 2 = its inverse
    std::vector<lofp_bs> gates;            // application order
    std::vector<int32_t> gate_cut, gate_layer, layer_start;
    std::vector<uint8_t> cut_gate;         // [D][nc]
    std::vector<int32_t> gate_at;          // [D][nc] gate id or -1
    std::vector<int8_t> fr_lo, fr_hi, br_lo, br_hi;  // [(D+1)][m]
    std::vector<uint8_t> stage_time;       // [(G+1)][nc]
    std::vector<int32_t> cut_ngates, cut_gates, ver_at;
    // contraction step program (built once per circuit)
    // device-side set-up enqueued on some stream; later users on other
    // streams wait for ready_ev
    bool pending_init = false;
    hipEvent_t ready_ev = nullptr;
    hipStream_t ready_stream = nullptr;
    // end of the last call's work on the per-call buffers below, and its stream
    hipEvent_t last_ev = nullptr;
    hipStream_t last_stream = nullptr;
    bool prog_built = false;
    bool prog_on_device = false;
    std::string prog_error;
    int nvars = 0;
    std::vector<int32_t> var_cut, var_time;
    std::vector<lofp::ContractStep> steps;
    std::vector<std::vector<int>> var_of;                    // [cut][version] -> variable or -1
    std::vector<std::array<lofp::host::FRef, 4>> fac;       // factors in cut-major order
    std::vector<int> fgate, fcut;
    std::map<int, std::unique_ptr<lofp::host::SplitProgram>> splits;
    // tuned ways of contracting: (S, (batch, fp32, state limit)) -> configuration
    using TuneKey = std::pair<std::vector<int32_t>, std::array<int, 3>>;
    std::map<TuneKey, lofp::host::SplitCfg> tuned;
    std::mutex mu;

    // device state (lazy)
    bool dev_ready = false;
    int n_tab = -1;
    int tab_stride = 0;
    DevBuf d_table, d_theta, d_phi, d_fr_lo, d_fr_hi, d_br_lo, d_br_hi, d_cut_gate, d_stage_time;
    DevBuf d_gate_cut, d_gate_layer, d_cut_ngates, d_cut_gates, d_ver_at, d_var_cut, d_var_time, d_steps;
    // per-call workspace
    DevBuf d_S, d_lo, d_hi, d_inf, d_C, d_E, d_count, d_slot_stage, d_off, d_coff, d_fa, d_fb, d_ba, d_bb;
    DevBuf d_levels, d_tab_mid, d_counters, d_T, d_out, d_ws, d_cfg, d_rankb;
    DevBuf d_ktab, d_kslot, d_kof, d_krep, d_kcnt, d_khull, d_klohi, d_kinf, d_jobs, d_kstate, d_korder;
    DevBuf d_ws2;                          // per-pattern workspace of the device-decided split
    std::vector<std::shared_ptr<lofp::host::SharedBlock>> blocks;   // pooled set-up blocks in use
    int32_t *h_pin = nullptr;              // small pinned readback buffer
    lofp::KeyLayoutState klay;             // layout of the key table and hulls
    std::vector<int32_t> S_dev;            // the S now held in d_S
    // S-only bounds of the last S asked for, and the state bounds under them
    // (the whole program; each split program by its split cut)
    std::vector<int32_t> sb_S;
    std::vector<int16_t> sb_lo, sb_hi;
    int64_t sb_prog = -1;
    std::map<int, int64_t> sb_split;
};


namespace lofp {
namespace host {

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


// The per-call buffers of a circuit serve every call on it, whatever its
// stream: a call first makes its stream wait for the previous call's work
// when that ran on another stream, and on leaving records where its own work
// ends (enqueued or not, whatever the status).
class StreamUse {
public:
    StreamUse(lofp_circuit_s &c, hipStream_t s) : c_(c), s_(s) {}
    StreamUse(const StreamUse &) = delete;
    StreamUse &operator=(const StreamUse &) = delete;
    hipError_t begin()
    {
        // a call being captured into a graph records no events (the graph's
        // circuit serves that graph alone)
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s_, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return hipSuccess;
        armed_ = true;
        if (c_.last_ev && c_.last_stream != s_) return hipStreamWaitEvent(s_, c_.last_ev, 0);
        return hipSuccess;
    }
    ~StreamUse()
    {
        if (!armed_) return;
        if (!c_.last_ev && hipEventCreateWithFlags(&c_.last_ev, hipEventDisableTiming) != hipSuccess) {
            c_.last_ev = nullptr;
            return;
        }
        if (hipEventRecord(c_.last_ev, s_) == hipSuccess) c_.last_stream = s_;
    }

private:
    lofp_circuit_s &c_;
    hipStream_t s_;
    bool armed_ = false;
};

lofp_status check_S(const lofp_circuit_s &c, const int32_t *S, int &n);
// A new circuit with the same compiled splitters (and exact swaps) as c, and
// buffers of its own.
lofp_status clone_circuit(const lofp_circuit_s &c, lofp_circuit_s **out);
// S-only bounds of S, cached on the circuit (the caller holds its lock).
void s_only_cached(lofp_circuit_s &c, const int32_t *S, int n);
void s_only_bounds(const lofp_circuit_s &c, const int32_t *S, int n, std::vector<int16_t> &lo,
                   std::vector<int16_t> &hi);
lofp_status device_init(lofp_circuit_s &c, int n, hipStream_t s);
lofp_status init_circuits(const std::vector<std::pair<lofp_circuit_s *, int>> &list, hipStream_t s);
lofp_status prepare_program(lofp_circuit_s &c, hipStream_t s);
void build_program(lofp_circuit_s &c);
SplitProgram *get_split(lofp_circuit_s &c, int rs);
// Record or wait for the circuit's device set-up so that `s` sees it.
lofp_status ready_on_stream(lofp_circuit_s &c, hipStream_t s);
int64_t program_state_bound(const lofp_circuit_s &c, const std::vector<int16_t> &lo, const std::vector<int16_t> &hi);

}  // namespace host
}  // namespace lofp
