// graph.cpp -- one amplitude call captured as a HIP graph and replayed.
//
// Batches of patterns that are evaluated again and again (new T values in
// the same buffer, the same circuit and S) pay the host work and the launch
// latency of the call's kernels once: the call is captured once into a
// graph and each replay launches the whole graph.  The contraction path of a
// call has no host read-back and no memset when the split is decided on the
// device, which is what makes it capturable.  The graph runs on a private
// copy of the circuit, so its buffers never move under later calls on the
// caller's circuit.
#include <hip/hip_runtime.h>

#include "host_internal.h"

struct lofp_graph_s {
    lofp_circuit_s *circ = nullptr;   // private copy, owns the graph's buffers
    hipStream_t stream = nullptr;     // capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace lofp;
using namespace lofp::host;

namespace {

void free_graph(lofp_graph_s *g)
{
    if (!g) return;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->circ) (void)lofp_circuit_destroy(g->circ);
    if (g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

}  // namespace

extern "C" {

lofp_status lofp_graph_create(lofp_circuit c, const int32_t *S, int32_t batch, const int32_t *T_dev,
                              lofp_c128 *out_dev, const lofp_opts *opts, lofp_graph *out)
{
    if (!c || !out) return fail(LOFP_EINVAL, "null circuit or out");
    if (batch <= 0 || !T_dev || !out_dev) return fail(LOFP_EINVAL, "need a batch of at least one pattern and T, out");
    if (batch > 32768) return fail(LOFP_ENOTSUP, "a captured call takes at most 32768 patterns");
    int n = 0;
    lofp_status rc = check_S(*c, S, n);
    if (rc != LOFP_OK) return rc;
    lofp_opts o{};
    o.method = LOFP_METHOD_AUTO;
    o.fwd_layer = -1;
    o.bwd_layer = -1;
    if (opts) o = *opts;
    if (o.method == LOFP_METHOD_PATHSUM) return fail(LOFP_ENOTSUP, "the path sum sizes its frontiers on the host: not capturable");
    o.method = LOFP_METHOD_CONTRACT;
    o.record_timing = 0;
    auto *g = new lofp_graph_s();
    {
        std::lock_guard<std::mutex> lk(c->mu);
        rc = clone_circuit(*c, &g->circ);
    }
    if (rc != LOFP_OK) { free_graph(g); return rc; }
    hipError_t e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
    if (e != hipSuccess) { free_graph(g); return fail(LOFP_EDEVICE, hipGetErrorString(e)); }
    // an ordinary call first: it sets the circuit up, tunes if asked, and
    // allocates every buffer, so the captured call allocates nothing
    rc = lofp_amplitudes_device(g->circ, S, batch, T_dev, out_dev, &o, g->stream, nullptr);
    if (rc == LOFP_OK) {
        e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) rc = fail(LOFP_EDEVICE, hipGetErrorString(e));
    }
    if (rc != LOFP_OK) { free_graph(g); return rc; }
    e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { free_graph(g); return fail(LOFP_EDEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e)); }
    rc = lofp_amplitudes_device(g->circ, S, batch, T_dev, out_dev, &o, g->stream, nullptr);
    const std::string msg = rc != LOFP_OK ? std::string(lofp_last_error()) : std::string();
    e = hipStreamEndCapture(g->stream, &g->graph);
    if (rc != LOFP_OK) { free_graph(g); return fail(rc, "captured call: " + msg); }
    if (e != hipSuccess || !g->graph) {
        free_graph(g);
        return fail(LOFP_ENOTSUP, std::string("the call could not be captured (a host read-back on this workload): ") +
                                      hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { free_graph(g); return fail(LOFP_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)); }
    *out = g;
    return LOFP_OK;
}

lofp_status lofp_graph_launch(lofp_graph g, void *stream)
{
    if (!g || !g->exec) return fail(LOFP_EINVAL, "null graph");
    const hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(LOFP_EDEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    return LOFP_OK;
}

lofp_status lofp_graph_destroy(lofp_graph g)
{
    if (!g) return fail(LOFP_EINVAL, "null graph");
    free_graph(g);
    return LOFP_OK;
}

}  // extern "C"
