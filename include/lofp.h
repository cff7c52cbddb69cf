/*
 * lofp.h -- C-ABI of the MI355X (gfx950) Feynman path-sum library.
 *
 * The library computes the exact amplitude <T|U_P|S> of a Fock input S and a
 * photon-detection pattern T through layers of locally connected two-mode
 * beam splitters (Sec. II of the paper).  A path is the sequence of
 * intermediate Fock configurations between beam splitters; its weight is the
 * product of single-beam-splitter transition amplitudes (Appendix) and the
 * amplitude is the sum over valid paths (Eq. (1)).
 *
 * Conventions (all calls):
 *   - Modes are numbered 0..m-1 from the top of the circuit.
 *   - A beam splitter acts on two modes a < b, usually adjacent (b = a + 1);
 *     mode a is its upper port (index 1 in Eq. (bs_matrix)), theta and phi
 *     are the two angles of
 *     Eq. (bs_matrix): [[cos t, -e^{-i p} sin t], [e^{i p} sin t, cos t]],
 *     rows = output ports, columns = input ports.
 *   - Layers are applied in the order given; inside a layer beam splitters
 *     must act on disjoint modes.  Any angle values are accepted.
 *   - S and T are int32 occupation vectors of length m.  If sum(S) != sum(T)
 *     the amplitude is exactly 0 (photon number is conserved, Sec. II).
 *   - Complex results are two doubles {re, im}.
 *   - Every call returns a lofp_status; on anything but LOFP_OK a message is
 *     available from lofp_last_error() (thread-local, valid until the next
 *     call on the same thread).  On error no output is written.
 *   - Results are bit-reproducible for a fixed (circuit, S, T, opts) and do
 *     not depend on the other patterns of the batch.
 *
 * Limits: m <= 32 modes and total photon number n <= 64 (LOFP_ENOTSUP
 * otherwise).
 */
#ifndef LOFP_H
#define LOFP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LOFP_OK = 0,
    LOFP_EINVAL = 1,   /* malformed argument (null pointer, bad mode, ...) */
    LOFP_ENOMEM = 2,   /* device or host allocation failed, or a state space
                          exceeds the 32-bit index range                     */
    LOFP_ENOTSUP = 3,  /* valid request outside the supported limits        */
    LOFP_EDEVICE = 4   /* HIP runtime error (message names the call)        */
} lofp_status;

/* One beam splitter, Eq. (bs_matrix), on modes a < b. */
typedef struct {
    int32_t a, b;
    double theta, phi;
} lofp_bs;

typedef struct {
    double re, im;
} lofp_c128;

/* Opaque circuit handle.  Owns a copy of the layer list, the light-cone
 * (reach) tables and, once a device call has been made, the device copy of
 * the beam-splitter transition tables and the workspace of its calls.
 * Immutable after creation; calls on one handle from several threads are
 * serialised internally, and a call on one stream waits (on the device) for
 * the previous call's work on the handle when that ran on another stream. */
typedef struct lofp_circuit_s *lofp_circuit;

enum {
    LOFP_METHOD_AUTO = 0,     /* contraction when its state fits, else path sum */
    LOFP_METHOD_PATHSUM = 1,  /* frontier split + depth-first path sum       */
    LOFP_METHOD_CONTRACT = 2  /* mode-axis layer-block contraction (Sec. II.C) */
};

enum {
    LOFP_PREC_FP64 = 0,       /* products, tables and sums in FP64           */
    LOFP_PREC_FP32 = 1        /* path products in FP32; tables and sums FP64 */
};

/* How the contraction treats a batch sharing S (Sec. II.C contracted from
 * both ends): each distinct top and bottom half of T contracted once and
 * joined per pattern, or one contraction per pattern.  The results agree to
 * rounding (the sums run in another order). */
enum {
    LOFP_SPLIT_AUTO = 0,      /* split when halves are shared, for batches of
                                 256 to 1024 patterns, and for smaller
                                 batches of circuits with at least 40
                                 splitters (two half-length chains in
                                 parallel beat one long chain)             */
    LOFP_SPLIT_NEVER = 1,     /* one contraction per pattern                 */
    LOFP_SPLIT_ALWAYS = 2     /* halves contracted and joined for any batch  */
};

typedef struct {
    int32_t method;        /* LOFP_METHOD_*                                    */
    int32_t precision;     /* LOFP_PREC_*                                      */
    int32_t fwd_layer;     /* frontier cut: forward frontier after this many
                              layers (-1 = chosen by the planner)             */
    int32_t bwd_layer;     /* backward frontier at this layer boundary
                              (-1 = planner); fwd_layer <= bwd_layer          */
    int32_t record_timing; /* 1: time each phase with HIP events (adds a
                              stream synchronisation at the end of the call) */
    int32_t frontier_budget_kb; /* path sum with fwd_layer = -1: the forward
                              frontier is merged up to the latest layer whose
                              frontier fits this many KiB (0 = a quarter of
                              the free device memory); the splitters between
                              the frontiers (at most 16) are enumerated
                              depth-first                                  */
    int32_t count_work;       /* with stats: also count the work done
                                 (stats->transitions); the counting kernels
                                 run slower, so timed calls leave it 0       */
    int32_t state_limit;      /* contraction: at most this many entries per
                                 state buffer (0 = as large as the state
                                 needs).  A result whose state would exceed
                                 the limit is NaN + NaN i; the call returns
                                 ENOMEM when stats are passed              */
    double fp32_rtol;         /* multi-circuit FP32 form: a result whose
                                 rounding bound exceeds fp32_rtol * |amp| is
                                 recomputed in FP64 (0 = 1e-6)               */
    int32_t autotune;         /* contraction with split = LOFP_SPLIT_AUTO: 1 =
                                 on the first call for this circuit, S and
                                 batch size, time the candidate ways to
                                 contract it (split cut, LDS per job, split
                                 or one job per pattern) on the device and
                                 keep the fastest for later calls with
                                 autotune = 1 (that first call synchronises
                                 the stream); 0 = the default way          */
    int32_t split;            /* contraction: LOFP_SPLIT_* (EINVAL otherwise) */
} lofp_opts;

/* Per-call statistics (filled when a non-null pointer is passed). */
typedef struct {
    int32_t batch;            /* patterns in the call                          */
    int32_t fwd_layer;        /* layer boundaries actually used                */
    int32_t bwd_layer;
    int32_t dfs_levels;       /* beam splitters enumerated depth-first         */
    int64_t frontier_states;  /* forward frontier entries over the batch       */
    int64_t backward_states;  /* backward frontier entries over the batch      */
    int64_t bfs_states;       /* states produced by all frontier expansions    */
    int64_t dfs_leaves;       /* complete middle paths evaluated               */
    int64_t dfs_edges;        /* depth-first tree edges taken (incl. leaves)   */
    int64_t transitions;      /* contraction (count_work): transitions with a
                                 nonzero source state                        */
    double ms_plan;           /* record_timing: bounds + state-space tables
                                 (contraction: bounds and key hulls)         */
    double ms_forward;        /*   forward frontier expansion                  */
    double ms_backward;       /*   backward frontier expansion                 */
    double ms_dfs;            /*   depth-first kernel                          */
    double ms_reduce;         /*   final compensated reduction (contraction
                                   split across the batch: the join)         */
    double ms_contract;       /*   contraction kernel                          */
    double ms_total;          /*   whole call on the stream                    */
    int32_t method_used;      /* LOFP_METHOD_PATHSUM or LOFP_METHOD_CONTRACT   */
    int32_t split_top_keys;   /* contraction split across the batch: distinct  */
    int32_t split_bottom_keys;/*   top / bottom halves of T (0 if not split)   */
    int32_t max_state;        /* contraction: entries of the largest state     */
    int32_t split_cut;        /* split contraction: the top half's last cut    */
    int32_t lds_kb;           /*   LDS per job (KiB)                           */
    int32_t tuned;            /* 1 if the way of contracting came from the tuner */
} lofp_stats;

/* Message for the last non-OK status on this thread ("" if none). */
const char *lofp_last_error(void);

/* Library version string. */
const char *lofp_version(void);

/* Build a circuit from n_layers layers; layer k holds layer_len[k] beam
 * splitters, stored consecutively in bs (host memory, copied).
 * Sec. II: the interferometer is a list of layers of two-mode beam splitters
 * with parameters (theta, phi).  Does not touch the GPU.
 * Distant pairs (b > a + 1; Sec. II.A allows connections between distant
 * modes) are compiled exactly to adjacent splitters: mode b is brought next
 * to a by exact swaps (theta = -pi/2, phi = 0, tables built with
 * cos theta = 0) on (b-1, b), ..., (a+1, a+2), the splitter acts on
 * (a, a+1), and the chain is undone by the inverse swaps (theta = pi/2) in
 * reverse order; every Fock amplitude is that of the given circuit (up to
 * rounding), and the light-cone bounds follow the compiled layers.  The
 * host queries of layers and cuts (lofp_light_cone, lofp_bounds,
 * lofp_bounds_batch) and lofp_path_counts return ENOTSUP for such circuits.
 * Errors: EINVAL for m < 2, negative lengths, a or b out of range, a >= b,
 * or a mode used twice in one layer; ENOTSUP for m > 32 or more than 250
 * layers after compiling distant pairs. */
lofp_status lofp_circuit_create(int32_t m, int32_t n_layers, const int32_t *layer_len,
                                const lofp_bs *bs, lofp_circuit *out);

lofp_status lofp_circuit_destroy(lofp_circuit c);

/* Light cone of one waveguide (Sec. II.B, Fig. light_cones): the output
 * waveguide of mode `mode` after `layer` layers (0 <= layer <= D) receives
 * photons only from inputs [*past_lo, *past_hi] and sends them only to
 * outputs [*fut_lo, *fut_hi] (0-based, inclusive).  Host only. */
lofp_status lofp_light_cone(lofp_circuit c, int32_t layer, int32_t mode, int32_t *past_lo,
                            int32_t *past_hi, int32_t *fut_lo, int32_t *fut_hi);

/* Cut bounds for one (S, T) (Sec. II.B light cones, tightened by photon
 * conservation): lo[t*(m-1)+r] <= #photons in modes 0..r after t layers
 * <= hi[t*(m-1)+r], for t = 0..D, r = 0..m-2.  lo/hi: host arrays of
 * (D+1)*(m-1) int32.  *feasible = 0 when no valid path exists.  Host only. */
lofp_status lofp_bounds(lofp_circuit c, const int32_t *S, const int32_t *T, int32_t *lo,
                        int32_t *hi, int32_t *feasible);

/* The same cut bounds for a batch of patterns, computed on the device by the
 * planner kernel that the amplitude calls run (one wave per pattern).  T:
 * host int32[batch][m]; lo, hi: host int32[batch][(D+1)*(m-1)] in the layout
 * of lofp_bounds; feasible: host int32[batch].  lo/hi of an infeasible
 * pattern are unspecified (lo > hi somewhere).  EINVAL for null arguments
 * or negative occupations.  Synchronises the default stream. */
lofp_status lofp_bounds_batch(lofp_circuit c, const int32_t *S, int32_t batch, const int32_t *T, int32_t *lo,
                              int32_t *hi, int32_t *feasible);

/* Single-beam-splitter transition table (Appendix): out[x1*(N+1)+y1] =
 * <y1, N-y1| BS_g |x1, N-x1> for beam splitter g (0-based, in application
 * order) and photon number N, computed on the device in FP64 by the same
 * kernel the path sum uses, copied to the host array out ((N+1)^2 entries). */
lofp_status lofp_bs_table(lofp_circuit c, int32_t gate, int32_t N, lofp_c128 *out);

/* Amplitudes <T_i|U_P|S> for a batch of patterns, device-resident form.
 * S: host int32[m].  T_dev: device int32[batch*m] (row-major).  out_dev:
 * device lofp_c128[batch].  stream: hipStream_t (NULL = default stream).
 * Kernels run on `stream`; the call synchronises that stream once to size
 * the frontier buffers, and returns with the results written in stream
 * order.  opts may be NULL (defaults); stats may be NULL.
 * Eq. (1) summed by the frontier split (forward and backward merged
 * frontiers, Schroedinger-Feynman interpolation of Sec. I) and depth-first
 * enumeration of the middle layers (method PATHSUM), or by the mode-axis
 * contraction of Sec. II.C (method CONTRACT).  Batches above 32768 patterns
 * run in passes of 32768 (stats then sum over the passes).  A result whose
 * contraction state did not fit its buffers (see opts->state_limit) is
 * NaN + NaN i; with stats the call then returns ENOMEM. */
lofp_status lofp_amplitudes_device(lofp_circuit c, const int32_t *S, int32_t batch,
                                   const int32_t *T_dev, lofp_c128 *out_dev,
                                   const lofp_opts *opts, void *stream, lofp_stats *stats);

/* Allocation-free form of lofp_amplitudes_device, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid allocation).  It runs the contraction one pattern
 * per block (method AUTO or CONTRACT; precision FP64 or FP32; state_limit
 * honoured; other options ignored) with every per-call buffer carved from
 * one fixed device array of the library (32 MiB per device, held until the
 * process ends); it calls no device allocation routine.
 * S: host int32[m].  T_dev: device int32[batch*m].  out_dev: device
 * lofp_c128[batch].  stream: hipStream_t (NULL = default).  Stream-ordered,
 * no synchronisation.  A result whose state did not fit is NaN + NaN i.
 * All calls on one device share the array, which keeps the last call's
 * contents: calls that overlap on one device race (order them on one stream
 * or synchronise between them).
 * Errors: EINVAL for null arguments, a batch whose buffers exceed the array
 * (the message gives the bytes needed), or a circuit whose tables and step
 * program are not yet on the device for this photon number (make one
 * lofp_amplitudes_device call with the contraction first); ENOTSUP for the
 * path-sum method or a state beyond 2^22 entries. */
lofp_status lofp_amplitudes_device_noalloc(lofp_circuit c, const int32_t *S, int32_t batch,
                                           const int32_t *T_dev, lofp_c128 *out_dev,
                                           const lofp_opts *opts, void *stream);

/* ---------------------------------------------------------------------------
 * One amplitude call captured as a HIP graph (batching: a batch evaluated
 * again and again pays the host planning and the kernel launches once).
 * lofp_graph_create makes one ordinary call of lofp_amplitudes_device (the
 * contraction; opts may ask for autotune) on a private copy of the circuit,
 * then captures a second call into a graph; the graph reads T_dev and writes
 * out_dev (device buffers the caller keeps alive and in place) each time it
 * is launched, with S and the batch size fixed.  The copy owns the graph's
 * workspace, so later calls on c do not disturb it.  Synchronises at
 * creation.  Errors: EINVAL for null arguments or batch < 1; ENOTSUP for the
 * path-sum method, batch > 32768, or a workload whose call needs a host
 * read-back (a contraction state above 2^20 entries in the split form, or
 * above 2^22 / beyond 1 GiB of workspace per pattern). */
typedef struct lofp_graph_s *lofp_graph;
lofp_status lofp_graph_create(lofp_circuit c, const int32_t *S, int32_t batch, const int32_t *T_dev,
                              lofp_c128 *out_dev, const lofp_opts *opts, lofp_graph *out);
/* Launch the captured call on `stream` (hipStream_t; NULL = default).
 * Launches on one graph must not overlap (they share its workspace). */
lofp_status lofp_graph_launch(lofp_graph g, void *stream);
lofp_status lofp_graph_destroy(lofp_graph g);

/* Host-memory form of lofp_amplitudes_device: T is host int32[batch*m], out
 * host lofp_c128[batch].
 * Copies in and out and synchronises; for convenience, not for timing. */
lofp_status lofp_amplitudes(lofp_circuit c, const int32_t *S, int32_t batch, const int32_t *T,
                            lofp_c128 *out, const lofp_opts *opts, lofp_stats *stats);

/* One amplitude, host memory, default options. */
lofp_status lofp_amplitude(lofp_circuit c, const int32_t *S, const int32_t *T, lofp_c128 *out);

/* Every output amplitude of one input (Sec. IV names computing all output
 * amplitudes as an extension): the C(m+n-1, n) patterns T with
 * sum(T) = sum(S), in decreasing lexicographic order of (t_0, ..., t_{m-1})
 * (the first puts every photon in mode 0, the last in mode m-1), each with
 * <T|U_P|S> computed on the device by lofp_amplitudes_device (opts may be
 * NULL) in passes of 32768 patterns.  T_out: host int32[capacity*m];
 * amp_out: host lofp_c128[capacity]; *count receives the number of
 * patterns.  With both outputs NULL only *count is set.  Synchronises the
 * default stream.  Errors: EINVAL for a null count, one output NULL, or a
 * capacity below the count; ENOTSUP above 2^31 patterns. */
lofp_status lofp_all_outputs(lofp_circuit c, const int32_t *S, int64_t capacity, int32_t *T_out,
                             lofp_c128 *amp_out, int64_t *count, const lofp_opts *opts);

/* The circuit the library evaluates, host only: each splitter on distant
 * modes (a, b) is compiled to adjacent ones (see lofp_circuit_create).
 * *n_layers receives the compiled depth; with layer_len (int32[depth]) and
 * bs (lofp_bs[capacity]) both non-NULL, the compiled layers are written
 * (EINVAL if capacity is below the compiled splitter count). */
lofp_status lofp_circuit_compiled(lofp_circuit c, int32_t *n_layers, int32_t *layer_len, lofp_bs *bs,
                                  int32_t capacity);

/* Number of valid paths of Eq. (1) for each pattern (conservation-valid
 * sequences of intermediate configurations from S to T_i, counted on the
 * device by the contraction in the counting semiring; exact below 2^53).
 * T: host int32[batch*m]; counts: host double[batch]. */
lofp_status lofp_path_counts(lofp_circuit c, const int32_t *S, int32_t batch, const int32_t *T,
                             double *counts);

/* ---------------------------------------------------------------------------
 * Many circuits per launch.
 * One request = one circuit, one S and one T (host memory, copied at the call).
 * Circuits may all differ in mode count, depth and angles. */
typedef struct {
    lofp_circuit circuit;
    const int32_t *S;   /* int32[m of that circuit] */
    const int32_t *T;   /* int32[m of that circuit] */
} lofp_request;

/* Amplitudes of `count` requests evaluated by the mode-axis contraction
 * (Sec. II.C) in one bounds launch and one contraction launch on `stream`;
 * each circuit's tables and step program stay resident on the device.  out:
 * host lofp_c128[count].  opts: precision and record_timing; method must be
 * AUTO or CONTRACT.  Synchronises `stream`.
 *
 * Precision FP32: transition products in FP32, sums in FP64, and for every
 * result a rounding bound |amp - exact| <= ((1 + f)^G - 1 + 2^-51) A_abs,
 * exact meaning the same sum in exact arithmetic over the FP64 tables; G is
 * the circuit's splitter count, A_abs the sum over paths of the products of
 * |Re W| + |Im W| (computed by a second, absolute pass), and
 * f = 4u/(1 - 4u) + (2(n+1)^2 + 2) 2^-53 with u = 2^-24 (about 4 G u A_abs).
 * A result whose bound exceeds opts->fp32_rtol * |amp| is recomputed in FP64
 * (its bound then has f = (2(n+1)^2 + 2) 2^-53).  The bound assumes no FP32
 * underflow.  err_bound (host double[count], may be NULL) receives each
 * result's bound; NaN for the FP64 form, which computes none.
 *
 * Errors: EINVAL for null fields or bad occupations, ENOTSUP for a circuit
 * the contraction cannot take, ENOMEM past 2^22 state entries. */
lofp_status lofp_amplitudes_multi(int32_t count, const lofp_request *req, lofp_c128 *out,
                                  double *err_bound, const lofp_opts *opts, void *stream, lofp_stats *stats);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of amplitude requests.
 * A worker thread admits whatever has been submitted (up to max_batch, while
 * the admitted workspace stays within memory_budget bytes), launches it as
 * one multi-circuit batch on the next free stream, and keeps admitting while
 * earlier batches run (up to `streams` batches in flight).  A result does
 * not depend on which other requests shared its batch.  The caller keeps each
 * circuit alive until its requests have completed. */
typedef struct lofp_server_s *lofp_server;

typedef struct {
    int32_t max_batch;      /* requests per launch (default 256)              */
    int32_t streams;        /* batches in flight, one HIP stream each (2, <=8) */
    int64_t memory_budget;  /* device workspace bytes admitted at once (1 GiB) */
    int32_t precision;      /* LOFP_PREC_* for every request; FP32 results
                               carry bounds and fall back to FP64 as in
                               lofp_amplitudes_multi                          */
    int32_t reserved;
    double fp32_rtol;       /* the fallback threshold (0 = 1e-6)              */
} lofp_server_opts;

typedef struct {
    int64_t submitted, completed, launches;
    double mean_batch;      /* requests per launch                            */
    double p50_ms, p99_ms, max_ms;   /* submit-to-completion latency          */
    int64_t fp64_fallbacks; /* FP32 results recomputed in FP64                */
    int64_t pathsum_fallbacks; /* requests the contraction refused (program or
                               state too large), summed by the path-sum form
                               on a planner thread instead                 */
} lofp_server_stats;

/* Start a server on the current device (opts may be NULL). */
lofp_status lofp_server_create(const lofp_server_opts *opts, lofp_server *out);
/* Queue one request (S, T: host int32[m], copied); *ticket identifies it.
 * Lengths and occupations are checked here (EINVAL); the request is planned
 * on the server's thread.  A request the contraction cannot take is summed
 * by the path-sum form instead (counted in pathsum_fallbacks); if that fails
 * too, its error (ENOMEM) comes from lofp_server_result. */
lofp_status lofp_server_submit(lofp_server s, lofp_circuit c, const int32_t *S, const int32_t *T,
                               uint64_t *ticket);
/* *done = 1 and out / latency_ms / err_bound filled (any may be NULL) once
 * the ticket has completed; wait = 1 blocks until then.  err_bound: the
 * result's rounding bound (FP32 form and its FP64 fallbacks; NaN for the
 * FP64 form).  A completed ticket is consumed.  EDEVICE if its batch failed;
 * the planning error (ENOTSUP, ENOMEM) if the request could not run. */
lofp_status lofp_server_result(lofp_server s, uint64_t ticket, int32_t wait, lofp_c128 *out,
                               double *latency_ms, double *err_bound, int32_t *done);
lofp_status lofp_server_get_stats(lofp_server s, lofp_server_stats *out);
/* Finish every queued request, stop the worker and free the server. */
lofp_status lofp_server_destroy(lofp_server s);

#ifdef __cplusplus
}
#endif

#endif /* LOFP_H */
