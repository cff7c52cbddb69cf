// lofp_device.h -- declarations shared by the kernel files and the host API.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "key_layout.h"
#include "lofp_core.h"

namespace lofp {

// Complex FP64 helpers (double2 = {re, im}).
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc)
{
    return make_double2(acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x);
}

// Compensated accumulator: running sum s and the accumulated rounding error
// c, each addition done with Knuth's branch-free TwoSum.
struct CSum {
    double s, c;
};
__device__ __forceinline__ void csum_add(CSum &a, double x)
{
    double t = a.s + x;
    double z = t - a.s;
    double e = (a.s - (t - z)) + (x - z);
    a.s = t;
    a.c += e;
}
__device__ __forceinline__ void csum_merge(CSum &a, const CSum &b)
{
    csum_add(a, b.s);
    a.c += b.c;
}

// exact small-integer quotient via the float reciprocal (values < 2^22)
__device__ __forceinline__ int qdiv(int a, int d, float inv)
{
    int q = __float2int_rz(__int2float_rn(a) * inv);
    int r = a - q * d;
    if (r < 0) { --q; r += d; }
    if (r >= d) { ++q; }
    return q;
}

// a table in global memory, read as pairs of doubles (lets the compiler use
// global loads with a 32-bit offset rather than flat ones)
typedef const double __attribute__((address_space(1))) gdouble;

// A result that could not be computed (a state larger than its buffers):
// NaN in both parts, so no caller takes it for an amplitude.
__device__ __forceinline__ double2 nan2()
{
    return make_double2(__builtin_nan(""), __builtin_nan(""));
}

// Find the pattern owning flattened index k: largest p with off[p] <= k.
__device__ __forceinline__ int find_pattern(const int64_t *off, int B, int64_t k)
{
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `stream` and return the hipError_t of the launch.

// a2: transition tables for every gate and every sector N <= n_tab of many
// circuits at once (max_gates: largest G).
struct TableJob {
    int G, n_tab, stride;
    const double *theta, *phi;
    double2 *table;
};
hipError_t launch_build_tables_multi(int count, const TableJob *jobs, int max_gates, hipStream_t stream);

// a1: per-pattern cut bounds.
hipError_t launch_bounds(int B, int m, int D, int n, const int32_t *S, const int32_t *T,
                         const int8_t *fr_lo, const int8_t *fr_hi, const int8_t *br_lo,
                         const int8_t *br_hi, const uint8_t *cut_gate, int16_t *lo, int16_t *hi,
                         int32_t *infeasible, hipStream_t stream);

// a1/a3: per (stage slot, pattern) rank tables and state counts.
hipError_t launch_stage_tables(int B, int m, int D, int n, int nslots, const int32_t *slot_stage,
                               const uint8_t *stage_time, const int16_t *lo, const int16_t *hi,
                               const int32_t *infeasible, int32_t *C, int32_t *E, int32_t *count,
                               int32_t *overflow, hipStream_t stream);

// a3: seed a frontier (single state per pattern with value 1).
hipError_t launch_seed(int B, const int64_t *off, double2 *vec, hipStream_t stream);

// a3: one beam splitter applied to a merged frontier (forward: stage g -> g+1;
// backward: stage g+1 -> g).
struct GateArgs {
    int B, m, n, D;
    int cut;                  // beam splitter on modes (cut, cut+1)
    const uint8_t *st_tgt;    // stage_time row of the stage being produced
    const uint8_t *st_src;    // stage_time row of the stage being read
    const int16_t *lo, *hi;   // [B][(D+1)(m-1)]
    const int32_t *C_tgt;     // [B][(m-1)(n+2)]
    const int32_t *E_src;     // [B][(m-1)(n+2)]
    const int64_t *off_tgt;   // [B+1]
    const int64_t *off_src;   // [B+1]
    const double2 *W;         // this gate's table (all sectors)
    const double2 *src;
    double2 *dst;
    int64_t total_tgt;
    const int32_t *xoff;       // [8][nbx+1] per-XCD chunk prefix over patterns x, x+8, ...
    int nbx;                   // ceil(B / 8)
    int grid;                  // 8 x the longest per-XCD chunk list
};
constexpr int kGateChunk = 256;
constexpr int kXcds = 8;       // workgroup b runs on XCD b % 8 (round-robin dispatch)

// Map a workgroup to (pattern, chunk within the pattern) so that all chunks
// of pattern p run on XCD p % 8 and share that XCD's L2.  Returns false for
// workgroups past the end of their XCD's list.
__device__ __forceinline__ bool xcd_chunk(const int32_t *xoff, int nbx, int B, int block, int &p, int &chunk)
{
    const int x = block % kXcds, j = block / kXcds;
    const int32_t *xo = xoff + (size_t)x * (nbx + 1);
    if (j >= xo[nbx]) return false;
    int lo = 0, hi = nbx - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (xo[mid] <= j) lo = mid; else hi = mid - 1;
    }
    p = x + kXcds * lo;
    chunk = j - xo[lo];
    return p < B;
}
hipError_t launch_gate(const GateArgs &a, bool forward, hipStream_t stream);

// a4: depth-first enumeration of the middle beam splitters.
struct DfsArgs {
    int B, m, n, D;
    int levels;               // number of middle beam splitters
    const int4 *level_info;   // [levels]: {cut, layer, table offset, 0}
    const double2 *tab;       // compact tables of the middle gates
    int tab_len;              // entries in tab
    const int16_t *lo, *hi;
    const int32_t *E_back;    // [B][(m-1)(n+2)] rank tables of the backward stage
    const uint32_t *cfg;      // [total][cfg_words] packed cut values of each entry
    const int32_t *rank_back; // [total] rank of each entry's configuration at s_b
    int cfg_words;
    const int64_t *off_front; // [B+1]
    const int64_t *off_back;  // [B+1]
    double2 *front;           // frontier values; overwritten by value * suffix sum
    const double2 *back;      // backward frontier values
    int64_t total;            // frontier entries
    const int32_t *xoff;      // [8][nbx+1] per-XCD chunk prefix (see xcd_chunk)
    int nbx;
    unsigned long long *work_counter;   // [8] one counter per XCD list
    unsigned long long *stat_leaves;
    unsigned long long *stat_edges;
    int fp32_products;        // 1: running products in FP32
};
constexpr int kDfsChunk = 256;
constexpr int kMaxDfsGates = 16;   // splitters enumerated depth-first (LDS stack depth)
constexpr int kDfsBlock = 128;
hipError_t launch_dfs(const DfsArgs &a, int grid, hipStream_t stream);
size_t dfs_lds_bytes(const DfsArgs &a);
int dfs_blocks_per_cu(const DfsArgs &a);   // resident k_dfs blocks per CU (0: unknown)

// a3/a4: per frontier entry, its packed cut values (cfg_words words of four
// 8-bit cut values) and its rank in the backward stage's state space.
struct AnnotateArgs {
    int B, m, n, D;
    const uint8_t *st_front;
    const int16_t *lo, *hi;
    const int32_t *C_front, *E_back;
    const int64_t *off_front;
    const int32_t *xoff;
    int nbx;
    int nchunks;               // grid size (8 x the longest per-XCD list)
    int cfg_words;
    uint32_t *cfg;
    int32_t *rank_back;
};
hipError_t launch_annotate(const AnnotateArgs &a, hipStream_t stream);

// a5: per-pattern compensated reduction: sum of vec over the pattern's
// entries, or of vec[i] * back[i] when back != nullptr.
hipError_t launch_reduce(int B, const int64_t *off, const double2 *vec, const double2 *back,
                         double2 *out, hipStream_t stream);

// a6: mode-axis contraction, one splitter per step.
constexpr int kMaxActive = 16;         // live versions in a contraction state
constexpr int kMaxContractVars = 1024; // free versions in a circuit
// LDS of one key job of a split contraction (KiB): three jobs share a CU
#ifndef LOFP_SPLIT_LDS_KB
#define LOFP_SPLIT_LDS_KB 52
#endif
enum { CREF_ZERO = 0, CREF_N = 1, CREF_SPRE = 2, CREF_TPRE = 3, CREF_NEW = 4, CREF_SUM = 5 };
struct ContractStep {
    int gate;
    int n_new, n_old, n_sum;
    int new_vars[kMaxActive];     // live free versions after the step (refs first)
    int old_vars[kMaxActive];     // live free versions before the step
    int new_to_old[kMaxActive];   // position in the old layout, or -1 if introduced
    int sum_vars[2];              // versions summed out by this step
    int sum_to_old[2];            // their old position, or -1 if introduced and summed here
    int ref_kind[4], ref_arg[4];  // cut before / after the splitter, cut below, cut above
};
struct ContractArgs {
    int B, m, n, D;
    const int32_t *S;         // [m]
    const int32_t *T;         // [B][m]
    const int16_t *lo, *hi;   // [B][(D+1)(m-1)]
    const int32_t *infeasible;
    int nvars;
    const int32_t *var_cut;   // [nvars]
    const int32_t *var_time;  // [nvars] time index whose bounds apply
    int nsteps;
    const ContractStep *steps;
    const double2 *table;
    int tab_stride;
    double2 *out;             // amplitudes, or counts in .x when count_only
    int count_only;
    int fp32;                 // 1: transition products in FP32, sums in FP64
    unsigned long long *stat_transitions;
    int max_states;           // entries per state buffer
    double2 *ws;              // [B][2][max_states] when the state does not fit LDS
    int32_t *overflow;
    int stats;                // count transitions into stat_transitions
    const int32_t *skip;      // if set and nonzero: do nothing (the batch was split)
    int lds_states;           // > 0 with ws set: a pattern whose own largest state
                              // fits this many entries keeps it in LDS, others in ws
    int block;                // threads per block: 64 or 256 (0: by max_states)
};
hipError_t launch_contract(const ContractArgs &a, hipStream_t stream);

// Multi-circuit batches: one job per (request) pattern, each with its own
// circuit program, tables, S, T and bounds.
struct ContractJob {
    int m, n, D, nvars, nsteps, tab_stride, max_states, fp32;
    const ContractStep *steps;
    const int32_t *var_cut, *var_time;
    const double2 *table;
    const int32_t *S, *T;        // this job's S and T (device)
    const int16_t *lo, *hi;      // this job's bounds [(D+1)(m-1)]
    const int32_t *infeasible;   // this job's flag
    double2 *out;                // this job's amplitude
    double2 *ws;                 // 2 * max_states entries, or nullptr (state in LDS)
    double2 *state_out;          // if set: write the final state here instead of summing it
    int state_cap;               // entries available at state_out
    int stats;                   // count transitions into the statistics counter
    int out_remap;               // state_out in another variable order: the
    uint64_t out_pos;            // final state's variable q goes to place
                                 // (out_pos >> 4q) & 15
    int32_t *ovf;                // set to 1 when the job's state did not fit
                                 // its buffers (nullptr: not recorded)
};
// Per-launch overrides for key jobs of a split contraction (0 / nullptr: use
// the job's own fields): one state size for every job, and per-job slices of
// a workspace and of a state output buffer.
struct MultiOverride {
    int max_states;
    double2 *ws_base;            // job i uses ws_base + i * 2 * max_states
    double2 *state_base;         // job i writes state_base + i * state_cap
    int state_cap;
    int lds_states;              // > 0: a job whose own largest state fits this
                                 // many entries keeps it in LDS, others in ws
    const int *order;            // block b runs job order[b] (nullptr: job b)
    const int *njobs;            // if set: *njobs jobs (blocks past it do nothing)
    int *next;                   // if set: block b takes job b, then jobs
                                 // grid + (this counter, zero at launch) until
                                 // *njobs are taken; block b uses workspace slice b
};
struct BoundsJob {
    int m, D, n;
    const int32_t *S, *T;
    const int8_t *fr_lo, *fr_hi, *br_lo, *br_hi;
    const uint8_t *cut_gate;
    int16_t *lo, *hi;
    int32_t *infeasible;
};
// max_span: the largest (D+1)(m-1) over the jobs (sizes the LDS of a wave).
hipError_t launch_bounds_multi(int count, const BoundsJob *jobs, int max_span, hipStream_t stream);
// lds_bytes: dynamic LDS per block (max over jobs); max_states: max over jobs
hipError_t launch_contract_multi(int count, const ContractJob *jobs, size_t lds_bytes, int max_states,
                                 bool state_in_lds, bool fp32, unsigned long long *stat_transitions,
                                 int32_t *overflow, hipStream_t stream,
                                 MultiOverride ov = MultiOverride{0, nullptr, nullptr, 0, 0, nullptr}, bool stats = false,
                                 bool abs = false);
// Largest state over the jobs (one thread per job), atomically maxed into *mx.
hipError_t launch_multi_sizes(int count, const ContractJob *jobs, int *mx, hipStream_t stream);
// Blocks of the multi-job contraction kernel that can be resident at once on
// the current device (the grid of its job-queue form).
int contract_multi_resident_blocks(size_t lds_bytes, int max_states);
// Fills n ints with v (a kernel, so that a captured call records no memset).
hipError_t launch_fill_i32(int32_t *p, size_t n, int32_t v, hipStream_t stream);

constexpr int kKeySubs = 64;   // claim counters per half (spread the atomics)
// Grouping of a batch by the halves of T (split contraction), per half h:
// a hash table over the distinct half-rows, whose slots carry the group's
// key number and the hull of its feasible members' intervals.
struct KeyArgs {
    int B, m, n, rs, cap, span;
    int64_t stride;                // rows per half of the layout (>= cap; key_layout.h)
    const int32_t *T;              // [B][m]
    const int16_t *lo, *hi;        // per pattern [B][span]
    const int32_t *infeasible;     // [B]
    unsigned long long *table;     // [2][stride] kKeyEmpty, or the row's hash (high
                                   // 32 bits) above the group's lowest member p
                                   // (p + B if p has the wrong photon number)
    int *slot;                     // [2][B] each pattern's slot
    int *slot_key;                 // [2][stride] key number of a claimed slot
    int *key_slot;                 // [2][kKeySubs][B] claimed slots per sub-counter
    int *count;                    // [2][kKeySubs] claims per sub-counter (slot
                                   // mod kKeySubs); zeroed by the order kernel
    int *hlo, *hhi;                // [2][stride][span] int32 hull per slot
    int16_t *klo, *khi;            // per key intervals (top keys at 0, bottom at B)
    unsigned long long *counters;  // [8] zeroed by the jobs kernel
    int *job_bucket;               // [2B] cost bucket of each job
    int *order;                    // [2B] jobs by decreasing cost bucket
    // decided on the device (launches sized for the worst case, no host
    // read-back): nullptr in the host-sized form
    int *ctl;                      // [8] split?, jobs, top keys, bottom keys,
                                   // next job to take (zeroed with the jobs)
    int small_min, small_max;      // batch sizes split without shared halves
};
// Insert every pattern's two half-rows; keys are numbered as their slots are
// claimed, so their numbers (not the results) depend on thread timing.
hipError_t launch_keys(const KeyArgs &a, hipStream_t stream);
// One contraction job per key from the two half templates; jobs[0, ntop) top.
// Also the dispatch order a.order: jobs by decreasing work (the sum over the
// job's steps of state entries times summed versions), in buckets of 2^(1/8).
// Leaves the table, the slot hulls and the counts empty for the next call.
hipError_t launch_key_jobs(const KeyArgs &a, int ntop, int nbot, const ContractJob &top, const ContractJob &bot,
                           ContractJob *jobs, int32_t *kinf, hipStream_t stream);
// Empties the table, the slot hulls and the counts without making jobs.
hipError_t launch_key_reset(const KeyArgs &a, int ntop, int nbot, hipStream_t stream);
// Device-decided form of launch_key_jobs (a.ctl set): the key counts are read
// on the device, which decides whether the batch is split (halves shared by
// at most 3/4 as many keys as patterns, or a batch size in
// [small_min, small_max]) and records it in a.ctl.  Split: one job per key
// (2B waves launched), top key k writing its state at state_base + k * cap,
// bottom key k at state_base + (B + k) * cap, overflow flags at
// kinf[2B + k] and kinf[3B + k]; then the dispatch order.  Not split: the
// slots are emptied.  Either way the table, hulls and counts are left empty.
hipError_t launch_key_jobs_dev(const KeyArgs &a, const ContractJob &top, const ContractJob &bot, ContractJob *jobs,
                               int32_t *kinf, double2 *state_base, int state_cap, hipStream_t stream);
struct JoinArgs {
    int B, m, n, D;
    const int16_t *lo, *hi;          // per pattern [B][span]
    const int32_t *infeasible;
    const int32_t *slot;             // [2][B] each pattern's slot per half
    const int32_t *slot_key;         // [2][stride] key number of each slot
    int64_t stride;                  // rows per half of the slot layout
    const int16_t *tlo, *thi;        // per top key [ntop][span]
    const int16_t *blo, *bhi;        // per bottom key [nbot][span]
    int nshared;
    int cidx[kMaxActive];            // interval index (time * (m-1) + cut) of each
                                     // crossing variable, in the top state's order;
                                     // both states are laid out in that order
    const double2 *top_state, *bot_state;
    int state_cap;
    const int32_t *top_ovf, *bot_ovf; // per key: its job's state did not fit
    const int32_t *split_flag;        // if set and zero: the batch was not split
    double2 *out;
};
hipError_t launch_join(const JoinArgs &a, hipStream_t stream);
size_t contract_job_lds_bytes(int nvars, int m, int max_states, bool state_in_lds);
// State entries per buffer that fit in 64 KiB of LDS beside a job's fixed
// LDS (the per-pattern choice of LDS or workspace uses it).
inline int contract_lds_room(int nvars, int m)
{
    const size_t fixed = contract_job_lds_bytes(nvars, m, 0, true), cap = 64 * 1024;
    return fixed < cap ? (int)((cap - fixed) / (2 * sizeof(double2))) : 0;
}
// LDS a block may allocate on the current device (64 KiB if the query fails)
size_t max_lds_per_block();
// Threads per contraction block for a largest state of max_states entries:
// one wave for small states (more patterns resident), four for large.
inline int contract_block_size(int max_states) { return max_states <= 512 ? 64 : 256; }
hipError_t launch_contract_sizes(const ContractArgs &a, int *max_size, hipStream_t stream);
// dynamic LDS of the contraction kernel (state buffers included when in LDS)
size_t contract_lds_bytes(const ContractArgs &a, bool state_in_lds);

}  // namespace lofp
