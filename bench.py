"""Benchmark: exact amplitudes <T|U_P|S> for a batch of output patterns.

Workload (default): m=16 modes, n=8 photons in the even modes, depth-8
brickwork of nearest-neighbour beam splitters (theta ~ U(0, pi/2), phi ~
U(0, 2 pi), seed 0), 4096 collision-free output patterns with every sorted
output mode within distance 8 of its sorted input mode.  One step = one call
of the library on the whole batch with inputs resident in HBM; the library
picks the form (mode-axis contraction when its state fits, as the paper does
for depth > 2, else merged frontiers + depth-first path enumeration); both
forms are reported, each with the roofline of its dominant kernel.

Prints one JSON line.  `value` is represented valid paths per second: the
number of conservation-valid paths of Eq. (1) summed over the batch (counted
exactly by the contraction in the counting semiring, outside the timed
region), divided by the time per step.  Amplitudes/s and the evaluated
leaves/edges per second are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector, dense
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--method", default="auto", choices=["auto", "pathsum", "contract"])
    ap.add_argument("--fwd-layer", type=int, default=-1)
    ap.add_argument("--bwd-layer", type=int, default=-1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=15.0)
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the path would shard patterns "
                                   "or frontier subtrees across GPUs, which is not built here",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2510_26408_amd import lofp, workloads

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    wl = workloads.make(args.config, seed=0)
    circ = lofp.Circuit(wl.m, wl.layers)
    method = {"auto": lofp.METHOD_AUTO, "pathsum": lofp.METHOD_PATHSUM, "contract": lofp.METHOD_CONTRACT}[args.method]
    T = torch.from_numpy(wl.Ts).to(dev)
    out = torch.zeros(wl.batch, dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream(dev)

    # represented paths (exact counts, outside the timed region)
    counts = circ.path_counts(wl.S, wl.Ts)
    paths_per_step = float(counts.sum())

    eager_ms, per_step, s_work, amps = measure(lofp, circ, wl, T, out, stream, method, args.fwd_layer,
                                               args.bwd_layer, args.steps, args.warmup)
    # the production form: the call tuned once and captured as a graph, each
    # step one replay of the whole call (contraction only; the path sum sizes
    # its frontiers on the host)
    graph = None
    if method != lofp.METHOD_PATHSUM and s_work["method_used"] == lofp.METHOD_CONTRACT:
        graph = measure_graph(lofp, circ, wl, T, out, stream, args.steps, args.warmup)
    ms = graph["ms_per_step"] if graph else eager_ms
    if graph:
        amps = graph["produced"]

    # parity on a sample (oracle = plain definition, CPU)
    import oracle

    idx = np.random.default_rng(1).choice(wl.batch, min(64, wl.batch), replace=False)
    ref, _ = oracle.amplitudes(wl.m, wl.S, wl.Ts[idx], wl.flat_circuit(), nthreads=host_threads())
    max_err = float(np.abs(amps[idx] - ref).max())

    s0 = s_work
    avg = lambda k: float(np.mean([s[k] for s in per_step]))
    leaves, edges = s0["dfs_leaves"], s0["dfs_edges"]
    res = {
        "metric": "paths/s & amplitudes/s at <=1e-12 err vs FP64 oracle; p50/p99 amplitude latency",
        "value": paths_per_step / (ms * 1e-3),
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.note, "name": wl.name, "m": wl.m, "n": wl.n, "depth": wl.depth,
                   "batch": wl.batch, "method": args.method, "fwd_layer": s0["fwd_layer"],
                   "bwd_layer": s0["bwd_layer"], "parallelism": "single-gpu"},
        "amplitudes_per_s": wl.batch / (ms * 1e-3),
        "represented_paths_per_step": paths_per_step,
        "max_abs_err_vs_oracle_sample64": max_err,
        "phases_ms": {k: avg(k) for k in ("ms_plan", "ms_forward", "ms_backward", "ms_dfs", "ms_reduce",
                                          "ms_contract", "ms_total")},
        "frontier_states": s0["frontier_states"],
        "backward_states": s0["backward_states"],
        "bfs_states": s0["bfs_states"],
        "dfs_levels": s0["dfs_levels"],
        "dfs_leaves_per_step": leaves,
        "dfs_edges_per_step": edges,
        "eager_ms_per_step": eager_ms,
    }
    if graph:
        res["config"]["form"] = "graph replay of the tuned call"
        res["graph"] = {k: v for k, v in graph.items() if k != "produced"}
    else:
        res["config"]["form"] = "eager call"

    # roofline of the dominant kernel, from HIP events on the launch stream
    used = s0["method_used"]
    res["config"]["method_used"] = "contract" if used == lofp.METHOD_CONTRACT else "pathsum"
    if used == lofp.METHOD_CONTRACT:
        kname = "k_contract_multi" if s0["split_top_keys"] > 0 else "k_contract"
        res["roofline"] = contract_roofline(kname, avg("ms_contract"), s0["transitions"], args.config)
        res["split_keys"] = [s0["split_top_keys"], s0["split_bottom_keys"]]
        res["max_state"] = s0["max_state"]
        # evaluated work beside the represented paths: transitions per second
        # of the whole step and of the contraction kernel
        res["transitions_per_step"] = s0["transitions"]
        res["transitions_per_s"] = s0["transitions"] / (ms * 1e-3)
    else:
        res["roofline"] = pathsum_roofline(s0, avg, args.config)
        res["leaves_per_s"] = leaves / (ms * 1e-3)
        res["edges_per_s"] = edges / (ms * 1e-3)
    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib * (1 << 20)
        xa = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        xb = torch.empty_like(xa)
        xb.copy_(xa)
        torch.cuda.synchronize()
        res["calib_copy_bytes"] = nb
        del xa, xb

    if not args.no_latency:
        res["latency_single_ms"] = single_latency(circ, wl, T, out, method, stream, torch, lofp)
        if graph:
            res["latency_single_graph_ms"] = single_latency_graph(circ, wl, T, stream, torch, lofp)
    if not args.no_variants:
        res["variants"] = variants(lofp, workloads, torch, dev, stream)

    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(oracle, wl, paths_per_step, args.cpu_budget_s)
    print(json.dumps(res), flush=True)


def single_latency(circ, wl, T, out, method, stream, torch, lofp):
    """Latency of one-pattern calls of the same form (p50/p99 over 50)."""
    lat = []
    o1 = out[:1]
    for i in range(60):
        torch.cuda.synchronize()
        a = time.perf_counter()
        circ.amplitudes_device(wl.S, T[i:i + 1].contiguous(), o1, lofp.make_opts(method=method), stream=stream)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat[10:])
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}


def single_latency_graph(circ, wl, T, stream, torch, lofp):
    """Latency of one pattern through a captured call (p50/p99 over 50
    replays, new pattern copied into the captured buffer each time)."""
    T1 = T[:1].clone()
    o1 = torch.zeros(1, dtype=torch.complex128, device=T.device)
    g = lofp.Graph(circ, wl.S, T1, o1, lofp.make_opts(method=lofp.METHOD_CONTRACT))
    lat = []
    try:
        for i in range(60):
            T1.copy_(T[i:i + 1])
            torch.cuda.synchronize()
            a = time.perf_counter()
            g.launch(stream)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - a) * 1e3)
    finally:
        g.close()
    lat = np.array(lat[10:])
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}


def measure_graph(lofp, circ, wl, T, out, stream, steps, warmup):
    """The tuned call captured as a graph: `steps` replays timed after
    `warmup`; the tuned choice and the eager tuned call's time beside it."""
    import torch

    opts = lofp.make_opts(method=lofp.METHOD_CONTRACT, autotune=True)
    st = lofp.Stats()
    circ.amplitudes_device(wl.S, T, out, opts, stream=stream, stats=st)   # tunes (first call)
    for _ in range(warmup):
        circ.amplitudes_device(wl.S, T, out, opts, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        circ.amplitudes_device(wl.S, T, out, opts, stream=stream)
    torch.cuda.synchronize()
    eager_tuned = (time.perf_counter() - t0) * 1e3 / steps
    timed = lofp.make_opts(method=lofp.METHOD_CONTRACT, autotune=True, record_timing=True)
    st = lofp.Stats()
    circ.amplitudes_device(wl.S, T, out, timed, stream=stream, stats=st)
    g = lofp.Graph(circ, wl.S, T, out, opts)
    try:
        for _ in range(warmup):
            g.launch(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.launch(stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        produced = out.cpu().numpy()
    finally:
        g.close()
    return {"ms_per_step": ms, "eager_tuned_ms_per_step": eager_tuned, "tuned_split_cut": st.split_cut,
            "tuned_lds_kb": st.lds_kb, "tuned_split": bool(st.split_top_keys > 0),
            "tuned_phases_ms": {"ms_plan": st.ms_plan, "ms_contract": st.ms_contract, "ms_join": st.ms_reduce},
            "produced": produced}


def traffic_for(kernel: str, key: str):
    """HBM bytes per launch (or per step, where the record says so) from the
    committed rocprofv3 counter summary of `kernel` on workload `key`, or None
    when there is no record for that workload or the kernel's source changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))[kernel]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("key") != key or hashlib.sha256(src).hexdigest()[:16] != rec["source_sha16"]:
        return None
    return rec.get("bytes_per_launch", rec.get("bytes_per_step"))


def contract_roofline(kernel, ms_k, transitions, key):
    # one complex FP64 multiply-add (8 flops) per state transition
    flops = 8.0 * transitions
    achieved = flops / (ms_k * 1e-3) / 1e12 if ms_k > 0 else 0.0
    return {"kernel": kernel, "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic_for(kernel, key),
            "avg_ms": ms_k, "algorithmic": "8 FP64 flops (complex multiply-add) per contraction transition "
                                           "with a nonzero source"}


def dfs_roofline(s0, avg, key):
    ms_dfs = avg("ms_dfs")
    flops = 6.0 * s0["dfs_edges"] + 8.0 * s0["dfs_leaves"]
    achieved = flops / (ms_dfs * 1e-3) / 1e12 if ms_dfs > 0 else 0.0
    return {"kernel": "k_dfs", "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": traffic_for("k_dfs", key), "avg_ms": ms_dfs,
            "algorithmic": "6 FP64 flops per tree edge (complex product) + 8 per leaf"}


def pathsum_roofline(s0, avg, name):
    ms_dfs, ms_fwd = avg("ms_dfs"), avg("ms_forward")
    key = f"{name}/pathsum/{s0['fwd_layer']}-{s0['bwd_layer']}"
    if ms_dfs >= ms_fwd and ms_dfs > 0:
        return dfs_roofline(s0, avg, key)
    # forward frontier: per produced state one 16 B write plus one 16 B read of
    # each predecessor (counted once: 32 B per state)
    byts = 32.0 * s0["bfs_states"]
    achieved = byts / (ms_fwd * 1e-3) / 1e9 if ms_fwd > 0 else 0.0
    return {"kernel": "k_gate (forward)", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for("k_gate", key), "avg_ms": ms_fwd,
            "algorithmic": "32 B per frontier state (one 16 B write, one 16 B read); achieved and traffic are "
                           "per step (all forward launches of one call)"}


def measure(lofp, circ, wl, T, out, stream, method, fwd, bwd, steps, warmup):
    """Time `steps` production calls (no statistics, no event timing) after
    `warmup`, then a few calls with HIP-event phase timing (the same kernels),
    then one call that counts the work done (its kernels carry counters and
    run slower; only its counts are used)."""
    import torch

    opts = lofp.make_opts(method=method, fwd_layer=fwd, bwd_layer=bwd)
    for _ in range(warmup):
        circ.amplitudes_device(wl.S, T, out, opts, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        circ.amplitudes_device(wl.S, T, out, opts, stream=stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    produced = out.cpu().numpy()   # the timed calls' output, for the parity check
    timed = lofp.make_opts(method=method, fwd_layer=fwd, bwd_layer=bwd, record_timing=True)
    per_step = []
    for _ in range(max(3, min(steps, 10))):
        st = lofp.Stats()
        circ.amplitudes_device(wl.S, T, out, timed, stream=stream, stats=st)
        per_step.append(st.as_dict())
    work = lofp.make_opts(method=method, fwd_layer=fwd, bwd_layer=bwd, count_work=True)
    st = lofp.Stats()
    circ.amplitudes_device(wl.S, T, out, work, stream=stream, stats=st)
    return ms, per_step, st.as_dict(), produced


def run_variant(lofp, workloads, torch, dev, stream, name, method, steps=5, fwd=-1, bwd=-1):
    wl = workloads.make(name, seed=0)
    circ = lofp.Circuit(wl.m, wl.layers)
    T = torch.from_numpy(wl.Ts).to(dev)
    o = torch.zeros(wl.batch, dtype=torch.complex128, device=dev)
    ms, sts, s0, produced = measure(lofp, circ, wl, T, o, stream, method, fwd, bwd, steps, 2)
    paths = float(circ.path_counts(wl.S, wl.Ts).sum())
    import oracle
    idx = np.random.default_rng(2).choice(wl.batch, min(64, wl.batch), replace=False)
    ref, _ = oracle.amplitudes(wl.m, wl.S, wl.Ts[idx], wl.flat_circuit(), nthreads=host_threads())
    avg = lambda k: float(np.mean([s[k] for s in sts]))
    out = {"workload": wl.note, "batch": wl.batch, "ms_per_step": ms, "amplitudes_per_s": wl.batch / (ms * 1e-3),
           "paths_per_s": paths / (ms * 1e-3),
           "max_abs_err_vs_oracle_sample": float(np.abs(produced[idx] - ref).max()),
           "phases_ms": {k: avg(k) for k in ("ms_plan", "ms_forward", "ms_backward", "ms_dfs", "ms_reduce",
                                             "ms_contract", "ms_total")}}
    if method == lofp.METHOD_CONTRACT:
        out["transitions"] = s0["transitions"]
        out["transitions_per_s"] = s0["transitions"] / (ms * 1e-3)
        kname = "k_contract_multi" if s0["split_top_keys"] > 0 else "k_contract"
        out["roofline"] = contract_roofline(kname, avg("ms_contract"), s0["transitions"], name)
    else:
        out.update({k: s0[k] for k in ("fwd_layer", "bwd_layer", "dfs_levels", "frontier_states",
                                        "backward_states", "bfs_states", "dfs_leaves", "dfs_edges")})
        out["leaves_per_s"] = s0["dfs_leaves"] / (ms * 1e-3)
        out["edges_per_s"] = s0["dfs_edges"] / (ms * 1e-3)
        out["bfs_states_per_s"] = s0["bfs_states"] / (ms * 1e-3)
        out["roofline"] = pathsum_roofline(s0, avg, name)
        if s0["dfs_levels"] > 0:
            # the depth-first kernel beside the dominant one
            out["roofline_dfs"] = dfs_roofline(s0, avg, f"{name}/pathsum/{s0['fwd_layer']}-{s0['bwd_layer']}")
    return out


def variants(lofp, workloads, torch, dev, stream):
    """The path-sum forms on the same batch, the contraction on the small
    single-pattern, the bunched and the m=32, n=16 workloads, and the served
    mixed-request workload."""
    return {"pathsum_c2": run_variant(lofp, workloads, torch, dev, stream, "c2", lofp.METHOD_PATHSUM, steps=3),
            "pathsum_dfs_c2": run_variant(lofp, workloads, torch, dev, stream, "c2", lofp.METHOD_PATHSUM, steps=2,
                                          fwd=5, bwd=6),
            "contract_c1": run_variant(lofp, workloads, torch, dev, stream, "c1", lofp.METHOD_CONTRACT, steps=50),
            "contract_c3": run_variant(lofp, workloads, torch, dev, stream, "c3", lofp.METHOD_CONTRACT, steps=20),
            "contract_c5": run_variant(lofp, workloads, torch, dev, stream, "c5", lofp.METHOD_CONTRACT, steps=20),
            "contract_c5_multi": c5_multi_variant(lofp, workloads, torch),
            "served_c4": serve_variant(lofp, workloads)}


def c5_multi_variant(lofp, workloads, torch, R=64, steps=5):
    """The 32-mode, depth-6 workload as R independent circuits (seeds 0..R-1)
    x 512 patterns each, all in one multi-circuit launch (one contraction job
    per pattern, every job with its own circuit's tables): the device time of
    that launch from HIP events, and its FP64 rate from the transitions the
    same jobs make (counted by single-circuit calls of the per-pattern
    contraction, 32 patterns at a time)."""
    wls = [workloads.make("c5", seed=r) for r in range(R)]
    circs = [lofp.Circuit(w.m, w.layers) for w in wls]
    items = [(c, w.S, T) for c, w in zip(circs, wls) for T in w.Ts]
    lofp.amplitudes_multi(items[:64])   # set-up of every circuit's tables is not timed below
    lofp.amplitudes_multi(items)
    ms = []
    for _ in range(steps):
        st = lofp.Stats()
        lofp.amplitudes_multi(items, lofp.make_opts(record_timing=True), st)
        ms.append(st.ms_contract)
    ms_k = float(np.median(ms))
    trans = 0
    for c, w in zip(circs[:8], wls[:8]):
        for i in range(0, w.batch, 32):
            st = lofp.Stats()
            c.amplitudes(w.S, w.Ts[i:i + 32], lofp.make_opts(method=lofp.METHOD_CONTRACT, count_work=True), st)
            trans += st.transitions
    trans_all = trans * R / 8.0   # counted on 8 of the R circuits, scaled
    rl = contract_roofline("k_contract_multi", ms_k, trans_all, "c5x64")
    rl["kernel"] = "k_contract_multi (multi-circuit)"
    return {"circuits": R, "patterns_per_circuit": wls[0].batch, "jobs": len(items), "device_ms": ms_k,
            "amplitudes_per_s": len(items) / (ms_k * 1e-3), "transitions_est": trans_all,
            "transitions_counted_on_circuits": 8, "roofline": rl}


def _serve(lofp, reqs, circs, precision, rate_hz=0.0, n_warm=0):
    """Serve reqs (saturated when rate_hz == 0, else at their Poisson arrival
    times); returns (amplitudes, bounds, latencies after warm-up, wall s, stats)."""
    srv = lofp.Server(max_batch=512, streams=3, precision=precision)
    try:
        t0 = time.perf_counter()
        tk = []
        for c, r in zip(circs, reqs):
            if rate_hz > 0:
                delay = r.arrival_s - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
            tk.append(srv.submit(c, r.S, r.T))
        res = [srv.result(t) for t in tk]
        wall = time.perf_counter() - t0
        st = srv.stats()
    finally:
        srv.close()
    amps = np.array([a for a, _, _ in res])
    bounds = np.array([b for _, _, b in res])
    lats = np.array([l for _, l, _ in res][n_warm:])
    return amps, bounds, lats, wall, st


def serve_variant(lofp, workloads, n_req=10000, n_warm=1000, rate_fracs=(0.25, 0.5, 0.75), repeats=3):
    """Served mixed requests: m in {12,16,24}, n=m/2, depth in {4,6,8}, a fresh
    circuit and pattern per request.  The FP64 form, and the FP32-product form
    (FP64 sums) with its per-result bound, a result whose bound exceeds
    1e-6 |amp| recomputed in FP64.  First the saturated throughput (everything
    submitted at once), then Poisson arrivals at fractions of it; p50/p99 from
    submit to completion, after the warm-up requests."""
    reqs = workloads.served_requests(n_req + n_warm, rate_hz=1.0, seed=7)
    circs = [lofp.Circuit(r.m, r.layers) for r in reqs]
    out = {"requests": n_req, "warmup": n_warm}
    # complex128 reference (multi-circuit batch, same library)
    f64 = lofp.amplitudes_multi([(c, r.S, r.T) for c, r in zip(circs, reqs)])
    nz = np.abs(f64) > 1e-14
    # unchecked FP32 products: the observed error and the a-priori bound
    raw, raw_b = lofp.amplitudes_multi([(c, r.S, r.T) for c, r in zip(circs, reqs)],
                                       lofp.make_opts(precision=lofp.PREC_FP32, fp32_rtol=1e300), bounds=True)
    rel_raw = np.abs(raw - f64)[nz] / np.abs(f64)[nz]
    ratio = raw_b[nz] / np.abs(f64)[nz]
    out["fp32_unchecked"] = {"max_rel_err_vs_c128": float(rel_raw.max()),
                             "median_rel_err_vs_c128": float(np.median(rel_raw)),
                             "median_bound_over_amp": float(np.median(ratio)),
                             "certifiable_at_1e-6": float((ratio <= 1e-6).mean())}
    seed = 8
    for name, prec, fracs in (("fp64", lofp.PREC_FP64, rate_fracs), ("fp32_checked", lofp.PREC_FP32, (0.5,))):
        # saturated: submit all at once (fresh circuits: the set-up is served too)
        circs_s = [lofp.Circuit(r.m, r.layers) for r in reqs]
        amps, bounds, _, wall, st = _serve(lofp, reqs, circs_s, prec)
        sat = len(reqs) / wall
        rel = float((np.abs(amps - f64)[nz] / np.abs(f64)[nz]).max()) if nz.any() else 0.0
        rec = {"precision": "fp32 products, fp64 sums, fp64 re-run above 1e-6 |amp|" if prec == lofp.PREC_FP32
               else "fp64", "saturated_amplitudes_per_s": sat, "max_rel_err_vs_c128": rel, "poisson": []}
        if prec == lofp.PREC_FP32:
            rec["fp64_fallback_fraction"] = st["fp64_fallbacks"] / len(reqs)
            rec["max_bound_over_amp"] = float((bounds[nz] / np.abs(amps[nz])).max())
        for frac in fracs:
            # Poisson arrivals at frac * saturated (fresh circuits, a new seed
            # per repeat); p50/p99 of each repeat and their medians, since
            # the tail moves with host thread scheduling from run to run
            rate = frac * sat
            reps = []
            for _ in range(repeats):
                reqs2 = workloads.served_requests(n_req + n_warm, rate_hz=rate, seed=seed)
                seed += 1
                circs2 = [lofp.Circuit(r.m, r.layers) for r in reqs2]
                _, _, lats, wall2, st2 = _serve(lofp, reqs2, circs2, prec, rate_hz=rate, n_warm=n_warm)
                reps.append({"offered_amplitudes_per_s": (n_req + n_warm) / wall2,
                             "p50_ms": float(np.percentile(lats, 50)), "p99_ms": float(np.percentile(lats, 99)),
                             "mean_batch": st2["mean_batch"], "launches": st2["launches"]})
            rec["poisson"].append({"rate_fraction": frac, "rate_hz": rate, "repeats": repeats,
                                   "p50_ms": float(np.median([r["p50_ms"] for r in reps])),
                                   "p99_ms": float(np.median([r["p99_ms"] for r in reps])),
                                   "p99_ms_range": [min(r["p99_ms"] for r in reps), max(r["p99_ms"] for r in reps)],
                                   "runs": reps})
        out[name] = rec
    return out


def host_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return os.cpu_count() or 1


def cpu_baseline(oracle, wl, paths_per_step, budget_s):
    """The oracle (Ryser on the composed unitary, long double) on the host's
    cores, over repeated passes of the batch until about `budget_s`."""
    threads = host_threads()
    circ = wl.flat_circuit()
    # size the sample from a short probe
    probe = min(wl.batch, 256)
    t0 = time.perf_counter()
    _, used = oracle.amplitudes(wl.m, wl.S, wl.Ts[:probe], circ, nthreads=threads)
    dt = time.perf_counter() - t0
    per_pat = dt / probe
    n_pat = int(min(wl.batch * 20000, max(probe, budget_s / max(per_pat, 1e-9))))
    reps, rem = divmod(n_pat, wl.batch)
    t0 = time.perf_counter()
    done = 0
    for _ in range(reps):
        oracle.amplitudes(wl.m, wl.S, wl.Ts, circ, nthreads=threads)
        done += wl.batch
    if rem:
        oracle.amplitudes(wl.m, wl.S, wl.Ts[:rem], circ, nthreads=threads)
        done += rem
    el = time.perf_counter() - t0
    amps_per_s = done / el
    return {"value": amps_per_s * paths_per_step / wl.batch, "unit": "paths/s", "cores": used, "kind": "oracle",
            "amplitudes_per_s": amps_per_s, "seconds": el,
            "sample": f"{done} pattern evaluations ({reps} full passes of the {wl.batch}-pattern batch + {rem}) "
                      f"by Ryser's formula on the composed unitary, OpenMP over patterns"}


if __name__ == "__main__":
    main()
