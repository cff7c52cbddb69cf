"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Tolerance (see check()): every amplitude within 1e-12 absolute of the oracle
(the stated target) and, where the oracle's values come with its own rounding
bound eb (Ryser's a-posteriori bound), also within 1e-9 |A| + 1e3 eb: nine
significant digits wherever the oracle itself resolves them, so a result of
zero (or a wrong digit) fails for every amplitude the oracle vouches for,
however small.  Measured on the benchmark workloads the GPU stays two orders
of magnitude inside both terms (largest relative error 4e-12 where
eb <= 1e-9 |A|; largest |error| / eb 0.07)."""
import math

import numpy as np
import pytest

import oracle
from paper_2510_26408_amd import lofp, workloads

pytestmark = pytest.mark.gpu
ATOL = 1e-12
RTOL = 1e-9          # relative agreement where the oracle resolves the amplitude
EB_FACTOR = 1e3      # slack in units of the oracle's own rounding bound
# one contraction per pattern: the reference the split contraction is checked against
NEVER_SPLIT = lofp.make_opts(method=lofp.METHOD_CONTRACT, split=lofp.SPLIT_NEVER)


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(autouse=True)
def gpu_only():
    _need_gpu()


def flat(layers):
    return [bs for l in layers for bs in l]


class Want(np.ndarray):
    """Oracle amplitudes carrying the oracle's rounding bound of each entry
    (``.eb``, same shape); indexing keeps the two aligned."""

    def __new__(cls, amps, eb):
        obj = np.asarray(amps).view(cls)
        obj.eb = np.asarray(eb, dtype=np.float64)
        return obj

    def __array_finalize__(self, obj):
        self.eb = getattr(obj, "eb", None)

    def __getitem__(self, k):
        r = super().__getitem__(k)
        if isinstance(r, Want) and self.eb is not None:
            r.eb = self.eb[k]
        return r


def check(got, want, atol=ATOL):
    eb = getattr(want, "eb", None)
    got, want = np.asarray(got), np.asarray(want)
    err = np.abs(got - want)
    assert err.max() <= atol, (err.max(), int(err.argmax()))
    if eb is not None and eb.shape == want.shape:
        lim = RTOL * np.abs(want) + EB_FACTOR * eb
        bad = np.flatnonzero(err.ravel() > lim.ravel())
        assert bad.size == 0, ("relative", int(bad[0]), float(err.ravel()[bad[0]]), float(np.abs(want).ravel()[bad[0]]),
                               float(eb.ravel()[bad[0]]))


def oracle_amps(wl_m, S, Ts, layers):
    amps, eb, _ = oracle.amplitudes(wl_m, S, Ts, flat(layers), nthreads=8, with_bound=True)
    return Want(amps, eb)


# ------------------------------------------------------------------ tables
def test_tables_match_oracle():
    wl = workloads.make("c1", seed=3)
    c = lofp.Circuit(wl.m, wl.layers)
    gates = flat(wl.layers)
    for g in (0, 5, len(gates) - 1):
        _, _, th, ph = gates[g]
        for N in range(0, 9):
            got = c.bs_table(g, N)                  # [x1, y1]
            want = oracle.bs_sector(th, ph, N).T    # oracle is [y1, x1]
            check(got, want, 1e-14 * max(1, N))


@pytest.mark.parametrize("N", [12, 24, 36, 48, 64])
def test_tables_at_high_photon_number(N):
    """Sectors up to the 64-photon limit against the closed-form sum in 40
    digits (the FP64 closed form would be off by 1e-11 at N = 40 and by 1e-8
    at N = 64; the recurrence the tables use stays near 1e-14)."""
    pytest.importorskip("mpmath")
    c = lofp.Circuit(2, [[(0, 1, 0.91, 2.2)], [(0, 1, 0.35, -1.3)]])
    for g, (th, ph) in enumerate(((0.91, 2.2), (0.35, -1.3))):
        got = c.bs_table(g, N)                      # [x1, y1]
        want = oracle.bs_sector_hp(th, ph, N).T     # [x1, y1]
        check(got, want, 2e-15 * (N + 1))


def test_table_special_angles():
    layers = [[(0, 1, 0.0, 1.0)], [(0, 1, math.pi / 2, 0.4)], [(0, 1, math.pi / 4, 2.0)]]
    c = lofp.Circuit(2, layers)
    for N in range(0, 7):
        assert np.array_equal(c.bs_table(0, N), np.eye(N + 1))
        check(c.bs_table(1, N), oracle.bs_sector(math.pi / 2, 0.4, N).T, 1e-13)
    assert abs(c.bs_table(2, 2)[1, 1]) < 1e-15   # Hong-Ou-Mandel


# ---------------------------------------------------------- small circuits
@pytest.mark.parametrize("method", [lofp.METHOD_PATHSUM, lofp.METHOD_CONTRACT])
def test_paper_correctness_protocol(method):
    """Sec. III.A: 6-mode inputs at depths 3..6, every output; probabilities sum
    to 1 and agree with the oracle."""
    cases = [((1, 1, 1, 1, 1, 1), 3), ((0, 0, 4, 0, 0, 4), 4), ((2, 0, 3, 0, 0, 3), 5), ((2, 0, 0, 2, 0, 2), 6)]
    for k, (S, D) in enumerate(cases):
        layers = workloads.random_brickwork(6, D, np.random.Generator(np.random.PCG64(40 + k)))
        pats = np.array(oracle.all_patterns(6, sum(S)), dtype=np.int32)
        c = lofp.Circuit(6, layers)
        got = c.amplitudes(S, pats, lofp.make_opts(method=method))
        want = oracle_amps(6, np.array(S), pats, layers)
        check(got, want)
        assert abs(np.sum(np.abs(got) ** 2) - 1) < 1e-12
        tvd = 0.5 * np.abs(np.abs(got) ** 2 - np.abs(want) ** 2).sum()
        assert tvd < 1e-13


@pytest.mark.parametrize("fl,bl", [(0, 0), (0, 4), (1, 2), (2, 2), (1, 3), (0, 1), (4, 4), (3, 4)])
def test_c1_all_patterns_every_cut(fl, bl):
    wl = workloads.make("c1", seed=0)
    pats = np.array(oracle.all_patterns(wl.m, wl.n), dtype=np.int32)
    c = lofp.Circuit(wl.m, wl.layers)
    st = lofp.Stats()
    got = c.amplitudes(wl.S, pats, lofp.make_opts(method=lofp.METHOD_PATHSUM, fwd_layer=fl, bwd_layer=bl), st)
    check(got, oracle_amps(wl.m, wl.S, pats, wl.layers))
    assert st.fwd_layer == fl and st.bwd_layer == bl


@pytest.mark.parametrize("D", [0, 1, 2, 3])
def test_shallow_and_empty_circuits(D):
    m = 6
    layers = workloads.random_brickwork(m, D, np.random.Generator(np.random.PCG64(7 + D)))
    S = np.array([1, 0, 2, 0, 1, 0], dtype=np.int32)
    pats = np.array(oracle.all_patterns(m, 4), dtype=np.int32)
    c = lofp.Circuit(m, layers)
    for method in (lofp.METHOD_PATHSUM, lofp.METHOD_CONTRACT):
        got = c.amplitudes(S, pats, lofp.make_opts(method=method))
        if D == 0:
            want = np.array([1.0 if np.array_equal(T, S) else 0.0 for T in pats])
        else:
            want = oracle_amps(m, S, pats, layers)
        check(got, want)


def test_exact_zero_for_infeasible_and_nonconserving():
    wl = workloads.make("c1", seed=0)
    c = lofp.Circuit(wl.m, wl.layers)
    T_far = np.zeros(wl.m, dtype=np.int32)
    T_far[4:8] = 1                       # four photons must all move by 4 in depth 4: impossible
    T_more = wl.Ts[0].copy()
    T_more[0] += 1
    for method in (lofp.METHOD_PATHSUM, lofp.METHOD_CONTRACT):
        got = c.amplitudes(wl.S, np.stack([T_far, T_more]), lofp.make_opts(method=method))
        assert got[0] == 0 and got[1] == 0


def test_single_photon_and_bunched():
    m, D = 7, 5
    layers = workloads.random_brickwork(m, D, np.random.Generator(np.random.PCG64(11)))
    U = oracle.compose(m, flat(layers))
    c = lofp.Circuit(m, layers)
    for s in range(m):
        S = np.eye(m, dtype=np.int32)[s]
        got = c.amplitudes(S, np.eye(m, dtype=np.int32))
        check(got, U[:, s])
    S = np.zeros(m, dtype=np.int32)
    S[3] = 5
    pats = np.array(oracle.all_patterns(m, 5), dtype=np.int32)
    for method in (lofp.METHOD_PATHSUM, lofp.METHOD_CONTRACT):
        check(c.amplitudes(S, pats, lofp.make_opts(method=method)), oracle_amps(m, S, pats, layers))


def test_empty_batch():
    wl = workloads.make("c1", seed=0)
    c = lofp.Circuit(wl.m, wl.layers)
    assert c.amplitudes(wl.S, np.zeros((0, wl.m), dtype=np.int32)).shape == (0,)


# ----------------------------------------------------- workload-shaped cases
@pytest.mark.parametrize("name,batch", [("c2", 24), ("c3", 48)])
def test_workloads_pathsum_and_contract(name, batch):
    wl = workloads.make(name, seed=1, batch=batch)
    c = lofp.Circuit(wl.m, wl.layers)
    want = oracle_amps(wl.m, wl.S, wl.Ts, wl.layers)
    for opts in (lofp.make_opts(method=lofp.METHOD_PATHSUM),
                 lofp.make_opts(method=lofp.METHOD_PATHSUM, fwd_layer=wl.depth - 4, bwd_layer=wl.depth - 2),
                 lofp.make_opts(method=lofp.METHOD_CONTRACT)):
        check(c.amplitudes(wl.S, wl.Ts, opts), want)


def test_c5_contraction():
    wl = workloads.make("c5", seed=1, batch=32)
    c = lofp.Circuit(wl.m, wl.layers)
    want = oracle_amps(wl.m, wl.S, wl.Ts, wl.layers)
    got = c.amplitudes(wl.S, wl.Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT))
    check(got, want)


def test_c2_full_batch_sampled():
    """Full 4096-pattern batch in the launch configuration the benchmark
    times; 64 sampled patterns checked against the oracle."""
    import torch
    wl = workloads.make("c2", seed=0)
    c = lofp.Circuit(wl.m, wl.layers)
    T = torch.from_numpy(wl.Ts).cuda()
    out = torch.zeros(wl.batch, dtype=torch.complex128, device="cuda")
    st = lofp.Stats()
    c.amplitudes_device(wl.S, T, out, lofp.make_opts(method=lofp.METHOD_PATHSUM, fwd_layer=5, bwd_layer=6), stats=st)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    idx = np.random.default_rng(0).choice(wl.batch, 64, replace=False)
    check(got[idx], oracle_amps(wl.m, wl.S, wl.Ts[idx], wl.layers))
    assert st.dfs_leaves > 0


# ------------------------------------------------------------ path counts
def test_path_counts_match_enumeration():
    for (m, D, S) in [(5, 4, (1, 0, 1, 0, 1)), (6, 5, (2, 0, 1, 0, 1, 0))]:
        layers = workloads.random_brickwork(m, D, np.random.Generator(np.random.PCG64(m + D)))
        pats = np.array(oracle.all_patterns(m, sum(S)), dtype=np.int32)
        c = lofp.Circuit(m, layers)
        got = c.path_counts(S, pats)
        want = [oracle.path_count_bruteforce(m, S, T, flat(layers)) for T in pats]
        assert np.array_equal(got, np.array(want, dtype=np.float64))


def test_leaf_count_matches_path_count_when_frontiers_are_endpoints():
    """With the forward frontier at S and the backward one at T, every valid
    path is enumerated once by the depth-first kernel."""
    wl = workloads.make("c1", seed=2)
    pats = np.array(oracle.all_patterns(wl.m, wl.n), dtype=np.int32)
    c = lofp.Circuit(wl.m, wl.layers)
    st = lofp.Stats()
    c.amplitudes(wl.S, pats, lofp.make_opts(method=lofp.METHOD_PATHSUM, fwd_layer=0, bwd_layer=wl.depth), st)
    assert st.dfs_leaves == int(c.path_counts(wl.S, pats).sum())


# ------------------------------------------------------------- determinism
def test_deterministic_and_independent_of_batch():
    """Repeated calls give the same bits.  One contraction per pattern gives
    each pattern the same bits alone and in any batch; the split form (the
    default for this circuit) agrees with it to rounding: its half states
    span the hull of the batch's intervals, so their sums take other terms
    in another order."""
    wl = workloads.make("c2", seed=5, batch=64)
    c = lofp.Circuit(wl.m, wl.layers)
    a = c.amplitudes(wl.S, wl.Ts)
    b = c.amplitudes(wl.S, wl.Ts)
    assert np.array_equal(a, b)
    pp = c.amplitudes(wl.S, wl.Ts, NEVER_SPLIT)
    check(a, pp, 1e-14)
    for p in (0, 17, 63):
        alone = c.amplitudes(wl.S, wl.Ts[p:p + 1], NEVER_SPLIT)
        assert alone[0] == pp[p]
        check(c.amplitudes(wl.S, wl.Ts[p:p + 1]), pp[p:p + 1], 1e-14)


# ------------------------------------------------------------ FP32 products
def test_fp32_products_within_bound():
    wl = workloads.make("c2", seed=3, batch=32)
    c = lofp.Circuit(wl.m, wl.layers)
    ref = c.amplitudes(wl.S, wl.Ts)
    f32 = c.amplitudes(wl.S, wl.Ts, lofp.make_opts(precision=lofp.PREC_FP32))
    err = np.abs(f32 - ref)
    # products of at most `levels` FP32 factors: relative error per path
    # <= (2 levels + 2) 2^-24; summed paths of magnitude <= 1 each
    assert err.max() < 1e-5


def test_frontier_budget_moves_the_cut_to_depth_first():
    """A small frontier budget makes the planner stop merging earlier and
    enumerate more splitters depth-first; the result does not change."""
    wl = workloads.make("c1", seed=6)
    pats = np.array(oracle.all_patterns(wl.m, wl.n), dtype=np.int32)
    c = lofp.Circuit(wl.m, wl.layers)
    st_big, st_small = lofp.Stats(), lofp.Stats()
    a = c.amplitudes(wl.S, pats, lofp.make_opts(method=lofp.METHOD_PATHSUM), st_big)
    b = c.amplitudes(wl.S, pats, lofp.make_opts(method=lofp.METHOD_PATHSUM, frontier_budget_kb=40), st_small)
    assert st_big.fwd_layer == st_big.bwd_layer == wl.depth - 2
    assert st_small.fwd_layer < st_small.bwd_layer and st_small.dfs_leaves > 0
    check(a, b)
    check(a, oracle_amps(wl.m, wl.S, pats, wl.layers))


def test_pathsum_state_space_overflow_is_reported():
    wl = workloads.make("c5", seed=0, batch=2)
    c = lofp.Circuit(wl.m, wl.layers)
    with pytest.raises(lofp.LofpError) as e:
        c.amplitudes(wl.S, wl.Ts, lofp.make_opts(method=lofp.METHOD_PATHSUM, fwd_layer=3, bwd_layer=3))
    assert e.value.status == lofp.ENOMEM


def test_auto_picks_contraction_and_matches_pathsum():
    wl = workloads.make("c2", seed=2, batch=32)
    c = lofp.Circuit(wl.m, wl.layers)
    st = lofp.Stats()
    a = c.amplitudes(wl.S, wl.Ts, lofp.make_opts(), st)
    assert st.method_used == lofp.METHOD_CONTRACT
    st2 = lofp.Stats()
    b = c.amplitudes(wl.S, wl.Ts, lofp.make_opts(method=lofp.METHOD_PATHSUM), st2)
    assert st2.method_used == lofp.METHOD_PATHSUM
    check(a, b)
    check(a, oracle_amps(wl.m, wl.S, wl.Ts, wl.layers))


# ------------------------------------------------- many circuits and serving
def _served(count, seed=0):
    reqs = workloads.served_requests(count, rate_hz=0.0, seed=seed)
    return [(lofp.Circuit(r.m, r.layers), r) for r in reqs]


def test_multi_circuit_batch_matches_oracle_and_single_calls():
    items = _served(24, seed=3)
    got = lofp.amplitudes_multi([(c, r.S, r.T) for c, r in items])
    for i, (c, r) in enumerate(items):
        want = oracle.amplitude(r.m, r.S, r.T, flat(r.layers))
        assert abs(got[i] - want) <= ATOL
        alone = c.amplitudes(r.S, r.T[None, :], NEVER_SPLIT)[0]
        assert alone == got[i]


def test_multi_fp32_products_within_bound():
    items = _served(24, seed=4)
    f64 = lofp.amplitudes_multi([(c, r.S, r.T) for c, r in items])
    f32, eb = lofp.amplitudes_multi([(c, r.S, r.T) for c, r in items], lofp.make_opts(precision=lofp.PREC_FP32),
                                    bounds=True)
    assert np.all(np.isfinite(eb)) and np.all(eb >= 0)
    # every returned result is certified to 1e-6 relative or came from the FP64 re-run
    assert np.all(np.abs(f32 - f64) <= eb + 1e-14)
    assert np.all((eb <= 1e-6 * np.abs(f32)) | (np.abs(f32 - f64) <= 1e-13))
    nz = np.abs(f64) > 1e-12
    rel = np.abs(f32 - f64)[nz] / np.abs(f64)[nz]
    assert rel.max() < 1e-5, rel.max()
    f64b = lofp.amplitudes_multi([(c, r.S, r.T) for c, r in items])
    assert np.all(np.isnan(lofp.amplitudes_multi([(c, r.S, r.T) for c, r in items], bounds=True)[1]))
    assert np.array_equal(f64, f64b)


def _growth(G, n, fp32):
    """The factor ((1 + f)^G - 1 + 4 * 2^-53)(1 + 2^-30) that multiplies the
    absolute form in the stated rounding bound."""
    u = 2.0 ** -24
    k = (n + 1) ** 2
    f = (4 * u / (1 - 4 * u) if fp32 else 0.0) + (2 * k + 2) * 2.0 ** -53
    return (math.expm1(G * math.log1p(f)) + 4 * 2.0 ** -53) * (1 + 2.0 ** -30)


def _small_items(count, seed):
    rng = np.random.default_rng(seed)
    items = []
    for i in range(count):
        m = int(rng.choice([6, 8, 9]))
        n = m // 2
        layers = _brickwork(m, int(rng.integers(3, 7)), seed * 100 + i)
        S = np.zeros(m, np.int32)
        T = np.zeros(m, np.int32)
        for _ in range(n):
            S[rng.integers(m)] += 1
            T[rng.integers(m)] += 1
        items.append((lofp.Circuit(m, layers), m, n, layers, S, T))
    return items


@pytest.mark.parametrize("rtol", [1e300, 1e-300])
def test_fp32_bound_is_the_absolute_form_and_holds(rtol):
    """The bound each FP32 result carries is the stated growth factor times the
    absolute form (checked against the oracle's absolute form), and it holds
    against the oracle's amplitude.  rtol 1e300: no result falls back;
    1e-300: every result is recomputed in FP64 and carries the FP64 bound."""
    items = _small_items(20, seed=21 if rtol > 1 else 22)
    amps, eb = lofp.amplitudes_multi([(c, S, T) for c, _, _, _, S, T in items],
                                     lofp.make_opts(precision=lofp.PREC_FP32, fp32_rtol=rtol), bounds=True)
    for i, (c, m, n, layers, S, T) in enumerate(items):
        circ = flat(layers)
        want = oracle.amplitude(m, S, T, circ)
        a_abs = oracle.absolute_form(m, S, T, circ)
        grow = _growth(len(circ), n, fp32=rtol > 1)
        assert abs(eb[i] - grow * a_abs) <= 1e-9 * grow * a_abs + 1e-300, (i, eb[i], grow * a_abs)
        assert abs(amps[i] - want) <= eb[i] + 1e-15 * max(1.0, a_abs)
        if rtol < 1:
            assert abs(amps[i] - want) <= ATOL


def test_server_results_same_alone_and_in_mix():
    items = _served(40, seed=5)
    alone = [lofp.amplitudes_multi([(c, r.S, r.T)])[0] for c, r in items]
    srv = lofp.Server(max_batch=16, streams=2)
    try:
        tickets = [srv.submit(c, r.S, r.T) for c, r in items]
        res = [srv.result(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    for i, (amp, lat, _) in enumerate(res):
        assert amp == alone[i]
        assert lat >= 0
    assert st["completed"] == len(items) and st["launches"] >= 3


# ------------------------------------------------------ split contraction
def test_split_contraction_full_c2_batch():
    """The 4096-pattern batch shares S: the contraction runs once per distinct
    top and bottom half of T and joins per pattern.  Checked against the
    oracle on a sample and against one contraction per pattern on every
    pattern."""
    wl = workloads.make("c2", seed=0)
    c = lofp.Circuit(wl.m, wl.layers)
    st = lofp.Stats()
    got = c.amplitudes(wl.S, wl.Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT), st)
    assert st.split_top_keys > 0 and st.split_bottom_keys > 0
    idx = np.random.default_rng(2).choice(wl.batch, 64, replace=False)
    check(got[idx], oracle_amps(wl.m, wl.S, wl.Ts[idx], wl.layers))
    ref = np.concatenate([c.amplitudes(wl.S, wl.Ts[i:i + 32], NEVER_SPLIT) for i in range(0, wl.batch, 32)])
    check(got, ref, 1e-14)


def test_split_contraction_invalid_rows_and_no_sharing():
    wl = workloads.make("c2", seed=4, batch=1024)
    Ts = wl.Ts.copy()
    Ts[5, 0] += 1          # wrong photon number: exact 0
    Ts[9] = 0
    Ts[9, -1] = wl.n       # all photons in the last mode: infeasible at depth 8
    c = lofp.Circuit(wl.m, wl.layers)
    st = lofp.Stats()
    got = c.amplitudes(wl.S, Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT), st)
    assert st.split_top_keys > 0
    assert got[5] == 0 and got[9] == 0
    ok = np.array([i for i in range(len(Ts)) if i not in (5, 9)])
    check(got[ok[:128]], oracle_amps(wl.m, wl.S, Ts[ok[:128]], wl.layers))
    # bunched patterns share few halves: a large batch falls back to one
    # contraction per pattern ...
    wl3 = workloads.make("c3", seed=4, batch=2048)
    c3 = lofp.Circuit(wl3.m, wl3.layers)
    st3 = lofp.Stats()
    got3 = c3.amplitudes(wl3.S, wl3.Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT), st3)
    assert st3.split_top_keys == 0
    check(got3[:64], oracle_amps(wl3.m, wl3.S, wl3.Ts[:64], wl3.layers))
    # ... while a batch of 256 to 1024 patterns is split for parallelism
    wl4 = workloads.make("c3", seed=4, batch=300)
    c4 = lofp.Circuit(wl4.m, wl4.layers)
    st4 = lofp.Stats()
    got4 = c4.amplitudes(wl4.S, wl4.Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT), st4)
    assert st4.split_top_keys > 0
    check(got4[:64], oracle_amps(wl4.m, wl4.S, wl4.Ts[:64], wl4.layers))
    unsplit = np.concatenate([c4.amplitudes(wl4.S, wl4.Ts[i:i + 32], NEVER_SPLIT)
                              for i in range(0, 64, 32)])
    check(got4[:64], unsplit, 1e-14)


def _brickwork(m, depth, seed):
    rng = np.random.default_rng(seed)
    layers = []
    for l in range(depth):
        layers.append([(a, a + 1, float(rng.uniform(0, np.pi / 2)), float(rng.uniform(0, 2 * np.pi)))
                       for a in range(l % 2, m - 1, 2)])
    return layers


def test_server_falls_back_to_the_path_sum():
    """A request the contraction cannot take (too many live cut versions) is
    summed by the path-sum form on a planner thread and completes with the
    oracle's amplitude (counted as a path-sum fallback); the requests around
    it are unaffected and equal their batch values."""
    good = _served(6, seed=11)
    bad_layers = _brickwork(8, 40, seed=12)
    bad = lofp.Circuit(8, bad_layers)
    S = np.array([1, 1, 1, 1, 0, 0, 0, 0], dtype=np.int32)
    T = np.array([0, 0, 0, 0, 1, 1, 1, 1], dtype=np.int32)
    with pytest.raises(lofp.LofpError) as ei:
        lofp.amplitudes_multi([(bad, S, T)])
    assert ei.value.status == lofp.ENOTSUP
    srv = lofp.Server(max_batch=8, streams=2)
    try:
        t_good = [srv.submit(c, r.S, r.T) for c, r in good]
        t_bad = srv.submit(bad, S, T)
        res = [srv.result(t) for t in t_good]
        amp_bad, lat_bad, _ = srv.result(t_bad)
        st = srv.stats()
    finally:
        srv.close()
    assert st["pathsum_fallbacks"] == 1 and lat_bad >= 0
    assert abs(amp_bad - oracle.amplitude(8, S, T, flat(bad_layers))) <= ATOL
    assert amp_bad == bad.amplitudes(S, T[None, :], lofp.make_opts(method=lofp.METHOD_PATHSUM))[0]
    want = lofp.amplitudes_multi([(c, r.S, r.T) for c, r in good])
    for (amp, _, _), w in zip(res, want):
        assert amp == w


def test_circuit_setup_memory_is_reused_and_tables_grow():
    """Circuits set up together share pooled device blocks that are reused
    after the circuits go away; a circuit first used with few photons gets
    larger tables when a later call brings more."""
    for rnd in range(3):
        items = _served(40, seed=20 + rnd)
        got = lofp.amplitudes_multi([(c, r.S, r.T) for c, r in items])
        for i in (0, 17, 39):
            c, r = items[i]
            assert abs(got[i] - oracle.amplitude(r.m, r.S, r.T, flat(r.layers))) <= ATOL
        del items, got
    layers = _brickwork(10, 6, seed=30)
    c = lofp.Circuit(10, layers)
    for S in (np.array([1, 0, 1, 0, 0, 0, 0, 0, 0, 0]), np.array([1, 1, 1, 1, 1, 1, 0, 0, 0, 0]),
              np.array([2, 0, 2, 0, 2, 0, 1, 0, 0, 0])):
        S = S.astype(np.int32)
        n = int(S.sum())
        Ts = np.array([p for p in oracle.all_patterns(10, n)][:64], dtype=np.int32)
        got = c.amplitudes(S, Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT))
        check(got, oracle_amps(10, S, Ts, layers))


def test_count_work_only_counts():
    """Counting the work done changes no result bit; without it the counter
    stays zero."""
    wl = workloads.make("c2", seed=2, batch=512)
    c = lofp.Circuit(wl.m, wl.layers)
    st0, st1 = lofp.Stats(), lofp.Stats()
    a = c.amplitudes(wl.S, wl.Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT), st0)
    b = c.amplitudes(wl.S, wl.Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT, count_work=True), st1)
    assert np.array_equal(a, b)
    assert st0.transitions == 0 and st1.transitions > 0


def test_server_fp32_bounds_and_fallbacks():
    """FP32 serving: results whose bound exceeds rtol * |amp| are recomputed in
    FP64 (counted; rtol 1e-300 sends back every result with a path); every
    returned result lies within its bound of the oracle."""
    items = _small_items(16, seed=23)
    for rtol, all_back in ((1e-300, True), (0.0, False)):
        srv = lofp.Server(max_batch=8, streams=2, precision=lofp.PREC_FP32, fp32_rtol=rtol)
        try:
            tickets = [srv.submit(c, S, T) for c, _, _, _, S, T in items]
            res = [srv.result(t) for t in tickets]
            st = srv.stats()
        finally:
            srv.close()
        assert st["completed"] == len(items)
        if all_back:
            # a result with no path has bound 0 and needs no re-run
            live = sum(oracle.absolute_form(m, S, T, flat(layers)) > 0 for _, m, _, layers, S, T in items)
            assert 0 < live < len(items) and st["fp64_fallbacks"] == live
        for (amp, lat, eb), (c, m, n, layers, S, T) in zip(res, items):
            want = oracle.amplitude(m, S, T, flat(layers))
            assert math.isfinite(eb) and eb >= 0
            assert abs(amp - want) <= eb + 1e-15
            assert lat >= 0
            if all_back:
                assert abs(amp - want) <= ATOL
            else:
                assert eb <= 1e-6 * abs(amp) or st["fp64_fallbacks"] > 0


# ------------------------------------------------------------------ planner
@pytest.mark.parametrize("case", ["c2", "c3", "deep", "served"])
def test_device_bounds_equal_host_bounds(case):
    """The planner kernel's intervals (one wave per pattern) are the host
    propagation's, integer for integer; feasibility likewise.  Covers single
    and bunched photons, a depth-20 circuit and a served request shape."""
    rng = np.random.default_rng(31)
    if case in ("c2", "c3"):
        wl = workloads.make(case, seed=0)
        m, layers, S, Ts = wl.m, wl.layers, wl.S, np.asarray(wl.Ts[:512], dtype=np.int32)
    elif case == "deep":
        m, layers = 8, _brickwork(8, 20, seed=32)
        S = np.array([1, 0, 1, 0, 1, 0, 1, 0], np.int32)
        Ts = np.zeros((200, m), np.int32)
        for row in Ts:
            for _ in range(4):
                row[rng.integers(m)] += 1
    else:
        r = workloads.served_requests(1, rate_hz=0.0, seed=33)[0]
        m, layers, S = r.m, r.layers, r.S
        Ts = np.zeros((200, m), np.int32)
        for row in Ts:
            for _ in range(int(np.sum(S))):
                row[min(m - 1, max(0, int(np.flatnonzero(S)[rng.integers(len(np.flatnonzero(S)))] + rng.integers(-3, 4))))] += 1
    Ts = Ts.copy()
    Ts[3, 0] += 1                      # wrong photon number: infeasible
    c = lofp.Circuit(m, layers)
    lo, hi, feas = c.bounds_batch(S, Ts)
    nfeas = 0
    for p in range(Ts.shape[0]):
        hl, hh, hf = c.bounds(S, Ts[p])
        assert feas[p] == hf, p
        if hf:
            nfeas += 1
            assert np.array_equal(lo[p], hl) and np.array_equal(hi[p], hh), p
    assert not feas[3] and nfeas > 0


# ----------------------------------------------------- high photon density
@pytest.mark.parametrize("m,D,S", [(3, 4, (12, 0, 8)), (4, 5, (10, 4, 0, 10))])
def test_high_photon_density_all_outputs(m, D, S):
    """Many photons per mode (20 and 24 photons in 3 and 4 modes): every output
    pattern by the contraction and by the path sum against an evolution with
    40-digit splitter sectors; the probabilities sum to one."""
    pytest.importorskip("mpmath")
    layers = _brickwork(m, D, seed=70 + m)
    circ = flat(layers)
    want_state = oracle.evolve_hp(m, S, circ)
    Ts = np.array(oracle.all_patterns(m, sum(S)), dtype=np.int32)
    want = np.array([want_state.get(tuple(t), 0j) for t in Ts])
    c = lofp.Circuit(m, layers)
    for method in (lofp.METHOD_CONTRACT, lofp.METHOD_PATHSUM):
        got = c.amplitudes(np.array(S, np.int32), Ts, lofp.make_opts(method=method))
        check(got, want)
        assert abs(np.sum(np.abs(got) ** 2) - 1.0) < 1e-12


def test_split_contraction_large_batch():
    """32768 patterns in one call (eight times the benchmark batch): the
    grouping, job and join grids at that size; a sample against the oracle,
    a slice against the same patterns in a smaller batch, repeated calls
    bit-identical."""
    wl = workloads.make("c2", seed=9, batch=32768)
    c = lofp.Circuit(wl.m, wl.layers)
    st = lofp.Stats()
    got = c.amplitudes(wl.S, wl.Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT), st)
    assert st.split_top_keys > 0 and st.split_bottom_keys > 0
    idx = np.random.default_rng(5).choice(wl.batch, 48, replace=False)
    check(got[idx], oracle_amps(wl.m, wl.S, wl.Ts[idx], wl.layers))
    part = c.amplitudes(wl.S, wl.Ts[:4096], lofp.make_opts(method=lofp.METHOD_CONTRACT))
    check(got[:4096], part, 1e-14)
    again = c.amplitudes(wl.S, wl.Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT))
    assert np.array_equal(got, again)


def test_split_contraction_shrinking_batches_on_one_circuit():
    """One circuit, split batches of falling size in a row (4096, then 904
    and 1000 patterns split for parallelism, then 300): each call's grouping
    reuses the table and hull layout of the first, and every result equals the
    unsplit contraction of the same rows (and the oracle on a sample)."""
    wl = workloads.make("c2", seed=6)
    c = lofp.Circuit(wl.m, wl.layers)
    opts = lofp.make_opts(method=lofp.METHOD_CONTRACT)
    unsplit = np.concatenate([c.amplitudes(wl.S, wl.Ts[i:i + 32], NEVER_SPLIT) for i in range(0, 1024, 32)])
    for lo_, hi_ in ((0, 4096), (100, 1004), (0, 1000), (700, 1000)):
        st = lofp.Stats()
        got = c.amplitudes(wl.S, wl.Ts[lo_:hi_], opts, st)
        assert st.split_top_keys > 0 and st.split_bottom_keys > 0, (lo_, hi_)
        assert not np.isnan(got).any()
        k = min(hi_, 1024) - lo_
        if k > 0:
            check(got[:k], unsplit[lo_:lo_ + k], 1e-14)
    idx = np.random.default_rng(8).choice(1024, 32, replace=False)
    check(unsplit[idx], oracle_amps(wl.m, wl.S, wl.Ts[idx], wl.layers))


def test_split_contraction_batch_in_two_passes():
    """A batch above the pass size (32768 + 1024 patterns) runs in two passes
    on one circuit, the second smaller: rows equal the same rows computed in
    chunks of at most 4096, stats sum over the passes, a sample equals the
    oracle."""
    wl = workloads.make("c2", seed=11, batch=33792)
    c = lofp.Circuit(wl.m, wl.layers)
    opts = lofp.make_opts(method=lofp.METHOD_CONTRACT)
    st = lofp.Stats()
    got = c.amplitudes(wl.S, wl.Ts, opts, st)
    assert st.batch == wl.batch and not np.isnan(got).any()
    chunks, keys = [], [0, 0]
    for i in range(0, wl.batch, 4096):
        sc = lofp.Stats()
        chunks.append(c.amplitudes(wl.S, wl.Ts[i:i + 4096], opts, sc))
        keys[0] += sc.split_top_keys
        keys[1] += sc.split_bottom_keys
    check(got, np.concatenate(chunks), 1e-14)
    # the two passes share more halves than nine chunks do
    assert 0 < st.split_top_keys <= keys[0] and 0 < st.split_bottom_keys <= keys[1]
    idx = np.random.default_rng(12).choice(wl.batch, 32, replace=False)
    check(got[idx], oracle_amps(wl.m, wl.S, wl.Ts[idx], wl.layers))


@pytest.mark.parametrize("batch", [16, 300])
def test_contraction_overflow_is_nan_without_stats_and_enomem_with(batch):
    """A state larger than its buffers (forced from the host with a state
    limit of two entries): without stats every affected result is NaN, with
    stats the call returns ENOMEM; the next call without the limit is right.
    16 patterns take one contraction per pattern, 300 the split contraction
    (whose jobs then have neither LDS room nor a workspace: they stop)."""
    wl = workloads.make("c2", seed=13, batch=batch)
    c = lofp.Circuit(wl.m, wl.layers)
    want = oracle_amps(wl.m, wl.S, wl.Ts, wl.layers)
    tight = lofp.make_opts(method=lofp.METHOD_CONTRACT, state_limit=2)
    got = c.amplitudes(wl.S, wl.Ts, tight)
    live = np.abs(want) > 0
    assert live.sum() > 0 and np.isnan(got[live]).all()
    with pytest.raises(lofp.LofpError) as e:
        c.amplitudes(wl.S, wl.Ts, tight, lofp.Stats())
    assert e.value.status == lofp.ENOMEM
    check(c.amplitudes(wl.S, wl.Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT)), want)


def test_small_batches_split_for_latency():
    """A circuit of 40 or more splitters splits even one pattern into its two
    halves (two half-length chains in parallel, then the join); a short one
    keeps one contraction per pattern unless asked.  Every form agrees with
    one contraction per pattern and with the oracle."""
    wl = workloads.make("c2", seed=9)
    c = lofp.Circuit(wl.m, wl.layers)
    for B in (1, 8, 40):
        Ts = wl.Ts[:B]
        ref = c.amplitudes(wl.S, Ts, NEVER_SPLIT)
        st = lofp.Stats()
        got = c.amplitudes(wl.S, Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT), st)
        assert st.split_top_keys > 0 and st.split_bottom_keys > 0, B
        check(got, ref, 1e-14)
        st = lofp.Stats()
        got = c.amplitudes(wl.S, Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT, split=lofp.SPLIT_ALWAYS), st)
        assert st.split_top_keys > 0
        check(got, ref, 1e-14)
        check(ref, oracle_amps(wl.m, wl.S, Ts, wl.layers))
    w1 = workloads.make("c1", seed=0)
    c1 = lofp.Circuit(w1.m, w1.layers)
    ref = c1.amplitudes(w1.S, w1.Ts[:1], NEVER_SPLIT)
    st = lofp.Stats()
    got = c1.amplitudes(w1.S, w1.Ts[:1], lofp.make_opts(method=lofp.METHOD_CONTRACT), st)
    assert st.split_top_keys == 0
    check(got, ref, 1e-14)
    st = lofp.Stats()
    got = c1.amplitudes(w1.S, w1.Ts[:1], lofp.make_opts(method=lofp.METHOD_CONTRACT, split=lofp.SPLIT_ALWAYS), st)
    assert st.split_top_keys > 0
    check(got, ref, 1e-14)
    check(ref, oracle_amps(w1.m, w1.S, w1.Ts[:1], w1.layers))
    with pytest.raises(lofp.LofpError):
        c1.amplitudes(w1.S, w1.Ts[:1], lofp.make_opts(method=lofp.METHOD_CONTRACT, split=3))


@pytest.mark.parametrize("m,D,seed", [(6, 2, 21), (7, 5, 22), (9, 4, 23), (12, 7, 24), (14, 6, 25), (20, 3, 26)])
def test_forced_split_join_many_shapes(m, D, seed):
    """The split contraction forced on brickwork circuits of several widths
    and depths: the join sums over one to six crossing versions and boxes
    from a single entry to several passes of a wave.  Every pattern agrees
    with one contraction per pattern, a sample with the oracle."""
    rng = np.random.default_rng(seed)
    layers = workloads.random_brickwork(m, D, rng)
    S = workloads.photons_even_modes(m)
    Ts = np.stack([workloads.sample_collision_free(rng, S, D) for _ in range(48)])
    c = lofp.Circuit(m, layers)
    st = lofp.Stats()
    got = c.amplitudes(S, Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT, split=lofp.SPLIT_ALWAYS), st)
    assert st.split_top_keys > 0 and st.split_bottom_keys > 0
    ref = c.amplitudes(S, Ts, NEVER_SPLIT)
    check(got, ref, 1e-14)
    check(got[:8], oracle_amps(m, S, Ts[:8], layers))


def test_c5_full_batch_split_for_parallelism():
    """The 32-mode, depth-6 workload at its full 512 patterns, in the launch
    the benchmark times (the batch split into top and bottom halves for
    parallelism): 64 patterns against the oracle, all 512 against the
    unsplit contraction."""
    wl = workloads.make("c5", seed=0)
    assert wl.batch == 512
    c = lofp.Circuit(wl.m, wl.layers)
    st = lofp.Stats()
    got = c.amplitudes(wl.S, wl.Ts, lofp.make_opts(), st)
    assert st.method_used == lofp.METHOD_CONTRACT and st.split_top_keys > 0
    idx = np.random.default_rng(14).choice(wl.batch, 64, replace=False)
    check(got[idx], oracle_amps(wl.m, wl.S, wl.Ts[idx], wl.layers))
    ref = np.concatenate([c.amplitudes(wl.S, wl.Ts[i:i + 32], NEVER_SPLIT) for i in range(0, wl.batch, 32)])
    check(got, ref, 1e-14)


def test_fp32_depth_first_products_within_bound():
    """The depth-first kernel's FP32 form (running path products in FP32,
    frontier values and sums in FP64), with the frontiers at S and T so that
    every splitter is enumerated: each result lies within the stated FP32
    bound ((1 + f)^G - 1 + 4 * 2^-53) A_abs of the oracle, and the FP64 form
    within 1e-12."""
    items = _small_items(16, seed=41)
    done = 0
    for c, m, n, layers, S, T in items:
        circ = flat(layers)
        if len(circ) > 16:
            continue
        done += 1
        want, eb = oracle.amplitude(m, S, T, circ, with_bound=True)
        a_abs = oracle.absolute_form(m, S, T, circ)
        o32 = lofp.make_opts(method=lofp.METHOD_PATHSUM, precision=lofp.PREC_FP32, fwd_layer=0,
                             bwd_layer=len(layers))
        st = lofp.Stats()
        got = c.amplitudes(S, T[None, :], o32, st)[0]
        assert st.dfs_levels == len(circ)
        if a_abs == 0:
            # no valid path: exactly zero (the permanent's own rounding may not be)
            assert got == 0 and abs(want) <= eb
        else:
            # the stated bound plus the oracle's own rounding bound
            assert abs(got - want) <= _growth(len(circ), n, fp32=True) * a_abs + eb, (abs(got - want), a_abs)
        o64 = lofp.make_opts(method=lofp.METHOD_PATHSUM, fwd_layer=0, bwd_layer=len(layers))
        assert abs(c.amplitudes(S, T[None, :], o64)[0] - want) <= ATOL
    assert done >= 6


# ------------------------------------------------- distant pairs, all outputs
def _distant_layers(m, depth, rng):
    """Random layers of disjoint pairs at distance 1 to 4."""
    layers = []
    for _ in range(depth):
        free = list(range(m))
        layer = []
        for _ in range(m // 2):
            a = int(rng.choice(free))
            cand = [b for b in free if a < b <= a + 4]
            if not cand:
                continue
            b = int(rng.choice(cand))
            free.remove(a)
            free.remove(b)
            layer.append((a, b, float(rng.uniform(0, np.pi / 2)), float(rng.uniform(0, 2 * np.pi))))
        layers.append(layer)
    return layers


@pytest.mark.parametrize("method", [lofp.METHOD_PATHSUM, lofp.METHOD_CONTRACT, lofp.METHOD_AUTO])
def test_distant_pairs_match_oracle(method):
    """Circuits whose layers connect modes up to four apart (compiled by the
    library to adjacent splitters) against the oracle, which takes the
    distant splitters as given (Ryser on their composed unitary)."""
    rng = np.random.default_rng(51)
    ran = 0
    for m, D in ((6, 4), (8, 3), (10, 3)):
        layers = _distant_layers(m, D, rng)
        S = np.zeros(m, np.int32)
        S[::2] = 1
        n = int(S.sum())
        Ts = np.zeros((40, m), np.int32)
        for row in Ts:
            for _ in range(n):
                row[rng.integers(m)] += 1
        c = lofp.Circuit(m, layers)
        try:
            got = c.amplitudes(S, Ts, lofp.make_opts(method=method))
        except lofp.LofpError as e:
            # the swap chains can make the contraction's state too large; the
            # forced contraction then says so (AUTO takes the path sum)
            assert method == lofp.METHOD_CONTRACT and e.status == lofp.ENOMEM, e
            continue
        ran += 1
        check(got, oracle_amps(m, S, Ts, layers))
    assert ran == 3 or (method == lofp.METHOD_CONTRACT and ran >= 1)


def test_all_outputs_paper_protocol():
    """Sec. III.A through the all-outputs call: every output of the four
    6-mode inputs, in the oracle's pattern order; probabilities sum to one
    and their total variation distance to the oracle's is below 1e-13."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_correctness_inputs.json")))
    for k, case in enumerate(g["cases"]):
        S, D = np.array(case["S"], np.int32), case["depth"]
        layers = workloads.random_brickwork(g["m"], D, np.random.Generator(np.random.PCG64(60 + k)))
        c = lofp.Circuit(g["m"], layers)
        Ts, amps = c.all_outputs(S)
        assert np.array_equal(Ts, np.array(oracle.all_patterns(g["m"], int(S.sum())), np.int32))
        want = oracle_amps(g["m"], S, Ts, layers)
        check(amps, want)
        p, q = np.abs(amps) ** 2, np.abs(want) ** 2
        assert abs(p.sum() - 1) < 1e-12
        assert 0.5 * np.abs(p - q).sum() <= g["tvd_vs_ryser_max"]


def test_all_outputs_distant_pairs_and_c2_size():
    """All outputs of a 7-mode circuit with distant pairs (norm one, oracle
    parity), and of the 16-mode, depth-8 workload's input: its 490314
    patterns in passes, the norm within 1e-11 and a sample against the
    oracle."""
    rng = np.random.default_rng(71)
    layers = _distant_layers(7, 4, rng)
    S = np.array([1, 0, 2, 0, 1, 0, 0], np.int32)
    c = lofp.Circuit(7, layers)
    Ts, amps = c.all_outputs(S)
    check(amps, oracle_amps(7, S, Ts, layers))
    assert abs(np.sum(np.abs(amps) ** 2) - 1) < 1e-12
    wl = workloads.make("c2", seed=0, batch=8)
    c2 = lofp.Circuit(wl.m, wl.layers)
    Ts2, amps2 = c2.all_outputs(wl.S)
    assert Ts2.shape == (490314, wl.m) and np.all(Ts2.sum(axis=1) == wl.n)
    assert abs(np.sum(np.abs(amps2) ** 2) - 1) < 1e-11
    idx = np.random.default_rng(72).choice(len(Ts2), 48, replace=False)
    check(amps2[idx], oracle_amps(wl.m, wl.S, Ts2[idx], wl.layers))


# ------------------------------------------------ graph capture and the tuner
def test_graph_replay_equals_eager_tuned_call():
    """The whole call captured as a graph (split decided on the device, way of
    contracting chosen by the tuner) replays bit-identical to the eager call
    with the same tuned choice, with eager work on the same circuit and
    synchronisations between replays; new T values in the captured buffer are
    picked up; the tuned and the default way agree to 1e-14."""
    import torch
    wl = workloads.make("c2", seed=0)
    c = lofp.Circuit(wl.m, wl.layers)
    T = torch.from_numpy(np.ascontiguousarray(wl.Ts)).cuda()
    opts = lofp.make_opts(method=lofp.METHOD_CONTRACT, autotune=True)
    eager = torch.zeros(wl.batch, dtype=torch.complex128, device="cuda")
    st = lofp.Stats()
    c.amplitudes_device(wl.S, T, eager, opts, stats=st)
    torch.cuda.synchronize()
    assert st.tuned == 1
    ref = eager.cpu().numpy()
    idx = np.random.default_rng(90).choice(wl.batch, 32, replace=False)
    check(ref[idx], oracle_amps(wl.m, wl.S, wl.Ts[idx], wl.layers))
    check(ref, c.amplitudes(wl.S, wl.Ts, lofp.make_opts(method=lofp.METHOD_CONTRACT)), 1e-14)
    out = torch.zeros(wl.batch, dtype=torch.complex128, device="cuda")
    g = lofp.Graph(c, wl.S, T, out, opts)
    try:
        for r in range(4):
            out.zero_()
            g.launch()
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref), r
            c.amplitudes(wl.S, wl.Ts[: 100 + 50 * r])   # eager work on the caller's circuit
        # new patterns in the captured buffer
        T2 = workloads.make("c2", seed=3).Ts
        T.copy_(torch.from_numpy(np.ascontiguousarray(T2)))
        g.launch()
        torch.cuda.synchronize()
        c.amplitudes_device(wl.S, T, eager, opts)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager.cpu().numpy())
        check(out.cpu().numpy()[:16], oracle_amps(wl.m, wl.S, T2[:16], wl.layers))
    finally:
        g.close()


@pytest.mark.parametrize("name,batch", [("c2", 1), ("c5", 512), ("c3", 300)])
def test_graph_small_and_other_workloads(name, batch):
    """Captured calls for a single pattern (split into its halves: the
    circuit is long), the 32-mode batch and a bunched batch, each replayed
    twice against the eager call."""
    import torch
    wl = workloads.make(name, seed=5, batch=batch)
    c = lofp.Circuit(wl.m, wl.layers)
    T = torch.from_numpy(np.ascontiguousarray(wl.Ts)).cuda()
    out = torch.zeros(wl.batch, dtype=torch.complex128, device="cuda")
    opts = lofp.make_opts(method=lofp.METHOD_CONTRACT)
    ref = c.amplitudes(wl.S, wl.Ts, opts)
    g = lofp.Graph(c, wl.S, T, out, opts)
    try:
        for _ in range(2):
            out.zero_()
            g.launch()
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref)
    finally:
        g.close()
    check(ref[:32], oracle_amps(wl.m, wl.S, wl.Ts[:32], wl.layers))
