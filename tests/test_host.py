"""CPU tests of the library's host side: the C-ABI exports what include/lofp.h
declares, input validation, the light cone of Sec. II.B (paper's worked
example), and exactness of the cut bounds against brute-force enumeration of
the configurations that lie on valid paths."""
import json
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2510_26408_amd import lofp, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "lofp.h")).read()
    return sorted(set(re.findall(r"\b(lofp_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lofp.load()
    out = subprocess.check_output(["nm", "-D", "--defined-only", lofp.LIB_PATH]).decode()
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    decl = declared_symbols()
    assert decl, "no declarations parsed"
    missing = [s for s in decl if s not in exported]
    assert not missing, missing
    assert set(decl) == set(lofp.EXPORTED)


def test_light_cone_matches_paper_example():
    g = json.load(open(os.path.join(GOLDEN, "light_cone_example.json")))
    M, D = g["M"], g["D"]
    layers = [[(a, a + 1, 0.1, 0.2) for a, _ in pairs] for pairs in workloads.brickwork_pairs(M, D)]
    c = lofp.Circuit(M, layers)
    (plo, phi), (flo, fhi) = c.light_cone(g["layer_j"], g["waveguide_mode_1based"] - 1)
    assert [plo + 1, phi + 1] == g["past_inputs_1based"]
    assert [flo + 1, fhi + 1] == g["future_outputs_1based"]


def test_validation_errors():
    with pytest.raises(lofp.LofpError) as e:
        lofp.Circuit(1, [])
    assert e.value.status == lofp.EINVAL
    with pytest.raises(lofp.LofpError) as e:
        lofp.Circuit(4, [[(0, 1, 0.1, 0.1), (1, 2, 0.1, 0.1)]])
    assert e.value.status == lofp.EINVAL
    with pytest.raises(lofp.LofpError) as e:
        lofp.Circuit(4, [[(0, 2, 0.1, 0.1), (2, 3, 0.1, 0.1)]])
    assert e.value.status == lofp.EINVAL
    with pytest.raises(lofp.LofpError) as e:
        lofp.Circuit(4, [[(2, 1, 0.1, 0.1)]])
    assert e.value.status == lofp.EINVAL
    with pytest.raises(lofp.LofpError) as e:
        lofp.Circuit(40, [])
    assert e.value.status == lofp.ENOTSUP
    c = lofp.Circuit(4, [[(0, 1, 0.1, 0.1)]])
    with pytest.raises(lofp.LofpError) as e:
        c.bounds([1, -1, 0, 0], [0, 0, 0, 0])
    assert e.value.status == lofp.EINVAL


def live_cut_values(m, S, T, layers):
    """For each layer boundary t, the set of cut vectors of configurations that
    lie on at least one valid path (brute force: forward reachable from S and
    backward reachable from T)."""
    def step(confs, layer):
        out = set()
        for c in confs:
            frontier = [list(c)]
            for (a, b, _, _) in layer:
                nxt = []
                for cc in frontier:
                    N = cc[a] + cc[b]
                    for y in range(N + 1):
                        d = list(cc)
                        d[a], d[b] = y, N - y
                        nxt.append(d)
                frontier = nxt
            out.update(tuple(x) for x in frontier)
        return out

    D = len(layers)
    fwd = [{tuple(S)}]
    for l in range(D):
        fwd.append(step(fwd[-1], layers[l]))
    bwd = [None] * (D + 1)
    bwd[D] = {tuple(T)}
    for l in range(D - 1, -1, -1):
        bwd[l] = step(bwd[l + 1], layers[l])
    live = [fwd[t] & bwd[t] for t in range(D + 1)]
    return [{tuple(np.cumsum(c)[:-1]) for c in live_t} for live_t in live]


@pytest.mark.parametrize("m,D,S,seed", [(6, 3, (1, 1, 1, 1, 1, 1), 0), (6, 4, (0, 0, 4, 0, 0, 4), 1),
                                        (6, 5, (2, 0, 3, 0, 0, 3), 2), (7, 4, (1, 0, 1, 0, 1, 0, 1), 3),
                                        (8, 4, (1, 1, 1, 1, 0, 0, 0, 0), 4)])
def test_bounds_are_exact_intervals(m, D, S, seed):
    rng = np.random.default_rng(seed)
    layers = workloads.random_brickwork(m, D, np.random.Generator(np.random.PCG64(seed)))
    c = lofp.Circuit(m, layers)
    n = sum(S)
    checked = 0
    for _ in range(12):
        T = np.zeros(m, dtype=np.int32)
        for _k in range(n):
            T[rng.integers(0, m)] += 1
        lo, hi, feas = c.bounds(S, T)
        live = live_cut_values(m, S, T, layers)
        assert feas == (len(live[0]) > 0)
        if not feas:
            continue
        checked += 1
        for t in range(D + 1):
            vals = np.array(sorted(live[t]))
            for r in range(m - 1):
                seen = set(vals[:, r])
                assert min(seen) == lo[t, r] and max(seen) == hi[t, r]
                assert seen == set(range(lo[t, r], hi[t, r] + 1))
    assert checked > 0


def test_infeasible_when_photon_numbers_differ():
    wl = workloads.make("c1")
    c = lofp.Circuit(wl.m, wl.layers)
    T = wl.Ts[0].copy()
    T[0] += 1
    _, _, feas = c.bounds(wl.S, T)
    assert not feas


def _distant_layers(m, depth, rng):
    """Random layers of disjoint pairs at distance 1 to 4 (some layers hold
    only adjacent pairs, some only distant ones)."""
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


@pytest.mark.parametrize("m", [3, 5, 8, 12])
def test_distant_pairs_compile_to_the_same_unitary(m):
    """A splitter on distant modes is compiled to adjacent splitters (a chain
    of theta = pi/2 splitters bringing the lower mode next to the upper one
    and back): the compiled circuit's unitary, composed by the oracle, equals
    the given circuit's; adjacent pairs pass through unchanged."""
    import oracle
    rng = np.random.default_rng(100 + m)
    layers = _distant_layers(m, 5, rng)
    assert any(b > a + 1 for l in layers for a, b, _, _ in l)
    c = lofp.Circuit(m, layers)
    comp = c.compiled_layers()
    assert all(b == a + 1 for l in comp for a, b, _, _ in l)
    flat = [bs for l in layers for bs in l]
    cflat = [bs for l in comp for bs in l]
    assert np.abs(oracle.compose(m, flat) - oracle.compose(m, cflat)).max() < 1e-14
    # one extra splitter per step of the chain, there and back
    assert len(cflat) == len(flat) + sum(2 * (b - a - 1) for a, b, _, _ in flat)
    adjacent = [[(0, 1, 0.3, 0.4)], [(1, 2, 0.5, 0.6)]]
    assert lofp.Circuit(3, adjacent).compiled_layers() == adjacent


def test_distant_pairs_refuse_host_layer_queries():
    c = lofp.Circuit(4, [[(0, 3, 0.2, 0.1)]])
    for call in (lambda: c.light_cone(0, 0), lambda: c.bounds([1, 0, 0, 0], [0, 0, 0, 1])):
        with pytest.raises(lofp.LofpError) as e:
            call()
        assert e.value.status == lofp.ENOTSUP
