"""Seeded synthetic workloads (circuits, input and output patterns).

This module holds input generation only: random beam-splitter parameters,
occupation patterns and the sampling rules that pick them.  It contains none
of the amplitude arithmetic and imports nothing else from this package, so the
GPU library, the tests and the CPU oracle can all draw the same inputs from it.

The paper's benchmarks use synthetic planar circuits of locally connected beam
splitters with theta and phi drawn uniformly (Sec. III); there is no dataset.
The five workloads below follow that recipe:

=====  ===========================================================================
c1     m=8, photons in modes 0..3, depth-4 brickwork, 1 collision-free pattern
c2     m=16, photons in even modes, depth-8 brickwork, 4096 collision-free patterns
c3     m=20, two photons in modes 0,4,8,12,16, depth 6, 2048 bunched patterns
c4     served mix: m in {12,16,24}, n=m/2 on even modes, depth in {4,6,8}
c5     m=32, photons in even modes, depth-6 brickwork, 512 collision-free patterns
=====  ===========================================================================

Brickwork: layer l (0-based) holds the pairs (0,1),(2,3),... when l is even and
(1,2),(3,4),... when l is odd; the lower-numbered mode of a pair is the BS's
upper port.  Parameters are drawn layer by layer, pair by pair in ascending
mode order, theta ~ U(0, pi/2) then phi ~ U(0, 2 pi), from numpy's PCG64.
Output patterns are drawn after the circuit from the same generator.

Collision-free patterns: n distinct modes drawn uniformly, redrawn until the
k-th smallest output mode lies within ``dist`` of the k-th smallest input mode
for every k (``dist`` = circuit depth).  Bunched patterns (c3): every photon of
source mode s lands uniformly in the set of modes that s can reach through the
circuit's pairs, and the pattern is the histogram.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

Layer = List[Tuple[int, int, float, float]]


@dataclasses.dataclass
class Workload:
    name: str
    m: int
    S: np.ndarray                 # int32[m]
    layers: List[Layer]           # per layer: (a, b, theta, phi), a < b
    Ts: np.ndarray                # int32[B, m]
    seed: int
    note: str = ""

    @property
    def n(self) -> int:
        return int(self.S.sum())

    @property
    def depth(self) -> int:
        return len(self.layers)

    @property
    def batch(self) -> int:
        return int(self.Ts.shape[0])

    def flat_circuit(self) -> List[Tuple[int, int, float, float]]:
        return [bs for layer in self.layers for bs in layer]

    @property
    def n_bs(self) -> int:
        return sum(len(l) for l in self.layers)


def brickwork_pairs(m: int, depth: int) -> List[List[Tuple[int, int]]]:
    return [[(a, a + 1) for a in range(l % 2, m - 1, 2)] for l in range(depth)]


def random_brickwork(m: int, depth: int, rng: np.random.Generator) -> List[Layer]:
    layers: List[Layer] = []
    for pairs in brickwork_pairs(m, depth):
        layer: Layer = []
        for (a, b) in pairs:
            theta = float(rng.uniform(0.0, math.pi / 2))
            phi = float(rng.uniform(0.0, 2 * math.pi))
            layer.append((a, b, theta, phi))
        layers.append(layer)
    return layers


def photons_even_modes(m: int) -> np.ndarray:
    S = np.zeros(m, dtype=np.int32)
    S[0::2] = 1
    return S


def sample_collision_free(rng: np.random.Generator, S: np.ndarray, dist: int) -> np.ndarray:
    m = S.shape[0]
    n = int(S.sum())
    src = np.repeat(np.arange(m), S)
    while True:
        out = np.sort(rng.choice(m, n, replace=False))
        if np.all(np.abs(out - src) <= dist):
            T = np.zeros(m, dtype=np.int32)
            T[out] = 1
            return T


def reach_set(layers: Sequence[Layer], m: int, src: int) -> List[int]:
    """Modes a photon entering at ``src`` can occupy after the whole circuit:
    a mode joins the set whenever a pair touches the set."""
    cur = {src}
    for layer in layers:
        nxt = set(cur)
        for (a, b, _t, _p) in layer:
            if a in cur or b in cur:
                nxt.add(a)
                nxt.add(b)
        cur = nxt
    return sorted(cur)


def sample_bunched(rng: np.random.Generator, S: np.ndarray, layers: Sequence[Layer]) -> np.ndarray:
    m = S.shape[0]
    T = np.zeros(m, dtype=np.int32)
    for s in range(m):
        if S[s] == 0:
            continue
        cone = reach_set(layers, m, s)
        for _ in range(int(S[s])):
            T[cone[int(rng.integers(0, len(cone)))]] += 1
    return T


def make(name: str, seed: int = 0, batch: Optional[int] = None) -> Workload:
    """Build one of the named workloads.  ``batch`` overrides the pattern count
    (tests use small batches of the same distribution)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if name == "c1":
        m, D = 8, 4
        S = np.zeros(m, dtype=np.int32)
        S[:4] = 1
        layers = random_brickwork(m, D, rng)
        B = 1 if batch is None else batch
        Ts = np.stack([sample_collision_free(rng, S, D) for _ in range(B)])
        note = "m=8 n=4 D=4 brickwork, collision-free pattern(s), |sorted out - sorted in| <= 4"
    elif name == "c2":
        m, D = 16, 8
        S = photons_even_modes(m)
        layers = random_brickwork(m, D, rng)
        B = 4096 if batch is None else batch
        Ts = np.stack([sample_collision_free(rng, S, D) for _ in range(B)])
        note = "m=16 n=8 D=8 brickwork, collision-free patterns, |sorted out - sorted in| <= 8"
    elif name == "c3":
        m, D = 20, 6
        S = np.zeros(m, dtype=np.int32)
        S[0::4] = 2
        layers = random_brickwork(m, D, rng)
        B = 2048 if batch is None else batch
        Ts = np.stack([sample_bunched(rng, S, layers) for _ in range(B)])
        note = "m=20 n=10 (2 photons in modes 0,4,..,16) D=6 brickwork, bunched patterns"
    elif name == "c5":
        m, D = 32, 6
        S = photons_even_modes(m)
        layers = random_brickwork(m, D, rng)
        B = 512 if batch is None else batch
        Ts = np.stack([sample_collision_free(rng, S, D) for _ in range(B)])
        note = "m=32 n=16 D=6 brickwork, collision-free patterns, |sorted out - sorted in| <= 6"
    else:
        raise ValueError(f"unknown workload {name!r}")
    return Workload(name=name, m=m, S=S, layers=layers, Ts=Ts.astype(np.int32), seed=seed, note=note)


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    m: int
    S: np.ndarray
    layers: List[Layer]
    T: np.ndarray


def served_requests(count: int, rate_hz: float, seed: int = 0) -> List[Request]:
    """c4: Poisson arrivals at ``rate_hz``; m uniform in {12,16,24}, n = m/2
    single photons in the even modes, depth uniform in {4,6,8}, a fresh circuit
    and one collision-free pattern (|sorted out - sorted in| <= depth) each."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    reqs: List[Request] = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate_hz)) if rate_hz > 0 else 0.0
        m = int(rng.choice([12, 16, 24]))
        D = int(rng.choice([4, 6, 8]))
        S = photons_even_modes(m)
        layers = random_brickwork(m, D, rng)
        T = sample_collision_free(rng, S, D)
        reqs.append(Request(rid=i, arrival_s=t, m=m, S=S, layers=layers, T=T))
    return reqs
