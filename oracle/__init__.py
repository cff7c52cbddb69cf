"""CPU oracle for <T|U_P|S> through beam-splitter circuits.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product library
(``paper_2510_26408_amd``) never imports, links or executes anything here, and
this package imports nothing from the product.

What it computes (the plain definition that the Feynman path sum reaches, Sec.
II and the Appendix of the paper):

    <T|U_P|S> = Per(U[T,S]) / sqrt(prod s_i! prod t_j!)

with U the product of embedded 2x2 matrices of Eq. (bs_matrix) in application
order, rows of U = output modes, columns = input modes.  The heavy lifting
(matrix composition, Ryser's permanent in long double, the single-BS permanent
of the Appendix, the unpruned path sum of Eq. (1)) is plain C in
``lofp_oracle.c``; this module adds ctypes marshalling and two small pure-Python
forms used only on tiny inputs:

* :func:`evolve` -- the full output state of S, one beam splitter at a time
  (Eq. (1) with equal intermediate configurations summed as they appear);
* :func:`path_count_bruteforce` -- enumeration of every valid path.

Circuits are passed as a flat list of beam splitters in application order,
``[(a, b, theta, phi), ...]``, where ``a`` is the upper mode (BS port 1).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, Iterable, List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lofp_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liblofp_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP) into oracle/_build."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.orc_permanent_ryser.argtypes = [ctypes.c_int, dp, dp, dp]
    lib.orc_permanent_brute.argtypes = [ctypes.c_int, dp, dp]
    lib.orc_bs_amplitude.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, dp]
    lib.orc_fock_amplitude.argtypes = [ctypes.c_int, dp, ip, ip, dp]
    lib.orc_compose.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip, dp, dp, dp]
    lib.orc_amplitude.argtypes = [ctypes.c_int, ip, ip, ctypes.c_int, ip, ip, dp, dp, dp, dp]
    lib.orc_amplitudes.argtypes = [ctypes.c_int, ip, ctypes.c_int, ip, ctypes.c_int, ip, ip, dp, dp,
                                   dp, dp, ctypes.c_int, ip]
    lib.orc_pathsum.argtypes = [ctypes.c_int, ip, ip, ctypes.c_int, ip, ip, dp, dp, dp, dp]
    for f in ("orc_permanent_ryser", "orc_permanent_brute", "orc_bs_amplitude", "orc_compose", "orc_fock_amplitude",
              "orc_amplitude", "orc_amplitudes", "orc_pathsum"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _circ_arrays(circuit: Sequence[Tuple[int, int, float, float]]):
    ma = np.ascontiguousarray([c[0] for c in circuit], dtype=np.int32)
    mb = np.ascontiguousarray([c[1] for c in circuit], dtype=np.int32)
    th = np.ascontiguousarray([c[2] for c in circuit], dtype=np.float64)
    ph = np.ascontiguousarray([c[3] for c in circuit], dtype=np.float64)
    return ma, mb, th, ph


def permanent(a: np.ndarray, with_bound: bool = False):
    """Ryser's formula (Gray-code order, long-double accumulation)."""
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[0]
    buf = np.ascontiguousarray(np.stack([a.real, a.imag], axis=-1).reshape(-1))
    out = np.zeros(2)
    eb = np.zeros(1)
    rc = _load().orc_permanent_ryser(n, _dptr(buf), _dptr(out), _dptr(eb))
    if rc:
        raise ValueError("permanent: bad size")
    v = complex(out[0], out[1])
    return (v, float(eb[0])) if with_bound else v


def permanent_bruteforce(a: np.ndarray) -> complex:
    """Sum over all n! permutations (the definition); n <= 10."""
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[0]
    buf = np.ascontiguousarray(np.stack([a.real, a.imag], axis=-1).reshape(-1))
    out = np.zeros(2)
    if _load().orc_permanent_brute(n, _dptr(buf), _dptr(out)):
        raise ValueError("permanent_bruteforce: n too large")
    return complex(out[0], out[1])


def bs_amplitude(theta: float, phi: float, x1: int, x2: int, y1: int, y2: int) -> complex:
    """Appendix: <y1,y2|BS|x1,x2> = Per(repeated BS entries)/sqrt(x1!x2!y1!y2!)."""
    out = np.zeros(2)
    if _load().orc_bs_amplitude(theta, phi, x1, x2, y1, y2, _dptr(out)):
        raise ValueError("bs_amplitude: bad occupations")
    return complex(out[0], out[1])


def bs_sector(theta: float, phi: float, N: int) -> np.ndarray:
    """(N+1)x(N+1) matrix W[y1, x1] of the N-photon sector of one BS."""
    W = np.zeros((N + 1, N + 1), dtype=np.complex128)
    for x1 in range(N + 1):
        for y1 in range(N + 1):
            W[y1, x1] = bs_amplitude(theta, phi, x1, N - x1, y1, N - y1)
    return W


def bs_sector_hp(theta: float, phi: float, N: int, dps: int = 40) -> np.ndarray:
    """The N-photon sector W[y1, x1] from the Appendix's closed-form sum
    (with the denominator (x2 - y1 + t)!, reading 1), evaluated in `dps`
    decimal digits with mpmath and rounded to complex128 at the end: a
    reference for large N, where the same sum in FP64 cancels badly."""
    import mpmath
    old = mpmath.mp.dps
    mpmath.mp.dps = dps
    try:
        th, ph = mpmath.mpf(theta), mpmath.mpf(phi)
        c, s = mpmath.cos(th), mpmath.sin(th)
        f = [mpmath.factorial(k) for k in range(N + 1)]
        W = np.zeros((N + 1, N + 1), dtype=np.complex128)
        for x1 in range(N + 1):
            x2 = N - x1
            for y1 in range(N + 1):
                y2 = N - y1
                tot = mpmath.mpf(0)
                for t in range(max(0, y1 - x2), min(x1, y1) + 1):
                    term = c ** (x2 - y1 + 2 * t) * s ** (x1 + y1 - 2 * t) / (f[t] * f[y1 - t] * f[x1 - t] * f[x2 - y1 + t])
                    tot += -term if (y1 - t) % 2 else term
                mag = mpmath.sqrt(f[x1] * f[x2] * f[y1] * f[y2]) * tot
                z = mag * mpmath.expj(ph * (x1 - y1))
                W[y1, x1] = complex(z)
        return W
    finally:
        mpmath.mp.dps = old


def fock_amplitude(U: np.ndarray, S, T) -> complex:
    """Per(U[T,S]) / sqrt(prod s! prod t!) for any square matrix U (rows = outputs)."""
    U = np.asarray(U, dtype=np.complex128)
    m = U.shape[0]
    buf = np.ascontiguousarray(np.stack([U.real, U.imag], axis=-1).reshape(-1))
    S = np.ascontiguousarray(S, dtype=np.int32)
    T = np.ascontiguousarray(T, dtype=np.int32)
    out = np.zeros(2)
    if _load().orc_fock_amplitude(m, _dptr(buf), _iptr(S), _iptr(T), _dptr(out)):
        raise ValueError("fock_amplitude: bad input")
    return complex(out[0], out[1])


def compose(m: int, circuit) -> np.ndarray:
    """U = L_K ... L_1 (m x m complex, rows = outputs)."""
    ma, mb, th, ph = _circ_arrays(circuit)
    out = np.zeros(2 * m * m)
    if _load().orc_compose(m, len(circuit), _iptr(ma), _iptr(mb), _dptr(th), _dptr(ph), _dptr(out)):
        raise ValueError("compose: bad circuit")
    return (out[0::2] + 1j * out[1::2]).reshape(m, m)


def amplitude(m: int, S, T, circuit, with_bound: bool = False):
    """<T|U_P|S> = Per(U[T,S]) / sqrt(prod s! prod t!)."""
    S = np.ascontiguousarray(S, dtype=np.int32)
    T = np.ascontiguousarray(T, dtype=np.int32)
    ma, mb, th, ph = _circ_arrays(circuit)
    out = np.zeros(2)
    eb = np.zeros(1)
    if _load().orc_amplitude(m, _iptr(S), _iptr(T), len(circuit), _iptr(ma), _iptr(mb), _dptr(th),
                             _dptr(ph), _dptr(out), _dptr(eb)):
        raise ValueError("amplitude: bad input")
    v = complex(out[0], out[1])
    return (v, float(eb[0])) if with_bound else v


def amplitudes(m: int, S, Ts, circuit, nthreads: int = 1, with_bound: bool = False):
    """Batch of patterns Ts (B x m) for one S; OpenMP over patterns.

    Returns (complex128[B], threads_used) or, with ``with_bound``,
    (complex128[B], float64[B] error bounds, threads_used)."""
    S = np.ascontiguousarray(S, dtype=np.int32)
    Ts = np.ascontiguousarray(Ts, dtype=np.int32).reshape(-1, m)
    ma, mb, th, ph = _circ_arrays(circuit)
    B = Ts.shape[0]
    out = np.zeros(2 * B)
    eb = np.zeros(max(B, 1))
    used = np.zeros(1, dtype=np.int32)
    if _load().orc_amplitudes(m, _iptr(S), B, _iptr(Ts), len(circuit), _iptr(ma), _iptr(mb),
                              _dptr(th), _dptr(ph), _dptr(out), _dptr(eb), int(nthreads),
                              _iptr(used)):
        raise ValueError("amplitudes: bad input")
    amps = out[0::2] + 1j * out[1::2]
    if with_bound:
        return amps, eb[:B].copy(), int(used[0])
    return amps, int(used[0])


def pathsum(m: int, S, T, circuit):
    """Eq. (1) by explicit enumeration (no pruning).  Returns (amp, n_valid_paths)."""
    S = np.ascontiguousarray(S, dtype=np.int32)
    T = np.ascontiguousarray(T, dtype=np.int32)
    ma, mb, th, ph = _circ_arrays(circuit)
    out = np.zeros(2)
    cnt = np.zeros(1)
    if _load().orc_pathsum(m, _iptr(S), _iptr(T), len(circuit), _iptr(ma), _iptr(mb), _dptr(th),
                           _dptr(ph), _dptr(out), _dptr(cnt)):
        raise ValueError("pathsum: bad input")
    return complex(out[0], out[1]), float(cnt[0])


def evolve(m: int, S, circuit) -> Dict[Tuple[int, ...], complex]:
    """Full output state of |S>: apply each BS to every configuration and sum
    equal configurations.  Pure Python; small m and n only."""
    state: Dict[Tuple[int, ...], complex] = {tuple(int(s) for s in S): 1.0 + 0j}
    cache: Dict[Tuple[int, int, int, int], complex] = {}
    for g, (a, b, th, ph) in enumerate(circuit):
        new: Dict[Tuple[int, ...], complex] = {}
        for conf, amp in state.items():
            x1, x2 = conf[a], conf[b]
            N = x1 + x2
            for y1 in range(N + 1):
                key = (g, x1, x2, y1)
                if key not in cache:
                    cache[key] = bs_amplitude(th, ph, x1, x2, y1, N - y1)
                c = list(conf)
                c[a], c[b] = y1, N - y1
                c = tuple(c)
                new[c] = new.get(c, 0j) + amp * cache[key]
        state = new
    return state


def evolve_hp(m: int, S, circuit, dps: int = 40) -> Dict[Tuple[int, ...], complex]:
    """Full output state of |S> like :func:`evolve`, with each splitter's
    sectors from :func:`bs_sector_hp` (40-digit closed form) instead of the
    permanent, so many photons per mode stay affordable; small m only."""
    state: Dict[Tuple[int, ...], complex] = {tuple(int(s) for s in S): 1.0 + 0j}
    sectors: Dict[Tuple[int, int], np.ndarray] = {}
    for g, (a, b, th, ph) in enumerate(circuit):
        new: Dict[Tuple[int, ...], complex] = {}
        for conf, amp in state.items():
            x1, x2 = conf[a], conf[b]
            N = x1 + x2
            if (g, N) not in sectors:
                sectors[(g, N)] = bs_sector_hp(th, ph, N, dps)
            W = sectors[(g, N)]
            for y1 in range(N + 1):
                c = list(conf)
                c[a], c[b] = y1, N - y1
                c = tuple(c)
                new[c] = new.get(c, 0j) + amp * W[y1, x1]
        state = new
    return state


def path_count_bruteforce(m: int, S, T, circuit) -> int:
    """Number of valid paths of Eq. (1): sequences of per-BS output splits that
    start at S and end at T.  Counting form of :func:`evolve`."""
    counts: Dict[Tuple[int, ...], int] = {tuple(int(s) for s in S): 1}
    for (a, b, _th, _ph) in circuit:
        new: Dict[Tuple[int, ...], int] = {}
        for conf, w in counts.items():
            N = conf[a] + conf[b]
            for y1 in range(N + 1):
                c = list(conf)
                c[a], c[b] = y1, N - y1
                c = tuple(c)
                new[c] = new.get(c, 0) + w
        counts = new
    return counts.get(tuple(int(t) for t in T), 0)


def absolute_form(m: int, S, T, circuit) -> float:
    """Sum over the valid paths of Eq. (1) of the product of |Re W| + |Im W|
    of each splitter's transition amplitude: the scale against which the
    rounding of path products is bounded.  Same dictionary evolution as
    :func:`evolve`, with the 1-norm of each weight; small m and n only."""
    state: Dict[Tuple[int, ...], float] = {tuple(int(s) for s in S): 1.0}
    for (a, b, th, ph) in circuit:
        new: Dict[Tuple[int, ...], float] = {}
        for conf, w in state.items():
            x1, x2 = conf[a], conf[b]
            N = x1 + x2
            for y1 in range(N + 1):
                t = bs_amplitude(th, ph, x1, x2, y1, N - y1)
                c = list(conf)
                c[a], c[b] = y1, N - y1
                c = tuple(c)
                new[c] = new.get(c, 0.0) + w * (abs(t.real) + abs(t.imag))
        state = new
    return state.get(tuple(int(t) for t in T), 0.0)


def all_patterns(m: int, n: int) -> List[Tuple[int, ...]]:
    """Every occupation tuple of n photons in m modes (C(m+n-1, n) of them)."""
    out: List[Tuple[int, ...]] = []

    def rec(i, left, cur):
        if i == m - 1:
            out.append(tuple(cur + [left]))
            return
        for k in range(left, -1, -1):
            rec(i + 1, left - k, cur + [k])

    rec(0, n, [])
    return out
