"""CPU oracle for the checkerboard Metropolis sweep of the 2D Ising model.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1906_06297_amd``) and never imports it.

Contents
  - ``ising_oracle.c``   plain C/OpenMP: Philox4x32-10, the threshold tables
                         (Metropolis and heat bath, Sec. 2), int8 lattice
                         init, half-sweep, sweeps, observables (paper Sec. 2,
                         Sec. 3.1, Fig. 2; Eq. (1)); the +-J spin glass named
                         in the conclusions.
  - ``exact.py``         exact results: enumeration, transfer matrix,
                         Kaufman's finite-lattice solution, Onsager, Eq. (7).
  - ``stats.py``         blocking standard errors and integrated
                         autocorrelation times.
  - ``arnet.py``         the learned proposal: masked-convolution network
                         forward and backward, absolute-value scales for
                         rounding bounds, Adam, the sampling and
                         Metropolis-Hastings uniforms and decisions.

The readings of the paper that the oracle fixes are listed at the top of
``ising_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "ising_oracle.c")]

DOMAIN_SWEEP = 0
DOMAIN_INIT = 1


def build(verbose: bool = False) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` (always recompiles)."""
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, *SOURCES, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    """Load the built oracle, building it first only if nothing is built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    L = ctypes.CDLL(LIB_PATH)
    i8p = ctypes.POINTER(ctypes.c_int8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    f64p = ctypes.POINTER(ctypes.c_double)
    c_i64, c_u64, c_u32, c_int, c_dbl = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
                                         ctypes.c_int, ctypes.c_double)
    sigs = {
        "orc_philox4x32_10": (None, [u32p, u32p, u32p]),
        "orc_site_uniform": (c_u32, [c_u64, c_u32, c_u64, c_i64]),
        "orc_thresholds": (None, [c_dbl, c_dbl, u64p]),
        "orc_thresholds_heatbath": (None, [c_dbl, c_dbl, u64p]),
        "orc_glass_sweeps": (None, [i8p, i8p, i8p, c_i64, c_dbl, c_dbl, c_u64, c_u32, c_i64, c_u64,
                                    i64p, i64p]),
        "orc_glass_observables": (None, [i8p, i8p, i8p, c_i64, i64p, i64p]),
        "orc_glass_couplings": (None, [i8p, i8p, c_i64, c_u64, c_u32]),
        "orc_sweeps_table": (None, [i8p, c_i64, u64p, c_u64, c_u32, c_i64, c_u64, i64p, i64p]),
        "orc_init": (None, [i8p, c_i64, c_u64, c_u32]),
        "orc_half_sweep": (None, [i8p, c_i64, c_int, u64p, c_u64, c_u32, c_u64]),
        "orc_observables": (None, [i8p, c_i64, i64p, i64p]),
        "orc_sweeps": (None, [i8p, c_i64, c_dbl, c_dbl, c_u64, c_u32, c_i64, c_u64, i64p, i64p]),
        "orc_batch_sweeps": (None, [i8p, i64p, i64p, f64p, ctypes.c_int32, c_dbl, u64p, u32p,
                                    c_i64, c_u64]),
        "orc_window_init": (None, [i8p, c_i64, c_i64, c_i64, c_i64, c_i64, c_u64, c_u32]),
        "orc_window_sweeps": (None, [i8p, c_i64, c_i64, c_i64, c_i64, c_i64, c_dbl, c_dbl, c_u64,
                                     c_u32, c_i64, c_u64]),
        "orc_max_threads": (c_int, []),
        "orc_set_threads": (None, [c_int]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _ptr(a: np.ndarray, ctype):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _check_L(L: int) -> None:
    if L < 4 or L % 2:
        raise ValueError(f"lattice size must be even and >= 4, got {L}")


# --------------------------------------------------------------------------- RNG
def philox4x32_10(ctr, key) -> tuple:
    """One Philox4x32-10 block (SC'11 generator) at counter ``ctr`` (4 words), key ``key`` (2)."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                            _ptr(out, ctypes.c_uint32))
    return tuple(int(v) for v in out)


def site_uniform(seed: int, stream: int, t: int, n: int) -> int:
    """The 32-bit uniform of colour-linear site ``n`` at half-sweep ``t``."""
    return int(lib().orc_site_uniform(seed, stream, t, n))


# --------------------------------------------------------------------- thresholds
RULES = ("metropolis", "heatbath")


def thresholds(beta: float, J: float, rule: str = "metropolis") -> np.ndarray:
    """T[a], a = 0..4 aligned neighbours: flip accepted iff r < T[a] (r uniform 32-bit).
    rule "metropolis": min(1, e^{-beta dE}); "heatbath": e^{-beta dE} / (e^{-beta dE} + 1)
    (Sec. 2)."""
    T = np.zeros(5, dtype=np.uint64)
    fn = {"metropolis": lib().orc_thresholds, "heatbath": lib().orc_thresholds_heatbath}[rule]
    fn(float(beta), float(J), _ptr(T, ctypes.c_uint64))
    return T


# ------------------------------------------------------------------------ lattice
def init(L: int, seed: int, stream: int = 0) -> np.ndarray:
    """Initial L x L int8 lattice (+1/-1) from the domain-1 Philox stream."""
    _check_L(L)
    s = np.zeros((L, L), dtype=np.int8)
    lib().orc_init(_ptr(s, ctypes.c_int8), L, seed, stream)
    return s


def half_sweep(s: np.ndarray, colour: int, T: np.ndarray, seed: int, stream: int, t: int) -> None:
    """In-place update of every site of ``colour`` (Sec. 2 checkerboard, Fig. 2)."""
    L = s.shape[0]
    _check_L(L)
    T = np.ascontiguousarray(T, dtype=np.uint64)
    lib().orc_half_sweep(_ptr(s, ctypes.c_int8), L, colour, _ptr(T, ctypes.c_uint64), seed,
                         stream, t)


def sweeps(s: np.ndarray, beta: float, J: float, seed: int, stream: int, nsweeps: int,
           rng_counter: int = 0, trace: bool = False, rule: str = "metropolis"):
    """In-place ``nsweeps`` full sweeps; returns (bond_trace, M_trace) if ``trace``."""
    L = s.shape[0]
    _check_L(L)
    assert s.dtype == np.int8 and s.shape == (L, L)
    if trace:
        bt = np.zeros(nsweeps, dtype=np.int64)
        mt = np.zeros(nsweeps, dtype=np.int64)
        bp, mp = _ptr(bt, ctypes.c_int64), _ptr(mt, ctypes.c_int64)
    else:
        bp = mp = None
    if rule == "metropolis":
        lib().orc_sweeps(_ptr(s, ctypes.c_int8), L, float(beta), float(J), seed, stream,
                         nsweeps, rng_counter, bp, mp)
    else:
        T = thresholds(beta, J, rule)
        lib().orc_sweeps_table(_ptr(s, ctypes.c_int8), L, _ptr(T, ctypes.c_uint64), seed, stream,
                               nsweeps, rng_counter, bp, mp)
    if trace:
        return bt, mt
    return None


def glass_sweeps(s: np.ndarray, Jr: np.ndarray, Jd: np.ndarray, beta: float, J: float, seed: int,
                 stream: int, nsweeps: int, rng_counter: int = 0, trace: bool = False):
    """+-J spin glass: in-place sweeps with bond signs Jr (to the right) and Jd
    (downwards), int8 +1/-1 arrays of the lattice's shape."""
    L = s.shape[0]
    _check_L(L)
    Jr = np.ascontiguousarray(Jr, dtype=np.int8)
    Jd = np.ascontiguousarray(Jd, dtype=np.int8)
    assert s.dtype == np.int8 and Jr.shape == Jd.shape == s.shape == (L, L)
    if trace:
        bt = np.zeros(nsweeps, dtype=np.int64)
        mt = np.zeros(nsweeps, dtype=np.int64)
        bp, mp = _ptr(bt, ctypes.c_int64), _ptr(mt, ctypes.c_int64)
    else:
        bp = mp = None
    lib().orc_glass_sweeps(_ptr(s, ctypes.c_int8), _ptr(Jr, ctypes.c_int8), _ptr(Jd, ctypes.c_int8),
                           L, float(beta), float(J), seed, stream, nsweeps, rng_counter, bp, mp)
    if trace:
        return bt, mt
    return None


def glass_couplings(L: int, seed: int, stream: int = 0) -> tuple:
    """Random bond signs (Jr, Jd) of the +-J glass from Philox domain 4."""
    _check_L(L)
    Jr = np.zeros((L, L), dtype=np.int8)
    Jd = np.zeros((L, L), dtype=np.int8)
    lib().orc_glass_couplings(_ptr(Jr, ctypes.c_int8), _ptr(Jd, ctypes.c_int8), L, seed, stream)
    return Jr, Jd


def glass_observables(s: np.ndarray, Jr: np.ndarray, Jd: np.ndarray) -> tuple:
    """(bond sum with the bond signs, M)."""
    L = s.shape[0]
    b, m = ctypes.c_int64(), ctypes.c_int64()
    lib().orc_glass_observables(_ptr(np.ascontiguousarray(s), ctypes.c_int8),
                                _ptr(np.ascontiguousarray(Jr, dtype=np.int8), ctypes.c_int8),
                                _ptr(np.ascontiguousarray(Jd, dtype=np.int8), ctypes.c_int8), L,
                                ctypes.byref(b), ctypes.byref(m))
    return int(b.value), int(m.value)


def observables(s: np.ndarray) -> tuple:
    """(bond_sum, M): bond_sum = sum over bonds of sigma_i sigma_j (E = -J*bond_sum)."""
    L = s.shape[0]
    b = ctypes.c_int64()
    m = ctypes.c_int64()
    lib().orc_observables(_ptr(np.ascontiguousarray(s), ctypes.c_int8), L, ctypes.byref(b),
                          ctypes.byref(m))
    return int(b.value), int(m.value)


def batch_sweeps(lattices: list, betas, J: float, seeds, streams, nsweeps: int,
                 rng_counter: int = 0) -> list:
    """Advance independent lattices (list of LxL int8 arrays); returns the new arrays."""
    Ls = np.array([a.shape[0] for a in lattices], dtype=np.int64)
    for L in Ls:
        _check_L(int(L))
    offsets = np.zeros(len(lattices), dtype=np.int64)
    offsets[1:] = np.cumsum(Ls * Ls)[:-1]
    flat = np.concatenate([a.reshape(-1) for a in lattices]).astype(np.int8)
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    streams = np.ascontiguousarray(streams, dtype=np.uint32)
    lib().orc_batch_sweeps(_ptr(flat, ctypes.c_int8), _ptr(offsets, ctypes.c_int64),
                           _ptr(Ls, ctypes.c_int64), _ptr(betas, ctypes.c_double),
                           len(lattices), float(J), _ptr(seeds, ctypes.c_uint64),
                           _ptr(streams, ctypes.c_uint32), nsweeps, rng_counter)
    return [flat[o:o + L * L].reshape(L, L).copy() for o, L in zip(offsets, Ls)]


def window_init(L: int, i0: int, j0: int, h: int, w: int, seed: int, stream: int = 0):
    win = np.zeros((h, w), dtype=np.int8)
    lib().orc_window_init(_ptr(win, ctypes.c_int8), L, i0, j0, h, w, seed, stream)
    return win


def window_sweeps(win: np.ndarray, L: int, i0: int, j0: int, beta: float, J: float, seed: int,
                  stream: int, nsweeps: int, rng_counter: int = 0) -> None:
    """Evolve a window in place; sites >= 2*nsweeps+1 from its edge are exact."""
    h, w = win.shape
    lib().orc_window_sweeps(_ptr(win, ctypes.c_int8), L, i0, j0, h, w, float(beta), float(J),
                            seed, stream, nsweeps, rng_counter)


def max_threads() -> int:
    return int(lib().orc_max_threads())


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))
