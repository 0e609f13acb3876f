"""CPU oracle, part 3: Python driver for the recursive enumerator.

TEST INFRASTRUCTURE ONLY (see the package docstring).

``solve(A, d)`` runs steps 1-4 of Algorithm 1 (exact LLL, kernel extraction,
exact Gram-Schmidt rounded to float64, R = (n+1) r_max^2) and the recursive
enumeration in ``enum_ref.c``; it returns the sorted set of binary solutions
together with the search counters.
"""
from __future__ import annotations

import ctypes as C
import os
import time
from dataclasses import dataclass, field

import numpy as np

from . import lattice

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_enum_ref.so")
_lib = None

EPS = 1e-9  # relative slack on both pruning tests (solutions lie on the l2 bound)


class _Args(C.Structure):
    _fields_ = [
        ("k", C.c_int), ("dim", C.c_int), ("m", C.c_int), ("n", C.c_int),
        ("bhat", C.c_void_p), ("mu", C.c_void_p), ("beta", C.c_void_p),
        ("basis", C.c_void_p), ("A", C.c_void_p), ("d", C.c_void_p),
        ("R", C.c_double), ("eps", C.c_double),
        ("rmax", C.c_int), ("hoelder", C.c_int), ("onedir", C.c_int), ("mode", C.c_int),
        ("split", C.c_int), ("nthreads", C.c_int),
        ("cap", C.c_int64), ("time_cap_s", C.c_double),
        ("sol", C.c_void_p), ("n_found", C.c_void_p), ("counters", C.c_void_p),
        ("level_counts", C.c_void_p), ("n_roots", C.c_void_p), ("timed_out", C.c_void_p),
        ("cvec", C.c_void_p), ("disc_budget", C.c_int), ("disc_count", C.c_int),
    ]


def _load():
    global _lib
    if _lib is None:
        src = os.path.join(_HERE, "enum_ref.c")
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
            from . import build as _b
            _b.build()
        lib = C.CDLL(_LIB_PATH)
        lib.orc_enumerate.argtypes = [C.POINTER(_Args)]
        lib.orc_enumerate.restype = C.c_int
        _lib = lib
    return _lib


@dataclass
class Result:
    solutions: np.ndarray  # uint8 (count, n), rows sorted lexicographically
    n_found: int
    evals: int
    nodes: int
    expansions: int
    leaves: int
    n_roots: int
    seconds: float
    timed_out: bool
    threads: int
    level_counts: np.ndarray | None = None  # (k, 3): evals, nodes, expansions per level
    extra: dict = field(default_factory=dict)


def sort_rows(x: np.ndarray) -> np.ndarray:
    """Lexicographic row sort (solution sets are compared as sorted arrays)."""
    x = np.asarray(x, dtype=np.uint8)
    if x.shape[0] == 0:
        return x
    idx = np.lexsort(x.T[::-1])
    return x[idx]


def enumerate_prepared(P: lattice.Prepared, *, split: int = 0, threads: int = 1,
                       mode: str = "all", cap: int = 1 << 16, hoelder: bool = True,
                       onedir: bool = True, eps: float = EPS, time_cap_s: float = 0.0,
                       level_counts: bool = False, disc_budget: int = -1,
                       disc_count: bool = False) -> Result:
    """Enumerate every v in the kernel lattice with ||v||_inf <= r_max and
    v_n = r_max (each solution once) on the basis held by ``P`` (binary:
    r_max = 1)."""
    lib = _load()
    k, dim, m, n = P.k, P.dim, P.m, P.n
    bhat = np.ascontiguousarray(P.bhat, dtype=np.float64)
    mu = np.ascontiguousarray(P.mu, dtype=np.float64)
    beta = np.ascontiguousarray(P.beta, dtype=np.float64)
    basis = np.ascontiguousarray(P.basis, dtype=np.int64)
    A = np.ascontiguousarray(P.A, dtype=np.int32)
    d = np.ascontiguousarray(P.d, dtype=np.int64)
    sol = np.zeros((max(cap, 1), n), dtype=np.uint8)
    n_found = np.zeros(1, dtype=np.int64)
    counters = np.zeros(4, dtype=np.int64)
    lvl = np.zeros((k, 3), dtype=np.int64) if level_counts else None
    n_roots = np.zeros(1, dtype=np.int64)
    timed_out = np.zeros(1, dtype=np.int32)
    a = _Args()
    a.k, a.dim, a.m, a.n = k, dim, m, n
    a.bhat, a.mu, a.beta = bhat.ctypes.data, mu.ctypes.data, beta.ctypes.data
    a.basis, a.A, a.d = basis.ctypes.data, A.ctypes.data, d.ctypes.data
    a.R = float((n + 1) * P.rmax * P.rmax)  # (n+1) r_max^2
    a.eps = eps
    a.rmax = int(P.rmax)
    cvec = None if P.cvec is None else np.ascontiguousarray(P.cvec, dtype=np.int64)
    a.cvec = cvec.ctypes.data if cvec is not None else None
    a.disc_budget = int(disc_budget)
    a.disc_count = int(bool(disc_count))
    a.hoelder = int(hoelder)
    a.onedir = int(onedir)
    a.mode = 1 if mode == "first" else 0
    a.split = int(split)
    a.nthreads = int(threads)
    a.cap = int(cap)
    a.time_cap_s = float(time_cap_s)
    a.sol, a.n_found, a.counters = sol.ctypes.data, n_found.ctypes.data, counters.ctypes.data
    a.level_counts = lvl.ctypes.data if lvl is not None else None
    a.n_roots, a.timed_out = n_roots.ctypes.data, timed_out.ctypes.data
    t0 = time.perf_counter()
    rc = lib.orc_enumerate(C.byref(a))
    dt = time.perf_counter() - t0
    if rc != 0:
        raise RuntimeError(f"orc_enumerate failed ({rc})")
    nf = int(n_found[0])
    sols = sort_rows(sol[: min(nf, cap)])
    return Result(solutions=sols, n_found=nf, evals=int(counters[0]), nodes=int(counters[1]),
                  expansions=int(counters[2]), leaves=int(counters[3]), n_roots=int(n_roots[0]),
                  seconds=dt, timed_out=bool(timed_out[0]), threads=int(threads),
                  level_counts=lvl)


def solve(A, d, *, N: int = lattice.DEFAULT_N, r=None, **kw) -> tuple[lattice.Prepared, Result]:
    """Steps 1-4 of Algorithm 1 plus the enumeration (r: upper bounds)."""
    P = lattice.prepare(A, d, N=N, r=r)
    return P, enumerate_prepared(P, **kw)


def verify(A, d, X, r=None) -> bool:
    """Independent exact check that every row x of X satisfies 0 <= x <= r
    (binary when r is None) and A x = d."""
    X = np.asarray(X)
    if X.size == 0:
        return True
    hi = 1 if r is None else np.asarray(r, dtype=np.int64)[None, :]
    if not np.all((X.astype(np.int64) >= 0) & (X.astype(np.int64) <= hi)):
        return False
    return bool(np.all(X.astype(np.int64) @ np.asarray(A, dtype=np.int64).T == np.asarray(d, dtype=np.int64)[None, :]))
