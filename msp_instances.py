"""Seeded synthetic market-split instances (inputs only).

This module draws the inputs that both the CPU oracle and the GPU path
consume. It holds none of the method's arithmetic: no embedding, no
reduction, no enumeration -- only random draws and the planted right-hand
side d = A x*.

Instance shapes follow the market split classes of the paper (Section 1 and
Section 3): n = 10 (m - 1) variables, m constraints, entries of A uniform in
[0, D).  The paper's benchmark instances are not available here, so the
right-hand side is *planted*: x* is drawn uniformly from {0,1}^n and
d = A x*, which makes every instance feasible, as the paper's instances are
by construction.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Instance:
    """One market-split feasibility instance A x = d, x in {0,1}^n."""

    A: np.ndarray  # int32 (m, n), row-major
    d: np.ndarray  # int64 (m,)
    x_planted: np.ndarray  # uint8 (n,), a known solution
    seed: int
    D: int

    @property
    def m(self) -> int:
        return int(self.A.shape[0])

    @property
    def n(self) -> int:
        return int(self.A.shape[1])


def planted(m: int, n: int, D: int, seed: int) -> Instance:
    """Draw A ~ U[0, D)^{m x n} (int32), x* ~ U{0,1}^n, d = A x* (int64).

    The draw order (A first, then x*) is fixed so that a seed names one
    instance on every machine.
    """
    if m < 1 or n < 1 or D < 1:
        raise ValueError("m, n and D must be positive")
    rng = np.random.default_rng(seed)
    A = rng.integers(0, D, size=(m, n), dtype=np.int32)
    x = rng.integers(0, 2, size=n).astype(np.uint8)
    d = A.astype(np.int64) @ x.astype(np.int64)
    return Instance(A=np.ascontiguousarray(A), d=d.astype(np.int64), x_planted=x, seed=seed, D=D)


def msp_class(m: int, D: int, seed: int) -> Instance:
    """Planted instance of the class (m, 10(m-1), D)."""
    return planted(m, 10 * (m - 1), D, seed)


def cornuejols_dawande(m: int, seed: int, D: int = 100) -> Instance:
    """The original generator: d_i = floor(sum_j a_ij / 2) (Section 1).

    These instances are usually infeasible; x_planted is all zeros and is
    *not* a solution.  Used only for exhaustive-run workloads.
    """
    n = 10 * (m - 1)
    rng = np.random.default_rng(seed)
    A = rng.integers(0, D, size=(m, n), dtype=np.int32)
    d = A.astype(np.int64).sum(axis=1) // 2
    return Instance(A=A, d=d.astype(np.int64), x_planted=np.zeros(n, np.uint8), seed=seed, D=D)


# ---- the workloads -----------------------------------------------------------

def single_small(seed: int = 1001) -> Instance:
    """m=3, n=20, D=100: small enough for a 2^20 brute-force cross-check."""
    return planted(3, 20, 100, seed)


def m6_set(seeds=range(2000, 2016)) -> list[Instance]:
    """16 planted instances of the class (6, 50, 100)."""
    return [planted(6, 50, 100, s) for s in seeds]


def mixed_batch(seeds=range(3000, 3096)) -> list[Instance]:
    """Uneven batch: m drawn uniformly from {5,6,7,8} (first draw of the
    instance's generator), n = 10(m-1), D = 50/100/200 by thirds of the batch."""
    seeds = list(seeds)
    out = []
    third = max(1, len(seeds) // 3)
    for i, s in enumerate(seeds):
        rng = np.random.default_rng(s)
        m = int(rng.integers(5, 9))
        D = (50, 100, 200)[min(2, i // third)]
        n = 10 * (m - 1)
        A = rng.integers(0, D, size=(m, n), dtype=np.int32)
        x = rng.integers(0, 2, size=n).astype(np.uint8)
        d = A.astype(np.int64) @ x.astype(np.int64)
        out.append(Instance(A=A, d=d, x_planted=x, seed=s, D=D))
    return out


def class_set(m: int, seeds) -> list[Instance]:
    """Four instances per D in (50, 100, 200), seeds consumed in order."""
    seeds = list(seeds)
    out = []
    for i, s in enumerate(seeds):
        D = (50, 100, 200)[min(2, i * 3 // len(seeds))]
        out.append(msp_class(m, D, s))
    return out


def m9_eval(seeds=range(4500, 4512)) -> list[Instance]:
    return class_set(9, seeds)


def m11_eval(seeds=range(5000, 5012)) -> list[Instance]:
    return class_set(11, seeds)


def train_set(seeds=range(4000, 4192)) -> list[Instance]:
    """m in {6,7,8} x D in {50,100,200}: 64 instances per m, D cycling."""
    out = []
    seeds = list(seeds)
    per_m = len(seeds) // 3
    for i, s in enumerate(seeds):
        m = 6 + min(2, i // per_m)
        D = (50, 100, 200)[i % 3]
        out.append(msp_class(m, D, s))
    return out


def signed_planted(m: int, n: int, lo: int, hi: int, seed: int) -> Instance:
    """A ~ U[lo, hi)^{m x n} (entries of either sign), x* ~ U{0,1}^n,
    d = A x* (the paper allows negative entries in A and d, Section 2)."""
    rng = np.random.default_rng(seed)
    A = rng.integers(lo, hi, size=(m, n), dtype=np.int32)
    x = rng.integers(0, 2, size=n).astype(np.uint8)
    d = A.astype(np.int64) @ x.astype(np.int64)
    return Instance(A=np.ascontiguousarray(A), d=d.astype(np.int64), x_planted=x, seed=seed, D=hi - lo)


@dataclass(frozen=True)
class BoxInstance:
    """A x = d with l_j <= x_j <= u_j (integers); x_planted lies in the box."""

    A: np.ndarray      # int32 (m, n)
    d: np.ndarray      # int64 (m,)
    lo: np.ndarray     # int32 (n,)
    hi: np.ndarray     # int32 (n,)
    x_planted: np.ndarray  # int64 (n,)
    seed: int


def box_planted(m: int, n: int, a_lo: int, a_hi: int, l_lo: int, l_hi: int, r_max: int, seed: int) -> BoxInstance:
    """A ~ U[a_lo, a_hi)^{m x n}, lower bounds l ~ U[l_lo, l_hi), widths
    r ~ U{1..r_max}, upper bounds u = l + r, x* ~ U{l..u} per coordinate,
    d = A x*."""
    rng = np.random.default_rng(seed)
    A = rng.integers(a_lo, a_hi, size=(m, n), dtype=np.int32)
    lo = rng.integers(l_lo, l_hi, size=n).astype(np.int32)
    r = rng.integers(1, r_max + 1, size=n).astype(np.int32)
    hi = (lo + r).astype(np.int32)
    x = lo.astype(np.int64) + np.array([rng.integers(0, int(ri) + 1) for ri in r], dtype=np.int64)
    d = A.astype(np.int64) @ x
    return BoxInstance(A=np.ascontiguousarray(A), d=d, lo=lo, hi=hi, x_planted=x, seed=seed)
