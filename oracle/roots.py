"""CPU oracle, part 6: subtree roots, their features and their labels.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Tree partitioning (paper, Section 4): the levels k-1 .. L of the enumeration
tree of Algorithm 1 are walked depth first with the same rules as the
recursive enumerator (zig-zag next(), l2 bound R(1+eps), Hoelder test of
Thm 2 with the one-direction cut, sign symmetry broken while every higher u
is zero); every node of level L that passes both tests is a subtree root,
listed in the order depth-first search meets it.  Pure Python, for small
trees only.

Root features (a project addition for ordering the roots; the definitions
below are the specification, written out in FP64 and stored as float32):
for root r at level L with prefix u_{k-1..L}, partial norm l and projected
vector w, R = n + 1, and per level j the centre y_j = sum_{i>j} u_i mu_{i,j}
(one running sum over i = j+1 .. k-1) and the zig-zag rank of u_j (its index in the sequence
u1, u1+s, u1-s, u1+2s, ... of next(), or u_j itself while every higher u is
zero):
    0 l/R            1 l/||w||_1 (0 if w = 0)   2 min(||w||_inf, 4)/4
    3 mean rank      4 fraction of ranks > 0    5 min(max rank, 8)/8
    6 fraction of u_j != 0   7 mean |u_j|       8 min(max |u_j|, 4)/4
    9 x_L^2 beta_L/R (x_L = u_L + y_L)          10 min(|x_L|, 2)/2
    11 (L/k) ln(max((R-l)/R, 1e-6))/8           12 r/roots
    13 fraction of coordinates with |w_j| > 17/16   14 L/k   15 m/16
The label of a root is 1 iff some solution's coefficient vector (sign chosen
as the enumeration meets it: first non-zero coefficient from the top
positive) has that root's prefix.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import enum as E

NFEAT = 16


@dataclass
class Root:
    u: list        # length k; entries below level L are 0
    l: float
    w: np.ndarray  # float64 (dim,)


def centre(P, u, t: int) -> float:
    """y_t = sum_{i=t+1}^{k-1} u_i mu_{i,t} (Algorithm 1) as one running sum in
    that index order, starting at 0.0."""
    y = 0.0
    for i in range(t + 1, P.k):
        y = y + float(u[i]) * float(P.mu[i, t])
    return y


def _zig_next(off: int, s: int) -> int:
    if off == 0:
        return s
    if (off > 0) == (s > 0):
        return -off
    return -off + s


def roots_dfs(P, split: int, eps: float = E.EPS, hoelder: bool = True, onedir_cut: bool = True):
    """Subtree roots at level L = k - split, in depth-first order."""
    k, dim = P.k, P.dim
    L = k - split
    assert 1 <= split <= k - 1
    R = float(P.n + 1)
    bound = R * (1.0 + eps)
    beta, bhat = P.beta, P.bhat
    u = [0] * k
    out: list[Root] = []

    def level(t, wpar, lpar, topzero):
        y = centre(P, u, t)
        c = -y
        if topzero:
            u1, s, onedir, dr = 0, 1, True, 1
        else:
            u1 = int(np.rint(c))
            s = 1 if float(u1) - c <= 0.0 else -1
            onedir, dr = False, 0
        off = 0
        val = u1
        while True:
            x = float(val) + y
            l = x * x * float(beta[t]) + lpar
            if l > bound:
                break
            w = x * bhat[t] + wpar
            u[t] = val
            fail = hoelder and l > float(np.cumsum(np.abs(w))[-1]) * (1.0 + eps)  # sequential sum
            if fail and not onedir_cut:
                pass
            elif fail:
                if onedir:
                    break
                off = _zig_next(off, s)
                val = u1 + off
                onedir = True
                dr = 1 if float(val) - c > 0.0 else -1
                continue
            elif t == L:
                out.append(Root(u=list(u), l=l, w=w.copy()))
            else:
                level(t - 1, w, l, topzero and val == 0)
            if onedir:
                val += dr
            else:
                off = _zig_next(off, s)
                val = u1 + off
        u[t] = 0

    level(k - 1, np.zeros(dim), 0.0, True)
    return out


def zigzag_rank(uj: int, y: float, topzero: bool) -> int:
    """Index of uj in the zig-zag sequence of a level with centre -y."""
    if topzero:
        return uj
    c = -y
    u1 = int(np.rint(c))
    s = 1 if float(u1) - c <= 0.0 else -1
    o = uj - u1
    if o == 0:
        return 0
    return 2 * abs(o) - 1 if (o > 0) == (s > 0) else 2 * abs(o)


def features(P, roots, L: int) -> np.ndarray:
    """float32 (len(roots), 16) per the definitions in the module docstring."""
    k, dim, m = P.k, P.dim, P.m
    R = float(P.n + 1)
    beta = P.beta
    F = np.zeros((len(roots), NFEAT), dtype=np.float64)
    lv = float(k - L)
    for r, rt in enumerate(roots):
        u = rt.u
        ranks, tz = [], True
        xL = 0.0
        for j in range(k - 1, L - 1, -1):
            y = centre(P, u, j)
            ranks.append(zigzag_rank(u[j], y, tz))
            if j == L:
                xL = float(u[j]) + y
            tz = tz and u[j] == 0
        pre = [u[j] for j in range(L, k)]
        a = np.abs(rt.w)
        l1 = float(np.sum(a))
        F[r, 0] = rt.l / R
        F[r, 1] = rt.l / l1 if l1 > 0 else 0.0
        F[r, 2] = min(float(np.max(a)), 4.0) / 4.0
        F[r, 3] = sum(ranks) / lv
        F[r, 4] = sum(1 for q in ranks if q > 0) / lv
        F[r, 5] = min(max(ranks), 8) / 8.0
        F[r, 6] = sum(1 for q in pre if q != 0) / lv
        F[r, 7] = sum(abs(q) for q in pre) / lv
        F[r, 8] = min(max(abs(q) for q in pre), 4) / 4.0
        F[r, 9] = (xL * xL) * float(beta[L]) / R
        F[r, 10] = min(abs(xL), 2.0) / 2.0
        F[r, 11] = (L / k) * math.log(max((R - rt.l) / R, 1e-6)) / 8.0
        F[r, 12] = r / len(roots)
        F[r, 13] = float(np.sum(a > 1.0625)) / dim
        F[r, 14] = L / k
        F[r, 15] = m / 16.0
    return F.astype(np.float32)


def coefficients(P, x) -> np.ndarray:
    """Integer coefficient vector u with sum_i u_i b_i = v, where v is the
    lattice vector of solution x (v_j = 2 x_j - 1, v_n = 1), signed so that
    its first non-zero entry from the top (i = k-1) is positive."""
    B = np.asarray(P.basis, dtype=np.int64)
    v = np.concatenate([2 * np.asarray(x, dtype=np.int64) - 1, [1]])
    sol, *_ = np.linalg.lstsq(B.T.astype(np.float64), v.astype(np.float64), rcond=None)
    u = np.rint(sol).astype(np.int64)
    if not np.array_equal(u @ B, v):
        raise ArithmeticError("solution vector is not in the kernel lattice")
    nz = np.nonzero(u)[0]
    if nz.size and u[nz[-1]] < 0:
        u = -u
    return u


def labels(P, roots, L: int, solutions) -> np.ndarray:
    """uint8 per root: 1 iff a solution lies in its subtree."""
    k = P.k
    prefixes = {tuple(int(c) for c in coefficients(P, x)[L:k]) for x in np.asarray(solutions)}
    return np.array([1 if tuple(rt.u[L:k]) in prefixes else 0 for rt in roots], dtype=np.uint8)
