"""CPU pins of the oracle's limited discrepancy search (paper, Section 3): a
path may take a value other than its level's first zig-zag value at most B
times.  Pinned by an independent pure-Python recursion on small instances,
by B >= depth reducing to the plain search, and by monotonicity in B."""
from __future__ import annotations

import numpy as np
import pytest

import msp_instances as mi
from oracle import enum as E
from oracle import lattice as L
from oracle import roots as RT


def _python_lds(P, B, eps=E.EPS):
    """Counters and solutions of the budgeted search, written out directly."""
    k, dim, n = P.k, P.dim, P.n
    R = float(n + 1)
    bound = R * (1.0 + eps)
    u = [0] * k
    cnt = [0, 0, 0, 0]
    sols = []

    def level(t, wpar, lpar, topzero, dsc):
        y = RT.centre(P, u, t)
        c = -y
        if topzero:
            u1, s, onedir, dr = 0, 1, True, 1
        else:
            u1 = int(np.rint(c))
            s = 1 if float(u1) - c <= 0.0 else -1
            onedir, dr = False, 0
        off, val = 0, u1
        while True:
            if B >= 0 and val != u1 and dsc >= B:
                break
            x = float(val) + y
            l = x * x * float(P.beta[t]) + lpar
            cnt[0] += 1
            if l > bound:
                break
            cnt[1] += 1
            w = x * P.bhat[t] + wpar
            u[t] = val
            if t > 0:
                if l > float(np.cumsum(np.abs(w))[-1]) * (1.0 + eps):
                    if onedir:
                        break
                    off = RT._zig_next(off, s)
                    val = u1 + off
                    onedir = True
                    dr = 1 if float(val) - c > 0.0 else -1
                    continue
                cnt[2] += 1
                level(t - 1, w, l, topzero and val == 0, dsc + (val != u1))
            else:
                cnt[3] += 1
                v = np.array(u, dtype=np.int64) @ P.basis
                if abs(v[n]) == 1:
                    v = v * v[n]
                    if np.all(np.abs(v[:n]) == 1):
                        x01 = ((v[:n] + 1) // 2).astype(np.uint8)
                        if np.array_equal(x01.astype(np.int64) @ P.A.T.astype(np.int64), P.d):
                            sols.append(x01)
            if onedir:
                val += dr
            else:
                off = RT._zig_next(off, s)
                val = u1 + off
        u[t] = 0

    level(k - 1, np.zeros(dim), 0.0, True, 0)
    return cnt, E.sort_rows(np.array(sols, dtype=np.uint8).reshape(-1, n))


@pytest.mark.parametrize("seed", [1001, 1002, 1003])
@pytest.mark.parametrize("B", [0, 1, 2, 4])
def test_budgeted_search_matches_python_recursion(seed, B):
    inst = mi.single_small(seed)
    P = L.prepare(inst.A, inst.d)
    cnt, sols = _python_lds(P, B)
    for split in (0, 3):
        r = E.enumerate_prepared(P, split=split, disc_budget=B)
        assert [r.evals, r.nodes, r.expansions, r.leaves] == cnt, (split, B)
        assert np.array_equal(r.solutions, sols)


@pytest.mark.parametrize("m,D,seed", [(4, 50, 7), (5, 100, 11)])
def test_budget_is_monotone_and_reaches_the_plain_search(m, D, seed):
    inst = mi.msp_class(m, D, seed)
    P = L.prepare(inst.A, inst.d)
    full = E.enumerate_prepared(P, split=4)
    prev_nodes, prev_set = -1, set()
    for B in (0, 1, 2, 3, 5, 8):
        r = E.enumerate_prepared(P, split=4, disc_budget=B)
        s = {tuple(x) for x in r.solutions}
        assert r.nodes >= prev_nodes and prev_set <= s
        assert s <= {tuple(x) for x in full.solutions}
        prev_nodes, prev_set = r.nodes, s
    r = E.enumerate_prepared(P, split=4, disc_budget=P.k)
    assert (r.evals, r.nodes, r.expansions, r.leaves) == (full.evals, full.nodes, full.expansions, full.leaves)
    assert np.array_equal(r.solutions, full.solutions)
