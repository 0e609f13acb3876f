"""CPU pins of the oracle's limited discrepancy search (paper, Section 3) under
both readings of a discrepancy: "rank", where the ranks of a path's values in
their levels' value orders (u1, u1+s, u1-s, ...; 0, 1, 2, ... on top-zero
levels) sum to at most the budget B, and "count", where each value other than
its level's first costs one, so a path departs from the heuristic's choice at
most B times.  Pinned by an independent pure-Python recursion on small
instances; by the solution set of each budget being exactly the solutions
whose own path, recovered from the solution vector's basis coordinates, is
within B; by a large budget reducing to the plain search; and by
monotonicity in B."""
from __future__ import annotations

import numpy as np
import pytest

import msp_instances as mi
from oracle import enum as E
from oracle import lattice as L
from oracle import roots as RT


def _rank(val, u1, s, topzero):
    """Position of val in its level's value order."""
    if topzero:
        return val
    o = val - u1
    if o == 0:
        return 0
    return 2 * abs(o) - 1 if (o > 0) == (s > 0) else 2 * abs(o)


def _cost(rank, count):
    return (1 if rank > 0 else 0) if count else rank


def _python_lds(P, B, eps=E.EPS, count=False):
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
            rank = _cost(_rank(val, u1, s, topzero), count)
            if B >= 0 and dsc + rank > B:
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
                level(t - 1, w, l, topzero and val == 0, dsc + rank)
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


@pytest.mark.parametrize("count", [False, True])
@pytest.mark.parametrize("seed", [1001, 1002, 1003])
@pytest.mark.parametrize("B", [0, 1, 2, 4])
def test_budgeted_search_matches_python_recursion(seed, B, count):
    inst = mi.single_small(seed)
    P = L.prepare(inst.A, inst.d)
    cnt, sols = _python_lds(P, B, count=count)
    for split in (0, 3):
        r = E.enumerate_prepared(P, split=split, disc_budget=B, disc_count=count)
        assert [r.evals, r.nodes, r.expansions, r.leaves] == cnt, (split, B)
        assert np.array_equal(r.solutions, sols)


@pytest.mark.parametrize("count", [False, True])
@pytest.mark.parametrize("m,D,seed", [(4, 50, 7), (5, 100, 11)])
def test_budget_is_monotone_and_reaches_the_plain_search(m, D, seed, count):
    inst = mi.msp_class(m, D, seed)
    P = L.prepare(inst.A, inst.d)
    full = E.enumerate_prepared(P, split=4)
    prev_nodes, prev_set = -1, set()
    for B in (0, 1, 2, 3, 5, 8):
        r = E.enumerate_prepared(P, split=4, disc_budget=B, disc_count=count)
        s = {tuple(x) for x in r.solutions}
        assert r.nodes >= prev_nodes and prev_set <= s
        assert s <= {tuple(x) for x in full.solutions}
        prev_nodes, prev_set = r.nodes, s
    r = E.enumerate_prepared(P, split=4, disc_budget=1 << 20, disc_count=count)
    assert (r.evals, r.nodes, r.expansions, r.leaves) == (full.evals, full.nodes, full.expansions, full.leaves)
    assert np.array_equal(r.solutions, full.solutions)


def _path_ranks(P, x):
    """Ranks of the values on the path that leads to solution x, top level
    first: u solves u B = v with v = (2x - 1, 1) (the enumerated sign has a
    positive top nonzero u); the centres along the path follow from u alone."""
    v = np.concatenate([2 * x.astype(np.int64) - 1, [1]])
    B = np.asarray(P.basis, dtype=np.int64)
    u = np.rint(np.linalg.lstsq(B.T.astype(np.float64), v.astype(np.float64), rcond=None)[0]).astype(np.int64)
    assert np.array_equal(u @ B, v)
    if u[np.nonzero(u)[0][-1]] < 0:
        u = -u
    out, topzero = [], True
    for t in range(P.k - 1, -1, -1):
        c = -RT.centre(P, [int(e) for e in u], t)
        u1 = int(np.rint(c))
        out.append(_rank(int(u[t]), u1, 1 if float(u1) - c <= 0.0 else -1, topzero))
        topzero = topzero and u[t] == 0
    return out


# instances with a solution whose path takes a value of rank 2 or more, where
# counting ranks and counting departures from u1 give different budgets
@pytest.mark.parametrize("count", [False, True])
@pytest.mark.parametrize("m,D,seed", [(5, 50, 1), (5, 50, 2), (5, 50, 14)])
def test_each_budget_finds_exactly_the_solutions_within_it(m, D, seed, count):
    inst = mi.msp_class(m, D, seed)
    P = L.prepare(inst.A, inst.d)
    full = E.enumerate_prepared(P, split=4, threads=4)
    paths = {tuple(x): _path_ranks(P, x) for x in full.solutions}
    assert any(max(r) >= 2 for r in paths.values())
    costs = {x: sum(_cost(q, count) for q in r) for x, r in paths.items()}
    assert len(set(costs.values())) >= 2                 # the budgets separate the solutions
    for B in range(0, max(costs.values()) + 2):
        r = E.enumerate_prepared(P, split=4, threads=4, disc_budget=B, disc_count=count)
        assert {tuple(x) for x in r.solutions} == {x for x, c in costs.items() if c <= B}, B


@pytest.mark.parametrize("m,D,seed", [(5, 50, 1), (5, 50, 2)])
def test_the_two_readings_differ_where_a_path_takes_a_later_value(m, D, seed):
    """The count reading charges a rank-2 value once, the rank reading twice,
    so some budget separates the two solution sets on these instances."""
    inst = mi.msp_class(m, D, seed)
    P = L.prepare(inst.A, inst.d)
    full = E.enumerate_prepared(P, split=4, threads=4)
    paths = [_path_ranks(P, x) for x in full.solutions]
    differ = False
    for B in range(0, 6):
        a = E.enumerate_prepared(P, split=4, threads=4, disc_budget=B)
        b = E.enumerate_prepared(P, split=4, threads=4, disc_budget=B, disc_count=True)
        sa, sb = {tuple(x) for x in a.solutions}, {tuple(x) for x in b.solutions}
        assert sa <= sb                      # a rank is never below its count
        assert a.nodes <= b.nodes
        differ = differ or sa != sb
    assert differ and any(max(r) >= 2 for r in paths)
