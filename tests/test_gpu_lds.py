"""GPU limited discrepancy search (paper, Section 3) against the oracle: the
budgeted exhaustive walk (same nodes, same solutions for each budget) under
both readings of a discrepancy (rank in the level's value order, or one per
departure from the level's first value), at m = 6..7 and at m = 11 (n = 100,
the wide walker variant), and the first-solution mode that raises the budget
pass by pass."""
from __future__ import annotations

import os

import numpy as np
import pytest
import torch

import msp_instances as mi
from oracle import enum as E
from oracle import lattice as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import paper_2508_08702_amd as M
    return M


@pytest.fixture(scope="module")
def ctx(M):
    c = M.Context(0)
    yield c
    c.close()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


_PREP = {}


def _prepared(m, D, seed):
    """The oracle's exact reduction of one planted instance, computed once."""
    key = (m, D, seed)
    if key not in _PREP:
        inst = mi.msp_class(m, D, seed)
        _PREP[key] = L.prepare(inst.A, inst.d)
    return _PREP[key]


@pytest.mark.parametrize("count", [0, 1])
@pytest.mark.parametrize("m,D,seed", [(6, 100, 2000), (6, 50, 2003), (7, 100, 4100),
                                      (11, 50, 5000), (11, 100, 5004), (11, 200, 5008)])
@pytest.mark.parametrize("B", [0, 1, 2, 4])
def test_budgeted_walk_matches_oracle(M, ctx, m, D, seed, B, count):
    inst = mi.msp_class(m, D, seed)
    P = _prepared(m, D, seed)
    ref = E.enumerate_prepared(P, split=6, threads=os.cpu_count() or 1, disc_budget=B, disc_count=bool(count))
    print(f"  budget {B} ({'count' if count else 'rank'}) m={m} D={D} seed={seed}: oracle {ref.nodes} nodes",
          flush=True)
    prm = M.msp_params_default(time_cap_ms=60000.0, disc_budget=B, disc_count=count)
    r = M.msp_enumerate(ctx, _dev(inst.A), _dev(inst.d), _dev(P.basis), params=prm)
    assert r.status == M.MSP_OK and r.n_found == ref.n_found
    assert np.array_equal(E.sort_rows(r.x.cpu().numpy()), ref.solutions)
    for key in ("evals", "nodes", "expansions", "leaves"):
        assert r.stats[key] == getattr(ref, key), key


@pytest.mark.parametrize("order", [0, 2])
def test_lds_mode_finds_verified_solutions(M, ctx, order):
    for m, D, seed in ((7, 100, 4102), (8, 200, 4152), (9, 50, 4500)):
        inst = mi.msp_class(m, D, seed)
        A, d = _dev(inst.A), _dev(inst.d)
        Bk = M.msp_reduce(ctx, A, d)
        r = M.msp_enumerate(ctx, A, d, Bk, params=M.msp_params_default(time_cap_ms=60000.0), mode=M.MSP_LDS,
                            order=order, cap=64)
        print(f"  lds m={m} seed={seed}: passes {r.stats['stages']} ttfs {r.stats['ttfs_ms']:.1f} ms", flush=True)
        assert r.status == M.MSP_OK and r.n_found >= 1
        assert E.verify(inst.A, inst.d, r.x.cpu().numpy())
        assert r.stats["stages"] >= 1 and r.stats["ttfs_ms"] > 0.0


def test_lds_mode_is_exhaustive_without_solutions(M, ctx):
    inst = mi.cornuejols_dawande(6, 33)
    d = inst.d.copy()
    d[0] = int(inst.A[0].astype(np.int64).sum()) + 1      # infeasible
    A, dd = _dev(inst.A), _dev(d)
    Bk = M.msp_reduce(ctx, A, dd)
    plain = M.msp_enumerate(ctx, A, dd, Bk)
    r = M.msp_enumerate(ctx, A, dd, Bk, mode=M.MSP_LDS)
    assert r.status == M.MSP_OK and r.n_found == 0 and plain.n_found == 0
    k = Bk.shape[0]
    assert r.stats["stages"] == min(k, 255) + 2          # every budget, then the unlimited walk
    assert r.stats["nodes"] >= plain.stats["nodes"]
