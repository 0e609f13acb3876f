"""First solutions from A and d by limited discrepancy search over shuffled
copies of the instance (paper, Section 4: the method on randomly reordered
input bases), through the C ABI: every returned row is one of the oracle's
solutions in the caller's variable order, one copy reproduces the LDS mode on
the given basis, an infeasible instance ends with the exhaustive pass, and
the arguments are checked."""
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


def _oracle_set(inst):
    P = L.prepare(inst.A, inst.d)
    ref = E.enumerate_prepared(P, split=6, threads=os.cpu_count() or 1)
    return {tuple(x) for x in ref.solutions}


@pytest.mark.parametrize("m,D,seed", [(6, 200, 2004), (7, 200, 4102)])
def test_one_copy_is_the_lds_mode_on_the_given_order(M, ctx, m, D, seed):
    inst = mi.msp_class(m, D, seed)
    sols = _oracle_set(inst)
    A, d = _dev(inst.A), _dev(inst.d)
    prm = M.msp_params_default(time_cap_ms=60000.0, restarts=1)
    print(f"  one copy m={m} D={D} seed={seed}: oracle solutions {len(sols)}", flush=True)
    r = M.msp_solve_first(ctx, A, d, params=prm)
    assert r.status == M.MSP_OK and r.n_found >= 1
    assert r.stats["copy"] == 0 and r.stats["copies"] == 1
    Bk = M.msp_reduce(ctx, A, d, prm)
    q = M.msp_enumerate(ctx, A, d, Bk, params=M.msp_params_default(time_cap_ms=60000.0), mode=M.MSP_LDS, cap=64)
    assert q.status == M.MSP_OK and q.stats["stages"] == r.stats["stages"]
    assert {tuple(x) for x in r.x.cpu().numpy()} <= sols
    if len(sols) == 1:
        assert np.array_equal(r.x.cpu().numpy(), q.x.cpu().numpy())


@pytest.mark.parametrize("bkz", [0, 10])
def test_shuffled_copies_return_oracle_solutions(M, ctx, bkz):
    hits = []
    for m, D, seed in ((5, 50, 1), (6, 50, 2003), (6, 100, 2001), (7, 100, 4101), (7, 50, 4100)):
        inst = mi.msp_class(m, D, seed)
        sols = _oracle_set(inst)
        A, d = _dev(inst.A), _dev(inst.d)
        for R, rs in ((4, 1), (16, 7)):
            prm = M.msp_params_default(time_cap_ms=60000.0, restarts=R, restart_seed=rs, bkz_block=bkz)
            print(f"  copies={R} seed={rs} bkz={bkz} m={m} D={D} seed={seed}", flush=True)
            r = M.msp_solve_first(ctx, A, d, params=prm, cap=64)
            assert r.status == M.MSP_OK and r.n_found >= 1
            x = r.x.cpu().numpy()
            assert x.shape[0] == min(r.n_found, 64)
            assert E.verify(inst.A, inst.d, x)
            assert {tuple(row) for row in x} <= sols
            assert r.stats["copies"] == R and 0 <= r.stats["copy"] < R
            assert r.stats["reduce_ms"] > 0.0 and r.stats["ttfs_ms"] >= r.stats["reduce_ms"]
            hits.append(r.stats["copy"])
    assert any(h > 0 for h in hits)      # rows found on shuffled copies came back in the given order


def test_one_row_capacity_keeps_the_hit(M, ctx):
    # several lanes can hit in the same pass: with room for one row the call
    # may report MSP_E_CAPACITY, and the row it returns is still a solution
    inst = mi.msp_class(5, 50, 1)
    sols = _oracle_set(inst)
    for R, rs in ((1, 1), (8, 5), (8, 9)):
        prm = M.msp_params_default(time_cap_ms=60000.0, restarts=R, restart_seed=rs)
        r = M.msp_solve_first(ctx, _dev(inst.A), _dev(inst.d), params=prm, cap=1)
        assert r.status in (M.MSP_OK, M.MSP_E_CAPACITY) and r.n_found >= 1
        x = r.x.cpu().numpy()
        assert x.shape[0] == 1 and tuple(x[0]) in sols
        assert (r.status == M.MSP_E_CAPACITY) == (r.n_found > 1)
        assert r.stats["copy"] >= 0 and r.stats["ttfs_ms"] > 0.0
    A, d = _dev(inst.A), _dev(inst.d)
    q = M.msp_enumerate(ctx, A, d, M.msp_reduce(ctx, A, d), params=M.msp_params_default(time_cap_ms=60000.0),
                        mode=M.MSP_LDS, cap=1)
    assert q.status in (M.MSP_OK, M.MSP_E_CAPACITY) and q.n_found >= 1 and q.stats["ttfs_ms"] > 0.0
    assert tuple(q.x.cpu().numpy()[0]) in sols


def test_learned_roots_on_reduced_copies(M, ctx):
    M.msp_model_init(ctx, 8)
    for m, D, seed in ((6, 100, 2000), (7, 200, 4102)):
        inst = mi.msp_class(m, D, seed)
        sols = _oracle_set(inst)
        prm = M.msp_params_default(time_cap_ms=60000.0, restarts=6, restart_seed=3, bkz_block=12)
        r = M.msp_solve_first(ctx, _dev(inst.A), _dev(inst.d), order=M.MSP_LEARNED, params=prm)
        assert r.status == M.MSP_OK and r.n_found >= 1 and r.stats["copies"] == 6
        assert {tuple(x) for x in r.x.cpu().numpy()} <= sols
        assert r.stats["ordering_ms"] > 0.0


def test_time_cap_ends_the_search(M, ctx):
    # an m=9 instance needs far more than 1 ms of search: the cap is reached
    inst = mi.msp_class(9, 100, 4504)
    prm = M.msp_params_default(time_cap_ms=1.0, restarts=4)
    r = M.msp_solve_first(ctx, _dev(inst.A), _dev(inst.d), params=prm)
    assert r.status == M.MSP_E_TIMEOUT
    if r.n_found:
        assert E.verify(inst.A, inst.d, r.x.cpu().numpy())


def test_infeasible_instance_ends_exhaustive(M, ctx):
    inst = mi.cornuejols_dawande(6, 31)
    d_np = inst.d.copy()
    d_np[0] = int(inst.A[0].astype(np.int64).sum()) + 1
    r = M.msp_solve_first(ctx, _dev(inst.A), _dev(d_np), params=M.msp_params_default(time_cap_ms=60000.0, restarts=4))
    assert r.status == M.MSP_OK and r.n_found == 0 and r.stats["copy"] == -1 and r.stats["copies"] == 4


def test_restart_arguments(M, ctx):
    inst = mi.msp_class(5, 100, 3)
    A, d = _dev(inst.A), _dev(inst.d)
    for R in (0, 65):
        with pytest.raises(M.MspError) as ei:
            M.msp_solve_first(ctx, A, d, params=M.msp_params_default(restarts=R))
        assert ei.value.code == M.MSP_E_ARG
