"""GPU batch path (msp_solve_batch) on the uneven batch of market split
instances: m drawn from 5..8 per instance, n = 10(m-1), D by thirds.

The batch reduces every instance in one LLL launch and then enumerates each
one, so its bases, solution sets and search-tree counters must equal those
of the single-instance calls; solution sets must equal the oracle's: for
m <= 6 the oracle runs here, for m = 7 and 8 its sets are stored
(tests/golden/batch_sets.json, written by tests/golden/make_batch_sets.py from
oracle/ alone).
"""
from __future__ import annotations

import os

import numpy as np
import pytest
import torch

import msp_instances as mi
from oracle import enum as E

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


@pytest.fixture(scope="module")
def batch():
    return mi.mixed_batch()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _oracle(inst):
    return E.solve(inst.A, inst.d, split=6, threads=os.cpu_count() or 1)[1]


def _run_batch(M, ctx, insts, params=None, **kw):
    print(f"  gpu batch of {len(insts)} seeds {insts[0].seed}..{insts[-1].seed}", flush=True)
    prm = params if params is not None else M.msp_params_default(time_cap_ms=60000.0)
    r = M.msp_solve_batch(ctx, [_dev(i.A) for i in insts], [_dev(i.d) for i in insts], params=prm, **kw)
    torch.cuda.synchronize()
    return r


def test_batch_equals_single_calls(M, ctx, batch):
    r = _run_batch(M, ctx, batch)
    assert r.rc == M.MSP_OK
    prm = M.msp_params_default(time_cap_ms=60000.0)
    for i, inst in enumerate(batch):
        assert r.status[i] == M.MSP_OK
        A, d = _dev(inst.A), _dev(inst.d)
        Bk = M.msp_reduce(ctx, A, d, prm)
        s = M.msp_enumerate(ctx, A, d, Bk, params=prm, cap=1024)
        assert s.status == M.MSP_OK
        assert r.n_found[i] == s.n_found
        xb = E.sort_rows(r.x[i].cpu().numpy())
        xs = E.sort_rows(s.x.cpu().numpy())
        assert np.array_equal(xb, xs), f"seed {inst.seed}"
        for key in ("evals", "nodes", "expansions", "leaves", "k"):
            assert r.stats[i][key] == s.stats[key], (inst.seed, key)
        assert E.verify(inst.A, inst.d, xb)
        assert any(np.array_equal(row, inst.x_planted) for row in xb)


def test_batch_oracle_parity_small_m(M, ctx, batch):
    small = _small(batch, 24)
    assert len(small) == 24
    r = _run_batch(M, ctx, small)
    assert r.rc == M.MSP_OK
    for i, inst in enumerate(small):
        ref = _oracle(inst)
        x = E.sort_rows(r.x[i].cpu().numpy())
        assert r.n_found[i] == ref.n_found, f"seed {inst.seed}"
        assert np.array_equal(x, ref.solutions), f"seed {inst.seed}"


def test_batch_oracle_parity_large_m(M, ctx, batch):
    import json
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_sets.json")
    stored = json.load(open(path))["instances"]
    large = [inst for inst in batch if inst.m >= 7]
    assert len(large) == len(stored) and {str(i.seed) for i in large} == set(stored)
    r = _run_batch(M, ctx, large)
    assert r.rc == M.MSP_OK
    for i, inst in enumerate(large):
        g = stored[str(inst.seed)]
        assert (g["m"], g["n"], g["D"]) == (inst.m, inst.n, int(inst.D))
        x = E.sort_rows(r.x[i].cpu().numpy())
        assert r.n_found[i] == g["n_found"], f"seed {inst.seed}"
        assert np.array_equal(x, E.sort_rows(np.array(g["solutions"], dtype=np.uint8).reshape(-1, inst.n))), \
            f"seed {inst.seed}"


def _small(batch, count):
    return [inst for inst in batch if inst.m <= 6][:count]


def test_batch_per_instance_status(M, ctx, batch):
    good = _small(batch, 3)
    bad_A = good[0].A.copy()
    bad_A[1] = bad_A[0]                                 # rank A < m
    bad_d = bad_A.astype(np.int64) @ good[0].x_planted.astype(np.int64)
    As = [_dev(good[0].A), _dev(bad_A), _dev(good[1].A), _dev(good[2].A)]
    ds = [_dev(good[0].d), _dev(bad_d), _dev(good[1].d), _dev(good[2].d)]
    prm = M.msp_params_default(time_cap_ms=60000.0)
    r = M.msp_solve_batch(ctx, As, ds, params=prm)
    torch.cuda.synchronize()
    assert r.status[1] == M.MSP_E_RANK and r.n_found[1] == 0 and r.x[1].shape[0] == 0
    assert r.rc == M.MSP_E_RANK
    for i, inst in ((0, good[0]), (2, good[1]), (3, good[2])):
        assert r.status[i] == M.MSP_OK
        assert r.n_found[i] == _oracle(inst).n_found


def test_batch_capacity_and_first(M, ctx, batch):
    insts = _small(batch, 6)
    ref = [_oracle(i) for i in insts]
    r = _run_batch(M, ctx, insts, cap=1)
    for i, inst in enumerate(insts):
        want = M.MSP_E_CAPACITY if ref[i].n_found > 1 else M.MSP_OK
        assert r.status[i] == want and r.n_found[i] == ref[i].n_found
        assert r.x[i].shape[0] == 1 and E.verify(inst.A, inst.d, r.x[i].cpu().numpy())
    r = _run_batch(M, ctx, insts, mode=M.MSP_FIRST, cap=64)
    assert r.rc == M.MSP_OK
    for i, inst in enumerate(insts):
        x = r.x[i].cpu().numpy()
        assert 1 <= x.shape[0] <= r.n_found[i] and E.verify(inst.A, inst.d, x)
        assert r.stats[i]["ttfs_ms"] >= 0.0


def test_batch_bad_arguments(M, ctx, batch):
    inst = batch[0]
    with pytest.raises(M.MspError):
        # m > n
        M.msp_solve_batch(ctx, [_dev(inst.A.T.copy())], [_dev(np.zeros(inst.n, np.int64))])
    with pytest.raises(ValueError):
        M.msp_solve_batch(ctx, [], [])


def test_autotune_picks_a_candidate_and_keeps_results(M, ctx, batch):
    tune = mi.mixed_batch(range(3900, 3932))[:8]          # tuning seeds, disjoint from the batch
    best, pts = M.msp_autotune(ctx, [_dev(i.A) for i in tune], [_dev(i.d) for i in tune],
                               params=M.msp_params_default(time_cap_ms=60000.0))
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert [p[0] for p in pts] == [c * cus for c in (128, 256, 512, 1024, 2048)]
    assert all(p[1] == M.MSP_OK and p[2] > 0 for p in pts)
    assert best.target_roots == min(pts, key=lambda p: p[2])[0] and best.split_depth == -1
    insts = batch[:12]
    tuned = _run_batch(M, ctx, insts, params=best)
    plain = _run_batch(M, ctx, insts)
    for i in range(len(insts)):
        assert tuned.status[i] == plain.status[i] == M.MSP_OK
        assert np.array_equal(E.sort_rows(tuned.x[i].cpu().numpy()), E.sort_rows(plain.x[i].cpu().numpy()))
        for key in ("evals", "nodes", "expansions", "leaves"):
            assert tuned.stats[i][key] == plain.stats[i][key], key


def test_tuned_roots_are_kept_per_shape_and_used_by_the_batch(M, ctx, batch):
    """msp_autotune keeps the fastest candidate of each (m, n bucket) group of
    its tuning batch; msp_solve_batch uses it for instances of those shapes,
    and the results do not change."""
    tune = mi.mixed_batch(range(3900, 3932))[:8]
    shapes = {(i.m, i.n) for i in tune}
    best, pts = M.msp_autotune(ctx, [_dev(i.A) for i in tune], [_dev(i.d) for i in tune],
                               params=M.msp_params_default(time_cap_ms=60000.0))
    cands = {p[0] for p in pts}
    for m, n in shapes:
        t = M.msp_tune_lookup(ctx, m, n)
        assert t in cands, (m, n, t)
        assert M.msp_tune_lookup(ctx, m, n, mode=M.MSP_FIRST) == 0     # only the tuned mode
    assert M.msp_tune_lookup(ctx, 3, 20) == 0                          # a shape not in the tuning batch
    insts = [i for i in batch if (i.m, i.n) in shapes][:6]
    assert insts
    tuned = _run_batch(M, ctx, insts)                                  # default params: the table applies
    fixed = _run_batch(M, ctx, insts, params=M.msp_params_default(target_roots=4096))
    for i, inst in enumerate(insts):
        assert tuned.status[i] == fixed.status[i] == M.MSP_OK
        assert tuned.stats[i]["roots"] != 0
        assert np.array_equal(E.sort_rows(tuned.x[i].cpu().numpy()), E.sort_rows(fixed.x[i].cpu().numpy()))
        for key in ("evals", "nodes", "expansions", "leaves"):
            assert tuned.stats[i][key] == fixed.stats[i][key], key
    with pytest.raises(M.MspError):
        M.msp_tune_lookup(ctx, 0, 20)


def test_batch_with_bkz_keeps_the_solution_sets(M, ctx, batch):
    """p.bkz_block applies to every instance of a batch (each kernel basis
    BKZ-reduced after the shared LLL launch): the solution sets are those of
    the LLL-only batch; the tree may change.  A block size of 1 is rejected."""
    insts = [i for i in batch if i.m <= 6][:6]
    plain = _run_batch(M, ctx, insts)
    bkz = _run_batch(M, ctx, insts, params=M.msp_params_default(time_cap_ms=60000.0, bkz_block=8))
    for i, inst in enumerate(insts):
        assert plain.status[i] == bkz.status[i] == M.MSP_OK
        assert np.array_equal(E.sort_rows(plain.x[i].cpu().numpy()), E.sort_rows(bkz.x[i].cpu().numpy()))
        assert E.verify(inst.A, inst.d, bkz.x[i].cpu().numpy())
    assert any(plain.stats[i]["nodes"] != bkz.stats[i]["nodes"] for i in range(len(insts)))
    with pytest.raises(M.MspError):
        _run_batch(M, ctx, insts[:2], params=M.msp_params_default(bkz_block=1))
