"""GPU parity: libmsp (through its C ABI) against the CPU oracle.

The GPU enumerates on the oracle's exactly reduced basis, so besides equal
solution sets the search-tree counters must agree: the centre and partial
norm recurrences are evaluated in the same order without fused operations,
so the l2 decisions are identical, and the Hoelder decisions differ only if
an l1 norm falls within rounding of its threshold.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import msp_instances as mi
from oracle import brute as B
from oracle import enum as E
from oracle import lattice as L

pytestmark = pytest.mark.gpu

GS_TOL = 1e-9  # relative agreement of Gram-Schmidt data with exact rationals


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


def _gpu_enum(M, ctx, inst, P, **kw):
    prm = M.msp_params_default(time_cap_ms=kw.pop("time_cap_ms", 60000.0))
    for key in ("split_depth", "hoelder", "onedir", "target_roots", "eps"):
        if key in kw:
            setattr(prm, key, kw.pop(key))
    print(f"  gpu enumerate m={inst.m} n={inst.n} seed={inst.seed} params split={prm.split_depth}", flush=True)
    r = M.msp_enumerate(ctx, _dev(inst.A), _dev(inst.d), _dev(P.basis), params=prm, **kw)
    torch.cuda.synchronize()
    return r, E.sort_rows(r.x.cpu().numpy())


def _check_gs(M, ctx, P):
    bh, mu, beta = M.msp_gram_schmidt(ctx, _dev(P.basis))
    bh, mu, beta = bh.cpu().numpy(), mu.cpu().numpy(), beta.cpu().numpy()
    gs = P.gs
    assert np.all(np.abs(beta - P.beta) <= GS_TOL * P.beta)
    for i in range(P.k):
        assert mu[i, i] == 1.0 and np.all(mu[i, i + 1:] == 0.0)
        for j in range(i):
            ex = float(gs.mu(i, j))
            assert abs(mu[i, j] - ex) <= GS_TOL * max(1.0, abs(ex))
        assert np.max(np.abs(bh[i] - P.bhat[i])) <= GS_TOL * np.max(np.abs(P.bhat[i]))


@pytest.mark.parametrize("seed,m,D", [(1001, 3, 100), (2000, 6, 100), (4500, 9, 50), (5000, 11, 50)])
def test_gram_schmidt_parity(M, ctx, seed, m, D):
    inst = mi.msp_class(m, D, seed) if m != 3 else mi.single_small(seed)
    P = L.prepare(inst.A, inst.d)
    _check_gs(M, ctx, P)


def test_config1_all_solutions_and_counts(M, ctx):
    inst = mi.single_small()
    P = L.prepare(inst.A, inst.d)
    ref = E.enumerate_prepared(P)
    bf = B.brute_force(inst.A, inst.d)
    for split in (0, 3, 17, -1):
        r, x = _gpu_enum(M, ctx, inst, P, split_depth=split)
        assert r.status == M.MSP_OK
        assert x.shape == bf.shape and (x == bf).all()
        st = r.stats
        assert (st["evals"], st["nodes"], st["expansions"], st["leaves"]) == (ref.evals, ref.nodes, ref.expansions, ref.leaves)


@pytest.mark.parametrize("seed", list(range(2000, 2016)))
def test_config2_m6_sets_and_counts(M, ctx, seed):
    inst = mi.planted(6, 50, 100, seed)
    P = L.prepare(inst.A, inst.d)
    ref = E.enumerate_prepared(P, split=8, threads=4)
    r, x = _gpu_enum(M, ctx, inst, P, split_depth=8)
    assert r.status == M.MSP_OK
    assert x.shape == ref.solutions.shape and (x == ref.solutions).all()
    assert any((row == inst.x_planted).all() for row in x)
    st = r.stats
    assert (st["evals"], st["nodes"], st["expansions"]) == (ref.evals, ref.nodes, ref.expansions)


@pytest.mark.parametrize("m,n,D,seed", [(2, 20, 5, 3), (2, 24, 5, 8), (1, 28, 10000, 3), (4, 22, 10, 103), (5, 40, 50, 11)])
def test_many_solution_instances(M, ctx, m, n, D, seed):
    inst = mi.planted(m, n, D, seed)
    P = L.prepare(inst.A, inst.d)
    ref = E.enumerate_prepared(P, split=4, threads=4, cap=1 << 20)
    r, x = _gpu_enum(M, ctx, inst, P, cap=1 << 20)
    assert r.status == M.MSP_OK and r.n_found == ref.n_found
    assert (x == ref.solutions).all()
    assert E.verify(inst.A, inst.d, x)
    assert r.stats["nodes"] == ref.nodes


def test_m7_m8_auto_split(M, ctx):
    for (m, D, seed) in [(7, 100, 5), (8, 200, 11)]:
        inst = mi.msp_class(m, D, seed)
        P = L.prepare(inst.A, inst.d)
        ref = E.enumerate_prepared(P, split=10, threads=8)
        r, x = _gpu_enum(M, ctx, inst, P)
        assert r.status == M.MSP_OK
        assert (x == ref.solutions).all()
        assert (r.stats["nodes"], r.stats["expansions"]) == (ref.nodes, ref.expansions)


def test_pruning_variants(M, ctx):
    inst = mi.planted(3, 20, 10, 40)
    P = L.prepare(inst.A, inst.d)
    for kw in ({"onedir": 0}, {"hoelder": 0}):
        ref = E.enumerate_prepared(P, onedir=kw.get("onedir", 1) == 1, hoelder=kw.get("hoelder", 1) == 1)
        r, x = _gpu_enum(M, ctx, inst, P, **kw)
        assert (x == ref.solutions).all() and r.stats["nodes"] == ref.nodes


def test_capacity_reports_true_total(M, ctx):
    inst = mi.planted(2, 20, 5, 3)
    P = L.prepare(inst.A, inst.d)
    ref = E.enumerate_prepared(P, cap=1 << 20)
    assert ref.n_found > 10
    r, x = _gpu_enum(M, ctx, inst, P, cap=7)
    assert r.status == M.MSP_E_CAPACITY and r.n_found == ref.n_found and x.shape[0] == 7
    allset = {row.tobytes() for row in ref.solutions}
    assert all(row.tobytes() in allset for row in x)


def test_first_mode(M, ctx):
    for (m, D, seed) in [(5, 50, 11), (6, 100, 2003), (7, 200, 6)]:
        inst = mi.msp_class(m, D, seed)
        P = L.prepare(inst.A, inst.d)
        ref = E.enumerate_prepared(P, split=6, threads=8)
        r, x = _gpu_enum(M, ctx, inst, P, mode=M.MSP_FIRST)
        assert r.status == M.MSP_OK and r.n_found >= 1
        allset = {row.tobytes() for row in ref.solutions}
        assert all(row.tobytes() in allset for row in x)
        assert r.stats["ttfs_ms"] >= 0.0


def test_time_cap_partial_subset(M, ctx):
    inst = mi.msp_class(8, 50, 9)
    P = L.prepare(inst.A, inst.d)
    r, x = _gpu_enum(M, ctx, inst, P, time_cap_ms=2.0, cap=1 << 12)
    assert r.status in (M.MSP_E_TIMEOUT, M.MSP_OK)
    assert E.verify(inst.A, inst.d, x)


def test_edge_shapes(M, ctx):
    """k = 2 and k = 3 (m close to n; N raised until the kernel is isolated)
    and an infeasible instance of the original generator (empty set)."""
    cases = [(mi.planted(5, 6, 3, 5), 1 << 20), (mi.planted(4, 6, 4, 2), 1 << 16), (mi.cornuejols_dawande(3, 9), 1024)]
    for inst, N in cases:
        P = L.prepare(inst.A, inst.d, N=N)
        ref = E.enumerate_prepared(P)
        for split in (0, P.k - 1, -1):
            r, x = _gpu_enum(M, ctx, inst, P, split_depth=split)
            assert r.status == M.MSP_OK and x.shape == ref.solutions.shape and (x == ref.solutions).all()
            assert r.stats["nodes"] == ref.nodes


def test_bad_arguments(M, ctx):
    inst = mi.single_small()
    P = L.prepare(inst.A, inst.d)
    A, d, Bs = _dev(inst.A), _dev(inst.d), _dev(P.basis)
    # the binding rejects a basis with too few rows before any library call ...
    with pytest.raises(ValueError):
        M.msp_enumerate(ctx, A, d, Bs[:-1].contiguous())
    # ... and the library rejects the same call made straight through the C ABI
    import ctypes as C
    m, n = inst.A.shape
    out = torch.zeros((4, n), dtype=torch.uint8, device=ctx.device)
    nf, st, prm0 = C.c_int64(0), M.Stats(), M.msp_params_default()
    rc = M.lib().msp_enumerate(ctx.handle, m, n, A.data_ptr(), d.data_ptr(), Bs.data_ptr(), P.k - 1, M.MSP_ALL,
                               M.MSP_PLAIN, C.byref(prm0), out.data_ptr(), 4, C.byref(nf), C.byref(st),
                               torch.cuda.current_stream(ctx.device).cuda_stream)
    assert rc == M.MSP_E_ARG
    prm = M.msp_params_default(split_depth=P.k)
    r = M.msp_enumerate(ctx, A, d, Bs, params=prm, raise_on_error=False)
    assert r.status == M.MSP_E_ARG


@pytest.mark.parametrize("seed", [6000, 6003])
def test_cornuejols_dawande_instances(M, ctx, seed):
    """The original generator, d_i = floor(sum_j a_ij / 2), m=7, n=60: the
    exhaustive walk on the oracle's basis gives the oracle's set and search
    counters, and the whole GPU path (GPU LLL basis) the same set."""
    import os
    inst = mi.cornuejols_dawande(7, seed)
    P = L.prepare(inst.A, inst.d)
    ref = E.enumerate_prepared(P, split=8, threads=os.cpu_count() or 1)
    r, x = _gpu_enum(M, ctx, inst, P)
    assert r.status == M.MSP_OK and r.n_found == ref.n_found
    assert np.array_equal(x, ref.solutions)
    for key in ("evals", "nodes", "expansions", "leaves"):
        assert r.stats[key] == getattr(ref, key), key
    A, d = _dev(inst.A), _dev(inst.d)
    Bk = M.msp_reduce(ctx, A, d)
    r2 = M.msp_enumerate(ctx, A, d, Bk, params=M.msp_params_default(time_cap_ms=60000.0))
    assert r2.status == M.MSP_OK
    assert np.array_equal(E.sort_rows(r2.x.cpu().numpy()), ref.solutions)


@pytest.mark.parametrize("m,n,D,seed,order", [(4, 30, 20, 7, 0), (7, 60, 100, 4100, 0), (5, 40, 10, 3, 2)])
def test_root_ranges_partition_the_walk(M, ctx, m, n, D, seed, order):
    """Walking the roots in three disjoint position ranges (a checkpoint and
    two resumptions) gives disjoint solution sets whose union is the full set,
    and counters that add up to the full walk's; a range past the last root
    walks nothing.  In depth-first and in learned root order."""
    inst = mi.planted(m, n, D, seed)
    P = L.prepare(inst.A, inst.d)
    if order == 2:
        M.msp_model_init(ctx, 5)
    A, d, Bk = _dev(inst.A), _dev(inst.d), _dev(P.basis)
    full = M.msp_enumerate(ctx, A, d, Bk, params=M.msp_params_default(time_cap_ms=60000.0), order=order,
                           cap=1 << 16)
    assert full.status == M.MSP_OK and full.stats["roots"] >= 3
    np_ = full.stats["roots"]
    cuts = [0, np_ // 3, 2 * np_ // 3, np_]
    xs, tot = [], {key: 0 for key in ("evals", "nodes", "expansions", "leaves")}
    for a, b in zip(cuts[:-1], cuts[1:]):
        prm = M.msp_params_default(time_cap_ms=60000.0, root_begin=a, root_count=(b - a if b < np_ else -1))
        r = M.msp_enumerate(ctx, A, d, Bk, params=prm, order=order, cap=1 << 16)
        assert r.status == M.MSP_OK and r.stats["roots"] == np_ and r.stats["initial_items"] == b - a
        xs.append(E.sort_rows(r.x.cpu().numpy()))
        for key in tot:
            tot[key] += r.stats[key]
    allx = np.concatenate(xs) if sum(len(x) for x in xs) else np.zeros((0, n), np.uint8)
    assert len(allx) == full.n_found == len({bytes(row) for row in allx})       # disjoint
    assert np.array_equal(E.sort_rows(allx), E.sort_rows(full.x.cpu().numpy()))
    assert np.array_equal(E.sort_rows(full.x.cpu().numpy()), E.solve(inst.A, inst.d)[1].solutions)
    for key in tot:
        assert tot[key] == full.stats[key], key
    past = M.msp_enumerate(ctx, A, d, Bk, params=M.msp_params_default(root_begin=np_ + 5), order=order)
    assert past.status == M.MSP_OK and past.n_found == 0 and past.stats["initial_items"] == 0
    with pytest.raises(M.MspError):
        M.msp_enumerate(ctx, A, d, Bk, params=M.msp_params_default(root_begin=-1))
    with pytest.raises(M.MspError):
        M.msp_enumerate(ctx, A, d, Bk, params=M.msp_params_default(root_count=5), mode=M.MSP_LDS)
