"""GPU parity with entries of either sign and with general box bounds
(paper, Section 2): msp_reduce + msp_enumerate on signed binary instances
against brute force over {0,1}^n and the oracle's counters on its own basis;
msp_solve_box (the substitution x := x - l in a kernel, the bounded path,
x' + l written back) against brute force over the box and the oracle on the
shifted problem; rejected bounds."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import msp_instances as mi
from oracle import brute as B
from oracle import enum as E
from oracle import lattice as L

from test_oracle_signs import box_brute_force, shifted_oracle

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


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_signed_binary_instances(M, ctx, seed):
    inst = mi.signed_planted(3, 20, -50, 50, seed)
    want = E.sort_rows(B.brute_force(inst.A, inst.d))
    A, d = _dev(inst.A), _dev(inst.d)
    prm = M.msp_params_default(time_cap_ms=60000.0)
    r = M.msp_enumerate(ctx, A, d, M.msp_reduce(ctx, A, d, prm), params=prm)
    assert r.status == M.MSP_OK
    assert np.array_equal(E.sort_rows(r.x.cpu().numpy()), want)
    # counters on the oracle's exact basis
    P = L.prepare(inst.A, inst.d)
    ref = E.enumerate_prepared(P, split=4, threads=4)
    r2 = M.msp_enumerate(ctx, A, d, _dev(P.basis), params=prm)
    assert np.array_equal(E.sort_rows(r2.x.cpu().numpy()), ref.solutions)
    for key in ("evals", "nodes", "expansions", "leaves"):
        assert r2.stats[key] == getattr(ref, key), key


@pytest.mark.parametrize("mode", ["all", "first", "lds"])
@pytest.mark.parametrize("seed", [11, 12, 13, 14])
def test_box_bounds(M, ctx, seed, mode):
    b = mi.box_planted(2, 8, -6, 7, -2, 2, 2, seed)
    want = box_brute_force(b.A, b.d, b.lo, b.hi)
    assert np.array_equal(shifted_oracle(b.A, b.d, b.lo, b.hi), want)
    md = {"all": M.MSP_ALL, "first": M.MSP_FIRST, "lds": M.MSP_LDS}[mode]
    r = M.msp_solve_box(ctx, _dev(b.A), _dev(b.d), _dev(b.lo), _dev(b.hi), mode=md,
                        params=M.msp_params_default(time_cap_ms=60000.0))
    assert r.status == M.MSP_OK
    x = r.x.cpu().numpy().astype(np.int64)
    assert np.all(x >= b.lo[None, :]) and np.all(x <= b.hi[None, :])
    assert np.all(x @ b.A.T.astype(np.int64) == b.d[None, :])
    got = x[np.lexsort(x.T[::-1])] if x.shape[0] else x
    if mode == "all":
        assert r.n_found == want.shape[0] and np.array_equal(got, want)
    else:
        assert r.n_found >= 1 and {tuple(v) for v in got} <= {tuple(v) for v in want}


def test_box_bounds_wider_instance(M, ctx):
    # n = 30 binary-width boxes around negative lower bounds: the oracle on the
    # shifted problem (brute force is out of reach) and every row verified
    b = mi.box_planted(4, 30, -20, 21, -3, 1, 1, 21)
    want = shifted_oracle(b.A, b.d, b.lo, b.hi)
    r = M.msp_solve_box(ctx, _dev(b.A), _dev(b.d), _dev(b.lo), _dev(b.hi),
                        params=M.msp_params_default(time_cap_ms=60000.0))
    assert r.status == M.MSP_OK
    x = r.x.cpu().numpy().astype(np.int64)
    assert np.array_equal(x[np.lexsort(x.T[::-1])], want)
    assert any(np.array_equal(v, b.x_planted) for v in x)


def test_box_bound_errors(M, ctx):
    b = mi.box_planted(2, 8, -6, 7, -2, 2, 2, 11)
    A, d = _dev(b.A), _dev(b.d)
    for lo, hi in ((b.lo, b.lo), (b.lo, b.lo + 256), (b.lo - (1 << 25), b.hi)):
        with pytest.raises(M.MspError) as e:
            M.msp_solve_box(ctx, A, d, _dev(np.asarray(lo, dtype=np.int32)), _dev(np.asarray(hi, dtype=np.int32)))
        assert e.value.code == M.MSP_E_ARG
