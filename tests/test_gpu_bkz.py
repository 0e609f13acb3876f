"""GPU BKZ of the kernel basis (msp_params.bkz_block): the reduced basis spans
the same lattice (equal Gram determinant, exact, and every vector in the
kernel of the extended system), the solution set is the oracle's, the first
vector is no longer than LLL's, and at m = 8 the enumeration tree shrinks."""
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


@pytest.mark.parametrize("m,D,seed,beta", [(6, 100, 2000, 8), (7, 100, 4100, 12), (8, 200, 4152, 16),
                                           (8, 50, 4002, 10)])
def test_bkz_basis_is_a_basis_and_keeps_the_solutions(M, ctx, m, D, seed, beta):
    inst = mi.msp_class(m, D, seed)
    A, d = _dev(inst.A), _dev(inst.d)
    print(f"  bkz m={m} D={D} seed={seed} beta={beta}", flush=True)
    B0 = M.msp_reduce(ctx, A, d).cpu().numpy()
    B1 = M.msp_reduce(ctx, A, d, M.msp_params_default(bkz_block=beta)).cpu().numpy()
    assert B1.shape == B0.shape
    n = inst.n
    for row in B1:   # in the kernel of A x = d x_{n+1} (binary embedding)
        assert np.array_equal(inst.A.astype(np.int64) @ (row[:n] + row[n]), 2 * inst.d * row[n])
    g0 = L.gram_schmidt_exact([[int(v) for v in r] for r in B0])
    g1 = L.gram_schmidt_exact([[int(v) for v in r] for r in B1])
    assert g0.d[-1] == g1.d[-1]   # same covolume: same lattice
    prm = M.msp_params_default(time_cap_ms=60000.0)
    r0 = M.msp_enumerate(ctx, A, d, _dev(B0), params=prm)
    r1 = M.msp_enumerate(ctx, A, d, _dev(B1), params=prm)
    assert r0.status == r1.status == M.MSP_OK
    x0, x1 = E.sort_rows(r0.x.cpu().numpy()), E.sort_rows(r1.x.cpu().numpy())
    assert np.array_equal(x0, x1)
    print(f"    nodes LLL {r0.stats['nodes']} BKZ {r1.stats['nodes']}", flush=True)
    # BKZ starts from the LLL basis and never lengthens its first vector
    assert int(B1[0] @ B1[0]) <= int(B0[0] @ B0[0])
    if m >= 8:  # where the tree is large, the better basis shrinks it
        assert r1.stats["nodes"] < r0.stats["nodes"]
    if m <= 7:
        ref = E.solve(inst.A, inst.d, split=6, threads=os.cpu_count() or 1)[1]
        assert np.array_equal(x1, ref.solutions)


def test_bkz_argument_check(M, ctx):
    inst = mi.msp_class(5, 100, 3)
    with pytest.raises(M.MspError):
        M.msp_reduce(ctx, _dev(inst.A), _dev(inst.d), M.msp_params_default(bkz_block=1))


@pytest.mark.parametrize("m,D,seed,beta", [(4, 100, 3, 10), (5, 100, 11, 8), (6, 100, 2000, 6)])
def test_bkz_output_satisfies_the_block_condition(M, ctx, m, D, seed, beta):
    """With tours enough to converge, no projected block of the GPU's BKZ
    basis holds a vector shorter than 0.999 ||b_hat_j||^2 (the insertion
    threshold), checked by the oracle's exact block enumeration; the LLL
    basis of the same instance violates it (so the check has teeth)."""
    from oracle import bkz as K
    inst = mi.msp_class(m, D, seed)
    A, d = _dev(inst.A), _dev(inst.d)
    B0 = M.msp_reduce(ctx, A, d).cpu().numpy()
    B1 = M.msp_reduce(ctx, A, d, M.msp_params_default(bkz_block=beta, bkz_tours=64)).cpu().numpy()
    assert K.bkz_violations(B0, beta)
    assert K.bkz_violations(B1, beta) == []


@pytest.mark.parametrize("m,n,D,seed,beta", [(6, 120, 50, 6100, 8), (12, 126, 100, 6101, 10)])
def test_bkz_with_the_basis_in_hbm(M, ctx, m, n, D, seed, beta):
    """k x dim int64 too large for LDS next to the Gram triangle and mu (k =
    115 and 115 here): the kernel works on the basis in HBM.  The output spans
    the same lattice (exact Gram determinant), lies in the kernel of the
    extended system, and its first vector is no longer than LLL's."""
    inst = mi.planted(m, n, D, seed)
    k, dim = n - m + 1, n + 1
    lds_without_basis = 8 * (k * (k + 1) // 2) + 8 * (k * (k - 1) // 2 + 1 + k) + 4 * (k + 6)
    assert lds_without_basis <= 160 * 1024 < lds_without_basis + 8 * k * dim
    A, d = _dev(inst.A), _dev(inst.d)
    print(f"  bkz in HBM m={m} n={n} k={k} beta={beta}", flush=True)
    B0 = M.msp_reduce(ctx, A, d).cpu().numpy()
    B1 = M.msp_reduce(ctx, A, d, M.msp_params_default(bkz_block=beta)).cpu().numpy()
    assert B1.shape == B0.shape == (k, dim)
    assert not np.array_equal(B0, B1)          # BKZ changed the basis
    for row in B1:
        assert np.array_equal(inst.A.astype(np.int64) @ (row[:n] + row[n]), 2 * inst.d * row[n])
    g0 = L.gram_schmidt_exact([[int(v) for v in r] for r in B0])
    g1 = L.gram_schmidt_exact([[int(v) for v in r] for r in B1])
    assert g0.d[-1] == g1.d[-1]
    assert int(B1[0] @ B1[0]) <= int(B0[0] @ B0[0])
