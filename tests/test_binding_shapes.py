"""CPU checks of the binding's shape validation: a mis-shaped tensor is
rejected with ValueError before any pointer reaches the library (the kernels
trust the sizes they are given).  A stand-in context on the CPU is enough,
because every check runs before the first library call."""
from __future__ import annotations

from types import SimpleNamespace

import pytest
import torch

import paper_2508_08702_amd as M

CPU = torch.device("cpu")
CTX = SimpleNamespace(device=CPU, handle=None)
m, n = 3, 20


def _A(mm=m, nn=n):
    return torch.zeros((mm, nn), dtype=torch.int32)


def _d(mm=m):
    return torch.zeros((mm,), dtype=torch.int64)


def _B(k=n - m + 1, dim=n + 1):
    return torch.zeros((k, dim), dtype=torch.int64)


@pytest.mark.parametrize("call", [
    lambda: M.msp_reduce(CTX, _A(), _d(m - 1)),
    lambda: M.msp_reduce(CTX, _A().reshape(-1), _d()),
    lambda: M.msp_enumerate(CTX, _A(), _d(m + 1), _B()),
    lambda: M.msp_enumerate(CTX, _A(), _d(), _B(dim=n)),
    lambda: M.msp_enumerate(CTX, _A(), _d(), _B(k=n - m)),
    lambda: M.msp_enumerate(CTX, _A(), _d(), _B(), out=torch.zeros((4, n - 1), dtype=torch.uint8)),
    lambda: M.msp_solve_first(CTX, _A(), _d(), out=torch.zeros((4, n + 1), dtype=torch.uint8)),
    lambda: M.msp_solve_first(CTX, _A(), _d(m - 1)),
    lambda: M.msp_solve_batch(CTX, [_A(), _A(4, 30)], [_d(), _d(3)]),
    lambda: M.msp_root_trace(CTX, _A(), _d(), _B(dim=n + 2)),
    lambda: M.msp_reduce_bounded(CTX, _A(), _d(), torch.ones((n - 1,), dtype=torch.int32)),
    lambda: M.msp_enumerate_bounded(CTX, _A(), _d(), torch.ones((n,), dtype=torch.int32), _B(k=2)),
    lambda: M.msp_model_score(CTX, torch.zeros((5, M.MSP_NFEAT - 1), dtype=torch.float32)),
    lambda: M.msp_model_grad(CTX, torch.zeros((5, M.MSP_NFEAT), dtype=torch.float32),
                             torch.zeros((4,), dtype=torch.uint8)),
    lambda: M.msp_model_train(CTX, torch.zeros((5, M.MSP_NFEAT), dtype=torch.float32),
                              torch.zeros((6,), dtype=torch.uint8)),
    lambda: M.msp_gram_schmidt(CTX, torch.zeros((5, 3), dtype=torch.int64)),
])
def test_mis_shaped_arguments_are_rejected_before_the_library(call):
    with pytest.raises(ValueError):
        call()


def test_well_shaped_arguments_pass_the_checks():
    assert M._check_instance(_A(), _d()) == (m, n)
    assert M._check_basis(_B(), m, n) == n - m + 1
    assert M._check_out(torch.zeros((7, n), dtype=torch.uint8), n) == 7
    M._check_bounds(torch.ones((n,), dtype=torch.int32), n)
    assert M._check_features(torch.zeros((9, M.MSP_NFEAT)), torch.zeros((9,), dtype=torch.uint8)) == 9
