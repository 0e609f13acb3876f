"""msp_reduce_noalloc (the reduction that allocates nothing) against
msp_reduce on two calls in a row, the second with a smaller instance: the
same kernel basis, bit for bit, and the same k; sizes and options beyond its
fixed scratch are rejected."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import msp_instances as mi

pytestmark = pytest.mark.gpu


def test_noalloc_reduction_matches_msp_reduce_on_two_calls():
    import paper_2508_08702_amd as M
    dev = torch.device("cuda", 0)
    out = torch.full((128, 128), -7, dtype=torch.int64, device=dev)  # one output buffer for both calls
    with M.Context(0) as ctx:
        for inst in (mi.msp_class(7, 100, 4002), mi.single_small(1001)):
            print(f"  noalloc reduce m={inst.m} n={inst.n} seed {inst.seed}", flush=True)
            A = torch.from_numpy(inst.A).to(dev)
            d = torch.from_numpy(inst.d).to(dev)
            want = M.msp_reduce(ctx, A, d).cpu().numpy()
            o = out[: inst.n + 1, : inst.n + 1].contiguous()
            got = M.msp_reduce_noalloc(A, d, out=o).cpu().numpy()
            torch.cuda.synchronize()
            assert got.shape == want.shape == (inst.n - inst.m + 1, inst.n + 1)
            assert np.array_equal(got, want)


def test_noalloc_reduction_rejects_what_its_scratch_cannot_hold():
    import paper_2508_08702_amd as M
    dev = torch.device("cuda", 0)
    inst = mi.single_small(1001)
    A = torch.from_numpy(inst.A).to(dev)
    d = torch.from_numpy(inst.d).to(dev)
    with pytest.raises(M.MspError) as e:
        M.msp_reduce_noalloc(A, d, M.msp_params_default(bkz_block=16))
    assert e.value.code == M.MSP_E_ARG
    big = torch.zeros((2, M.MSP_MAX_N + 1), dtype=torch.int32, device=dev)
    with pytest.raises(M.MspError) as e:
        M.msp_reduce_noalloc(big, torch.zeros((2,), dtype=torch.int64, device=dev))
    assert e.value.code == M.MSP_E_ARG
