"""What the trained root-scoring model gains over the plain order, measured
without clocks: on held-out planted instances (m=8, n=70, seeds 4600-4611,
not in the training set 4000-4191) an exhaustive trace labels every subtree
root; the position of the first root with a solution below it is compared
between depth-first order and the model's order (best score first).  The
committed model must move that position forward on the median instance by a
large factor, and a random-weight model (a control) must not."""
from __future__ import annotations

import os
import statistics

import numpy as np
import pytest
import torch

import msp_instances as mi

pytestmark = pytest.mark.gpu

MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2508_08702_amd",
                     "order_model.npy")


def _first_positive(label, key):
    order = np.argsort(-key, kind="stable")
    return int(np.nonzero(label[order])[0][0])


def test_learned_order_ranks_solution_subtrees_first():
    import paper_2508_08702_amd as M
    ctx = M.Context(0)
    try:
        traces = []
        for i in range(12):
            inst = mi.msp_class(8, (50, 100, 200)[i // 4], 4600 + i)
            A = torch.from_numpy(inst.A).to("cuda:0")
            d = torch.from_numpy(inst.d).to("cuda:0")
            print(f"  trace m=8 D={inst.D} seed={inst.seed}", flush=True)
            Bk = M.msp_reduce(ctx, A, d)
            tr = M.msp_root_trace(ctx, A, d, Bk)
            lab = tr.label.cpu().numpy().astype(bool)
            assert lab.any() and tr.n_found >= 1
            traces.append((tr.feat, lab))
        plain = [int(np.nonzero(lab)[0][0]) for _, lab in traces]
        M.msp_model_set(ctx, np.load(MODEL))
        learned = [_first_positive(lab, M.msp_model_score(ctx, f).cpu().numpy()) for f, lab in traces]
        M.msp_model_init(ctx, 12345)
        control = [_first_positive(lab, M.msp_model_score(ctx, f).cpu().numpy()) for f, lab in traces]
        mp, ml, mc = statistics.median(plain), statistics.median(learned), statistics.median(control)
        print(f"  median first-positive position: plain {mp}, learned {ml}, random-weight control {mc}")
        assert ml * 10 <= mp
        assert ml * 10 <= mc
    finally:
        ctx.close()
