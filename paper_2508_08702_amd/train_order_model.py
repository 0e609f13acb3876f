"""Train the root-scoring model on traces the enumerator logs.

    python -m paper_2508_08702_amd.train_order_model [--out FILE] [--epochs 30]

For every instance of the training set (planted market split instances,
m in {6, 7, 8}, n = 10(m-1), D in {50, 100, 200}, seeds 4000-4191) this runs
the exhaustive GPU enumeration with root tracing (msp_root_trace): each
subtree root gets its 16 features and the label "a solution lies below".
With --bkz the traced bases are BKZ-reduced first.
The traces stay on the device; the model (16 -> 64 -> 64 -> 1, BF16 weights)
is trained on them by the library's own kernels (msp_model_train) and its
FP32 master weights are written with numpy.save.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import msp_instances as mi  # noqa: E402

from . import (Context, msp_model_get, msp_model_init, msp_model_train, msp_params_default,  # noqa: E402
               msp_reduce, msp_root_trace, msp_train_params_default)

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "order_model.npy")


def collect(ctx, insts, log=print, bkz=0):
    dev = ctx.device
    prm = msp_params_default(time_cap_ms=120000.0, bkz_block=bkz)
    feats, labels = [], []
    t0 = time.time()
    for i, inst in enumerate(insts):
        A = torch.from_numpy(inst.A).to(dev)
        d = torch.from_numpy(inst.d).to(dev)
        basis = msp_reduce(ctx, A, d, prm)
        tr = msp_root_trace(ctx, A, d, basis, params=prm)
        feats.append(tr.feat)
        labels.append(tr.label)
        if i % 16 == 15:
            log(f"traced {i + 1}/{len(insts)} instances, {time.time() - t0:.1f} s")
    return torch.cat(feats), torch.cat(labels)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--init-seed", type=int, default=1)
    ap.add_argument("--bkz", type=int, default=0, help="BKZ block size of the traced bases (0: LLL)")
    args = ap.parse_args()
    ctx = Context(0)
    F, Y = collect(ctx, mi.train_set(), log=lambda s: print(s, flush=True), bkz=args.bkz)
    print(f"dataset: {F.shape[0]} roots, {int(Y.sum())} with a solution below", flush=True)
    msp_model_init(ctx, args.init_seed)
    t0 = time.time()
    losses = msp_model_train(ctx, F, Y, msp_train_params_default(epochs=args.epochs, lr=args.lr, batch=args.batch))
    torch.cuda.synchronize()
    print(f"trained {args.epochs} epochs in {time.time() - t0:.1f} s; loss per epoch "
          + " ".join(f"{x:.4f}" for x in losses), flush=True)
    np.save(args.out, msp_model_get(ctx))
    print(f"wrote {args.out}", flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
