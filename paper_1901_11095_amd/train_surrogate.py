"""Train the learned surrogate on the GPU and write its weights.

    python -m paper_1901_11095_amd.train_surrogate [--epochs N] [--out PATH] [--eval-shape S]

With the defaults this reproduces the committed weights: 32 seeded 256^3 volumes whose
faults, chaotic bodies and SNR are drawn from their seeds (2M labelled voxels per epoch, 96
epochs, batch 64, cosine learning rate 1e-3 -> 1e-4).  `--volumes 8 --no-mix` trains on the
8-volume set at one noise level.  Afterwards it reports the error of the surrogate against
the plain method on a held-out volume (seed 99) before and after the tile check with exact
fallback.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import sal, surrogate, synth


def evaluate(net, V: torch.Tensor, L=16, bound=0.02, frac=0.02):
    """Errors of the surrogate against the plain FP32 method on one device volume, before
    and after the tile check with exact fallback."""
    ctx = sal.Saliency(L=L)
    st_ref = torch.zeros(8, dtype=torch.float64, device="cuda")
    Sr_ref = torch.empty((3,) + tuple(V.shape), dtype=torch.float32, device="cuda")
    S_ref = ctx.saliency(V, S_raw_out=Sr_ref, stats_out=st_ref)
    pred = net.infer(V)
    rng = (st_ref[1::2][:3] - st_ref[0::2][:3]).float().reshape(3, 1, 1, 1)
    raw_err = ((pred - Sr_ref).abs() / rng)
    S_pred = sal.normalize_combine(ctx, pred.clone(), V)
    out = {"raw_rel_max": float(raw_err.max()), "raw_rel_mean": float(raw_err.mean()),
           "S_abs_max_before": float((S_pred - S_ref).abs().max()),
           "S_abs_mean_before": float((S_pred - S_ref).abs().mean())}
    del S_pred
    # tiles within the bound before any fallback
    t = 32
    te = raw_err.amax(0)
    del raw_err
    n0, n1, n2 = V.shape
    tiles = te[:n0 // t * t, :n1 // t * t, :n2 // t * t].reshape(n0 // t, t, n1 // t, t, n2 // t, t)
    tmax = tiles.amax(dim=(1, 3, 5))
    out["tiles_within_bound"] = float((tmax <= bound).float().mean())
    res = surrogate.infer_with_fallback(net, ctx, V, frac=frac, bound=bound)
    out["checked_tiles"] = len(res["tiles"])
    out["checked_over_bound"] = int((res["tile_err"] > bound).sum())
    out["S_abs_max_after"] = float((res["S"] - S_ref).abs().max())
    out["S_abs_mean_after"] = float((res["S"] - S_ref).abs().mean())
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    d = surrogate.TrainConfig()
    ap.add_argument("--epochs", type=int, default=d.epochs)
    ap.add_argument("--batch", type=int, default=d.batch)
    ap.add_argument("--lr", type=float, default=d.lr)
    ap.add_argument("--shape", type=int, default=d.shape[0])
    ap.add_argument("--out", default=surrogate.WEIGHTS)
    ap.add_argument("--eval-shape", type=int, default=256)
    ap.add_argument("--volumes", type=int, default=d.n_volumes)
    ap.add_argument("--no-mix", action="store_true",
                    help="one noise level and structure count for every training volume")
    ap.add_argument("--eval-survey", action="store_true",
                    help="also evaluate on the 512 x 1024 x 1024 survey volume")
    args = ap.parse_args(argv)
    cfg = surrogate.TrainConfig(epochs=args.epochs, batch=args.batch, lr=args.lr,
                                shape=(args.shape,) * 3, n_volumes=args.volumes,
                                seeds=tuple(range(10, 10 + args.volumes)), mix=not args.no_mix)
    t0 = time.time()
    net, cfg = surrogate.train(cfg, log=lambda s: print(s, flush=True))
    torch.cuda.synchronize()
    print("trained in %.1f s" % (time.time() - t0), flush=True)
    surrogate.save(net, cfg, args.out)
    print("wrote", args.out, flush=True)
    shape = (args.eval_shape,) * 3
    V = torch.from_numpy(synth.make_volume(**surrogate.volume_kwargs(99, shape))).cuda()
    ev = {"held_out_%d" % args.eval_shape: evaluate(net, V)}
    del V
    if args.eval_survey:
        V = torch.from_numpy(synth.workload("survey512x1024x1024")).cuda()
        ev["survey512x1024x1024"] = evaluate(net, V)
        del V
    print(json.dumps({"eval": ev, "loss_history": cfg.history}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
