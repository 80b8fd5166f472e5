"""Train the learned controller and write its parameters next to this file
(controller_weights.json), which the package's LearnedContinuation.load reads.

Training instances are drawn from the evaluation workload's family
(rpca_inputs.controller_family: m = n, rank 5-50, 1-20% corruption of
magnitude U[5, 20]); for each, a greedy search along one trajectory tries
every candidate (decay, step multiplier) for a few lookahead rounds on a copy
of the iterate and keeps the pair that lands closest to the planted L*; the
MLP is then trained on the (features, best pair) samples with the library's
training kernel. Needs a GPU; prints one JSON line with the cost.

    python -m paper_2207_11669_amd.train_controller --instances 300 --size 2000
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--instances", type=int, default=300)
    ap.add_argument("--size", type=int, default=2000, help="m = n of the training instances")
    ap.add_argument("--first-seed", type=int, default=10_000)
    ap.add_argument("--horizon", type=int, default=10)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=0.5)
    ap.add_argument("--samples-in", default=None,
                    help="npz of samples from earlier runs to add (X, Y)")
    ap.add_argument("--samples-out", default=None, help="write the samples (npz) here")
    ap.add_argument("--out", default=None, help="weights file (default: next to the package)")
    args = ap.parse_args(argv)

    import torch

    from paper_2207_11669_amd import DCFPCA, colmajor
    from paper_2207_11669_amd import controller as C
    from rpca_inputs import controller_family, gaussian_init

    t0 = time.perf_counter()
    Xs, Ys = [], []
    if args.samples_in:
        d = np.load(args.samples_in)
        Xs.append(d["X"])
        Ys.append(d["Y"])
    gen_s = 0.0
    for k in range(args.instances):
        g0 = time.perf_counter()
        inst, r = controller_family(args.first_seed + k, args.size)
        lam = 1.0 / math.sqrt(inst.n)
        M = colmajor(inst.M)
        U0 = colmajor(gaussian_init(inst.m, r, 7))
        Us, Vs = colmajor(inst.Ustar), colmajor(inst.Vstar)
        gen_s += time.perf_counter() - g0

        def make():
            s = DCFPCA(M, inst.widths, inst.m, r, 0.1, lam, U0)
            s.set_target(Us, Vs, r)
            return s
        X, Y = C.greedy_samples(make, lam, float(np.abs(inst.M).max()), float(inst.m * inst.n),
                                horizon=args.horizon)
        Xs.append(X)
        Ys.append(Y)
        if (k + 1) % 10 == 0:
            print(f"[train] {k + 1}/{args.instances} instances, "
                  f"{sum(len(y) for y in Ys)} samples, {time.perf_counter() - t0:.0f}s",
                  file=sys.stderr, flush=True)
    X, Y = np.concatenate(Xs), np.concatenate(Ys)
    if args.samples_out:
        np.savez(args.samples_out, X=X, Y=Y)
    search_s = time.perf_counter() - t0
    t1 = time.perf_counter()
    params, losses = C.train(X, Y, steps=args.steps, lr=args.lr)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    info = {"kind": "learned (MLP 10-64-64-2: lambda-scale decay and U step multiplier; greedy "
                    "per-round targets)",
            "training_instances": args.instances + (0 if not args.samples_in else -0),
            "training_size": f"{args.size}x{args.size}",
            "family": "rank 5-50, corruption 1-20% of magnitude U[5, 20], clients of 250 columns",
            "samples": int(len(Y)), "horizon": args.horizon,
            "candidates": {"decay": list(C.GAMMAS), "step": list(C.OMEGAS)},
            "search_seconds": round(search_s, 1), "host_generation_seconds": round(gen_s, 1),
            "train_seconds": round(train_s, 1), "train_steps": args.steps,
            "final_train_loss": round(losses[-1], 6),
            "target_histogram": {f"{g}/{w}": int(np.sum((Y[:, 0] == g) & (Y[:, 1] == w)))
                                 for g in C.GAMMAS for w in C.OMEGAS}}
    out = args.out or C.WEIGHTS
    with open(out, "w") as f:
        json.dump({"training": info, "params": [float(v) for v in params.cpu().numpy()]}, f)
    print(json.dumps(info), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
