#!/usr/bin/env python3
"""The paper's synthetic experiments (Section 4) run on the GPU path.

    python experiments.py phase        # relative error over (rank, corruption) levels
    python experiments.py rank         # upper-bound rank p = 2r: singular-value error
    python experiments.py local-steps  # convergence for K local steps per round
    python experiments.py controller   # learned lambda controller vs fixed schedules

Instances follow Section 4.1's problem generation: L* = U0 V0^T with N(0, 1)
factors, and round(s m n) corrupted entries of value +-sqrt(m n) with a fair
sign. The paper leaves lambda and rho unstated; these runs use lambda =
1/sqrt(n) and rho = 0.1 (as the benchmark workloads do). The U step follows
the section's setting where it names one (the gradient step with K local
steps and eta0 / sqrt(t + 1), the paper's decaying rate); --u-mode closed and
--continuation (lambda_t = max(lambda, max|M| 0.8^t)) are offered beside it.
The library fits ranks up to 128, so the rank-level grid runs at the paper's
m = n = 500 (ranks 25 .. 100 = 0.05 n .. 0.2 n) and the upper-bound-rank
table up to its n = 1000 row (p = 100); its n = 5000 row (p = 500) is beyond
that range. Each command prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def _instance(n: int, r: int, s: float, E: int, seed: int):
    from rpca_inputs import equal_widths, planted_instance
    mag = math.sqrt(n * n)
    return planted_instance(n, equal_widths(n, E), r, s, values="signed", lo=mag, hi=mag, seed=seed)


def _solver(args) -> dict:
    if args.u_mode == "closed":
        return dict(u_mode="closed", K=args.K)
    return dict(u_mode="grad", eta0=args.eta, eta_sched=args.sched, K=args.K)


def _run(inst, r: int, rounds: int, continuation: bool, seed: int = 7, **kw):
    """Rounds of the GPU path from U^(0) ~ N(0, 1); returns L (m x n, FP64)."""
    import torch

    from paper_2207_11669_amd import DCFPCA, colmajor
    from rpca_inputs import gaussian_init
    lam = 1.0 / math.sqrt(inst.n)
    U0 = gaussian_init(inst.m, r, seed)
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, 0.1, lam, colmajor(U0), **kw)
    done = 0
    if continuation:
        lam0 = float(np.abs(inst.M).max())
        while done < rounds:
            lt = max(lam, lam0 * 0.8 ** done)
            s.set_lambda(lt)
            s.step(1)
            done += 1
            if lt == lam:
                break
    s.step(rounds - done)
    L, _ = s.get_LS(-1)
    torch.cuda.synchronize()
    out = L[:, :inst.m].T.double().cpu().numpy()
    s.close()
    return out


def _relerr(L, inst) -> float:
    Ls = inst.Ustar @ inst.Vstar.T
    return float(np.linalg.norm(L - Ls) / np.linalg.norm(Ls))


def phase(args) -> dict:
    """Relative error over rank r in [0.05 n, 0.2 n] and corruption s in
    [0.05, 0.3] (the paper's Fig. on sparsity and rank levels, m = n = 500)."""
    n = args.n
    ranks = [round(f * n) for f in (0.05, 0.10, 0.15, 0.20)]
    fracs = [0.05, 0.10, 0.15, 0.20, 0.25, 0.30]
    grid = []
    for r in ranks:
        row = []
        for sfrac in fracs:
            inst = _instance(n, r, sfrac, args.clients, seed=1000 * r + int(100 * sfrac))
            row.append(_relerr(_run(inst, r, args.rounds, args.continuation, **_solver(args)), inst))
        grid.append(row)
        print(f"[phase] r={r}: " + " ".join(f"{e:.2e}" for e in row), file=sys.stderr, flush=True)
    return {"experiment": "phase", "n": n, "E": args.clients, "rounds": args.rounds,
            "continuation": args.continuation, "solver": _solver(args), "ranks": ranks,
            "corruption": fracs, "relerr": grid}


def rank(args) -> dict:
    """Fit rank p = 2 r with r = 0.05 n, s = 0.05: relative singular-value
    error max_i |sigma_i(L) - sigma_i(L*)| / sigma_r(L*) over i <= p (the
    paper's table of relative singular value errors). Fits above rank 128
    are outside the library's range."""
    rows = []
    for n in args.sizes:
        r = round(0.05 * n)
        p = 2 * r
        if p > 128:
            rows.append({"n": n, "r": r, "p": p, "skipped": "p > 128"})
            continue
        inst = _instance(n, r, 0.05, args.clients, seed=n)
        t0 = time.perf_counter()
        L = _run(inst, p, args.rounds, args.continuation, **_solver(args))
        secs = time.perf_counter() - t0
        sl = np.linalg.svd(L, compute_uv=False)[:p]
        ss = np.zeros(p)
        ss[:r] = np.linalg.svd(inst.Ustar @ inst.Vstar.T, compute_uv=False)[:r]
        err = float(np.max(np.abs(sl - ss)) / ss[r - 1])
        rows.append({"n": n, "r": r, "p": p, "sv_error": err,
                     "tail_ratio": float(sl[r] / sl[r - 1]), "relerr": _relerr(L, inst),
                     "seconds": round(secs, 3)})
        print(f"[rank] {rows[-1]}", file=sys.stderr, flush=True)
    return {"experiment": "rank", "rounds": args.rounds, "continuation": args.continuation,
            "solver": _solver(args), "E": args.clients, "rows": rows}


def local_steps(args) -> dict:
    """Relative error per round for K local steps per round (GRAD step,
    constant eta, E clients; the paper's ablation on local iterations)."""
    n = args.n
    r = round(0.05 * n)
    inst = _instance(n, r, 0.05, args.clients, seed=7)
    import torch

    from paper_2207_11669_amd import DCFPCA, colmajor
    from rpca_inputs import gaussian_init
    lam = 1.0 / math.sqrt(inst.n)
    U0 = gaussian_init(inst.m, r, 7)
    curves = {}
    for K in args.ks:
        s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, 0.1, lam, colmajor(U0),
                   u_mode="grad", eta0=args.eta, K=K)
        errs = []
        for _ in range(args.rounds):
            s.step(1)
            L, _ = s.get_LS(-1)
            torch.cuda.synchronize()
            errs.append(_relerr(L[:, :inst.m].T.double().cpu().numpy(), inst))
        s.close()
        curves[str(K)] = errs
        print(f"[local-steps] K={K}: " + " ".join(f"{e:.2e}" for e in errs[::max(1, len(errs) // 10)]),
              file=sys.stderr, flush=True)
    return {"experiment": "local-steps", "n": n, "r": r, "E": args.clients, "eta": args.eta,
            "rounds": args.rounds, "relerr_per_round": curves}


def _trajectory(s, budget: int, every: int = 5, start: int = 0):
    """Planted-target error every `every` rounds up to `budget` rounds
    (counting `start` already run): [(rounds, error), ...]."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = [(start, s.target_error(), 0.0)]
    done = start
    while done < budget:
        s.step(every)
        done += every
        out.append((done, s.target_error(), time.perf_counter() - t0))
    return out


def _first(traj, tol, offset_s: float = 0.0):
    """(rounds, seconds) at the first check with error <= tol, or None."""
    hit = next(((k, t) for k, e, t in traj if e <= tol), None)
    return None if hit is None else [hit[0], round(hit[1] + offset_s, 4)]


def controller(args) -> dict:
    """The learned lambda controller: greedy-search targets on method-
    generated training instances, MLP training on the GPU, and rounds to a
    relative error against the planted L* for the plain method, the fixed
    continuation and the learned one on held-out instances."""
    import torch

    from paper_2207_11669_amd import DCFPCA, colmajor
    from paper_2207_11669_amd import controller as C
    from rpca_inputs import controller_family, gaussian_init, recipe

    def family(seed):
        return controller_family(seed, args.train_n)

    def session(inst, r, lam, target=True):
        s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, 0.1, lam,
                   colmajor(gaussian_init(inst.m, r, 7)))
        if target:
            s.set_target(colmajor(inst.Ustar), colmajor(inst.Vstar), inst.Ustar.shape[1])
        return s

    def cases():
        for k in range(args.train_instances):
            inst, r = family(10_000 + k)
            lam = 1.0 / math.sqrt(inst.n)
            yield ((lambda inst=inst, r=r, lam=lam: session(inst, r, lam)), lam,
                   float(np.abs(inst.M).max()), float(inst.m * inst.n))

    t0 = time.perf_counter()
    params, (X, Y), losses = C.fit(cases(), horizon=args.horizon, steps=args.steps, lr=args.lr)
    torch.cuda.synchronize()
    print(f"[controller] {len(Y)} greedy samples from {args.train_instances} instances, trained "
          f"in {time.perf_counter() - t0:.1f}s; decay histogram " +
          str({g: int(np.sum(Y == g)) for g in C.GAMMAS}) +
          f"; loss {losses[0]:.4f} -> {losses[-1]:.4f}", file=sys.stderr, flush=True)

    evals = []
    cases = [("held-out", 20_000 + k) for k in range(args.eval_instances)]
    if args.large_eval:
        cases.append(("m=8000 n=32000 r=40 s=0.15 E=32", None))
    for name, seed in cases:
        if seed is None:
            inst, r = recipe("plain_8000x32000_r40", seed=0), 40
        else:
            inst, r = family(seed)
        lam = 1.0 / math.sqrt(inst.n)
        lam0 = float(np.abs(inst.M).max())
        budget = args.budget if seed is not None else args.large_budget
        row = {"instance": name, "m": inst.m, "n": inst.n, "r": r}
        trajs = {}
        for cname, ctl in (("plain", None), ("fixed_0.8", C.FixedContinuation(0.8)),
                           ("learned", C.LearnedContinuation(params))):
            s = session(inst, r, lam)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ctrl = C.run_controlled(s, lam, lam0, ctl, float(inst.m * inst.n),
                                    judge=cname == "learned") if ctl else \
                {"control_rounds": 0, "gammas": []}
            control_s = time.perf_counter() - t1
            trajs[cname] = _trajectory(s, budget, start=ctrl["control_rounds"])
            row[cname] = {"control_rounds": ctrl["control_rounds"],
                          "control_seconds": round(control_s, 4),
                          "final_relerr": trajs[cname][-1][1]}
            s.close()
        # The three runs end at the same fixed point (lambda ends at its
        # target): rounds to 1e-2 and to within 5% of the best error seen.
        floor = min(e for tr in trajs.values() for _, e, _ in tr)
        for cname, tr in trajs.items():
            off = row[cname]["control_seconds"]
            # [rounds, seconds] at the first check at or below the tolerance;
            # seconds include the controlled rounds and the checks (a
            # synchronising Gram evaluation every 5 rounds).
            row[cname]["to_1e-2"] = _first(tr, 1e-2, off)
            row[cname]["to_1e-4"] = _first(tr, 1e-4, off)
            row[cname]["to_floor_5pct"] = _first(tr, 1.05 * floor, off)
        row["floor"] = floor
        evals.append(row)
        print(f"[controller] {name} seed={seed} floor={floor:.2e}: " + "; ".join(
            f"{c}: 1e-2@{row[c]['to_1e-2']} 1e-4@{row[c]['to_1e-4']} floor@{row[c]['to_floor_5pct']}"
            for c in ("plain", "fixed_0.8", "learned")), file=sys.stderr, flush=True)
    return {"experiment": "controller", "train_instances": args.train_instances,
            "train_n": args.train_n, "samples": int(len(Y)), "horizon": args.horizon,
            "decays": list(C.GAMMAS), "train_loss": losses, "eval": evals}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    def solver_args(p, K, eta, rounds):
        p.add_argument("--u-mode", default="grad", choices=["grad", "closed"])
        p.add_argument("--K", type=int, default=K)
        p.add_argument("--eta", type=float, default=eta)
        p.add_argument("--sched", default="sqrt", choices=["sqrt", "const"])
        p.add_argument("--rounds", type=int, default=rounds)
        p.add_argument("--continuation", action="store_true")
    a = sub.add_parser("phase")
    a.add_argument("--n", type=int, default=500)
    a.add_argument("--clients", type=int, default=5)
    solver_args(a, 2, 0.05, 200)
    b = sub.add_parser("rank")
    b.add_argument("--sizes", type=int, nargs="+", default=[200, 500, 1000, 5000])
    b.add_argument("--clients", type=int, default=5)
    solver_args(b, 2, 0.05, 200)
    c = sub.add_parser("local-steps")
    c.add_argument("--n", type=int, default=500)
    c.add_argument("--clients", type=int, default=10)
    c.add_argument("--rounds", type=int, default=30)
    c.add_argument("--eta", type=float, default=0.01)
    c.add_argument("--ks", type=int, nargs="+", default=[1, 2, 5, 10])
    d = sub.add_parser("controller")
    d.add_argument("--train-instances", type=int, default=40)
    d.add_argument("--train-n", type=int, default=256)
    d.add_argument("--horizon", type=int, default=15)
    d.add_argument("--steps", type=int, default=2000)
    d.add_argument("--lr", type=float, default=0.5)
    d.add_argument("--eval-instances", type=int, default=12)
    d.add_argument("--budget", type=int, default=1000)
    d.add_argument("--large-budget", type=int, default=6000)
    d.add_argument("--no-large-eval", dest="large_eval", action="store_false")
    args = ap.parse_args()
    fn = {"phase": phase, "rank": rank, "local-steps": local_steps, "controller": controller}[args.cmd]
    print(json.dumps(fn(args)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
