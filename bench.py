#!/usr/bin/env python3
"""DCF-PCA benchmark on one MI355X: rounds of Algorithm 1 per second, and the
wall time to a relative error of 1e-4 against the planted low-rank part.

Headline workload (`value`, rounds/s in FP32): m = 20000, n = 100000, planted
rank 64 with singular values geometric from 100 down to 1, 5% of the entries
corrupted (Bernoulli) with magnitude U[1, 100] and a random sign, E = 50
clients of 2000 columns, r = 64, lambda = 1/sqrt(n), rho = 0.1, closed-form U
step, K = 1. Inputs are synthetic, seeded, and resident in HBM before timing.
The FP32 context is created with RPCA_FLAG_SPARSE_S, so that the autotuner
(run before timing) chooses between handing S from the S-pass to the next
V-pass in sparse form and rebuilding it; both give bitwise the same rounds.

Next to it, on the same workload: BF16 rounds (BF16 copies of M, U and V on
BF16 MFMA) and three-product BF16 rounds (FP32 M, hi/lo splits), each with its
rounds/s and its error against the FP64 oracle on the workload's 2000 x 2000
sub-instance after a fixed schedule of low-precision rounds followed by FP32
closing rounds.

Time to relative error 1e-4 (where it is reachable): m = 8000, n = 32000,
planted rank 40, 15% corruption with magnitude U[5, 20], E = 32, r = 40, for
plain FP32 rounds, the fixed lambda continuation, the learned controller, and
the learned controller driving three-product BF16 rounds, each with the launch
shape the autotuner picked on a context of its own.

The FP64 CPU oracle is timed on bounded samples of both workloads, on all the
host's cores and on one.

--rank fits another rank than the workload's (up to 128; the BF16 legs need
64 or less), for the upper-bound rank setting of Section 4.2; the line then
names the fitted rank and reads the byte counters of that fit.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DCF-PCA iters/sec + time-to-relerr 1e-4 (BF16/learned vs plain FP32), 1 GPU"
WORKLOAD = "geom_20000x100000_r64"
EVAL_WORKLOAD = "plain_8000x32000_r40"
SUB_WORKLOAD = "geom_2000x2000_r64"
WORKLOADS = ("geom_20000x100000_r64", "plain_4000x8000_r20", "uneven_10000_r32",
             "plain_8000x32000_r40", "plain_500x500_r5")
HBM_PEAK_GBS = 8000.0
# Dense MFMA peaks of one MI355X, per algorithmic flop: three-product BF16
# rounds run three BF16 products per product of the method.
MFMA_PEAK_TFS = {"fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0 / 3}
KERNEL_SRCS = [os.path.join(ROOT, "paper_2207_11669_amd", "csrc", f)
               for f in ("rpca_device.h", "rpca_internal.h", "rpca_vpass_kernel.h",
                         "rpca_vpass.hip", "rpca_vpass_q.hip", "rpca_vpass_s.hip",
                         "rpca_spass_kernel.h", "rpca_spass.hip", "rpca_spass_q.hip",
                         "rpca_spass_s.hip", "rpca_bf16.hip", "rpca_tail.hip")]


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def traffic_file(workload: str, precision: str = "fp32") -> str:
    suffix = "" if precision == "fp32" else f"_{precision}"
    return os.path.join(ROOT, "profiles", f"traffic_{workload}{suffix}.json")


def kernel_costs(m: int, n: int, E: int, r: int, precision: str = "fp32",
                 sparse: bool = False, nnz: float = 0.0) -> dict:
    """Algorithmic HBM bytes and flops per launch of the two streaming kernels,
    for the default round (K = 1, one V/S alternation, S not stored densely).

    V-pass: reads M once (4 B per entry; 2 B in BF16 rounds, which read their
    BF16 copy), U, the previous U and V, and writes W = (M - S)^T U (n x r);
    flops: 2r per entry to rebuild the residual U_old V_old^T and 2r per entry
    for W.
    S-pass: reads M once (4 B, or 2 B in BF16), U and V, writes the
    per-client U-step terms (E x m x r); flops: 2r per entry for U V^T and 2r
    for Lambda V. Factor operands count at their own width (4 B, or 2 B).
    With the sparse handoff (sparse, nnz = the support size of S) the S-pass
    also writes S's nonzero values and their positions (4 B per nonzero, 8 B
    per 256 entries) and the V-pass reads them instead of rebuilding S: no
    previous factors, 2r flops per entry."""
    elem = m * n
    w = 2 if precision == "bf16" else 4
    s_bytes = 4 * nnz + elem / 32
    if sparse:
        return {
            "vpass": {"bytes": w * elem + w * m * r + 4 * n * r + s_bytes, "flops": 2 * r * elem},
            "spass": {"bytes": w * elem + w * (m * r + n * r) + 4 * E * m * r + s_bytes,
                      "flops": 4 * r * elem},
        }
    return {
        "vpass": {"bytes": w * elem + w * (2 * m * r + n * r) + 4 * n * r, "flops": 4 * r * elem},
        "spass": {"bytes": w * elem + w * (m * r + n * r) + 4 * E * m * r, "flops": 4 * r * elem},
    }


def roofline_of(cost: dict, avg_s: float, precision: str = "fp32") -> dict:
    """Bound = the resource whose peak gives the longer time for this kernel's
    algorithmic work (HBM at 8 TB/s; dense MFMA at 157.3 TFLOP/s in FP32,
    2.5 PFLOP/s in BF16)."""
    peak = MFMA_PEAK_TFS[precision]
    t_hbm = cost["bytes"] / (HBM_PEAK_GBS * 1e9)
    t_mfma = cost["flops"] / (peak * 1e12)
    hbm = {"bound": "hbm", "achieved": cost["bytes"] / avg_s / 1e9, "peak": HBM_PEAK_GBS,
           "unit": "GB/s"}
    mfma = {"bound": "mfma", "achieved": cost["flops"] / avg_s / 1e12,
            "peak": peak, "unit": "TFLOP/s"}
    main, other = (mfma, hbm) if t_mfma > t_hbm else (hbm, mfma)
    for d in (main, other):
        d["frac"] = round(d["achieved"] / d["peak"], 4)
        d["achieved"] = round(d["achieved"], 2)
    main["other"] = other
    return main


def src_hash() -> str:
    """Hash of the kernel sources, which the hardware counters were taken on."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_sample_rate(inst, U0, r, rho, lam, threads=None) -> dict:
    """One round of the FP64 oracle over a prefix of the clients (about 1/16
    of the columns), after an untimed warm-up on a sliver, scaled to the full
    column count (a round's work is linear in n); `threads` limits the BLAS
    threads (None: all)."""
    import contextlib

    import numpy as np
    import oracle.reference as O
    from threadpoolctl import threadpool_info, threadpool_limits
    blocks = inst.blocks()
    ncols, k = 0, 0
    while k < len(blocks) and ncols < inst.n / 16:
        ncols += blocks[k].shape[1]
        k += 1
    sub = [np.asarray(b, dtype=np.float64) for b in blocks[:k]]
    ctx = threadpool_limits(limits=threads) if threads else contextlib.nullcontext()
    with ctx:
        used = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        O.dcfpca([b[:, :8] for b in sub[:1]], r, rho, lam, 1, U0, record=False)
        t0 = time.perf_counter()
        O.dcfpca(sub, r, rho, lam, 1, U0, record=False)
        dt = (time.perf_counter() - t0) * inst.n / ncols
    return {"value": round(1.0 / dt, 5), "cores": int(used),
            "sample": f"one round of the FP64 numpy oracle over the first {k} of {inst.E} clients "
                      f"({ncols} of {inst.n} columns, m={inst.m}, r={r}), time scaled by "
                      f"{inst.n / ncols:.2f} to the full instance"}


def cpu_baseline(inst, U0, r, rho, lam, eval_inst=None, eval_U0=None, eval_r=None) -> dict:
    """The oracle as it stands, timed on this host: all cores and one core,
    on the headline workload and (when given) the evaluation workload."""
    allc = oracle_sample_rate(inst, U0, r, rho, lam)
    one = oracle_sample_rate(inst, U0, r, rho, lam, threads=1)
    out = {"value": allc["value"], "unit": "iters/s", "cores": allc["cores"], "kind": "oracle",
           "sample": allc["sample"], "cpu_model": cpu_model(),
           "host_cpus": os.cpu_count(), "single_thread_value": one["value"]}
    if eval_inst is not None:
        ea = oracle_sample_rate(eval_inst, eval_U0, eval_r, rho, 1.0 / math.sqrt(eval_inst.n))
        e1 = oracle_sample_rate(eval_inst, eval_U0, eval_r, rho, 1.0 / math.sqrt(eval_inst.n),
                                threads=1)
        out["eval_workload"] = {"workload": EVAL_WORKLOAD, "value": ea["value"],
                                "cores": ea["cores"], "single_thread_value": e1["value"],
                                "sample": ea["sample"]}
    return out


def continuation(lam: float, lam0: float, gamma: float = 0.8) -> list:
    """lambda_t = max(lambda, lambda0 gamma^t) up to the first round at lambda."""
    out = []
    while not out or out[-1] > lam:
        out.append(max(lam, lam0 * gamma ** len(out)))
    return out


def measure(M_cols, inst, r, rho, lam, U0_cols, args, precision: str, workload: str) -> dict:
    """Rounds/s of one precision on a resident instance: warm-up rounds, the
    autotuner, then `steps` rounds between HIP events on the library's stream,
    and per-kernel HIP events over `profile_rounds` more rounds. `workload`
    names the counter file (the workload, with the fitted rank when it is
    not the workload's)."""
    import torch

    from paper_2207_11669_amd import DCFPCA
    eta0 = 0.0 if args.u_mode == "closed" else 1e-4
    s = DCFPCA(M_cols, inst.widths, inst.m, r, rho, lam, U0_cols, u_mode=args.u_mode, eta0=eta0,
               graph=args.graph, bf16=precision == "bf16", bf16x3=precision == "bf16x3",
               sparse_s=not args.no_sparse_s and precision == "fp32")
    log(f"{precision}: warmup {args.warmup}")
    s.step(args.warmup)
    if args.launch_shape:
        keys = ("row_splits", "column_groups", "spass_phases", "vpass_queue", "spass_queue",
                "sparse_s")
        s.set_launch_shape(**dict(zip(keys, (int(x) for x in args.launch_shape.split(",")))))
        shape = s.launch_shape()
    else:
        shape = s.autotune(args.autotune) if args.autotune > 0 else s.launch_shape()
    torch.cuda.synchronize()
    first = s.rounds  # rounds run before the timed ones (warm-up and autotuner)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    log(f"{precision}: timing {args.steps} rounds from round {first}")
    ev0.record(s.stream)
    s.step(args.steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    st = s.stats()
    if not math.isfinite(st["objective"]):
        raise RuntimeError(f"{precision}: non-finite objective")
    log(f"{precision}: per-kernel events over {args.profile_rounds} rounds")
    prof = s.profile(args.profile_rounds)
    s.close()
    sparse = bool(shape.get("sparse_s"))
    costs = kernel_costs(inst.m, inst.n, inst.E, r, precision, sparse, st["nnz"])
    total = {k: v[0] * v[1] for k, v in prof.items()}
    dom = max(("vpass", "spass"), key=lambda k: total[k])
    roof = roofline_of(costs[dom], prof[dom][0] / 1e3, precision)
    # The launch shape selects the kernel instance of an FP32 pass: counters
    # are kept per instance ("spass:phases=2", "vpass:column_groups=1", ...).
    variant = dom
    if precision == "fp32":
        variant += (f":phases={shape['spass_phases']}" if dom == "spass"
                    else f":column_groups={shape['column_groups']}")
        variant += ":sparse" if sparse else ""
    traffic = None
    path = traffic_file(workload, precision)
    if os.path.exists(path):
        with open(path) as f:
            tr = json.load(f)
        if tr.get("kernel_source_sha256_16") == src_hash():
            per = tr.get("bytes_per_launch", {})
            traffic = per.get(variant, per.get(dom))
    roof.update({"traffic": traffic, "kernel": variant, "s_support": st["nnz"],
                 "algorithmic_bytes": costs[dom]["bytes"], "algorithmic_flops": costs[dom]["flops"],
                 "avg_launch_us": {k: round(v[0] * 1e3, 2) for k, v in prof.items()},
                 "launches_per_round": {k: v[1] / args.profile_rounds for k, v in prof.items()}})
    return {"iters_per_s": round(args.steps / (ms / 1e3), 2), "ms_per_step": round(ms / args.steps, 5),
            "autotuned_launch_shape": shape, "timed_from_round": first, "roofline": roof}


def error_vs_oracle(precision: str, low_rounds: int, closing_rounds: int) -> dict:
    """Relative Frobenius error of L and S against the FP64 oracle on the
    2000 x 2000 sub-instance of the headline recipe (rank 64, geometric
    spectrum, 5% corruption of magnitude U[1, 100], one client, r = 64):
    after `low_rounds` rounds in `precision`, and after `closing_rounds`
    further FP32 rounds (against the oracle's iterate after as many rounds)."""
    import numpy as np
    import torch

    import oracle.reference as O
    from paper_2207_11669_amd import DCFPCA, colmajor
    from rpca_inputs import gaussian_init, recipe
    inst = recipe(SUB_WORKLOAD, seed=0)
    r, rho = 64, 0.1
    lam = 1.0 / math.sqrt(inst.n)
    U0 = gaussian_init(inst.m, r, 7)
    a = O.dcfpca(inst.blocks(), r, rho, lam, low_rounds, U0, record=False)
    b = O.dcfpca(inst.blocks(), r, rho, lam, closing_rounds, a.U, S0=a.S, t0=low_rounds,
                 record=False)

    def LS(s):
        L, S = s.get_LS(-1)
        torch.cuda.synchronize()
        return (L[:, :inst.m].T.double().cpu().numpy(), S[:, :inst.m].T.double().cpu().numpy())

    def rel(x, y):
        return float(np.linalg.norm(x - y) / np.linalg.norm(y))

    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, rho, lam, colmajor(U0),
               bf16=precision == "bf16", bf16x3=precision == "bf16x3")
    s.step(low_rounds)
    L1, S1 = LS(s)
    if precision != "fp32":
        s.set_precision("fp32")
    s.step(closing_rounds)
    L2, S2 = LS(s)
    s.close()
    return {"instance": f"{SUB_WORKLOAD} (m=n=2000, r=64, one client)",
            "schedule": f"{low_rounds} {precision} rounds, then {closing_rounds} fp32 rounds",
            f"after_{low_rounds}_{precision}_rounds": {"relL": rel(L1, a.L_full()),
                                                        "relS": rel(S1, a.S_full())},
            f"after_{closing_rounds}_fp32_closing_rounds": {"relL": rel(L2, b.L_full()),
                                                            "relS": rel(S2, b.S_full())}}


def tuned_shape(M_cols, inst, r, rho, lam, U0_cols, args, precision: str) -> dict:
    """Launch shape picked by the autotuner on a context of its own (FP32:
    with RPCA_FLAG_SPARSE_S, so that it also decides the sparse handoff), so
    that the timed runs below start from U^(0) with a tuned shape."""
    import torch

    from paper_2207_11669_amd import DCFPCA
    eta0 = 0.0 if args.u_mode == "closed" else 1e-4
    s = DCFPCA(M_cols, inst.widths, inst.m, r, rho, lam, U0_cols, u_mode=args.u_mode, eta0=eta0,
               bf16x3=precision == "bf16x3", sparse_s=precision == "fp32")
    s.step(max(args.warmup, 5))
    shape = s.autotune(args.autotune) if args.autotune > 0 else s.launch_shape()
    torch.cuda.synchronize()
    s.close()
    return shape


def time_to_target(M_cols, inst, r, rho, lam, U0_cols, args, target, max_rounds,
                   schedule=None, ctl=None, lam0=None, precision="fp32", shape=None) -> dict:
    """Wall time from U^(0) until ||U V^T - X Y^T||_F / ||X Y^T||_F <= 1e-4 for
    the target factors (X, Y), checked every 10 rounds with r x r Gram
    matrices (L is never formed) by rpca_solve. With a lambda schedule (a
    list, or a controller deciding round by round from the recorded
    statistics), its rounds run first and count."""
    import torch

    from paper_2207_11669_amd import DCFPCA
    from paper_2207_11669_amd import controller as C
    eta0 = 0.0 if args.u_mode == "closed" else 1e-4
    sparse = bool(shape and shape.get("sparse_s"))
    s2 = DCFPCA(M_cols, inst.widths, inst.m, r, rho, lam, U0_cols, u_mode=args.u_mode,
                eta0=eta0, bf16x3=precision == "bf16x3", sparse_s=sparse)
    if shape:
        s2.set_launch_shape(**shape)
    s2.set_target(*target)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pre = 0
    for lt in schedule or []:
        s2.set_lambda(lt)
        s2.step(1)
        pre += 1
    ctrl = None
    if ctl is not None:
        ctrl = C.run_controlled(s2, lam, lam0, ctl, float(inst.m) * inst.n)
        pre += ctrl["control_rounds"]
    s2.set_lambda(lam)
    done, err = s2.solve(max_rounds - pre, 1e-4, check_every=10)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    s2.close()
    out = {"tol": 1e-4, "reached": bool(err <= 1e-4), "rounds": pre + done,
           "seconds": round(secs, 4), "final_relerr": err, "max_rounds": max_rounds,
           "check_every": 10, "precision": precision, "launch_shape": shape}
    if ctrl is not None:
        out["control"] = {"rounds": ctrl["control_rounds"], "rejected": ctrl["rejected"],
                          "decays": [round(g, 3) for g in ctrl["gammas"]],
                          "steps": [round(w, 3) for w in ctrl["omegas"]]}
    return out


def learned_controller():
    """The learned controller with the parameters committed next to the
    package (paper_2207_11669_amd/controller_weights.json, written by
    paper_2207_11669_amd/train_controller.py on instances of the evaluation
    workload's family), and the description of their training."""
    from paper_2207_11669_amd import controller as C
    ctl, info = C.LearnedContinuation.load()
    log(f"learned controller: {info.get('training_instances')} training instances of "
        f"{info.get('training_size')}")
    return ctl, info


def relerr_suite(args, dev) -> tuple:
    """Time to relative error 1e-4 against L* on the evaluation workload for
    plain FP32 rounds, the fixed continuation, the learned controller and the
    learned controller with three-product BF16 rounds."""
    import numpy as np
    import torch

    from paper_2207_11669_amd import colmajor
    from rpca_inputs import RECIPES, gaussian_init, recipe
    log(f"generating {EVAL_WORKLOAD}")
    inst = recipe(EVAL_WORKLOAD, seed=0)
    cfg = RECIPES[EVAL_WORKLOAD]
    r, rho = cfg["r"], cfg["rho"]
    lam = 1.0 / math.sqrt(inst.n)
    U0 = gaussian_init(inst.m, r, 7)
    M_cols = colmajor(inst.M, device=dev)
    U0_cols = colmajor(U0, device=dev)
    target = (colmajor(inst.Ustar, device=dev), colmajor(inst.Vstar, device=dev), cfg["rstar"])
    lam0 = float(np.abs(inst.M).max())
    out = {"workload": EVAL_WORKLOAD, "m": inst.m, "n": inst.n, "E": inst.E, "r": r,
           "planted_rank": cfg["rstar"], "corruption": cfg["s"], "lambda": lam, "rho": rho}
    log("launch shapes for the timed runs (autotuner, on contexts of their own)")
    sh32 = tuned_shape(M_cols, inst, r, rho, lam, U0_cols, args, "fp32")
    sh3 = tuned_shape(M_cols, inst, r, rho, lam, U0_cols, args, "bf16x3")
    log("time to 1e-4: plain fp32")
    out["plain_fp32"] = time_to_target(M_cols, inst, r, rho, lam, U0_cols, args, target,
                                       args.relerr_rounds, shape=sh32)
    log("time to 1e-4: fixed continuation")
    sched = continuation(lam, lam0)
    out["fixed_continuation"] = dict(
        time_to_target(M_cols, inst, r, rho, lam, U0_cols, args, target, args.relerr_rounds,
                       schedule=sched, shape=sh32),
        kind="lambda_t = max(lambda, max|M| 0.8^t)", schedule_rounds=len(sched))
    ctl, info = learned_controller()
    out["controller_training"] = info
    log("time to 1e-4: learned controller")
    out["learned"] = time_to_target(M_cols, inst, r, rho, lam, U0_cols, args, target,
                                    args.relerr_rounds, ctl=ctl, lam0=lam0, shape=sh32)
    log("time to 1e-4: learned controller, three-product BF16 rounds")
    out["learned_bf16x3"] = time_to_target(M_cols, inst, r, rho, lam, U0_cols, args, target,
                                           args.relerr_rounds, ctl=ctl, lam0=lam0,
                                           precision="bf16x3", shape=sh3)
    base = out["plain_fp32"]["seconds"]
    out["speedup_vs_plain_fp32"] = {k: round(base / out[k]["seconds"], 3)
                                    for k in ("fixed_continuation", "learned", "learned_bf16x3")
                                    if out[k]["reached"] and out["plain_fp32"]["reached"]}
    del M_cols, U0_cols, target
    torch.cuda.empty_cache()
    return out, inst, U0, r


def copy_calibration() -> int:
    import torch
    n = (256 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.zeros(n, dtype=torch.float32, device="cuda:0")
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))
    return 0


def hbm_ceiling() -> int:
    """What plain streaming kernels of the runtime reach on this GPU, as a
    practical HBM ceiling beside the 8 TB/s peak: torch's device copy (read
    and write), sum (read) and fill (write) of 4 GiB, each timed over 10
    launches with HIP events after one untimed launch."""
    import torch
    n = 1 << 30
    x = torch.empty(n, dtype=torch.float32, device="cuda:0").normal_()
    y = torch.empty_like(x)
    z = torch.empty((), dtype=torch.float32, device="cuda:0")

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps / 1e3

    out = {}
    for name, fn, nbytes in (("copy", lambda: y.copy_(x), 8 * n),
                             ("sum", lambda: torch.sum(x, dim=0, out=z), 4 * n),
                             ("fill", lambda: x.fill_(1.0), 4 * n)):
        sec = timed(fn)
        out[name] = {"bytes": nbytes, "ms": round(sec * 1e3, 4),
                     "GB_per_s": round(nbytes / sec / 1e9, 1)}
    print(json.dumps({"hbm_ceiling": out}))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default=WORKLOAD, choices=WORKLOADS,
                    help="workload of the timed rounds (default: the 20000 x 100000, r = 64 "
                         "geometric-spectrum workload)")
    ap.add_argument("--rank", type=int, default=0,
                    help="fitted rank r instead of the workload's (1 .. 128)")
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--u-mode", default="closed", choices=["closed", "grad"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "bf16x3"],
                    help="arithmetic of the headline rounds' streaming passes")
    ap.add_argument("--graph", action="store_true",
                    help="replay steady-state rounds from HIP graphs (RPCA_FLAG_GRAPH)")
    ap.add_argument("--no-sparse-s", action="store_true",
                    help="create the FP32 contexts without RPCA_FLAG_SPARSE_S (by default the "
                         "flag is set and the autotuner decides whether FP32 rounds hand S from "
                         "the S-pass to the next V-pass in sparse form or rebuild it)")
    ap.add_argument("--autotune", type=int, default=20, metavar="ROUNDS",
                    help="before timing, pick the launch shapes with rpca_autotune (ROUNDS timed "
                         "rounds per candidate); 0 keeps the defaults")
    ap.add_argument("--launch-shape", default="", metavar="RS,CG,PH,VQ,SQ[,SP]",
                    help="pin the launch shape instead of autotuning it: V-pass row splits, "
                         "column groups per wave, S-pass column phases, V-pass and S-pass "
                         "persistent launch forms (0/1), and the sparse S handoff (0/1; "
                         "not with --no-sparse-s)")
    ap.add_argument("--profile-rounds", type=int, default=20)
    ap.add_argument("--relerr-rounds", type=int, default=6000,
                    help="round budget of the time-to-relerr runs")
    ap.add_argument("--low-rounds", type=int, default=20,
                    help="low-precision rounds before the FP32 closing rounds in the error check")
    ap.add_argument("--closing-rounds", type=int, default=20)
    ap.add_argument("--no-mixed", action="store_true", help="skip the BF16 legs")
    ap.add_argument("--no-relerr", action="store_true", help="skip the time-to-relerr legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device to device three times (a kernel of known "
                         "traffic, to scale hardware byte counters) and exit")
    ap.add_argument("--hbm-ceiling", action="store_true",
                    help="time torch's copy, sum and fill of 4 GiB (a practical HBM ceiling) "
                         "and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.hbm_ceiling:
        return hbm_ceiling()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the DCF-PCA path here runs every client on a "
              "single MI355X, so --gpus must be 1.", file=sys.stderr)
        return 2

    import torch

    from paper_2207_11669_amd import colmajor
    from rpca_inputs import RECIPES, gaussian_init, recipe

    workload = args.workload
    cfg = RECIPES[workload]
    r, rho = (args.rank or cfg["r"]), cfg["rho"]
    # Counters of a fit at another rank live in a file of their own.
    tag = workload if r == cfg["r"] else f"{workload}_fit{r}"
    log(f"generating {workload}")
    inst = recipe(workload, seed=0)
    lam = 1.0 / math.sqrt(inst.n)
    U0 = gaussian_init(inst.m, r, 7)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    M_cols = colmajor(inst.M, device=dev)
    U0_cols = colmajor(U0, device=dev)
    torch.cuda.synchronize()

    head = measure(M_cols, inst, r, rho, lam, U0_cols, args, args.precision, tag)
    mixed = None
    if not args.no_mixed and args.precision == "fp32" and r <= 64:
        mixed = {}
        for prec in ("bf16", "bf16x3"):
            mixed[prec] = measure(M_cols, inst, r, rho, lam, U0_cols, args, prec, tag)
            mixed[prec]["speedup_vs_fp32"] = round(mixed[prec]["iters_per_s"] /
                                                   head["iters_per_s"], 3)
            log(f"{prec}: error against the FP64 oracle on the 2000 x 2000 sub-instance")
            mixed[prec]["error_vs_fp64_oracle"] = error_vs_oracle(prec, args.low_rounds,
                                                                  args.closing_rounds)
        mixed["fp32_error_vs_fp64_oracle"] = error_vs_oracle("fp32", args.low_rounds,
                                                             args.closing_rounds)
    del M_cols, U0_cols
    torch.cuda.empty_cache()

    relerr = eval_inst = eval_U0 = eval_r = None
    if not args.no_relerr:
        relerr, eval_inst, eval_U0, eval_r = relerr_suite(args, dev)

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        cpu = cpu_baseline(inst, U0, r, rho, lam, eval_inst, eval_U0, eval_r)

    out = {
        "metric": METRIC, "value": head["iters_per_s"], "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "bf16x3": "bf16x3 (hi/lo splits, f32 M)"}[
            args.precision],
        "data": "synthetic",
        "config": {"workload": workload, "m": inst.m, "n": inst.n, "E": inst.E, "r": r,
                   "planted_rank": cfg["rstar"], "corruption": cfg["s"], "lambda": lam,
                   "rho": rho, "K": 1, "inner": 1, "u_mode": args.u_mode,
                   "graph": bool(args.graph), "sparse_s_flag": not args.no_sparse_s,
                   "precision": args.precision,
                   "autotuned_launch_shape": head["autotuned_launch_shape"],
                   "timed_from_round": head["timed_from_round"]},
        "roofline": head["roofline"],
        "mixed_precision": mixed,
        "time_to_relerr": relerr,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
