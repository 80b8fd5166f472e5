"""Shared helpers for the GPU parity tests: run the HIP path and the FP64
oracle on the same seeded instance and compare what is unique (L and S)."""
from __future__ import annotations

import math
import sys

import numpy as np

import oracle.reference as O
from rpca_inputs import Instance, gaussian_init


def announce(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def run_gpu(inst: Instance, U0: np.ndarray, r: int, rho: float, lam: float, T: int,
            shape: dict | None = None, **kw):
    import torch

    from paper_2207_11669_amd import DCFPCA, colmajor
    M_cols = colmajor(inst.M)
    U0_cols = colmajor(U0)
    s = DCFPCA(M_cols, inst.widths, inst.m, r, rho, lam, U0_cols, **kw)
    if shape:
        s.set_launch_shape(**shape)
    s.step(T)
    L, S = s.get_LS(-1)
    torch.cuda.synchronize()
    m = inst.m
    Lg = L[:, :m].T.double().cpu().numpy()
    Sg = S[:, :m].T.double().cpu().numpy()
    hist = [s.stats(t) for t in range(max(0, T - min(T, 4096)), T)]
    return s, Lg, Sg, hist


def run_oracle(inst: Instance, U0: np.ndarray, r: int, rho: float, lam: float, T: int,
               K: int = 1, inner: int = 1, u_mode: str = "closed", eta0: float = 0.0,
               eta_sched: str = "const", store_s: bool = False, sparse_s: bool = False):
    # store_s and sparse_s choose how the HIP path keeps S between its passes;
    # the oracle's arithmetic has no such choice.
    return O.dcfpca(inst.blocks(), r, rho, lam, T, U0, K=K, inner=inner, u_mode=u_mode,
                    eta0=eta0, eta_sched=eta_sched)


def rel(a: np.ndarray, b: np.ndarray) -> float:
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


def default_lam(inst: Instance) -> float:
    return 1.0 / math.sqrt(inst.n)


def init_for(inst: Instance, r: int, seed: int) -> np.ndarray:
    return gaussian_init(inst.m, r, seed)


TOL = 1e-5


def parity(inst: Instance, r: int, T: int, seed: int = 7, rho: float = 0.1, lam=None,
           tol: float = TOL, shape: dict | None = None, **kw):
    """Run both paths for T rounds and require relative Frobenius differences
    <= tol on L and on S (shape: launch shapes of the HIP path)."""
    lam = default_lam(inst) if lam is None else lam
    U0 = init_for(inst, r, seed)
    announce(f"m={inst.m} widths={inst.widths[:8]}{'...' if inst.E > 8 else ''} r={r} T={T} "
             f"{kw} shape={shape}")
    s, Lg, Sg, hist = run_gpu(inst, U0, r, rho, lam, T, shape=shape, **kw)
    res = run_oracle(inst, U0, r, rho, lam, T, **kw)
    eL = rel(Lg, res.L_full())
    eS = rel(Sg, res.S_full())
    announce(f"relL={eL:.3e} relS={eS:.3e}")
    assert eL <= tol, eL
    assert eS <= tol, eS
    return s, Lg, Sg, hist, res
