"""Round-by-round lambda control for DCF-PCA: a fixed continuation and a
learned one driven by the library's MLP (rpca_mlp_*).

The paper fixes lambda. A controller runs the same rounds but chooses each
round's lambda_t = lambda * s_t with a scale s_t >= 1 that only decreases,
s_t = max(1, s_{t-1} g_t), starting from s_0 = lambda0 / lambda (by default
lambda0 = max|M|, so that no entry is thresholded at first and L takes the
bulk of M before S takes the outliers). Once s reaches 1 the plain method
runs on, so the fixed point is the plain method's; the plain fixed-lambda
rounds are also the fallback when the controller has decided nothing after
max_control rounds. The fixed continuation uses g_t = 0.8. The learned
controller takes g_t in [0.5, 1] from the MLP, fed with eight features of the
last recorded rounds (all scale-free).

Training targets come from a per-round greedy search: from the current state,
each candidate decay is tried for a few lookahead rounds on a copy of the
iterate (rpca_copy_state), and the one whose iterate is closest to the
planted L* wins.
"""
from __future__ import annotations

import math
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

from .binding import DCFPCA, mlp_forward, mlp_param_count, mlp_train_step

GAMMAS = (0.5, 0.6, 0.7, 0.8, 0.9, 1.0)
N_FEATURES = 8


def features(st: dict, prev: Optional[dict], scale: float, gamma_prev: float, t: int,
             lam: float, mn: float) -> List[float]:
    """Eight scale-free features of the last finished round (st, recorded at
    lambda * scale) and the one before it (prev)."""
    lt = lam * scale
    sat = st["lambda_fro_sq"] / max(mn * lt * lt, 1e-300)        # ||Lambda||^2 / (mn lambda_t^2)
    nnz = st["nnz"] / mn                                          # fraction of S's support
    du = math.log10(st["du_sq"] / max(st["u_sq"], 1e-300) + 1e-12) / 12.0 + 1.0
    grow = 0.0
    if prev is not None and prev["u_sq"] > 0:
        grow = max(-1.0, min(1.0, math.log(max(st["u_sq"], 1e-300) / prev["u_sq"])))
    l1 = math.log10(st["l1"] / max(mn * lt, 1e-300) + 1e-12) / 6.0
    return [math.log10(max(scale, 1.0)) / 4.0, min(t, 100) / 100.0, min(sat, 1.0), nnz, du,
            grow, gamma_prev, l1]


class FixedContinuation:
    def __init__(self, gamma: float = 0.8):
        self.gamma = float(gamma)

    def decide(self, feats: Sequence[float]) -> float:
        return self.gamma


class LearnedContinuation:
    """g_t from the MLP (inference on the GPU, rpca_mlp_forward)."""

    def __init__(self, params):
        self.params = params  # FP32 CUDA tensor of mlp_param_count() floats

    def decide(self, feats: Sequence[float]) -> float:
        import torch
        x = torch.tensor([list(feats)], dtype=torch.float32, device=self.params.device)
        g = float(mlp_forward(self.params, x).cpu()[0])
        # Fallback for a non-finite proposal: the fixed continuation's decay.
        return g if math.isfinite(g) else 0.8


def run_controlled(s: DCFPCA, lam: float, lam0: float, controller, mn: float,
                   max_control: int = 200) -> dict:
    """Run the controlled rounds on session s until the scale reaches 1 (or
    max_control rounds); leaves lambda at its target. Returns the decays."""
    scale = max(1.0, lam0 / lam)
    gammas: List[float] = []
    prev = None
    t = 0
    g = 1.0
    while scale > 1.0 and t < max_control:
        s.set_lambda(lam * scale)
        s.step(1)
        st = s.stats(-1)
        g = float(min(1.0, max(0.5, controller.decide(features(st, prev, scale, g, t, lam, mn)))))
        gammas.append(g)
        prev = st
        scale = max(1.0, scale * g)
        t += 1
    s.set_lambda(lam)
    return {"control_rounds": t, "gammas": gammas}


def greedy_samples(make_session: Callable[[], DCFPCA], lam: float, lam0: float, mn: float,
                   horizon: int = 5, gammas: Sequence[float] = GAMMAS,
                   max_control: int = 80) -> Tuple[np.ndarray, np.ndarray]:
    """(features, best decay) pairs along one greedy trajectory: at each round
    every candidate decay runs `horizon` lookahead rounds on a copy of the
    iterate, and the one closest to the target (set on the sessions) wins.
    make_session returns a fresh session with the target registered."""
    main, probe = make_session(), make_session()
    scale = max(1.0, lam0 / lam)
    X, Y = [], []
    prev = None
    g = 1.0
    t = 0
    main.set_lambda(lam * scale)
    main.step(1)
    while scale > 1.0 and t < max_control:
        st = main.stats(-1)
        f = features(st, prev, scale, g, t, lam, mn)
        errs = []
        for cand in gammas:
            probe.copy_state_from(main)
            sc = scale
            for _ in range(horizon):
                sc = max(1.0, sc * cand)
                probe.set_lambda(lam * sc)
                probe.step(1)
            errs.append(probe.target_error())
        g = float(gammas[int(np.argmin(errs))])
        X.append(f)
        Y.append(g)
        prev = st
        scale = max(1.0, scale * g)
        main.set_lambda(lam * scale)
        main.step(1)
        t += 1
    main.close()
    probe.close()
    return np.asarray(X, dtype=np.float32), np.asarray(Y, dtype=np.float32)


def init_params(seed: int = 0) -> np.ndarray:
    """Scaled Gaussian weights (1/sqrt(fan-in)), zero biases."""
    rng = np.random.default_rng(seed)
    h, k = 64, N_FEATURES
    parts = [rng.standard_normal(h * k) / math.sqrt(k), np.zeros(h),
             rng.standard_normal(h * h) / math.sqrt(h), np.zeros(h),
             rng.standard_normal(h) / math.sqrt(h), np.zeros(1)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == mlp_param_count()
    return p


def train(X: np.ndarray, Y: np.ndarray, steps: int = 2000, lr: float = 0.5, seed: int = 0,
          device="cuda") -> Tuple["object", List[float]]:
    """Full-batch gradient descent on the GPU (rpca_mlp_train_step); returns
    the parameters (CUDA tensor) and the loss every 100 steps."""
    import torch
    p = torch.from_numpy(init_params(seed)).to(device)
    x = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(device)
    y = torch.from_numpy(np.ascontiguousarray(Y, dtype=np.float32)).to(device)
    ws = torch.empty(int(x.shape[0]) * mlp_param_count(), dtype=torch.float32, device=device)
    losses = []
    for k in range(steps):
        if k % 100 == 0:
            pred = mlp_forward(p, x)
            losses.append(float(0.5 * torch.mean((pred - y) ** 2)))
        mlp_train_step(p, x, y, lr, ws)
    return p, losses


def fit(cases, horizon: int = 15, steps: int = 2000, lr: float = 0.5, seed: int = 0):
    """Train the learned controller: greedy samples along each training case,
    then full-batch gradient descent. cases yields (make_session, lam, lam0,
    mn) per training instance, make_session returning a fresh session with
    the planted target registered. Returns (params, samples, losses)."""
    Xs, Ys = [], []
    for make_session, lam, lam0, mn in cases:
        X, Y = greedy_samples(make_session, lam, lam0, mn, horizon=horizon)
        Xs.append(X)
        Ys.append(Y)
    X, Y = np.concatenate(Xs), np.concatenate(Ys)
    params, losses = train(X, Y, steps=steps, lr=lr, seed=seed)
    return params, (X, Y), losses
