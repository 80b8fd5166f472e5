"""Fitted ranks above 64 (five to eight 16-rank tiles; the paper's upper-bound
rank experiments, Section 4.2 and Table 1, fit p = 0.1 n and more): the FP32
passes with one column group per V-pass wave and one S-pass column phase,
full rank tiles, and a standalone finalize. Against the FP64 oracle on ragged
rows and client widths, in both U steps and with local steps; clients
narrower than the rank against the oracle's own sensitivity to FP32 there;
bitwise across launch forms, row splits, sparse S and graph replay; the
relative error against a target of rank above 64."""
import numpy as np
import pytest

import oracle.reference as O
from gpu_helpers import (announce, default_lam, init_for, parity, rel, run_gpu, run_oracle,
                         TOL)
from rpca_inputs import planted_instance

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("r", [65, 80, 100, 128])
def test_wide_rank_parity(r):
    """Fitted rank above the planted one, as in the upper-bound experiments;
    every client at least r columns wide."""
    inst = planted_instance(333, [150, 130, 201, 177], 12, 0.05, values="uniform", hi=10.0,
                            seed=80 + r)
    s, _Lg, _Sg, hist, res = parity(inst, r, 25, u_mode="closed")
    for g, o in zip(hist, res.history):
        assert g["t"] == o["t"]
        assert abs(g["objective"] - o["objective"]) <= 1e-5 * abs(o["objective"])
        assert abs(g["u_sq"] - o["u_sq"]) <= 1e-5 * o["u_sq"]
    s.close()


def test_wide_rank_high_planted_rank():
    """A planted rank of 90 fitted at r = 96."""
    inst = planted_instance(400, [200, 250], 90, 0.05, values="uniform", hi=10.0, seed=91)
    parity(inst, 96, 30, u_mode="closed")[0].close()


def test_wide_rank_grad_and_local_steps():
    """Gradient U step with the decaying step size, K = 2 local steps of two
    V/S alternations each (stored S, per-client finalize); closed-form local
    steps."""
    inst = planted_instance(250, [60, 90, 33], 8, 0.05, values="signed", lo=2.0, hi=8.0,
                            seed=92)
    parity(inst, 72, 15, u_mode="grad", eta0=2e-3, eta_sched="sqrt", K=2,
           inner=2)[0].close()
    inst = planted_instance(250, [130, 140, 125], 8, 0.05, values="signed", lo=2.0, hi=8.0,
                            seed=93)
    parity(inst, 120, 15, u_mode="closed", K=2, inner=1)[0].close()


def _closed_U_rounded_P(V, S, M, rho, n_i, n):
    """The oracle's closed-form U step with P = (M - S) V rounded to FP32
    once (its only change)."""
    r = V.shape[1]
    A = V.T @ V + (rho * n_i / n) * np.eye(r)
    P = ((M - S) @ V).astype(np.float32).astype(np.float64)
    return np.linalg.solve(A, P.T).T


@pytest.mark.parametrize("case", ["r128_K1", "r120_K2"])
def test_wide_rank_narrow_clients(case):
    """Clients narrower than the rank: V_i^T V_i is singular and A_i =
    (V_i^T V_i + c_i I)^{-1} has eigenvalues 1/c_i = n / (rho n_i) on its null
    space, where the closed-form step's output cancels exactly in exact
    arithmetic and any FP32 error of P = (M - S) V_i comes out multiplied by
    1/c_i. The bar is the larger of 1e-5 and delta, the difference that
    rounding P to FP32 once per step (nothing else) makes to the oracle's own
    trajectory."""
    if case == "r128_K1":
        inst = planted_instance(333, [64, 150, 80, 129], 12, 0.05, values="uniform", hi=10.0,
                                seed=208)
        r, T, kw = 128, 25, dict(u_mode="closed")
    else:
        inst = planted_instance(250, [60, 90, 33], 8, 0.05, values="signed", lo=2.0, hi=8.0,
                                seed=92)
        r, T, kw = 120, 15, dict(u_mode="closed", K=2, inner=1)
    lam = default_lam(inst)
    U0 = init_for(inst, r, 7)
    ref = run_oracle(inst, U0, r, 0.1, lam, T, **kw)
    keep = O.closed_U
    O.closed_U = _closed_U_rounded_P
    try:
        pert = run_oracle(inst, U0, r, 0.1, lam, T, **kw)
    finally:
        O.closed_U = keep
    delta = max(rel(pert.L_full(), ref.L_full()), rel(pert.S_full(), ref.S_full()))
    s, Lg, Sg, _ = run_gpu(inst, U0, r, 0.1, lam, T, **kw)
    s.close()
    eL, eS = rel(Lg, ref.L_full()), rel(Sg, ref.S_full())
    tol = max(TOL, delta)
    announce(f"{case}: widths={inst.widths} relL={eL:.3e} relS={eS:.3e}; P rounded once: "
             f"delta={delta:.3e}; bar {tol:.3e}")
    assert eL <= tol and eS <= tol


def _snap(s):
    import torch
    L, S = s.get_LS(-1)
    torch.cuda.synchronize()
    return L[:, :s.m].cpu().numpy(), S[:, :s.m].cpu().numpy(), s.stats()


def _trajectory(inst, r, rounds, shape=None, **kw):
    from paper_2207_11669_amd import DCFPCA, colmajor
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, 0.1, default_lam(inst),
               colmajor(init_for(inst, r, 5)), **kw)
    if shape:
        s.set_launch_shape(**shape)
    out = []
    for chunk in (1, 2, rounds - 3):
        s.step(chunk)
        out.append(_snap(s))
    s.close()
    return out


def _same(a, b):
    return all(np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) and x[2] == y[2]
               for x, y in zip(a, b))


def test_wide_rank_forms_are_bitwise():
    """Persistent tile-queue launches, sparse S and graph replay run the same
    sums in the same order as the per-tile launches with S rebuilt, at the
    default row splits and at 7 (whose V-pass chunks start on odd 16-row
    tiles of the S-pass strips). (Another row split count sums W's partials
    in another order.)"""
    inst = planted_instance(1007, [9, 300, 177, 64, 410], 10, 0.06, values="uniform", hi=10.0,
                            seed=93, support="bernoulli")
    r = 128
    queue = dict(vpass_queue=1, spass_queue=1)
    for splits in (None, 7):
        rs = {} if splits is None else dict(row_splits=splits)
        base = _trajectory(inst, r, 9, shape=rs)
        variants = {
            "queue": dict(shape={**rs, **queue}),
            "sparse": dict(sparse_s=True, shape=rs),
            "sparse_queue": dict(sparse_s=True, shape={**rs, **queue}),
            "graph": dict(graph=True, shape=rs),
        }
        for name, kw in variants.items():
            other = _trajectory(inst, r, 9, **kw)
            same = _same(base, other)
            announce(f"r={r} row splits {splits or 'default'}, {name}: bitwise={same} "
                     f"relL={rel(other[-1][0], base[-1][0]):.2e} nnz={other[-1][2]['nnz']:.0f}")
            assert same, name


def test_wide_rank_shapes_and_autotune():
    from paper_2207_11669_amd import DCFPCA, RpcaError, colmajor
    inst = planted_instance(700, [300, 250, 120], 10, 0.05, values="uniform", hi=10.0, seed=94)
    r = 112
    U0 = init_for(inst, r, 6)
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, 0.1, default_lam(inst), colmajor(U0))
    shape = s.launch_shape()
    assert shape["column_groups"] == 1 and shape["spass_phases"] == 1
    for kw in (dict(column_groups=4), dict(spass_phases=2)):
        with pytest.raises(RpcaError, match="ranks above 64"):
            s.set_launch_shape(**kw)
    assert s.launch_shape() == shape
    s.step(2)
    picked = s.autotune(2)
    announce(f"r={r} autotune picked {picked}")
    assert picked["column_groups"] == 1 and picked["spass_phases"] == 1
    s.step(3)
    T = s.rounds
    import torch
    L, S = s.get_LS(-1)
    torch.cuda.synchronize()
    La = L[:, :inst.m].T.double().cpu().numpy()
    Sa = S[:, :inst.m].T.double().cpu().numpy()
    res = run_oracle(inst, U0, r, 0.1, default_lam(inst), T)
    eL, eS = rel(La, res.L_full()), rel(Sa, res.S_full())
    announce(f"autotuned run, {T} rounds, vs the oracle: relL={eL:.3e} relS={eS:.3e}")
    assert eL <= TOL and eS <= TOL
    s.close()


@pytest.mark.parametrize("r,rstar", [(80, 100), (128, 30), (40, 128)])
def test_wide_rank_target_error(r, rstar):
    """rpca_target_error with factor widths above 64 on either side, against
    the same distance formed in FP64 from the returned factors."""
    import torch

    from paper_2207_11669_amd import DCFPCA, colmajor
    inst = planted_instance(300, [120, 70, 100], 8, 0.05, values="uniform", hi=10.0, seed=95)
    rng = np.random.default_rng(96)
    Us = rng.standard_normal((inst.m, rstar))
    Vs = rng.standard_normal((inst.n, rstar)) / np.sqrt(rstar)
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, 0.1, default_lam(inst),
               colmajor(init_for(inst, r, 7)))
    s.step(5)
    s.set_target(colmajor(Us), colmajor(Vs), rstar)
    got = s.target_error()
    U, V = s.get_factors()
    torch.cuda.synchronize()
    Un = U[:, :inst.m].T.double().cpu().numpy()
    Vn = V[:, :inst.n].T.double().cpu().numpy()
    Ls = Us.astype(np.float32).astype(np.float64) @ Vs.astype(np.float32).astype(np.float64).T
    want = rel(Un @ Vn.T, Ls)
    announce(f"r={r} rstar={rstar}: target error {got:.9e} vs FP64 {want:.9e}")
    assert abs(got - want) <= 1e-9 * want
    s.close()


def test_wide_rank_schedule_stored_s_and_copy():
    """Rank 100: a lambda continuation with the sparse S handoff (rounds after
    a lambda change rebuild S) against the oracle run with the same schedule,
    each round's objective included; stored S (RPCA_FLAG_STORE_S) bitwise equal
    to rebuilt S; and rpca_copy_state mid-run continuing bitwise."""
    import math

    import torch

    from paper_2207_11669_amd import DCFPCA, colmajor
    inst = planted_instance(400, [150, 130, 120], 10, 0.08, values="signed", lo=5.0, hi=20.0,
                            seed=97)
    r = 100
    lam = float(np.float32(1.0 / math.sqrt(inst.n)))
    U0 = init_for(inst, r, 8)
    lam0 = float(np.abs(inst.M).max())
    sched = [max(lam, lam0 * 0.8 ** t) for t in range(30)] + [lam] * 6
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, 0.1, lam, colmajor(U0), sparse_s=True)
    for lt in sched:
        s.set_lambda(lt)
        s.step(1)
    L, S = s.get_LS(-1)
    torch.cuda.synchronize()
    Lg = L[:, :inst.m].T.double().cpu().numpy()
    Sg = S[:, :inst.m].T.double().cpu().numpy()
    res = O.dcfpca(inst.blocks(), r, 0.1, lam, len(sched), U0, lam_schedule=sched)
    eL, eS = rel(Lg, res.L_full()), rel(Sg, res.S_full())
    hist = [s.stats(t) for t in range(len(sched))]
    ef = max(abs(g["objective"] - o["objective"]) / abs(o["objective"])
             for g, o in zip(hist, res.history))
    announce(f"r={r} continuation with sparse S: relL={eL:.3e} relS={eS:.3e} "
             f"max objective rel={ef:.3e}")
    assert eL <= TOL and eS <= TOL and ef <= TOL
    s.close()

    lam_d = default_lam(inst)
    _, L1, S1, _ = run_gpu(inst, U0, r, 0.1, lam_d, 12)
    _, L2, S2, _ = run_gpu(inst, U0, r, 0.1, lam_d, 12, store_s=True)
    same = np.array_equal(L1, L2) and np.array_equal(S1, S2)
    announce(f"r={r} rebuilt vs stored S: bitwise={same}")
    assert same

    a = DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, 0.1, lam_d, colmajor(U0), sparse_s=True)
    b = DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, 0.1, lam_d, colmajor(U0), sparse_s=True)
    a.step(5)
    b.copy_state_from(a)
    a.step(4)
    b.step(4)
    snaps = []
    for x in (a, b):
        L, S = x.get_LS(-1)
        torch.cuda.synchronize()
        snaps.append((L.cpu().numpy(), S.cpu().numpy(), x.stats()))
    a.close()
    b.close()
    same = (np.array_equal(snaps[0][0], snaps[1][0]) and np.array_equal(snaps[0][1], snaps[1][1])
            and snaps[0][2] == snaps[1][2])
    announce(f"r={r} copy_state mid-run: bitwise={same}")
    assert same
