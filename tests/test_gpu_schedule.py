"""A lambda schedule (rpca_set_lambda between rounds) against the FP64
oracle run with the same schedule: L and S to the FP32 bar, and each round's
recorded objective evaluated at that round's lambda."""
import math

import numpy as np
import pytest

from gpu_helpers import TOL, announce, init_for, rel
import oracle.reference as O
from rpca_inputs import planted_instance

pytestmark = pytest.mark.gpu


def _continuation(inst, lam, T, gamma=0.8):
    mx = float(np.abs(inst.M).max())
    # The library keeps lambda in FP32; hand the oracle the same values.
    return [float(np.float32(max(lam, mx * gamma ** t))) for t in range(T)]


@pytest.mark.parametrize("bf16", [False, True])
def test_lambda_continuation_matches_oracle(bf16):
    """300 x 300, rank 5, 10% corrupted with magnitude U[5, 20], three clients,
    r = 5, lambda_t = max(1/sqrt(300), max|M| 0.8^t) for 40 rounds (it reaches
    the target at round 33), then 10 more rounds at the target. BF16 rounds
    are held to their own bar (5u, u = 2^-8)."""
    import torch

    from paper_2207_11669_amd import DCFPCA, colmajor
    inst = planted_instance(300, [100, 100, 100], 5, 0.10, values="signed", lo=5.0, hi=20.0,
                            seed=3)
    lam = float(np.float32(1.0 / math.sqrt(inst.n)))
    U0 = init_for(inst, 5, 7)
    sched = _continuation(inst, lam, 40) + [lam] * 10
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, 5, 0.1, lam, colmajor(U0), bf16=bf16)
    for lt in sched:
        s.set_lambda(lt)
        s.step(1)
    L, S = s.get_LS(-1)
    torch.cuda.synchronize()
    Lg = L[:, :inst.m].T.double().cpu().numpy()
    Sg = S[:, :inst.m].T.double().cpu().numpy()
    res = O.dcfpca(inst.blocks(), 5, 0.1, lam, len(sched), U0, lam_schedule=sched)
    eL, eS = rel(Lg, res.L_full()), rel(Sg, res.S_full())
    hist = [s.stats(t) for t in range(len(sched))]
    ef = max(abs(g["objective"] - o["objective"]) / abs(o["objective"])
             for g, o in zip(hist, res.history))
    relerr = rel(Lg, inst.Ustar @ inst.Vstar.T)
    announce(f"continuation bf16={bf16}: relL={eL:.3e} relS={eS:.3e} max objective rel={ef:.3e} "
             f"relerr vs L*={relerr:.3e}")
    tol = 2e-2 if bf16 else TOL
    assert eL <= tol and eS <= tol and ef <= tol


def test_set_lambda_rules():
    """rpca_set_lambda refuses negative or non-finite values and the stored-S
    form; a graph-replayed run with a mid-run lambda change equals the eager
    run bitwise."""
    import torch

    from paper_2207_11669_amd import DCFPCA, RpcaError, colmajor
    inst = planted_instance(200, [64, 100, 36], 4, 0.05, values="uniform", hi=10.0, seed=9)
    U0 = init_for(inst, 4, 2)
    lam = 1.0 / math.sqrt(inst.n)
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, 4, 0.1, lam, colmajor(U0))
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(RpcaError):
            s.set_lambda(bad)
    st = DCFPCA(colmajor(inst.M), inst.widths, inst.m, 4, 0.1, lam, colmajor(U0), store_s=True)
    with pytest.raises(RpcaError):
        st.set_lambda(0.5)
    outs = []
    for graph in (False, True):
        g = DCFPCA(colmajor(inst.M), inst.widths, inst.m, 4, 0.1, lam, colmajor(U0), graph=graph)
        g.step(6)
        g.set_lambda(3 * lam)
        g.step(7)
        g.set_lambda(lam)
        g.step(8)
        L, S = g.get_LS(-1)
        torch.cuda.synchronize()
        outs.append((L.cpu().numpy(), S.cpu().numpy(),
                     [g.stats(t)["objective"] for t in range(21)]))
        g.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


@pytest.mark.parametrize("mode,eta", [("closed", 0.0), ("grad", 2e-3)])
def test_step_multiplier_matches_oracle(mode, eta):
    """U steps multiplied by omega (rpca_set_step), changing between rounds,
    against the oracle run with the same multipliers; omega = 1 is the plain
    step bitwise."""
    import torch

    from paper_2207_11669_amd import DCFPCA, colmajor
    inst = planted_instance(300, [100, 70, 130], 5, 0.10, values="signed", lo=5.0, hi=20.0,
                            seed=8)
    lam = 1.0 / math.sqrt(inst.n)
    U0 = init_for(inst, 5, 7)
    omegas = [1.3] * 12 + [0.8] * 8 + [1.0] * 10
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, 5, 0.1, lam, colmajor(U0), u_mode=mode,
               eta0=eta)
    for w in omegas:
        s.set_step(w)
        s.step(1)
    L, S = s.get_LS(-1)
    torch.cuda.synchronize()
    Lg, Sg = L[:, :inst.m].T.double().cpu().numpy(), S[:, :inst.m].T.double().cpu().numpy()
    res = O.dcfpca(inst.blocks(), 5, 0.1, lam, len(omegas), U0, u_mode=mode, eta0=eta,
                   omega_schedule=omegas)
    eL, eS = rel(Lg, res.L_full()), rel(Sg, res.S_full())
    announce(f"step multipliers ({mode}): relL={eL:.3e} relS={eS:.3e}")
    assert eL <= TOL and eS <= TOL
    # omega = 1 set explicitly is the plain step, bit for bit.
    a = DCFPCA(colmajor(inst.M), inst.widths, inst.m, 5, 0.1, lam, colmajor(U0), u_mode=mode,
               eta0=eta)
    b = DCFPCA(colmajor(inst.M), inst.widths, inst.m, 5, 0.1, lam, colmajor(U0), u_mode=mode,
               eta0=eta)
    b.set_step(1.0)
    a.step(10)
    b.step(10)
    La, Sa = a.get_LS(-1)
    Lb, Sb = b.get_LS(-1)
    torch.cuda.synchronize()
    assert torch.equal(La, Lb) and torch.equal(Sa, Sb)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_target_objective_matches_oracle(precision):
    """Each round's objective at the problem's lambda (rpca_stats
    objective_target: the Huber form, S at its optimum) along a continuation,
    against the oracle's; in rounds at that lambda it is the recorded
    objective itself."""
    from paper_2207_11669_amd import DCFPCA, colmajor
    inst = planted_instance(300, [100, 100, 100], 5, 0.10, values="signed", lo=5.0, hi=20.0,
                            seed=3)
    lam = float(np.float32(1.0 / math.sqrt(inst.n)))
    U0 = init_for(inst, 5, 7)
    sched = _continuation(inst, lam, 40) + [lam] * 10
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, 5, 0.1, lam, colmajor(U0),
               bf16x3=precision == "bf16x3")
    for lt in sched:
        s.set_lambda(lt)
        s.step(1)
    res = O.dcfpca(inst.blocks(), 5, 0.1, lam, len(sched), U0, lam_schedule=sched)
    tol = TOL if precision == "fp32" else 2e-5
    worst = 0.0
    for t, (lt, o) in enumerate(zip(sched, res.history)):
        g = s.stats(t)
        worst = max(worst, abs(g["objective_target"] - o["objective_target"]) / o["objective_target"])
        if lt == lam:
            assert g["objective_target"] == g["objective"]
    announce(f"target objective ({precision}): worst relative difference {worst:.3e}")
    assert worst <= tol
