"""The controller's pieces on the GPU: the MLP kernels against the FP64
reference (oracle/controller.py), rpca_copy_state (a copied iterate continues
bitwise like the original), and the controlled lambda schedule."""
import math

import numpy as np
import pytest

from gpu_helpers import announce, default_lam, init_for
import oracle.controller as OC
from rpca_inputs import planted_instance

pytestmark = pytest.mark.gpu


def _mlp_case(seed, n):
    rng = np.random.default_rng(seed)
    p = (0.3 * rng.standard_normal(OC.N_PARAMS)).astype(np.float32)
    X = rng.standard_normal((n, OC.N_IN)).astype(np.float32)
    T = np.stack([rng.uniform(OC.G_MIN, 1.0, n), rng.uniform(OC.W_MIN, OC.W_MAX, n)],
                 axis=1).astype(np.float32)
    return p, X, T


def test_mlp_forward_matches_reference():
    import torch

    from paper_2207_11669_amd import mlp_forward, mlp_param_count
    assert mlp_param_count() == OC.N_PARAMS
    p, X, _ = _mlp_case(3, 300)
    y = mlp_forward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    yo, _ = OC.forward(p.astype(np.float64), X.astype(np.float64))
    err = float(np.max(np.abs(y - yo)))
    announce(f"mlp forward: max abs diff {err:.2e}")
    assert err <= 1e-5


def test_mlp_train_step_matches_reference():
    """One gradient step: the GPU's parameter update equals the FP64
    reference's to FP32 accuracy, and repeats bitwise."""
    import torch

    from paper_2207_11669_amd import mlp_train_step
    p, X, T = _mlp_case(4, 200)
    outs = []
    for _ in range(2):
        pg = torch.from_numpy(p.copy()).cuda()
        ws = torch.empty(200 * OC.N_PARAMS, dtype=torch.float32, device="cuda")
        mlp_train_step(pg, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), 0.3, ws)
        outs.append(pg.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    d_gpu = outs[0].astype(np.float64) - p
    d_ref = OC.sgd_step(p.astype(np.float64), X, T, 0.3) - p
    err = float(np.linalg.norm(d_gpu - d_ref) / np.linalg.norm(d_ref))
    announce(f"mlp step: relative update difference {err:.2e}")
    assert err <= 1e-4


def test_copy_state_continues_bitwise():
    """A fresh session that takes over another's iterate (mid-run, after a
    lambda change) continues bitwise like the original, including its
    recorded statistics; sessions of other parameters are refused."""
    import torch

    from paper_2207_11669_amd import DCFPCA, RpcaError, colmajor
    inst = planted_instance(260, [90, 70, 100], 4, 0.05, values="uniform", hi=10.0, seed=12)
    U0 = init_for(inst, 5, 3)
    lam = default_lam(inst)
    M = colmajor(inst.M)
    a = DCFPCA(M, inst.widths, inst.m, 5, 0.1, lam, colmajor(U0))
    a.step(7)
    a.set_lambda(2 * lam)
    a.step(2)
    b = DCFPCA(M.clone(), inst.widths, inst.m, 5, 0.1, lam, colmajor(init_for(inst, 5, 9)))
    b.copy_state_from(a)
    for s in (a, b):
        s.step(3)
        s.set_lambda(lam)
        s.step(4)
    La, Sa = a.get_LS(-1)
    Lb, Sb = b.get_LS(-1)
    torch.cuda.synchronize()
    assert torch.equal(La, Lb) and torch.equal(Sa, Sb)
    assert a.rounds == b.rounds == 16
    assert [a.stats(t)["objective"] for t in range(16)] == [b.stats(t)["objective"] for t in range(16)]
    c = DCFPCA(M, inst.widths, inst.m, 6, 0.1, lam, colmajor(init_for(inst, 6, 3)))
    with pytest.raises(RpcaError):
        c.copy_state_from(a)


def test_fixed_continuation_controller_schedule():
    """run_controlled with the fixed decay 0.8 applies lambda_t = lambda
    max(1, s0 0.8^t) until the scale reaches 1, then leaves lambda at its
    target; each round's record carries its lambda (objective uses it)."""
    from paper_2207_11669_amd import DCFPCA, colmajor
    from paper_2207_11669_amd import controller as C
    inst = planted_instance(200, [100, 100], 4, 0.1, values="signed", lo=5.0, hi=20.0, seed=2)
    lam = default_lam(inst)
    lam0 = float(np.abs(inst.M).max())
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, 4, 0.1, lam, colmajor(init_for(inst, 4, 1)))
    out = C.run_controlled(s, lam, lam0, C.FixedContinuation(0.8), float(inst.m * inst.n),
                           judge=False)
    expect = math.ceil(math.log(lam / lam0) / math.log(0.8))
    assert out["control_rounds"] == expect and all(g == 0.8 for g in out["gammas"])
    s.step(1)
    st = s.stats(-1)
    assert st["t"] == expect
