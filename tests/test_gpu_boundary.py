"""The C ABI's boundary behaviour on the GPU: the library's own draw of
U^(0) (Algorithm 1 leaves the start open; rpca_init with U0 = NULL), and the
poisoning rule: a non-finite objective makes rpca_solve return
RPCA_ENONFINITE, after which every call on the context returns RPCA_ESTATE."""
import math

import numpy as np
import pytest

from gpu_helpers import announce, default_lam, rel, run_oracle
from rpca_inputs import planted_instance, splitmix_gaussian_init

pytestmark = pytest.mark.gpu


def test_null_U0_draws_the_documented_start_and_matches_the_oracle():
    """U^(0) drawn on the device from the seed equals the host-side draw of
    the same published rule (SplitMix64 counters, Box-Muller in FP64, FP32
    rounding) to within one FP32 ulp (device and host libm may differ in the
    last bits of a double), and the run from it matches the oracle started
    from the host draw."""
    import torch

    from paper_2207_11669_amd import DCFPCA, colmajor
    inst = planted_instance(203, [70, 33, 90], 4, 0.05, values="uniform", hi=10.0, seed=31)
    r, lam, seed = 5, default_lam(inst), 0xC0FFEE
    announce(f"NULL U0: m={inst.m} widths={inst.widths} r={r} seed={seed}")
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, 0.1, lam, None, seed=seed)
    U, _ = s.get_factors()
    torch.cuda.synchronize()
    Ud = U[:, :inst.m].T.double().cpu().numpy()
    Uh = splitmix_gaussian_init(inst.m, r, seed)
    ulp = np.spacing(np.abs(Uh).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(Ud - Uh) <= ulp), float(np.max(np.abs(Ud - Uh) / ulp))
    announce(f"device draw equals host draw bitwise: {np.array_equal(Ud, Uh)}")
    T = 30
    s.step(T)
    L, S = s.get_LS(-1)
    torch.cuda.synchronize()
    Lg = L[:, :inst.m].T.double().cpu().numpy()
    Sg = S[:, :inst.m].T.double().cpu().numpy()
    res = run_oracle(inst, Ud, r, 0.1, lam, T)
    eL, eS = rel(Lg, res.L_full()), rel(Sg, res.S_full())
    announce(f"NULL U0 run vs oracle: relL={eL:.3e} relS={eS:.3e}")
    assert eL <= 1e-5 and eS <= 1e-5


def _assert_poisoned(s):
    from paper_2207_11669_amd import RpcaError
    from paper_2207_11669_amd.binding import RPCA_ESTATE
    for call in (lambda: s.step(1), lambda: s.solve(5, 0.0, 1), lambda: s.get_LS(-1),
                 lambda: s.stats(-1), lambda: s.get_factors(), lambda: s.set_lambda(0.1),
                 lambda: s.set_launch_shape(row_splits=1)):
        with pytest.raises(RpcaError) as ei:
            call()
        assert ei.value.status == RPCA_ESTATE, ei.value


def test_non_finite_entry_poisons_the_context():
    """A NaN entry of M makes the first checked round's objective NaN:
    rpca_solve returns RPCA_ENONFINITE, then every call RPCA_ESTATE."""
    from paper_2207_11669_amd import DCFPCA, RpcaError, colmajor
    from paper_2207_11669_amd.binding import RPCA_ENONFINITE
    inst = planted_instance(140, [30, 45, 25], 3, 0.05, values="uniform", hi=10.0, seed=21)
    M = inst.M.copy()
    M[17, 40] = np.nan
    announce("NaN entry in M: expect RPCA_ENONFINITE then RPCA_ESTATE")
    s = DCFPCA(colmajor(M), inst.widths, inst.m, 3, 0.1, default_lam(inst),
               colmajor(splitmix_gaussian_init(inst.m, 3, 1)))
    with pytest.raises(RpcaError) as ei:
        s.solve(20, 0.0, check_every=5)
    assert ei.value.status == RPCA_ENONFINITE
    _assert_poisoned(s)


def test_diverging_gradient_step_poisons_the_context():
    """The paper's gradient step with a step size far above 1/L (Theorem 1
    needs eta < 1/L) diverges: with K = 1 the consensus step is U - (eta/E)
    (rho U - sum_i P_i), whose linear part multiplies U by 1 - eta rho / E =
    -32 per round here while the data term shrinks like 1/|U|, so U
    overflows FP32 within a few dozen rounds and the objective turns
    infinite or NaN (arithmetic only), which the solve loop detects; the
    context is then poisoned."""
    from paper_2207_11669_amd import DCFPCA, RpcaError, colmajor
    from paper_2207_11669_amd.binding import RPCA_ENONFINITE
    inst = planted_instance(140, [30, 45, 25], 3, 0.05, values="uniform", hi=10.0, seed=22)
    announce("GRAD with eta0 = 1000: expect RPCA_ENONFINITE then RPCA_ESTATE")
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, 3, 0.1, default_lam(inst),
               colmajor(splitmix_gaussian_init(inst.m, 3, 2)), u_mode="grad", eta0=1000.0)
    with pytest.raises(RpcaError) as ei:
        s.solve(200, 0.0, check_every=10)
    assert ei.value.status == RPCA_ENONFINITE
    _assert_poisoned(s)
