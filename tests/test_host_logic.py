"""Host-side logic that needs no GPU: the lambda continuation schedule, the
controller's features and decisions, and the parameter rules of the
precision flags."""
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_continuation_schedule():
    """max(lambda, lambda0 0.8^t) down to the first round at lambda, strictly
    decreasing before it; a start at or below lambda is one round."""
    from bench import continuation
    lam, lam0 = 0.0111803, 46.78
    c = continuation(lam, lam0)
    assert c[0] == lam0 and c[-1] == lam
    assert all(b < a for a, b in zip(c, c[1:]))
    assert len(c) == math.ceil(math.log(lam / lam0) / math.log(0.8)) + 1
    assert continuation(1.0, 0.5) == [1.0]


def test_controller_features_are_scale_free():
    """The ten features stay in fixed ranges, and scaling M (hence lambda,
    the statistics and the objective) leaves them unchanged."""
    from paper_2207_11669_amd import controller as C
    st = dict(t=3, objective=5.0, lambda_fro_sq=12.0, nnz=900.0, du_sq=0.02, u_sq=40.0,
              v_sq=30.0, l1=300.0)
    prev = dict(st, u_sq=38.0)
    st["objective_target"], prev["objective_target"] = 6.0, 6.5
    f = C.features(st, prev, 20.0, 0.8, 3, 0.05, 1e4, 1.3)
    assert len(f) == C.N_FEATURES and all(math.isfinite(x) for x in f)
    assert 0.0 <= f[2] <= 1.0 and 0.0 <= f[3] <= 1.0 and -1.0 <= f[5] <= 1.0
    assert -1.0 <= f[9] < 0.0 and abs(f[8] - 0.3) < 1e-12
    k = 7.0  # M -> k M: Lambda, S scale by k; U, V by sqrt(k); lambda by k
    st2 = dict(st, lambda_fro_sq=st["lambda_fro_sq"] * k * k, l1=st["l1"] * k,
               du_sq=st["du_sq"] * k, u_sq=st["u_sq"] * k,
               objective_target=st["objective_target"] * k * k)
    prev2 = dict(prev, u_sq=prev["u_sq"] * k, objective_target=prev["objective_target"] * k * k)
    f2 = C.features(st2, prev2, 20.0, 0.8, 3, 0.05 * k, 1e4, 1.3)
    assert np.allclose(f, f2, rtol=1e-12, atol=1e-12)


def test_controller_decisions():
    from paper_2207_11669_amd import controller as C
    assert C.FixedContinuation(0.8).decide([0.0] * C.N_FEATURES) == (0.8, 1.0)
    assert C.GAMMAS == (0.5, 0.6, 0.7, 0.8, 0.9, 1.0) and C.OMEGAS[0] == 1.0


def test_precision_flag_rules():
    """Both BF16 flags need the rebuilt-S form; the three-product flag alone
    adds only the factor splits to the workspace (no copies of M)."""
    from paper_2207_11669_amd import make_params, params_error, workspace_bytes
    for flag in ("bf16", "bf16x3"):
        for kw in (dict(K=2), dict(inner=2), dict(store_s=True)):
            p, _k = make_params(100, [30, 70], 5, 0.1, 0.1, **{flag: True}, **kw)
            msg = params_error(p)
            assert msg is not None and "RPCA_FLAG_BF16" in msg, (flag, kw, msg)
    p32, _a = make_params(4000, [500] * 16, 20, 0.1, 0.01)
    px3, _b = make_params(4000, [500] * 16, 20, 0.1, 0.01, bf16x3=True)
    pb, _c = make_params(4000, [500] * 16, 20, 0.1, 0.01, bf16=True)
    b32, bx3, bb = workspace_bytes(p32), workspace_bytes(px3), workspace_bytes(pb)
    assert b32 < bx3 < b32 + 8 * 2 * (4096 + 8192) * 64 * 2
    assert bb >= bx3 + 2 * 2 * 4096 * 8192


def test_splitmix64_counter_form_matches_the_published_generator():
    """The counter form used for U^(0) equals the stateful SplitMix64
    recurrence (state += golden-ratio increment, output the state's mix),
    whose first outputs for seed 0 are the published e220a8397b1dcdaf,
    6e789e6aa1b965f4, 06c45d188009454f."""
    from rpca_inputs import splitmix64_outputs
    mask = (1 << 64) - 1

    def mix(z):
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        return z ^ (z >> 31)

    assert [int(x) for x in splitmix64_outputs(0, 0, 3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    for seed in (1, 12345, (1 << 64) - 7):
        state, ref = seed, []
        for _ in range(40):
            state = (state + 0x9E3779B97F4A7C15) & mask
            ref.append(mix(state))
        assert [int(x) for x in splitmix64_outputs(seed, 0, 40)] == ref
        assert [int(x) for x in splitmix64_outputs(seed, 17, 5)] == ref[17:22]


def test_splitmix_gaussian_init_is_standard_normal():
    """Box-Muller on the SplitMix64 uniforms: mean 0, variance 1, and the
    normal's 1-sigma and 2-sigma masses, within sampling error at 2e5 draws;
    distinct seeds give distinct starts; the layout is entry (i, c) from
    counter pair k = c m + i."""
    from rpca_inputs import splitmix64_outputs, splitmix_gaussian_init
    U = splitmix_gaussian_init(4000, 50, 9)
    x = U.ravel()
    assert abs(x.mean()) < 0.01 and abs(x.var() - 1.0) < 0.01
    assert abs(np.mean(np.abs(x) < 1.0) - 0.682689) < 0.005
    assert abs(np.mean(np.abs(x) < 2.0) - 0.954500) < 0.003
    assert not np.array_equal(U, splitmix_gaussian_init(4000, 50, 10))
    i, c, m = 123, 7, 4000
    k = c * m + i
    a, b = (int(v) >> 11 for v in splitmix64_outputs(9, 2 * k, 2))
    z = math.sqrt(-2.0 * math.log(1.0 - a * 2.0 ** -53)) * math.cos(2.0 * math.pi * b * 2.0 ** -53)
    assert U[i, c] == float(np.float32(z))
