"""The paper's synthetic experiments (Section 4.2) as `experiments.py` runs
them on the GPU path: the upper-bound-rank table's n = 200 and n = 1000
(fitted rank 100) rows against the values the paper prints, the local-steps
ablation's ordering, and the recovery boundary of the rank/corruption grid,
small and at the paper's m = n = 500 (ranks up to 100)."""
import argparse
import os
import sys

import pytest

from gpu_helpers import announce

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _args(**kw):
    base = dict(u_mode="grad", K=2, eta=0.05, sched="sqrt", rounds=200, continuation=False,
                clients=5)
    base.update(kw)
    return argparse.Namespace(**base)


def test_upper_bound_rank_n200_within_the_papers_table():
    """Table 1 (Section 4.2, upper-bound rank): n = 200, r = 10, fitted rank
    p = 20, s = 0.05. The paper prints a relative singular-value error of
    0.0286 for this row; with lambda = 1/sqrt(n), rho = 0.1, the gradient
    step with K = 2 and eta0 / sqrt(t + 1), 200 rounds, the error must not
    exceed it, and the surplus singular values stay small against sigma_r."""
    import experiments
    out = experiments.rank(_args(sizes=[200]))
    row = out["rows"][0]
    announce(f"rank n=200: {row}")
    assert row["p"] == 20 and row["sv_error"] <= 0.0286
    assert row["tail_ratio"] < 0.05


def test_local_steps_converge_faster_per_round():
    """Fig. 4's ablation: more local steps per round reach a lower error
    after the same number of communication rounds (gradient step, constant
    eta, E = 10)."""
    import experiments
    out = experiments.local_steps(argparse.Namespace(n=200, clients=10, rounds=20, eta=0.01,
                                                     ks=[1, 10]))
    c1, c10 = out["relerr_per_round"]["1"], out["relerr_per_round"]["10"]
    announce(f"local steps n=200: K=1 {c1[-1]:.3e}, K=10 {c10[-1]:.3e} after 20 rounds")
    assert c10[-1] < 0.5 * c1[-1]


def test_recovery_boundary_of_the_phase_grid():
    """Fig. 2 (sparsity and rank levels): low rank and sparse corruption is
    recovered, high rank with dense corruption is not."""
    import experiments
    out = experiments.phase(_args(n=120))
    grid = out["relerr"]
    announce(f"phase n=120 ranks {out['ranks']}: corner errors {grid[0][0]:.2e} "
             f"(r=0.05n, s=0.05), {grid[-1][-1]:.2e} (r=0.2n, s=0.3)")
    assert grid[0][0] < 1e-2
    assert grid[-1][-1] > 0.1


def test_upper_bound_rank_n1000_within_the_papers_table():
    """Table 1's n = 1000 row: r = 50, fitted rank p = 100, s = 0.05; the
    paper prints 0.0398. (This configuration's first rounds are chaotic:
    gradient steps against corruptions of +-1000 move the oracle's own L by
    1.5e-5 after one round and by O(1) after ten for a perturbation of U^(0)
    at FP32 rounding, so element-wise parity is checked on the stable
    instances of the rank-above-64 tests; here the metric the paper prints.)"""
    import experiments
    out = experiments.rank(_args(sizes=[1000]))
    row = out["rows"][0]
    announce(f"rank n=1000: {row}")
    assert row["p"] == 100 and row["sv_error"] <= 0.0398


def test_recovery_grid_at_the_papers_size():
    """Fig. 2 at m = n = 500 (ranks 25 .. 100, corruption 0.05 .. 0.3, 200
    rounds of the gradient step with K = 2): rank 0.05 n is recovered up to
    s = 0.2, rank 0.2 n at no corruption level."""
    import experiments
    out = experiments.phase(_args(n=500))
    grid = out["relerr"]
    announce(f"phase n=500 ranks {out['ranks']}: " +
             " | ".join(" ".join(f"{e:.1e}" for e in row) for row in grid))
    assert out["ranks"] == [25, 50, 75, 100]
    assert all(e < 1e-2 for e in grid[0][:4])
    assert all(e > 0.1 for e in grid[-1])
