"""Persistent launches over a tile queue (launch forms vpass_queue and
spass_queue): the resident work-groups take the streaming passes' tiles from a
counter in the workspace, each tile writing its own slots, so the rounds are
bitwise those of one work-group per tile whatever the timing. Checked on
instances with more tiles than resident work-groups (so the queue is really
walked), in every precision and S layout, under graph replay, and against the
oracle."""
import numpy as np
import pytest

from gpu_helpers import announce, default_lam, init_for, parity, rel
from rpca_inputs import loguniform_widths, planted_instance

pytestmark = pytest.mark.gpu

STATIC = dict(vpass_queue=0, spass_queue=0)
QUEUE = dict(vpass_queue=1, spass_queue=1)


def _instance(r_star=6, seed=51):
    # 48 clients of 40..300 columns, m = 6000: 47 x 48 = 2256 S-pass tiles and
    # about 1100 V-pass tiles, more than the resident work-groups of either.
    widths = loguniform_widths(48, 40, 300, seed=seed)
    return planted_instance(6000, widths, r_star, 0.05, values="uniform", hi=10.0, seed=seed,
                            support="bernoulli")


def _trajectory(inst, r, shape, rounds=12, **kw):
    import torch

    from paper_2207_11669_amd import DCFPCA, colmajor
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, 0.1, default_lam(inst),
               colmajor(init_for(inst, r, 3)), **kw)
    s.set_launch_shape(**shape)
    out = []
    for chunk in (1, 4, rounds - 5):
        s.step(chunk)
        L, S = s.get_LS(-1)
        torch.cuda.synchronize()
        out.append((L.cpu().numpy(), S.cpu().numpy(), s.stats()))
    s.close()
    return out


CASES = {
    "fp32_two_phases": (20, dict(spass_phases=2, column_groups=1), {}),
    "fp32_one_phase_four_groups": (33, dict(spass_phases=1, column_groups=4), {}),
    "fp32_stored_S": (20, dict(spass_phases=2), dict(store_s=True)),
    "fp32_K2_grad": (8, dict(spass_phases=2), dict(K=2, u_mode="grad", eta0=1e-4)),
    "bf16": (40, {}, dict(bf16=True)),
    "bf16x3": (64, {}, dict(bf16x3=True)),
    "fp32_graph": (20, {}, dict(graph=True)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_queue_is_bitwise_the_per_tile_grid(name):
    r, shape, kw = CASES[name]
    inst = _instance()
    announce(f"queue vs per-tile grid: {name}, m={inst.m}, E={inst.E}, n={inst.n}, r={r}")
    a = _trajectory(inst, r, dict(shape, **STATIC), **kw)
    b = _trajectory(inst, r, dict(shape, **QUEUE), **kw)
    for k, ((La, Sa, sa), (Lb, Sb, sb)) in enumerate(zip(a, b)):
        same = np.array_equal(La, Lb) and np.array_equal(Sa, Sb) and sa == sb
        announce(f"checkpoint {k} (round {sa['t']:.0f}): bitwise={same} relL={rel(Lb, La):.2e}")
        assert same


def test_queue_parity_with_oracle():
    """Both passes on the queue, FP32, against the FP64 oracle."""
    widths = loguniform_widths(40, 40, 400, seed=7)
    inst = planted_instance(2500, widths, 5, 0.05, values="uniform", hi=10.0, seed=7,
                            support="bernoulli")
    parity(inst, 8, 20, u_mode="closed", shape=QUEUE)
