"""Rounds replayed from HIP graphs (RPCA_FLAG_GRAPH) against the same rounds
launched eagerly: bitwise equal L, S and round statistics at every checkpoint,
with the library's own eager work (statistics flush, S emission) and host
synchronisations between the replays."""
import numpy as np
import pytest

from gpu_helpers import announce, default_lam, init_for
from rpca_inputs import planted_instance

pytestmark = pytest.mark.gpu


def _run(inst, U0, lam, graph):
    import torch

    from paper_2207_11669_amd import DCFPCA, colmajor
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, 4, 0.1, lam, colmajor(U0),
               u_mode="closed", graph=graph)
    out = []
    for chunk in (1, 5, 6, 2, 7):
        s.step(chunk)
        L, S = s.get_LS(-1)
        st = s.stats()
        torch.cuda.synchronize()
        out.append((L[:, :inst.m].cpu().numpy(), S[:, :inst.m].cpu().numpy(), st))
    s.close()
    return out


def test_graph_replay_matches_eager():
    inst = planted_instance(300, [100, 77, 120], 4, 0.05, values="uniform", hi=10.0, seed=21)
    U0 = init_for(inst, 4, 3)
    lam = default_lam(inst)
    eager = _run(inst, U0, lam, graph=False)
    graph = _run(inst, U0, lam, graph=True)
    for k, ((Le, Se, ste), (Lg, Sg, stg)) in enumerate(zip(eager, graph)):
        same = np.array_equal(Le, Lg) and np.array_equal(Se, Sg) and ste == stg
        announce(f"checkpoint {k}: round {ste['t']:.0f} bitwise={same}")
        assert same
