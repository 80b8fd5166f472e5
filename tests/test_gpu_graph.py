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


def test_autotune_keeps_parity():
    """The V-pass autotuner runs real rounds under several launch shapes (row
    split counts, 1 or 4 column groups per wave); the trajectory still matches
    the oracle's for the same number of rounds, and the pick is one of the
    candidates."""
    import torch

    import oracle.reference as O
    from gpu_helpers import rel
    from paper_2207_11669_amd import DCFPCA, colmajor
    inst = planted_instance(2000, [500, 500, 500, 500], 6, 0.05, values="uniform", hi=10.0,
                            seed=23)
    U0 = init_for(inst, 8, 4)
    lam = default_lam(inst)
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, 8, 0.1, lam, colmajor(U0), u_mode="closed")
    s.step(3)
    shape = s.autotune(3)
    v, g = shape["row_splits"], shape["column_groups"]
    s.step(4)
    T = s.rounds
    L, S = s.get_LS(-1)
    torch.cuda.synchronize()
    Lg = L[:, :inst.m].T.double().cpu().numpy()
    Sg = S[:, :inst.m].T.double().cpu().numpy()
    res = O.dcfpca(inst.blocks(), 8, 0.1, lam, T, U0)
    eL, eS = rel(Lg, res.L_full()), rel(Sg, res.S_full())
    announce(f"autotune picked {v} row splits, {g} column groups; {T} rounds; "
             f"relL={eL:.3e} relS={eS:.3e}")
    assert 1 <= v <= 64 and g in (1, 4) and eL <= 1e-5 and eS <= 1e-5
    s.close()
