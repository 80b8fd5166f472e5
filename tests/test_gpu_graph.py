"""Rounds replayed from HIP graphs (RPCA_FLAG_GRAPH) against the same rounds
launched eagerly: bitwise equal L, S and round statistics at every checkpoint,
with the library's own eager work (statistics flush, S emission) and host
synchronisations between the replays."""
import numpy as np
import pytest

from gpu_helpers import announce, default_lam, init_for, parity, rel, run_gpu
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
    """The autotuner runs real rounds under several launch shapes (V-pass row
    split counts, 1 or 4 column groups per wave; 1 or 2 S-pass column
    phases); the trajectory still matches the oracle's for the same number of
    rounds, and the pick is one of the candidates."""
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
    v, g, ph = shape["row_splits"], shape["column_groups"], shape["spass_phases"]
    s.step(4)
    T = s.rounds
    L, S = s.get_LS(-1)
    torch.cuda.synchronize()
    Lg = L[:, :inst.m].T.double().cpu().numpy()
    Sg = S[:, :inst.m].T.double().cpu().numpy()
    res = O.dcfpca(inst.blocks(), 8, 0.1, lam, T, U0)
    eL, eS = rel(Lg, res.L_full()), rel(Sg, res.S_full())
    announce(f"autotune picked {v} row splits, {g} column groups, {ph} S-pass phases; "
             f"{T} rounds; "
             f"relL={eL:.3e} relS={eS:.3e}")
    assert 1 <= v <= 64 and g in (1, 4) and ph in (1, 2) and s.launch_shape() == shape
    assert eL <= 1e-5 and eS <= 1e-5
    s.close()


SHAPES = {"two_phases": {"spass_phases": 2}, "one_phase": {"spass_phases": 1}}


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("r,widths", [(5, [100, 16, 9, 77, 300]), (20, [40, 21, 130, 64]),
                                      (32, [600, 40, 1100]), (36, [36, 90, 200]),
                                      (64, [64, 150, 80])])
def test_spass_shapes_parity(name, r, widths):
    """Both S-pass column-phase counts match the oracle on every rank-tile
    count, with clients of one 16-column chunk or less (a phase with no chunk
    when there are two), ragged chunk tails, and clients of more than 16
    V-finish groups (client factors summed over several blocks of groups)."""
    inst = planted_instance(333, widths, min(r, 12), 0.05, values="uniform", hi=10.0,
                            seed=40 + r)
    parity(inst, r, 25, u_mode="closed", shape=SHAPES[name])


def test_spass_one_phase_grad_and_stored_S():
    """One S-pass column phase: the gradient step with one-column clients
    matches the oracle, and stored-S rounds run the same summation as
    rebuilt-S ones (bitwise equal trajectories)."""
    inst = planted_instance(203, [1, 17, 33, 64, 5, 100], 5, 0.06, values="signed", lo=2.0,
                            hi=8.0, seed=4)
    parity(inst, 7, 40, u_mode="grad", eta0=1e-3, shape={"spass_phases": 1})
    inst = planted_instance(333, [100, 77, 120], 4, 0.05, values="uniform", hi=10.0, seed=19)
    U0 = init_for(inst, 4, 3)
    lam = default_lam(inst)
    one = {"spass_phases": 1}
    _, L1, S1, _ = run_gpu(inst, U0, 4, 0.1, lam, 30, shape=one)
    _, L2, S2, _ = run_gpu(inst, U0, 4, 0.1, lam, 30, shape=one, store_s=True)
    announce(f"one phase, rebuilt vs stored: relL={rel(L1, L2):.3e} "
             f"bitwise={np.array_equal(L1, L2) and np.array_equal(S1, S2)}")
    assert np.array_equal(L1, L2) and np.array_equal(S1, S2)


def test_set_launch_shape_rejects_bad_values():
    from paper_2207_11669_amd import DCFPCA, RpcaError, colmajor
    inst = planted_instance(200, [60, 70], 3, 0.05, values="uniform", hi=10.0, seed=2)
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, 3, 0.1, default_lam(inst),
               colmajor(init_for(inst, 3, 1)), u_mode="closed")
    before = s.launch_shape()
    for kw, frag in ((dict(row_splits=-1), "row splits"), (dict(row_splits=1000), "row splits"),
                     (dict(column_groups=2), "column groups"), (dict(spass_phases=3), "phases"),
                     (dict(vpass_queue=2), "launch forms"), (dict(spass_queue=-1), "launch forms")):
        with pytest.raises(RpcaError, match=frag):
            s.set_launch_shape(**kw)
        assert s.launch_shape() == before
    s.set_launch_shape(row_splits=1, column_groups=4, spass_phases=1)
    assert s.launch_shape() == {"row_splits": 1, "column_groups": 4, "spass_phases": 1,
                                "vpass_queue": 0, "spass_queue": 0, "sparse_s": 0}
    s.step(2)
    assert np.isfinite(s.stats()["objective"])
    s.close()
