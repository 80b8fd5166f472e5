"""Mixed-precision rounds (RPCA_FLAG_BF16) against the FP64 oracle.

BF16 rounds round M, U, V and Lambda (or M - S) to BF16 (8-bit significand,
unit roundoff u = 2^-8) before the rank-r contractions, with FP32
accumulation. Their trajectories therefore follow the oracle only to a few u:
the bar for BF16 rounds is a relative Frobenius difference on L and S of at
most 5u ~ 2e-2 after a fixed number of rounds, on instances where lambda is
well above the BF16 resolution of M's entries (lambda >> 2^-9 |M_ij| for the
uncorrupted entries; otherwise the soft-threshold's input is rounding noise).
FP32 closing rounds started from a BF16 iterate must land on the oracle's
trajectory to the FP32 bar (1e-5), since the method forgets its starting
point along the way."""
import numpy as np
import pytest

from gpu_helpers import TOL, announce, default_lam, init_for, rel, run_gpu, run_oracle
import oracle.reference as O
from rpca_inputs import planted_instance, recipe

pytestmark = pytest.mark.gpu

BF16_TOL = 2e-2  # 5 u, u = 2^-8


def _gpu_LS(s, m):
    import torch
    L, S = s.get_LS(-1)
    torch.cuda.synchronize()
    return L[:, :m].T.double().cpu().numpy(), S[:, :m].T.double().cpu().numpy()


def _session(inst, U0, r, lam, rho=0.1, **kw):
    from paper_2207_11669_amd import DCFPCA, colmajor
    return DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, rho, lam, colmajor(U0), **kw)


def test_bf16_rounds_follow_oracle():
    """m = n = 500, rank 5, lambda = 1/sqrt(500) ~ 0.045 against entries of
    M of size ~2 (BF16 resolution ~4e-3): 100 BF16 rounds stay within 5u of
    the FP64 trajectory, and the recorded objective within 5u of the oracle's."""
    inst = recipe("plain_500x500_r5", seed=0)
    U0 = init_for(inst, 5, 7)
    lam = default_lam(inst)
    s = _session(inst, U0, 5, lam, bf16=True)
    s.step(100)
    Lb, Sb = _gpu_LS(s, inst.m)
    res = run_oracle(inst, U0, 5, 0.1, lam, 100)
    eL, eS = rel(Lb, res.L_full()), rel(Sb, res.S_full())
    fo = s.stats(99)["objective"]
    ef = abs(fo - res.history[99]["objective"]) / res.history[99]["objective"]
    announce(f"bf16 100 rounds: relL={eL:.3e} relS={eS:.3e} objective rel={ef:.3e}")
    assert eL <= BF16_TOL and eS <= BF16_TOL and ef <= BF16_TOL


def test_fp32_closing_rounds_reach_fp32_bar():
    """100 BF16 rounds, then FP32 rounds: after 300 FP32 rounds L and S agree
    with the oracle's 400-round iterate to the FP32 bar."""
    inst = recipe("plain_500x500_r5", seed=0)
    U0 = init_for(inst, 5, 7)
    lam = default_lam(inst)
    s = _session(inst, U0, 5, lam, bf16=True)
    s.step(100)
    s.set_precision("fp32")
    s.step(300)
    Lr, Sr = _gpu_LS(s, inst.m)
    res = run_oracle(inst, U0, 5, 0.1, lam, 400)
    eL, eS = rel(Lr, res.L_full()), rel(Sr, res.S_full())
    announce(f"bf16 100 + fp32 300 vs oracle 400: relL={eL:.3e} relS={eS:.3e}")
    assert eL <= TOL and eS <= TOL


def test_bf16_geometric_2000_subinstance_error():
    """The 2000 x 2000 single-client instance of the large geometric-spectrum
    workload (rank 64, sigma 100 -> 1, 5% corrupted with magnitude U[1, 100]),
    r = 64: error of 10 BF16 rounds against the FP64 oracle, and of 10 FP32
    rounds for comparison."""
    inst = recipe("geom_2000x2000_r64", seed=0)
    U0 = init_for(inst, 64, 7)
    lam = default_lam(inst)
    res = run_oracle(inst, U0, 64, 0.1, lam, 10)
    out = {}
    for bf16 in (False, True):
        s = _session(inst, U0, 64, lam, bf16=bf16)
        s.step(10)
        L, S = _gpu_LS(s, inst.m)
        out[bf16] = (rel(L, res.L_full()), rel(S, res.S_full()))
        s.close()
    announce(f"geom 2000 r64, 10 rounds: bf16 relL={out[True][0]:.3e} relS={out[True][1]:.3e}; "
             f"fp32 relL={out[False][0]:.3e} relS={out[False][1]:.3e}")
    assert max(out[False]) <= TOL
    assert max(out[True]) <= BF16_TOL


@pytest.mark.parametrize("r,widths", [(20, [12, 90, 50]), (40, [30, 100, 70])])
def test_narrow_client_closed_step(r, widths):
    """CLOSED step with a client too narrow to give every S-pass phase a
    column chunk (FP32: two phases of 16-column chunks; BF16: four phases of
    32-column chunks), so some phases of its work-groups sweep nothing; rho = 5
    keeps V_i^T V_i + c_i I well conditioned at n_i < r."""
    inst = planted_instance(300, widths, 4, 0.05, values="uniform", hi=10.0, seed=23)
    U0 = init_for(inst, r, 7)
    res = run_oracle(inst, U0, r, 5.0, 0.1, 10)
    _, Lg, Sg, _ = run_gpu(inst, U0, r, 5.0, 0.1, 10)
    eL, eS = rel(Lg, res.L_full()), rel(Sg, res.S_full())
    _, Lh, Sh, _ = run_gpu(inst, U0, r, 5.0, 0.1, 10, bf16=True)
    hL, hS = rel(Lh, res.L_full()), rel(Sh, res.S_full())
    announce(f"r={r} widths={widths}: fp32 relL={eL:.3e} relS={eS:.3e}; bf16 relL={hL:.3e} relS={hS:.3e}")
    assert eL <= TOL and eS <= TOL
    assert hL <= BF16_TOL and hS <= BF16_TOL


@pytest.mark.parametrize("r", [20, 40, 64])
def test_bf16_pass_forms_follow_oracle(r):
    """One-product BF16 rounds with either form of each pass -- the factor
    operands in each wave's registers (V-pass column groups 4, S-pass phases
    2) or staged in LDS (column groups 1: four 64-column tiles per V-pass
    work-group; phases 1: four waves of 32 rows over the same S-pass chunks)
    -- on ragged m (301), clients of 1-3 tiles and a last V-pass work-group
    with two tiles stay within 5u of the FP64 trajectory after 20 rounds; the
    staged forms give the same bits from one work-group per tile and from
    the tile queues."""
    import torch
    inst = planted_instance(301, [70, 190, 130, 96], 4, 0.05, values="uniform", lo=5.0, hi=10.0,
                            seed=29)
    U0 = init_for(inst, r, 7)
    lam, T = 0.1, 20
    res = run_oracle(inst, U0, r, 0.1, lam, T)
    out = {}
    for cg, ph, q in ((4, 2, 0), (1, 2, 0), (4, 1, 0), (1, 1, 0), (1, 1, 1)):
        s, Lg, Sg, _ = run_gpu(inst, U0, r, 0.1, lam, T, bf16=True,
                               shape=dict(column_groups=cg, spass_phases=ph, vpass_queue=q,
                                          spass_queue=q))
        out[(cg, ph, q)] = (Lg, Sg)
        eL, eS = rel(Lg, res.L_full()), rel(Sg, res.S_full())
        announce(f"bf16 r={r} column_groups={cg} spass_phases={ph} queues={q}: "
                 f"relL={eL:.3e} relS={eS:.3e}")
        assert eL <= BF16_TOL and eS <= BF16_TOL
        del s
        torch.cuda.synchronize()
    assert np.array_equal(out[(1, 1, 0)][0], out[(1, 1, 1)][0])
    assert np.array_equal(out[(1, 1, 0)][1], out[(1, 1, 1)][1])


def test_bf16_deterministic_and_switchable():
    """BF16 rounds are bitwise reproducible; precision can go BF16 -> FP32 ->
    BF16; a context created without the flag refuses BF16."""
    from paper_2207_11669_amd import RpcaError
    inst = planted_instance(260, [90, 70, 110], 4, 0.05, values="uniform", hi=10.0, seed=5)
    U0 = init_for(inst, 8, 3)
    lam = default_lam(inst)
    outs = []
    for _ in range(2):
        s = _session(inst, U0, 8, lam, bf16=True)
        s.step(7)
        s.set_precision("fp32")
        s.step(5)
        s.set_precision("bf16")
        s.step(6)
        outs.append(_gpu_LS(s, inst.m))
        s.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    s = _session(inst, U0, 8, lam)
    with pytest.raises(RpcaError):
        s.set_precision("bf16")


def test_bf16_graph_replay_matches_eager():
    """HIP-graph replay of BF16 round pairs gives bitwise the eager result."""
    inst = planted_instance(300, [64, 100, 36], 5, 0.05, values="uniform", hi=10.0, seed=8)
    U0 = init_for(inst, 5, 2)
    lam = default_lam(inst)
    outs = []
    for graph in (False, True):
        s = _session(inst, U0, 5, lam, bf16=True, graph=graph)
        s.step(11)
        outs.append(_gpu_LS(s, inst.m))
        s.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


# Three-product BF16 rounds (RPCA_FLAG_BF16X3): hi/lo splits carry 16
# significand bits, and the dropped lo.lo term and the lo roundings leave a
# relative error of about 2^-17 ~ 7.6e-6 per product; the bar is 2e-5 (the
# FP32 bar's order, with room for the trajectory's amplification).
X3_TOL = 2e-5


def test_bf16x3_rounds_follow_oracle():
    """100 three-product rounds on the 500 x 500 instance and 3 rounds of the
    full 4000 x 8000, r = 20 workload (where plain BF16 rounds stall) stay
    within 2e-5 of the FP64 trajectory."""
    from gpu_helpers import run_gpu
    for name, r, T in (("plain_500x500_r5", 5, 100), ("plain_4000x8000_r20", 20, 3)):
        inst = recipe(name, seed=0)
        U0 = init_for(inst, r, 7)
        lam = default_lam(inst)
        _, Lg, Sg, _ = run_gpu(inst, U0, r, 0.1, lam, T, bf16x3=True)
        res = run_oracle(inst, U0, r, 0.1, lam, T)
        eL, eS = rel(Lg, res.L_full()), rel(Sg, res.S_full())
        announce(f"bf16x3 {name} T={T}: relL={eL:.3e} relS={eS:.3e}")
        assert eL <= X3_TOL and eS <= X3_TOL


@pytest.mark.parametrize("r,widths", [(20, [12, 90, 50]), (40, [30, 100, 70]), (64, [70, 90])])
def test_bf16x3_ragged_and_rank_tiles(r, widths):
    """Ragged m (row 300 is not a multiple of 32), narrow clients and every
    rank-tile count; rho = 5 keeps n_i < r well conditioned."""
    from gpu_helpers import run_gpu
    inst = planted_instance(301, widths, 4, 0.05, values="uniform", hi=10.0, seed=23)
    U0 = init_for(inst, r, 7)
    res = run_oracle(inst, U0, r, 5.0, 0.1, 10)
    _, Lh, Sh, _ = run_gpu(inst, U0, r, 5.0, 0.1, 10, bf16x3=True)
    hL, hS = rel(Lh, res.L_full()), rel(Sh, res.S_full())
    announce(f"bf16x3 r={r} widths={widths}: relL={hL:.3e} relS={hS:.3e}")
    assert hL <= X3_TOL and hS <= X3_TOL


@pytest.mark.parametrize("r", [20, 64])
def test_bf16x3_vpass_tiles_follow_oracle(r):
    """Three-product rounds with one and with two 64-column tiles per V-pass
    work-group (column groups 1 and 4) on ragged m, clients of 1-3 tiles and
    an odd tile count stay within the three-product bar of the FP64
    trajectory (rho = 1 keeps the closed-form step well conditioned for
    clients of 70 columns at r = 64); each gives the same bits from the
    per-group grid and from the tile queue."""
    import torch
    from gpu_helpers import run_gpu
    inst = planted_instance(301, [70, 190, 130, 96], 4, 0.05, values="uniform", hi=10.0, seed=31)
    U0 = init_for(inst, r, 7)
    res = run_oracle(inst, U0, r, 1.0, 0.1, 10)
    out = {}
    for cg in (1, 4):
        for q in (0, 1):
            s, Lg, Sg, _ = run_gpu(inst, U0, r, 1.0, 0.1, 10, bf16x3=True,
                                   shape=dict(column_groups=cg, vpass_queue=q))
            out[(cg, q)] = (Lg, Sg)
            eL, eS = rel(Lg, res.L_full()), rel(Sg, res.S_full())
            announce(f"bf16x3 r={r} column_groups={cg} vpass_queue={q}: relL={eL:.3e} relS={eS:.3e}")
            assert eL <= X3_TOL and eS <= X3_TOL
            del s
            torch.cuda.synchronize()
        assert np.array_equal(out[(cg, 0)][0], out[(cg, 1)][0])
        assert np.array_equal(out[(cg, 0)][1], out[(cg, 1)][1])


def test_precision_rules_and_switching():
    """A context made with RPCA_FLAG_BF16X3 alone starts in three-product
    rounds, refuses plain BF16 (it holds no BF16 copy of M), and switches to
    FP32 and back bitwise reproducibly; a context with RPCA_FLAG_BF16 can run
    all three precisions."""
    from paper_2207_11669_amd import RpcaError
    inst = planted_instance(260, [90, 70, 110], 4, 0.05, values="uniform", hi=10.0, seed=5)
    U0 = init_for(inst, 8, 3)
    lam = default_lam(inst)
    outs = []
    for _ in range(2):
        s = _session(inst, U0, 8, lam, bf16x3=True)
        with pytest.raises(RpcaError):
            s.set_precision("bf16")
        s.step(5)
        s.set_precision("fp32")
        s.step(4)
        s.set_precision("bf16x3")
        s.step(3)
        outs.append(_gpu_LS(s, inst.m))
        s.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    s = _session(inst, U0, 8, lam, bf16=True)
    for prec in ("bf16x3", "fp32", "bf16"):
        s.set_precision(prec)
        s.step(2)
    s.close()
