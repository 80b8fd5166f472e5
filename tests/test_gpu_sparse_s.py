"""Sparse S between the passes (RPCA_FLAG_SPARSE_S): each FP32 S-pass also
writes S (eq. "optS") as a slot word plus packed nonzero float4 slots per
16 x 16 tile, and the next V-pass reads those instead of rebuilding S from the
previous factors. S is the same bit for bit, so whole trajectories must be
bitwise those without the flag: in every launch shape and form, at ranks
that take the quad path and the full rank tiles, on ragged rows and client
widths (narrower than one tile too), under graph replay, across lambda
changes and precision switches (where the library falls back to the
rebuild), across rpca_copy_state, and with every entry of S nonzero (full
tiles). Then against the FP64 oracle."""
import numpy as np
import pytest

from gpu_helpers import announce, default_lam, init_for, parity, rel
from rpca_inputs import loguniform_widths, planted_instance

pytestmark = pytest.mark.gpu


def _instance(m=1007, seed=61):
    # Ragged: m is not a multiple of 16, widths are not multiples of 16, and
    # two clients are narrower than one 16-column tile.
    widths = [9, 13] + loguniform_widths(14, 17, 300, seed=seed)
    return planted_instance(m, widths, 5, 0.08, values="uniform", hi=10.0, seed=seed,
                            support="bernoulli")


def _session(inst, r, lam=None, shape=None, **kw):
    from paper_2207_11669_amd import DCFPCA, colmajor
    lam = default_lam(inst) if lam is None else lam
    s = DCFPCA(colmajor(inst.M), inst.widths, inst.m, r, 0.1, lam,
               colmajor(init_for(inst, r, 3)), **kw)
    if shape:
        s.set_launch_shape(**shape)
    return s


def _snap(s):
    """L, S (rows below m; the rows up to the leading dimension are padding
    the library does not write) and the last round's statistics."""
    import torch
    L, S = s.get_LS(-1)
    torch.cuda.synchronize()
    return L[:, :s.m].cpu().numpy(), S[:, :s.m].cpu().numpy(), s.stats()


def _same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def _trajectory(inst, r, shape=None, rounds=9, lam=None, schedule=None, precisions=None,
                sparse_per_round=None, **kw):
    """Checkpoints after rounds 1, 2 and `rounds`. schedule: lambda per round
    (scaled from the default); precisions: precision per round;
    sparse_per_round: the launch shape's sparse choice per round."""
    s = _session(inst, r, lam=lam, shape=shape, **kw)
    lam0 = default_lam(inst) if lam is None else lam
    out = []
    for t in range(rounds):
        if schedule is not None:
            s.set_lambda(lam0 * schedule[t])
        if precisions is not None:
            s.set_precision(precisions[t])
        if sparse_per_round is not None:
            s.set_launch_shape(sparse_s=sparse_per_round[t])
        s.step(1)
        if t in (0, 1, rounds - 1):
            out.append(_snap(s))
    s.close()
    return out


def _differences(x, y):
    out = []
    for part, u, v in (("L", x[0], y[0]), ("S", x[1], y[1])):
        if not np.array_equal(u, v):
            bad = ~((u == v) | (np.isnan(u) & np.isnan(v)))
            idx = np.argwhere(bad)
            out.append(f"{part}: {int(bad.sum())} entries differ, first at {idx[0].tolist()}: "
                       f"{u[tuple(idx[0])]!r} vs {v[tuple(idx[0])]!r}")
    out += [f"{k}: {x[2][k]!r} vs {y[2][k]!r}" for k in x[2] if x[2][k] != y[2][k]]
    return "; ".join(out)


def _compare(name, a, b):
    for k, (x, y) in enumerate(zip(a, b)):
        same = _same(x, y)
        announce(f"{name} checkpoint {k} (round {y[2]['t']:.0f}): bitwise={same} "
                 f"relL={rel(y[0], x[0]):.2e} nnz={y[2]['nnz']:.0f}")
        if not same:
            announce(f"{name} checkpoint {k}: {_differences(x, y)}")
        assert same


SHAPES = {
    "r5_static_g1_p2": (5, dict(column_groups=1, spass_phases=2, vpass_queue=0, spass_queue=0)),
    "r12_queue_g4_p1": (12, dict(column_groups=4, spass_phases=1, vpass_queue=1, spass_queue=1)),
    "r20_queue_g4_p1": (20, dict(column_groups=4, spass_phases=1, vpass_queue=1, spass_queue=1)),
    "r33_static_g4_p2": (33, dict(column_groups=4, spass_phases=2, vpass_queue=0, spass_queue=0)),
    "r64_queue_g1_p2": (64, dict(column_groups=1, spass_phases=2, vpass_queue=1, spass_queue=0)),
    "r64_static_g4_p1": (64, dict(column_groups=4, spass_phases=1, vpass_queue=0, spass_queue=1)),
}


@pytest.mark.parametrize("name", list(SHAPES))
def test_sparse_is_bitwise_the_rebuild(name):
    r, shape = SHAPES[name]
    inst = _instance()
    announce(f"sparse S vs rebuild: {name}, m={inst.m}, widths={inst.widths}")
    a = _trajectory(inst, r, shape)
    b = _trajectory(inst, r, shape, sparse_s=True)
    _compare(name, a, b)


def test_sparse_row_splits():
    """More row splits than the default (V-pass chunks start on odd 16-row
    tiles of the 32-row strips the S-pass waves write)."""
    inst = _instance(m=2001, seed=62)
    shape = dict(row_splits=7, column_groups=1)
    announce(f"sparse S, 7 row splits: m={inst.m}")
    _compare("splits", _trajectory(inst, 20, shape), _trajectory(inst, 20, shape, sparse_s=True))


def test_sparse_full_tiles():
    """lambda = 0: S = M - U V^T, every entry nonzero, every tile's 256 value
    slots in use."""
    inst = _instance(seed=63)
    announce("sparse S with every entry nonzero (lambda = 0)")
    a = _trajectory(inst, 8, lam=0.0, rounds=4)
    _compare("full, rebuild twice", a, _trajectory(inst, 8, lam=0.0, rounds=4))
    b = _trajectory(inst, 8, lam=0.0, rounds=4, sparse_s=True)
    assert b[-1][2]["nnz"] >= 0.99 * inst.m * inst.n
    _compare("full", a, b)


def test_sparse_graph_replay():
    inst = _instance(seed=64)
    announce("sparse S under graph replay")
    a = _trajectory(inst, 20, rounds=10, graph=True)
    b = _trajectory(inst, 20, rounds=10, graph=True, sparse_s=True)
    _compare("graph", a, b)


def test_sparse_lambda_changes():
    """A round after a lambda change rebuilds S (the sparse S holds the old
    lambda's); later rounds at a constant lambda read it again."""
    inst = _instance(seed=65)
    sched = [8.0, 8.0, 4.0, 2.0, 2.0, 1.0, 1.0, 1.0, 1.0]
    announce("sparse S across lambda changes")
    a = _trajectory(inst, 20, schedule=sched)
    b = _trajectory(inst, 20, schedule=sched, sparse_s=True)
    _compare("lambda", a, b)


def test_sparse_precision_switches():
    """Three-product BF16 rounds write no sparse S: the first FP32 round after
    them rebuilds; BF16 rounds after FP32 ones ignore the sparse S."""
    inst = _instance(seed=66)
    prec = ["bf16x3", "bf16x3", "fp32", "fp32", "bf16x3", "fp32", "fp32", "fp32", "fp32"]
    announce("sparse S across precision switches")
    a = _trajectory(inst, 20, precisions=prec, bf16x3=True)
    b = _trajectory(inst, 20, precisions=prec, bf16x3=True, sparse_s=True)
    _compare("precision", a, b)


def test_sparse_shape_switches():
    """The launch shape's sparse choice switched between rounds (as the
    autotuner does): a round after a rebuilt one rebuilds S, and the
    trajectory stays bitwise the rebuild's; a context without the flag refuses
    the sparse choice."""
    from paper_2207_11669_amd import RpcaError
    inst = _instance(seed=68)
    per_round = [1, 1, 0, 1, 1, 0, 0, 1, 1]
    announce("sparse S across launch-shape switches")
    a = _trajectory(inst, 20)
    b = _trajectory(inst, 20, sparse_per_round=per_round, sparse_s=True)
    _compare("switches", a, b)
    s = _session(inst, 20)
    assert s.launch_shape()["sparse_s"] == 0
    with pytest.raises(RpcaError, match="RPCA_FLAG_SPARSE_S"):
        s.set_launch_shape(sparse_s=1)
    s.close()
    s = _session(inst, 20, sparse_s=True)
    assert s.launch_shape()["sparse_s"] == 1
    with pytest.raises(RpcaError, match="sparse"):
        s.set_launch_shape(sparse_s=2)
    s.close()


def test_sparse_copy_state():
    """rpca_copy_state carries the sparse S and its validity: a copy taken
    mid-run continues bitwise like the original and like the rebuild."""
    inst = _instance(seed=67)
    announce("sparse S across rpca_copy_state")
    ref = _trajectory(inst, 20, rounds=6)
    s = _session(inst, 20, sparse_s=True)
    c = _session(inst, 20, sparse_s=True)
    s.step(3)
    c.copy_state_from(s)
    s.step(3)
    c.step(3)
    a, b = _snap(s), _snap(c)
    s.close()
    c.close()
    assert _same(a, b)
    _compare("copy", [ref[-1]], [b])


def test_sparse_parity_with_oracle():
    widths = loguniform_widths(30, 40, 400, seed=9)
    inst = planted_instance(2500, widths, 5, 0.05, values="uniform", hi=10.0, seed=9,
                            support="bernoulli")
    parity(inst, 8, 20, u_mode="closed", sparse_s=True)
