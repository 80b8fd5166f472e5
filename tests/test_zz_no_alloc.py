"""rpca_init_static: the allocation-free variant of rpca_init (workspace in
the library's static device array) against rpca_init with a caller-owned
workspace, through the C ABI, on two problems in a row, the second smaller,
each compared with the existing entry point's output bit for bit (same
kernels, same launch shapes, same summation orders). Also its size limit and
its one-context-per-GPU rule."""
import numpy as np
import pytest

from gpu_helpers import announce, default_lam, rel
from rpca_inputs import planted_instance, splitmix_gaussian_init

pytestmark = pytest.mark.gpu


def _LS(s, m):
    import torch
    L, S = s.get_LS(-1)
    torch.cuda.synchronize()
    return L[:, :m].T.double().cpu().numpy(), S[:, :m].T.double().cpu().numpy()


def _pair(inst, r, T, **kw):
    from paper_2207_11669_amd import DCFPCA, colmajor
    lam = default_lam(inst)
    U0 = colmajor(splitmix_gaussian_init(inst.m, r, 5))
    M = colmajor(inst.M)
    a = DCFPCA(M, inst.widths, inst.m, r, 0.1, lam, U0, static_workspace=True, **kw)
    a.step(T)
    La, Sa = _LS(a, inst.m)
    hist_a = [a.stats(t)["objective"] for t in range(T)]
    a.close()
    b = DCFPCA(M, inst.widths, inst.m, r, 0.1, lam, U0, **kw)
    b.step(T)
    Lb, Sb = _LS(b, inst.m)
    hist_b = [b.stats(t)["objective"] for t in range(T)]
    b.close()
    return (La, Sa, hist_a), (Lb, Sb, hist_b)


def test_static_workspace_matches_caller_workspace_twice_then_smaller():
    big = planted_instance(300, [100, 120, 90], 6, 0.05, values="uniform", hi=10.0, seed=41)
    small = planted_instance(150, [40, 50], 3, 0.05, values="uniform", hi=10.0, seed=42)
    for inst, r, kw in ((big, 8, {}), (small, 4, {}), (small, 4, dict(u_mode="grad", eta0=1e-3))):
        announce(f"static workspace: m={inst.m} widths={inst.widths} r={r} {kw}")
        (La, Sa, ha), (Lb, Sb, hb) = _pair(inst, r, 25, **kw)
        announce(f"static vs caller workspace: relL={rel(La, Lb):.3e} relS={rel(Sa, Sb):.3e} "
                 f"bitwise={np.array_equal(La, Lb) and np.array_equal(Sa, Sb)}")
        assert rel(La, Lb) <= 1e-5 and rel(Sa, Sb) <= 1e-5
        assert np.array_equal(La, Lb) and np.array_equal(Sa, Sb) and ha == hb


def test_static_workspace_limits():
    """Parameters needing more than the static array are refused with
    RPCA_EWORKSPACE; a second live context on the same GPU with RPCA_ESTATE,
    and creation works again once the first is destroyed."""
    from paper_2207_11669_amd import DCFPCA, RpcaError, colmajor, make_params, workspace_bytes
    from paper_2207_11669_amd.binding import RPCA_ESTATE, RPCA_EWORKSPACE
    inst = planted_instance(200, [60, 70], 3, 0.05, values="uniform", hi=10.0, seed=43)
    M = colmajor(inst.M)
    lam = default_lam(inst)
    p, _k = make_params(200, [60, 70], 3, 0.1, lam, store_s=True)
    assert workspace_bytes(p) < (64 << 20)
    # A wide stored-S problem whose workspace exceeds 64 MiB (m x n x 4 B of S).
    import torch
    wide = torch.zeros((5000, 4000), dtype=torch.float32, device="cuda")
    with pytest.raises(RpcaError) as ei:
        DCFPCA(wide, [5000], 4000, 4, 0.1, 0.01, None, store_s=True, static_workspace=True)
    assert ei.value.status == RPCA_EWORKSPACE and "static workspace" in str(ei.value)
    a = DCFPCA(M, inst.widths, inst.m, 3, 0.1, lam, None, static_workspace=True)
    with pytest.raises(RpcaError) as ei:
        DCFPCA(M, inst.widths, inst.m, 3, 0.1, lam, None, static_workspace=True)
    assert ei.value.status == RPCA_ESTATE
    a.close()
    b = DCFPCA(M, inst.widths, inst.m, 3, 0.1, lam, None, static_workspace=True)
    b.step(3)
    b.close()
