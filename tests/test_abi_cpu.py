"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/rpca.h declares, validates parameters, and sizes its
workspace; the product path never touches the oracle."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2207_11669_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2207_11669_amd import build
        build.build()
    return binding.load_library()


def test_exports_every_declared_function(lib):
    from paper_2207_11669_amd import declared_functions
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name


def test_parameter_validation_messages(lib):
    from paper_2207_11669_amd import make_params, params_error
    ok, _k = make_params(100, [30, 70], 5, 0.1, 0.1)
    assert params_error(ok) is None
    # Ranks up to 128 in FP32; the mixed-precision flags up to 64.
    for r in (64, 65, 100, 128):
        ok, _k = make_params(100, [30, 70], r, 0.1, 0.1)
        assert params_error(ok) is None, r
    ok, _k = make_params(100, [30, 70], 64, 0.1, 0.1, bf16=True)
    assert params_error(ok) is None
    cases = [
        (dict(m=0, widths=[3], r=1, rho=0.1, lam=0.1), "m must"),
        (dict(m=1 << 26, widths=[3], r=1, rho=0.1, lam=0.1), "m must"),
        (dict(m=10, widths=[3, 0], r=1, rho=0.1, lam=0.1), "n_i"),
        (dict(m=10, widths=[3], r=0, rho=0.1, lam=0.1), "r must"),
        (dict(m=10, widths=[3], r=129, rho=0.1, lam=0.1), "r must"),
        (dict(m=10, widths=[3], r=65, rho=0.1, lam=0.1, bf16=True), "r <= 64"),
        (dict(m=10, widths=[3], r=65, rho=0.1, lam=0.1, bf16x3=True), "r <= 64"),
        (dict(m=10, widths=[3], r=2, rho=0.0, lam=0.1), "rho"),
        (dict(m=10, widths=[3], r=2, rho=0.1, lam=-1.0), "lambda"),
        (dict(m=10, widths=[3], r=2, rho=0.1, lam=0.1, K=0), "K must"),
        (dict(m=10, widths=[3], r=2, rho=0.1, lam=0.1, inner=0), "inner"),
        (dict(m=10, widths=[3], r=2, rho=0.1, lam=0.1, u_mode="grad", eta0=0.0), "eta0"),
    ]
    for kw, frag in cases:
        p, _k = make_params(**kw)
        msg = params_error(p)
        assert msg is not None and frag in msg, (kw, msg)


def test_workspace_bytes_grow_with_problem(lib):
    from paper_2207_11669_amd import make_params, workspace_bytes
    p1, _a = make_params(4000, [500] * 16, 20, 0.1, 0.01, store_s=True)
    p2, _b = make_params(4000, [500] * 16, 20, 0.1, 0.01, K=2)
    p3, _c = make_params(8000, [500] * 16, 20, 0.1, 0.01, store_s=True)
    p4, _d = make_params(4000, [500] * 16, 20, 0.1, 0.01)
    b1, b2, b3, b4 = (workspace_bytes(p) for p in (p1, p2, p3, p4))
    # A stored S alone is m * n * 4 bytes; K > 1 stores S and per-client factors.
    assert b1 >= 4000 * 8000 * 4
    assert b2 > b1 and b3 > b1
    # With S rebuilt each round (K = 1, one alternation) no m x n buffer exists.
    assert b4 < 4000 * 8000 * 4 // 2
    assert b1 % 256 == 0 and b4 % 256 == 0


def test_product_path_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2207_11669_amd")
    for dirpath, _dirs, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "oracle/" not in text, f


def test_bf16_flag_rules_and_workspace(lib):
    """RPCA_FLAG_BF16 needs the rebuilt-S form (K = 1, one alternation, no
    stored S); its workspace holds two BF16 copies of M (2 B per entry each,
    columns padded to 64 per client, rows to 128)."""
    from paper_2207_11669_amd import make_params, params_error, workspace_bytes
    for kw in (dict(K=2), dict(inner=2), dict(store_s=True)):
        p, _k = make_params(100, [30, 70], 5, 0.1, 0.1, bf16=True, **kw)
        msg = params_error(p)
        assert msg is not None and "RPCA_FLAG_BF16" in msg, (kw, msg)
    p32, _a = make_params(4000, [500] * 16, 20, 0.1, 0.01)
    p16, _b = make_params(4000, [500] * 16, 20, 0.1, 0.01, bf16=True)
    assert params_error(p16) is None
    extra = workspace_bytes(p16) - workspace_bytes(p32)
    mp, nvp = 4096, 16 * 512
    assert extra >= 2 * 2 * mp * nvp
    assert extra < 2 * 2 * mp * nvp + 16 * (mp + nvp) * 64 * 4


def test_sparse_s_flag_rules_and_workspace(lib):
    """RPCA_FLAG_SPARSE_S needs the rebuilt-S form; its workspace holds, per
    16 x 16 tile of (rows rounded to 128, widths rounded to 64 per client),
    one 64-bit slot word and room for 64 float4 slots: 4.03125 B per entry."""
    from paper_2207_11669_amd import make_params, params_error, workspace_bytes
    for kw in (dict(K=2), dict(inner=2), dict(store_s=True)):
        p, _k = make_params(100, [30, 70], 5, 0.1, 0.1, sparse_s=True, **kw)
        msg = params_error(p)
        assert msg is not None and "RPCA_FLAG_SPARSE_S" in msg, (kw, msg)
    ok, _o = make_params(100, [30, 70], 5, 0.1, 0.1, sparse_s=True, bf16=True, graph=True)
    assert params_error(ok) is None
    p0, _a = make_params(1000, [100, 9, 300], 20, 0.1, 0.01)
    p1, _b = make_params(1000, [100, 9, 300], 20, 0.1, 0.01, sparse_s=True)
    mp, nvp = 1024, 128 + 64 + 320
    tiles = (mp // 16) * (nvp // 16)
    extra = workspace_bytes(p1) - workspace_bytes(p0)
    assert tiles * (8 + 1024) <= extra <= tiles * (8 + 1024) + 2 * 256


def test_size_limits_of_the_32_bit_buffer_ranges(lib):
    """Factor layouts are addressed with 32-bit byte ranges: (m rounded up to
    128) x (r rounded up to 16) x 4 B and (sum of the widths rounded up to 64)
    x (r rounded up to 16) x 4 B must stay below 2^31; one past either edge is
    refused with a message, the edge itself accepted."""
    from paper_2207_11669_amd import make_params, params_error
    # r = 64 (RP = 64): m rounded up to 128 must be < 2^23.
    ok, _a = make_params((1 << 23) - 128, [64], 64, 0.1, 0.1)
    assert params_error(ok) is None
    bad, _b = make_params((1 << 23) - 127, [64], 64, 0.1, 0.1)
    msg = params_error(bad)
    assert msg is not None and "m rounded up to 128" in msg, msg
    # r = 16 (RP = 16): the same bound is 2^25 rows, beyond which m < 2^26 decides.
    ok16, _c = make_params((1 << 25) - 128, [64], 16, 0.1, 0.1)
    assert params_error(ok16) is None
    # Columns: widths rounded up to 64 and summed, times RP = 64, below 2^29 floats.
    w_ok = [(1 << 22), (1 << 22) - 64]
    okc, _d = make_params(100, w_ok, 64, 0.1, 0.1)
    assert params_error(okc) is None
    badc, _e = make_params(100, [(1 << 22), (1 << 22) - 64, 1], 64, 0.1, 0.1)
    msg = params_error(badc)
    assert msg is not None and "n_i rounded up to 64" in msg, msg


def test_init_rejects_bad_workspace_before_any_device_call(lib):
    """rpca_init checks the workspace on the host: NULL, too small and
    misaligned workspaces give RPCA_EWORKSPACE (nothing is enqueued), and
    rpca_last_error(NULL) names the cause. The device pointers are never
    dereferenced on these paths, so stand-in addresses serve."""
    import ctypes

    from paper_2207_11669_amd import binding as B
    p, _k = B.make_params(64, [32, 32], 4, 0.1, 0.1)
    need = B.workspace_bytes(p)
    fake = 1 << 20  # 16-byte and 256-byte aligned stand-in address
    ptrs = (ctypes.c_void_p * 2)(fake, fake + 64 * 32 * 4)
    lds = (ctypes.c_int64 * 2)(64, 64)
    ctx = ctypes.c_void_p()
    cases = [(None, need, "NULL"), (fake, need - 256, "need"), (fake + 128, need, "aligned")]
    for ws, size, frag in cases:
        st = lib.rpca_init(ctypes.byref(ctx), ctypes.byref(p), ptrs, lds, ctypes.c_void_p(fake),
                           64, ctypes.c_void_p(ws), size, None)
        assert st == B.RPCA_EWORKSPACE, (ws, size, st)
        assert ctx.value is None
        assert frag in B.last_init_error(), B.last_init_error()
    # Invalid parameters are reported the same way (RPCA_EINVAL).
    bad, _b = B.make_params(64, [32, 32], 0, 0.1, 0.1)
    st = lib.rpca_init(ctypes.byref(ctx), ctypes.byref(bad), ptrs, lds, None, 0,
                       ctypes.c_void_p(fake), need, None)
    assert st == B.RPCA_EINVAL and "r must" in B.last_init_error()
