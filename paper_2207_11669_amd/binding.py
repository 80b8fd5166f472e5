"""ctypes binding of librpca.so (the C ABI in include/rpca.h).

Argument marshalling only: every step of the DCF-PCA round runs in the HIP
library. PyTorch provides device memory (inputs, outputs and the workspace)
and the stream. There is no fallback: if the library is missing, loading it
raises.

Storage convention: a column-major m x n matrix with leading dimension ld is
held in a contiguous torch tensor of shape (n, ld) -- row j of the tensor is
column j of the matrix. `colmajor(X)` builds one from an (m, n) array and
`.T[:m]` of such a tensor views it back as m x n.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_uint32,
                    c_uint64, c_void_p)
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "librpca.so")
ROOT = os.path.dirname(HERE)
HEADER = os.path.join(ROOT, "include", "rpca.h")

RPCA_OK = 0
RPCA_EINVAL = -1
RPCA_EWORKSPACE = -2
RPCA_EDEVICE = -3
RPCA_ENONFINITE = -4
RPCA_ESTATE = -5
RPCA_WARN_THM2 = 1

U_MODES = {"grad": 0, "closed": 1}
ETA_SCHEDS = {"const": 0, "sqrt": 1}


class RpcaParams(ctypes.Structure):
    _fields_ = [
        ("m", c_int64),
        ("E", c_int32),
        ("n_cols", POINTER(c_int64)),
        ("r", c_int32),
        ("rho", c_double),
        ("lam", c_double),
        ("K", c_int32),
        ("inner", c_int32),
        ("u_mode", c_int32),
        ("eta0", c_double),
        ("eta_sched", c_int32),
        ("flags", c_uint32),
        ("seed", c_uint64),
    ]


class RpcaStats(ctypes.Structure):
    _fields_ = [(k, c_double) for k in
                ("t", "objective", "lambda_fro_sq", "nnz", "du_sq", "u_sq", "v_sq", "l1",
                 "objective_target")]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class RpcaLaunchShape(ctypes.Structure):
    _fields_ = [("vsplit", c_int32), ("vcols", c_int32), ("sphases", c_int32),
                ("vqueue", c_int32), ("squeue", c_int32), ("sparse", c_int32)]

    def as_dict(self) -> dict:
        return {"row_splits": int(self.vsplit), "column_groups": int(self.vcols),
                "spass_phases": int(self.sphases), "vpass_queue": int(self.vqueue),
                "spass_queue": int(self.squeue), "sparse_s": int(self.sparse)}


class RpcaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rpca status {status}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librpca.so (built in-tree by paper_2207_11669_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch wheels carry their own HIP runtime; loading torch first makes the
    # library bind to that same runtime, so that torch's streams and device
    # pointers are valid in it.
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    vp = c_void_p
    sigs = {
        "rpca_params_error": (c_char_p, [POINTER(RpcaParams)]),
        "rpca_workspace_bytes": (c_int32, [POINTER(RpcaParams), POINTER(c_size_t)]),
        "rpca_init": (c_int32, [POINTER(vp), POINTER(RpcaParams), POINTER(vp), POINTER(c_int64),
                                vp, c_int64, vp, c_size_t, vp]),
        "rpca_init_static": (c_int32, [POINTER(vp), POINTER(RpcaParams), POINTER(vp),
                                       POINTER(c_int64), vp, c_int64, vp]),
        "rpca_step": (c_int32, [vp, c_int32]),
        "rpca_autotune": (c_int32, [vp, c_int32, POINTER(RpcaLaunchShape)]),
        "rpca_get_launch_shape": (c_int32, [vp, POINTER(RpcaLaunchShape)]),
        "rpca_set_launch_shape": (c_int32, [vp, POINTER(RpcaLaunchShape)]),
        "rpca_set_precision": (c_int32, [vp, c_int32]),
        "rpca_set_lambda": (c_int32, [vp, c_double]),
        "rpca_set_step": (c_int32, [vp, c_double]),
        "rpca_copy_state": (c_int32, [vp, vp]),
        "rpca_mlp_param_count": (c_int64, []),
        "rpca_mlp_forward": (c_int32, [vp, vp, c_int64, vp, vp]),
        "rpca_mlp_train_step": (c_int32, [vp, vp, vp, c_int64, c_float, vp, vp]),
        "rpca_solve": (c_int32, [vp, c_int32, c_double, c_int32, POINTER(c_int32),
                                 POINTER(c_double)]),
        "rpca_set_target": (c_int32, [vp, vp, c_int64, vp, c_int64, c_int32]),
        "rpca_target_error": (c_int32, [vp, POINTER(c_double)]),
        "rpca_get_LS": (c_int32, [vp, c_int32, vp, c_int64, vp, c_int64]),
        "rpca_get_factors": (c_int32, [vp, vp, c_int64, vp, c_int64]),
        "rpca_get_stats": (c_int32, [vp, c_int64, POINTER(RpcaStats)]),
        "rpca_profile": (c_int32, [vp, c_int32, POINTER(c_double), POINTER(c_int64)]),
        "rpca_rounds": (c_int64, [vp]),
        "rpca_last_error": (c_char_p, [vp]),
        "rpca_destroy": (None, [vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


RPCA_FLAG_STORE_S = 1
RPCA_FLAG_GRAPH = 2
RPCA_FLAG_BF16 = 4
RPCA_FLAG_BF16X3 = 8
RPCA_FLAG_SPARSE_S = 16
PRECISIONS = {"fp32": 0, "bf16": 1, "bf16x3": 2}


def make_params(m: int, widths: Sequence[int], r: int, rho: float, lam: float, K: int = 1,
                inner: int = 1, u_mode: str = "closed", eta0: float = 0.0,
                eta_sched: str = "const", store_s: bool = False, graph: bool = False,
                bf16: bool = False, bf16x3: bool = False, seed: int = 0,
                sparse_s: bool = False):
    """Build an rpca_params struct; returns (params, n_cols array to keep alive)."""
    ncols = (c_int64 * len(widths))(*[int(w) for w in widths])
    flags = ((RPCA_FLAG_STORE_S if store_s else 0) | (RPCA_FLAG_GRAPH if graph else 0)
             | (RPCA_FLAG_BF16 if bf16 else 0) | (RPCA_FLAG_BF16X3 if bf16x3 else 0)
             | (RPCA_FLAG_SPARSE_S if sparse_s else 0))
    p = RpcaParams(m=int(m), E=len(widths), n_cols=ncols, r=int(r), rho=float(rho),
                   lam=float(lam), K=int(K), inner=int(inner), u_mode=U_MODES[u_mode],
                   eta0=float(eta0), eta_sched=ETA_SCHEDS[eta_sched], flags=flags,
                   seed=int(seed) & 0xFFFFFFFFFFFFFFFF)
    return p, ncols


def params_error(p: RpcaParams) -> Optional[str]:
    msg = load_library().rpca_params_error(ctypes.byref(p))
    return None if msg is None else msg.decode()


def workspace_bytes(p: RpcaParams) -> int:
    out = c_size_t(0)
    st = load_library().rpca_workspace_bytes(ctypes.byref(p), ctypes.byref(out))
    if st != RPCA_OK:
        raise RpcaError(st, params_error(p) or "invalid parameters")
    return int(out.value)


def _ld(m: int) -> int:
    return (m + 3) // 4 * 4


def colmajor(X, device="cuda", ld: Optional[int] = None):
    """(m, n) array -> contiguous FP32 tensor (n, ld) holding X column-major."""
    import numpy as np
    import torch
    X = np.asarray(X, dtype=np.float32)
    m, n = X.shape
    ld = _ld(m) if ld is None else int(ld)
    if ld == m and X.T.flags["C_CONTIGUOUS"]:
        # Already column-major with no padding rows: upload as is.
        return torch.from_numpy(X.T).to(device)
    buf = np.zeros((n, ld), dtype=np.float32)
    buf[:, :m] = X.T
    return torch.from_numpy(buf).to(device)


class DCFPCA:
    """One DCF-PCA problem on one GPU (Algorithm 1 of arXiv 2207.11669).

    M_cols: (n, ldm) FP32 CUDA tensor, M column-major (see `colmajor`); client i
    owns columns offsets[i]:offsets[i+1] in order. U0_cols: (r, ldu) tensor
    with U^(0) column-major, or None: the library draws U^(0) on the device
    from `seed` (i.i.d. N(0, 1), the rule stated with rpca_init). bf16=True
    static_workspace=True creates the context with rpca_init_static (the
    library's static device workspace; no workspace tensor is allocated).
    bf16=True creates the context with
    RPCA_FLAG_BF16: rounds run in BF16 until set_precision("fp32").
    bf16x3=True (RPCA_FLAG_BF16X3): rounds run as three-product BF16.
    sparse_s=True (RPCA_FLAG_SPARSE_S): FP32 rounds hand S from the S-pass to
    the next V-pass in sparse form instead of rebuilding it.
    """

    def __init__(self, M_cols, widths: Sequence[int], m: int, r: int, rho: float, lam: float,
                 U0_cols, K: int = 1, inner: int = 1, u_mode: str = "closed",
                 eta0: float = 0.0, eta_sched: str = "const", store_s: bool = False,
                 graph: bool = False, stream=None, bf16: bool = False, bf16x3: bool = False,
                 seed: int = 0, static_workspace: bool = False, sparse_s: bool = False):
        import torch
        self._lib = load_library()
        if not (M_cols.is_cuda and M_cols.dtype == torch.float32 and M_cols.is_contiguous()):
            raise ValueError("M_cols must be a contiguous float32 CUDA tensor")
        if U0_cols is not None and not (U0_cols.is_cuda and U0_cols.dtype == torch.float32
                                        and U0_cols.is_contiguous()):
            raise ValueError("U0_cols must be a contiguous float32 CUDA tensor or None")
        self.m, self.r = int(m), int(r)
        self.widths = [int(w) for w in widths]
        self.n = sum(self.widths)
        if M_cols.shape[0] != self.n:
            raise ValueError("M_cols must have one row per column of M")
        self.ldm = int(M_cols.shape[1])
        self.params, self._ncols = make_params(m, self.widths, r, rho, lam, K, inner, u_mode,
                                               eta0, eta_sched, store_s, graph, bf16, bf16x3,
                                               seed, sparse_s)
        err = params_error(self.params)
        if err:
            raise ValueError(err)
        self.device = M_cols.device
        self.M_cols = M_cols  # borrowed by the library: keep it alive
        self.ws = None if static_workspace else torch.empty(
            workspace_bytes(self.params), dtype=torch.uint8, device=self.device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
            if graph and stream.cuda_stream == 0:
                # Graph capture needs a stream other than the null stream.
                stream = torch.cuda.Stream(self.device)
        self.stream = stream
        # Inputs were written on the caller's stream; order the library's work
        # after them. Outputs are handed back the same way (see _hand_back).
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        base = M_cols.data_ptr()
        ptrs, lds, off = [], [], 0
        for w in self.widths:
            ptrs.append(base + off * self.ldm * 4)
            lds.append(self.ldm)
            off += w
        self._ptrs = (c_void_p * len(ptrs))(*ptrs)
        self._ldms = (c_int64 * len(lds))(*lds)
        ctx = c_void_p()
        u0 = c_void_p(U0_cols.data_ptr()) if U0_cols is not None else c_void_p(None)
        ldu = int(U0_cols.shape[1]) if U0_cols is not None else 0
        if static_workspace:
            st = self._lib.rpca_init_static(ctypes.byref(ctx), ctypes.byref(self.params),
                                            self._ptrs, self._ldms, u0, ldu,
                                            c_void_p(self.stream.cuda_stream))
        else:
            st = self._lib.rpca_init(ctypes.byref(ctx), ctypes.byref(self.params), self._ptrs,
                                     self._ldms, u0, ldu, c_void_p(self.ws.data_ptr()),
                                     self.ws.numel(), c_void_p(self.stream.cuda_stream))
        if st < 0:
            raise RpcaError(st, "rpca_init failed: " + last_init_error())
        self.warning = st
        self.ctx = ctx

    def _check(self, st: int):
        if st != RPCA_OK:
            raise RpcaError(st, self._lib.rpca_last_error(self.ctx).decode())

    def _hand_back(self):
        """Order the caller's current stream after the library's work."""
        import torch
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.wait_stream(self.stream)

    def step(self, rounds: int = 1):
        self._check(self._lib.rpca_step(self.ctx, int(rounds)))

    def autotune(self, rounds: int = 10) -> dict:
        """Pick the launch shapes of the V-pass and the FP32 S-pass by timing
        real rounds; returns them as {"row_splits", "column_groups",
        "spass_phases", "vpass_queue", "spass_queue", "sparse_s"}."""
        k = RpcaLaunchShape()
        self._check(self._lib.rpca_autotune(self.ctx, int(rounds), ctypes.byref(k)))
        return k.as_dict()

    def launch_shape(self) -> dict:
        k = RpcaLaunchShape()
        self._check(self._lib.rpca_get_launch_shape(self.ctx, ctypes.byref(k)))
        return k.as_dict()

    def set_launch_shape(self, row_splits: int | None = None, column_groups: int | None = None,
                         spass_phases: int | None = None, vpass_queue: int | None = None,
                         spass_queue: int | None = None, sparse_s: int | None = None):
        """Fix the launch shapes (rpca_set_launch_shape); None keeps a value."""
        cur = self.launch_shape()
        pick = lambda key, v: cur[key] if v is None else int(v)  # noqa: E731
        k = RpcaLaunchShape(pick("row_splits", row_splits), pick("column_groups", column_groups),
                            pick("spass_phases", spass_phases), pick("vpass_queue", vpass_queue),
                            pick("spass_queue", spass_queue), pick("sparse_s", sparse_s))
        self._check(self._lib.rpca_set_launch_shape(self.ctx, ctypes.byref(k)))

    def copy_state_from(self, other: "DCFPCA"):
        """Take over other's whole iterate (same parameters; see rpca_copy_state)."""
        self._check(self._lib.rpca_copy_state(self.ctx, other.ctx))

    def set_lambda(self, lam: float):
        """lambda of the following rounds (rebuilt-S form only)."""
        self._check(self._lib.rpca_set_lambda(self.ctx, float(lam)))

    def set_step(self, omega: float):
        """Multiplier of the U step for the following rounds (1: the method's)."""
        self._check(self._lib.rpca_set_step(self.ctx, float(omega)))

    def set_precision(self, precision: str):
        """Precision of the following rounds' streaming passes: "fp32", "bf16" or
        "bf16x3"."""
        self._check(self._lib.rpca_set_precision(self.ctx, PRECISIONS[precision]))

    def solve(self, max_rounds: int, tol: float, check_every: int = 1):
        done, metric = c_int32(0), c_double(0.0)
        self._check(self._lib.rpca_solve(self.ctx, int(max_rounds), float(tol), int(check_every),
                                         ctypes.byref(done), ctypes.byref(metric)))
        return int(done.value), float(metric.value)

    def set_target(self, Ustar_cols, Vstar_cols, rstar: int):
        self._target = (Ustar_cols, Vstar_cols)
        self._check(self._lib.rpca_set_target(self.ctx, c_void_p(Ustar_cols.data_ptr()),
                                              int(Ustar_cols.shape[1]),
                                              c_void_p(Vstar_cols.data_ptr()),
                                              int(Vstar_cols.shape[1]), int(rstar)))

    def target_error(self) -> float:
        out = c_double(0.0)
        self._check(self._lib.rpca_target_error(self.ctx, ctypes.byref(out)))
        return float(out.value)

    def get_LS(self, client: int = -1):
        """(L, S) as (ncols, ld) column-major tensors of the client (or all)."""
        import torch
        ncols = self.n if client < 0 else self.widths[client]
        ld = _ld(self.m)
        L = torch.empty((ncols, ld), dtype=torch.float32, device=self.device)
        S = torch.empty((ncols, ld), dtype=torch.float32, device=self.device)
        self._check(self._lib.rpca_get_LS(self.ctx, int(client), c_void_p(L.data_ptr()), ld,
                                          c_void_p(S.data_ptr()), ld))
        self._hand_back()
        return L, S

    def get_factors(self):
        """(U, V) as (r, ldu) and (r, ldv) column-major tensors."""
        import torch
        ldu, ldv = _ld(self.m), _ld(self.n)
        U = torch.empty((self.r, ldu), dtype=torch.float32, device=self.device)
        V = torch.empty((self.r, ldv), dtype=torch.float32, device=self.device)
        self._check(self._lib.rpca_get_factors(self.ctx, c_void_p(U.data_ptr()), ldu,
                                               c_void_p(V.data_ptr()), ldv))
        self._hand_back()
        return U, V

    def stats(self, round_index: int = -1) -> dict:
        out = RpcaStats()
        self._check(self._lib.rpca_get_stats(self.ctx, int(round_index), ctypes.byref(out)))
        return out.as_dict()

    PHASES = ("vpass", "spass", "client_factor", "uupdate", "finalize", "vfinal")

    def profile(self, rounds: int) -> dict:
        """Average launch duration (ms) and launch count per kernel phase."""
        avg = (c_double * len(self.PHASES))()
        cnt = (c_int64 * len(self.PHASES))()
        self._check(self._lib.rpca_profile(self.ctx, int(rounds), avg, cnt))
        return {ph: (float(avg[k]), int(cnt[k])) for k, ph in enumerate(self.PHASES)}

    @property
    def rounds(self) -> int:
        return int(self._lib.rpca_rounds(self.ctx))

    def close(self):
        if getattr(self, "ctx", None):
            self._lib.rpca_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def last_init_error() -> str:
    """Cause of the last failed context creation on this thread."""
    return load_library().rpca_last_error(None).decode()


def mlp_param_count() -> int:
    return int(load_library().rpca_mlp_param_count())


def mlp_forward(params, x, stream=None):
    """MLP outputs (n, 2) -- the decay and the step multiplier -- for the rows
    of x ((n, 10) FP32 CUDA tensor); params: FP32 CUDA tensor of
    mlp_param_count() floats."""
    import torch
    n = int(x.shape[0])
    y = torch.empty((n, 2), dtype=torch.float32, device=x.device)
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    s = load_library().rpca_mlp_forward(c_void_p(params.data_ptr()), c_void_p(x.data_ptr()), n,
                                        c_void_p(y.data_ptr()), c_void_p(st.cuda_stream))
    if s != RPCA_OK:
        raise RpcaError(s, "rpca_mlp_forward failed")
    return y


def mlp_train_step(params, x, target, lr: float, grad_ws, stream=None):
    """One gradient-descent step of params on the mean squared-error loss
    (target: (n, 2) FP32 CUDA tensor)."""
    import torch
    n = int(x.shape[0])
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    s = load_library().rpca_mlp_train_step(c_void_p(params.data_ptr()), c_void_p(x.data_ptr()),
                                           c_void_p(target.data_ptr()), n, float(lr),
                                           c_void_p(grad_ws.data_ptr()), c_void_p(st.cuda_stream))
    if s != RPCA_OK:
        raise RpcaError(s, "rpca_mlp_train_step failed")


def declared_functions(header: str = HEADER):
    """Names of the functions include/rpca.h declares."""
    import re
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rpca_[a-z_A-Z0-9]+)\s*\(", text)))
