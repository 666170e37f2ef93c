"""ctypes binding of liblogm.so (include/logm.h).

Argument marshalling only: every step of the computation runs in the HIP library.
PyTorch supplies device memory (tensors, workspace) and the current stream.  If the
library has not been built, every entry point raises ``LibraryNotBuilt``; there is
no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblogm.so")

LOGM_R64 = 0
LOGM_C128 = 1

STATUS = {
    0: "LOGM_OK",
    1: "LOGM_EINVAL",
    2: "LOGM_ENOTSUP",
    3: "LOGM_EWORKSPACE",
    4: "LOGM_ENONFINITE",
    5: "LOGM_ESINGULAR",
    6: "LOGM_ENOCONV",
    7: "LOGM_EHIP",
}

# Every symbol include/logm.h declares.
EXPORTS = (
    "logm_default_opts",
    "logm_strerror",
    "logm_workspace_size",
    "logm_forward",
    "logm_forward_noalloc",
    "logm_backward_workspace_size",
    "logm_backward",
    "logm_forward_taped",
    "logm_backward_taped",
    "logm_batched_workspace_size",
    "logm_batched_f64",
    "logm_batched_autotune",
    "logm_batched_set_split",
    "logm_batched_c128_workspace_size",
    "logm_batched_c128",
    "logm_gemm_f64",
    "logm_inverse_f64",
    "logm_sqrt_f64",
    "logm_poly_f64",
    "logm_normest_f64",
    "logm_balance_f64",
    "logm_autotune",
    "logm_scheme",
    "logm_profile_enable",
    "logm_profile_reset",
    "logm_profile_get",
    "logm_version",
)


class LibraryNotBuilt(RuntimeError):
    pass


class LogmError(RuntimeError):
    def __init__(self, code: int, where: str, detail: int = 0):
        self.code = code
        self.status = STATUS.get(code, str(code))
        msg = f"{where}: {self.status}"
        if detail:
            msg += f" (hipError {detail})"
        super().__init__(msg)


class LogmOpts(ctypes.Structure):
    _fields_ = [
        ("k_max", ctypes.c_int32),
        ("max_sqrt", ctypes.c_int32),
        ("db_max_iter", ctypes.c_int32),
        ("theta_source", ctypes.c_int32),
        ("graph_fp32", ctypes.c_int32),
        ("balance", ctypes.c_int32),
        ("pivot_search", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class LogmInfo(ctypes.Structure):
    _fields_ = [
        ("s", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("n_inv", ctypes.c_int32),
        ("n_gemm", ctypes.c_int32),
        ("n_matvec", ctypes.c_int32),
        ("n_est", ctypes.c_int32),
        ("db_iters", ctypes.c_int32 * 64),
        ("flops", ctypes.c_double),
        ("norm1_b", ctypes.c_double),
        ("norm1_b2", ctypes.c_double),
        ("status_detail", ctypes.c_int32),
        ("n_inv_reordered", ctypes.c_int32),
        ("n_order_rejected", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {
            "s": self.s,
            "k": self.k,
            "m": self.m,
            "n_inv": self.n_inv,
            "n_gemm": self.n_gemm,
            "n_matvec": self.n_matvec,
            "n_est": self.n_est,
            "db_iters": [int(self.db_iters[i]) for i in range(self.s)],
            "flops": self.flops,
            "norm1_b": self.norm1_b,
            "norm1_b2": self.norm1_b2,
            "n_inv_reordered": self.n_inv_reordered,
            "n_order_rejected": self.n_order_rejected,
        }


_LIB = None

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f64 = ctypes.c_double
_sz = ctypes.c_size_t


def load_library(path: str = LIB_PATH):
    """Load liblogm.so and declare the C signatures (raises if absent)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise LibraryNotBuilt(
            f"{path} is missing: build the HIP library first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    sig = {
        "logm_default_opts": (None, [ctypes.POINTER(LogmOpts)]),
        "logm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "logm_workspace_size": (ctypes.c_int, [_i32, _i64, ctypes.POINTER(LogmOpts), ctypes.POINTER(_sz)]),
        "logm_forward": (ctypes.c_int, [_i32, _i64, _vp, _i64, _vp, _i64, ctypes.POINTER(LogmOpts),
                                        ctypes.POINTER(LogmInfo), _vp, _sz, _vp]),
        "logm_forward_noalloc": (ctypes.c_int, [_i64, _vp, _i64, _vp, _i64, ctypes.POINTER(LogmOpts),
                                                ctypes.POINTER(LogmInfo), _vp]),
        "logm_backward_workspace_size": (ctypes.c_int, [_i32, _i64, ctypes.POINTER(LogmOpts),
                                                        ctypes.POINTER(_sz)]),
        "logm_backward": (ctypes.c_int, [_i32, _i64, _vp, _i64, _vp, _i64, _vp, _i64, ctypes.POINTER(LogmOpts),
                                         ctypes.POINTER(LogmInfo), _vp, _sz, _vp]),
        "logm_forward_taped": (ctypes.c_int, [_i32, _i64, _vp, _i64, _vp, _i64, ctypes.POINTER(LogmOpts),
                                              ctypes.POINTER(LogmInfo), _vp, _sz, _vp]),
        "logm_backward_taped": (ctypes.c_int, [_i32, _i64, _vp, _i64, _vp, _i64, ctypes.POINTER(LogmOpts),
                                               ctypes.POINTER(LogmInfo), _vp, _sz, _vp]),
        "logm_batched_workspace_size": (ctypes.c_int, [_i32, _i64, _i32, ctypes.POINTER(_sz)]),
        "logm_batched_f64": (ctypes.c_int, [_i32, _i32, _i64, _vp, _vp, _vp, _vp, ctypes.POINTER(LogmOpts),
                                            _vp, _vp, _sz, _vp]),
        "logm_batched_autotune": (ctypes.c_int, [_i32, _i32, _i64, _vp, _vp, _vp, _vp, ctypes.POINTER(LogmOpts),
                                                 _vp, _vp, _sz, _vp, ctypes.POINTER(_i32),
                                                 ctypes.POINTER(_f64)]),
        "logm_batched_set_split": (_i32, [_i32]),
        "logm_batched_c128_workspace_size": (ctypes.c_int, [_i32, _i64, _i32, ctypes.POINTER(_sz)]),
        "logm_batched_c128": (ctypes.c_int, [_i32, _i32, _i64, _vp, _vp, _vp, _vp, ctypes.POINTER(LogmOpts),
                                             _vp, _vp, _sz, _vp]),
        "logm_gemm_f64": (ctypes.c_int, [_i64, _i64, _i64, _f64, _vp, _i64, _vp, _i64, _f64, _vp, _i64, _vp]),
        "logm_inverse_f64": (ctypes.c_int, [_i64, _vp, _i64, _vp, _i64, ctypes.POINTER(_f64), _vp, _sz, _vp]),
        "logm_sqrt_f64": (ctypes.c_int, [_i64, _vp, _i64, _vp, _i64, _i32, ctypes.POINTER(_i32), _vp, _sz, _vp]),
        "logm_poly_f64": (ctypes.c_int, [_i64, _i32, _i32, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp]),
        "logm_normest_f64": (ctypes.c_int, [_i64, _vp, _i64, _vp, _i64, _i32, _i32, ctypes.POINTER(_f64),
                                            ctypes.POINTER(_i32), _vp, _sz, _vp]),
        "logm_balance_f64": (ctypes.c_int, [_i64, _vp, _i64, _vp, _i64, _vp, _vp, ctypes.POINTER(_i32), _vp,
                                            _sz, _vp]),
        "logm_autotune": (ctypes.c_int, [_i64, _vp, _sz, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_f64)]),
        "logm_scheme": (ctypes.c_int, [_i32, _i32, ctypes.POINTER(_f64), ctypes.POINTER(_f64),
                                       ctypes.POINTER(_f64), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                       ctypes.POINTER(_f64)]),
        "logm_profile_enable": (None, [_i32]),
        "logm_profile_reset": (None, []),
        "logm_profile_get": (ctypes.c_int, [ctypes.POINTER(_i64), ctypes.POINTER(_f64),
                                            ctypes.POINTER(_f64), ctypes.POINTER(_f64)]),
        "logm_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def lib():
    return load_library()


def _check(rc: int, where: str, detail: int = 0):
    if rc != 0:
        raise LogmError(rc, where, detail)


# ------------------------------------------------------------ host tables ---
def default_opts() -> LogmOpts:
    o = LogmOpts()
    lib().logm_default_opts(ctypes.byref(o))
    return o


def strerror(code: int) -> str:
    return lib().logm_strerror(code).decode()


def version() -> str:
    return lib().logm_version().decode()


def workspace_size(n: int, opts: LogmOpts | None = None, dtype: int = LOGM_R64) -> int:
    b = _sz(0)
    _check(lib().logm_workspace_size(dtype, n, ctypes.byref(opts) if opts else None, ctypes.byref(b)),
           "logm_workspace_size")
    return b.value


def scheme(k: int, theta_source: int = 0):
    """(h, g, y, m_k, Theta) as the library holds them."""
    h = (_f64 * 64)()
    g = (_f64 * 64)()
    y = (_f64 * 16)()
    nh = _i32(0)
    m = _i32(0)
    th = _f64(0)
    _check(lib().logm_scheme(k, theta_source, h, g, y, ctypes.byref(nh), ctypes.byref(m), ctypes.byref(th)),
           "logm_scheme")
    return list(h[: nh.value]), list(g[: nh.value]), list(y[: k + 2]), m.value, th.value


def profile_enable(on: bool = True):
    lib().logm_profile_enable(1 if on else 0)


def profile_reset():
    lib().logm_profile_reset()


def profile_get() -> dict:
    n = _i64(0)
    ms = _f64(0)
    fl = _f64(0)
    by = _f64(0)
    lib().logm_profile_get(ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by))
    return {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}


# ------------------------------------------------------------ device calls ---
def _torch():
    import torch
    return torch


def _stream_ptr(t):
    torch = _torch()
    return _vp(torch.cuda.current_stream(t.device).cuda_stream)


def _as_matrix(A, name="A", allow_complex: bool = False):
    torch = _torch()
    if not isinstance(A, torch.Tensor) or A.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    ok = (torch.float64, torch.complex128) if allow_complex else (torch.float64,)
    if A.dtype not in ok:
        raise TypeError(f"{name} must be " + (" or ".join(str(t) for t in ok)))
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError(f"{name} must be a square matrix")
    if A.stride(1) != 1:
        A = A.contiguous()
    return A


def _workspace(n: int, device, workspace=None, dtype: int = LOGM_R64):
    torch = _torch()
    need = workspace_size(n, dtype=dtype)
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < need:
            raise ValueError(f"workspace needs {need} bytes")
        return workspace
    return torch.empty(need, dtype=torch.uint8, device=device)


def logm(A, k_max: int = 9, max_sqrt: int = 50, db_max_iter: int = 30, theta_source: int = 0,
         out=None, workspace=None, graph_fp32: bool = False, balance: bool = False,
         pivot_search: bool = False):
    """L = log(A) on the GPU (Algorithm 1), A float64 or complex128.  Returns (L, info
    dict).  graph_fp32 runs the graph products on the fp32 matrix cores (see
    logm_opts); complex A runs on its 2n x 2n real representation; pivot_search
    searches pivots in every inversion instead of trying the previous row order."""
    torch = _torch()
    A = _as_matrix(A, allow_complex=True)
    n = A.shape[0]
    dt = LOGM_C128 if A.dtype == torch.complex128 else LOGM_R64
    L = out if out is not None else torch.empty((n, n), dtype=A.dtype, device=A.device)
    o = default_opts()
    o.k_max, o.max_sqrt, o.db_max_iter, o.theta_source = k_max, max_sqrt, db_max_iter, theta_source
    o.graph_fp32 = 1 if graph_fp32 else 0
    o.balance = 1 if balance else 0
    o.pivot_search = 1 if pivot_search else 0
    ws = _workspace(n, A.device, workspace, dt)
    info = LogmInfo()
    rc = lib().logm_forward(dt, n, _vp(A.data_ptr()), A.stride(0), _vp(L.data_ptr()), L.stride(0),
                            ctypes.byref(o), ctypes.byref(info), _vp(ws.data_ptr()), ws.numel(),
                            _stream_ptr(A))
    _check(rc, "logm_forward", info.status_detail)
    return L, info.as_dict()


NOALLOC_MAX_N = 256


def logm_noalloc(A, k_max: int = 9, max_sqrt: int = 50, db_max_iter: int = 30, theta_source: int = 0,
                 out=None, pivot_search: bool = False):
    """L = log(A) through logm_forward_noalloc: real A, n <= 256, no workspace (the
    library's fixed device array) and no device allocation.  Returns (L, info dict)."""
    torch = _torch()
    A = _as_matrix(A)
    n = A.shape[0]
    L = out if out is not None else torch.empty((n, n), dtype=A.dtype, device=A.device)
    o = default_opts()
    o.k_max, o.max_sqrt, o.db_max_iter, o.theta_source = k_max, max_sqrt, db_max_iter, theta_source
    o.pivot_search = 1 if pivot_search else 0
    info = LogmInfo()
    rc = lib().logm_forward_noalloc(n, _vp(A.data_ptr()), A.stride(0), _vp(L.data_ptr()), L.stride(0),
                                    ctypes.byref(o), ctypes.byref(info), _stream_ptr(A))
    _check(rc, "logm_forward_noalloc", info.status_detail)
    return L, info.as_dict()


def backward_workspace_size(n: int, opts: LogmOpts | None = None, tape_mats: int = 0,
                            dtype: int = LOGM_R64) -> int:
    """Workspace bytes of the reverse mode; ``tape_mats`` extra matrices lengthen the
    ring of taped inverses (see logm_backward)."""
    b = _sz(0)
    _check(lib().logm_backward_workspace_size(dtype, n, ctypes.byref(opts) if opts else None,
                                              ctypes.byref(b)), "logm_backward_workspace_size")
    return b.value + tape_mats * _bwd_mat_bytes(2 * n if dtype == LOGM_C128 else n)


def _bwd_mat_bytes(n: int) -> int:
    n_pad = (n + 63) // 64 * 64
    return (n_pad * n_pad * 8 + 255) // 256 * 256


def logm_backward(A, G, k_max: int = 9, max_sqrt: int = 50, db_max_iter: int = 30,
                  theta_source: int = 0, out=None, workspace=None, tape_mats: int | None = None):
    """gradA = d<G, log A>/dA on the GPU (reverse mode of Algorithm 1).  Returns
    (gradA, info dict of the forward pass run inside the call).  Complex A, G give
    gradA = L_log(A^H, G).

    ``tape_mats`` extra matrices lengthen the ring of taped inverses (default: room
    for 100 inverses in all), so that roots whose inverses are still in the ring are
    not replayed."""
    torch = _torch()
    A = _as_matrix(A, allow_complex=True)
    G = _as_matrix(G, "G", allow_complex=True)
    n = A.shape[0]
    if G.shape != A.shape or G.device != A.device or G.dtype != A.dtype:
        raise ValueError("G must match A in shape, dtype and device")
    dt = LOGM_C128 if A.dtype == torch.complex128 else LOGM_R64
    gA = out if out is not None else torch.empty((n, n), dtype=A.dtype, device=A.device)
    o = default_opts()
    o.k_max, o.max_sqrt, o.db_max_iter, o.theta_source = k_max, max_sqrt, db_max_iter, theta_source
    if tape_mats is None:
        tape_mats = max(0, 100 - 2 * db_max_iter)
    need = backward_workspace_size(n, o, tape_mats, dt)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=A.device)
    elif workspace.numel() * workspace.element_size() < backward_workspace_size(n, o, 0, dt):
        raise ValueError("workspace smaller than logm_backward_workspace_size")
    info = LogmInfo()
    rc = lib().logm_backward(dt, n, _vp(A.data_ptr()), A.stride(0), _vp(G.data_ptr()), G.stride(0),
                             _vp(gA.data_ptr()), gA.stride(0), ctypes.byref(o), ctypes.byref(info),
                             _vp(workspace.data_ptr()), workspace.numel(), _stream_ptr(A))
    _check(rc, "logm_backward", info.status_detail)
    return gA, info.as_dict()


class Tape:
    """Workspace of a taped forward pass (logm_forward_taped), consumed by
    logm_backward_taped; holds the root checkpoints and taped inverses on the GPU.
    complex=True tapes a complex128 pass (run on the 2n x 2n real representation)."""

    def __init__(self, n: int, device, tape_mats: int | None = None, k_max: int = 9, max_sqrt: int = 50,
                 db_max_iter: int = 30, theta_source: int = 0, complex: bool = False):
        torch = _torch()
        self.n = n
        self.dt = LOGM_C128 if complex else LOGM_R64
        self.dtype = torch.complex128 if complex else torch.float64
        self.opts = default_opts()
        o = self.opts
        o.k_max, o.max_sqrt, o.db_max_iter, o.theta_source = k_max, max_sqrt, db_max_iter, theta_source
        if tape_mats is None:
            tape_mats = max(0, 100 - 2 * db_max_iter)
        self.ws = torch.empty(backward_workspace_size(n, o, tape_mats, self.dt), dtype=torch.uint8,
                              device=device)


def logm_forward_taped(A, tape: Tape, out=None):
    """L = log(A), leaving the reverse-mode tape in ``tape``.  Returns (L, info)."""
    torch = _torch()
    A = _as_matrix(A, allow_complex=True)
    n = A.shape[0]
    if n != tape.n or A.dtype != tape.dtype:
        raise ValueError("tape built for another size or dtype")
    L = out if out is not None else torch.empty((n, n), dtype=A.dtype, device=A.device)
    info = LogmInfo()
    rc = lib().logm_forward_taped(tape.dt, n, _vp(A.data_ptr()), A.stride(0), _vp(L.data_ptr()), L.stride(0),
                                  ctypes.byref(tape.opts), ctypes.byref(info), _vp(tape.ws.data_ptr()),
                                  tape.ws.numel(), _stream_ptr(A))
    _check(rc, "logm_forward_taped", info.status_detail)
    return L, info.as_dict()


def logm_backward_taped(G, tape: Tape, out=None):
    """gradA = d<G, log A>/dA from the tape of the last logm_forward_taped."""
    torch = _torch()
    G = _as_matrix(G, "G", allow_complex=True)
    n = G.shape[0]
    if n != tape.n or G.dtype != tape.dtype:
        raise ValueError("tape built for another size or dtype")
    gA = out if out is not None else torch.empty((n, n), dtype=G.dtype, device=G.device)
    info = LogmInfo()
    rc = lib().logm_backward_taped(tape.dt, n, _vp(G.data_ptr()), G.stride(0), _vp(gA.data_ptr()), gA.stride(0),
                                   ctypes.byref(tape.opts), ctypes.byref(info), _vp(tape.ws.data_ptr()),
                                   tape.ws.numel(), _stream_ptr(G))
    _check(rc, "logm_backward_taped", info.status_detail)
    return gA, info.as_dict()


def _autograd_function():
    torch = _torch()

    class LogmFunction(torch.autograd.Function):
        """log(A) with the hand-written reverse mode of the HIP library: the forward
        tapes what the backward needs (logm_forward_taped / logm_backward_taped)."""

        @staticmethod
        def forward(ctx, A):
            tape = Tape(A.shape[0], A.device, complex=A.dtype == torch.complex128)
            L, _ = logm_forward_taped(A, tape)
            ctx.tape = tape
            return L

        @staticmethod
        def backward(ctx, gL):
            gA, _ = logm_backward_taped(gL.contiguous(), ctx.tape)
            ctx.tape = None
            return gA

    return LogmFunction


_LOGM_FN = None


def logm_autograd(A):
    """log(A) as a differentiable torch op (the forward keeps its tape until backward)."""
    global _LOGM_FN
    if _LOGM_FN is None:
        _LOGM_FN = _autograd_function()
    return _LOGM_FN.apply(A)


class BatchPlan:
    """Device-side description of a batch of small matrices (packed row-major);
    complex=True plans a complex128 batch (n_i <= 64, through real representations)."""

    def __init__(self, dims, device, complex: bool = False):
        torch = _torch()
        self.dims_host = [int(d) for d in dims]
        if not self.dims_host:
            raise ValueError("empty batch")
        offs, tot = [], 0
        for d in self.dims_host:
            offs.append(tot)
            tot += d * d
        self.offsets_host = offs
        self.total = tot
        self.n_max = max(self.dims_host)
        self.device = device
        self.dims = torch.tensor(self.dims_host, dtype=torch.int32, device=device)
        self.offsets = torch.tensor(offs, dtype=torch.int64, device=device)
        self.complex = bool(complex)
        self.dtype = torch.complex128 if self.complex else torch.float64
        by = _sz()
        if self.complex:
            _check(lib().logm_batched_c128_workspace_size(len(dims), tot, self.n_max, ctypes.byref(by)),
                   "logm_batched_c128_workspace_size")
        else:
            _check(lib().logm_batched_workspace_size(len(dims), tot, self.n_max, ctypes.byref(by)),
                   "logm_batched_workspace_size")
        self.ws = torch.empty(by.value, dtype=torch.uint8, device=device)
        self.status = torch.empty(4 * len(dims), dtype=torch.int32, device=device)

    def pack(self, mats):
        torch = _torch()
        flat = torch.empty(self.total, dtype=self.dtype, device=self.device)
        for M, o, d in zip(mats, self.offsets_host, self.dims_host):
            flat[o:o + d * d] = torch.as_tensor(M, dtype=self.dtype).reshape(-1).to(self.device)
        return flat

    def unpack(self, flat):
        return [flat[o:o + d * d].reshape(d, d) for o, d in zip(self.offsets_host, self.dims_host)]


def logm_batched(A_flat, plan: "BatchPlan", L_flat=None, k_max: int = 9, max_sqrt: int = 50,
                 db_max_iter: int = 30, theta_source: int = 0):
    """L_i = log(A_i) for a packed batch (one persistent launch, decisions on the
    device).  Returns (L_flat, status tensor [batch, 4]: code, s, k, DB iterations);
    does not synchronise.  A complex128 batch needs a plan made with complex=True."""
    torch = _torch()
    if A_flat.dtype != plan.dtype or A_flat.numel() != plan.total or not A_flat.is_contiguous():
        raise ValueError("A_flat must be a contiguous packed batch of the plan's dtype and size")
    if L_flat is None:
        L_flat = torch.empty_like(A_flat)
    if L_flat.dtype != plan.dtype or L_flat.numel() != plan.total or not L_flat.is_contiguous():
        raise ValueError("L_flat must be a contiguous packed batch of the plan's dtype and size")
    o = default_opts()
    o.k_max, o.max_sqrt, o.db_max_iter, o.theta_source = k_max, max_sqrt, db_max_iter, theta_source
    fn, name = ((lib().logm_batched_c128, "logm_batched_c128") if plan.complex
                else (lib().logm_batched_f64, "logm_batched_f64"))
    rc = fn(len(plan.dims_host), plan.n_max, plan.total, _vp(plan.dims.data_ptr()),
            _vp(plan.offsets.data_ptr()), _vp(A_flat.data_ptr()), _vp(L_flat.data_ptr()),
            ctypes.byref(o), _vp(plan.status.data_ptr()), _vp(plan.ws.data_ptr()),
            plan.ws.numel(), _stream_ptr(A_flat))
    _check(rc, name)
    return L_flat, plan.status.view(-1, 4)


def autotune_batched(A_flat, plan: "BatchPlan", k_max: int = 9, max_sqrt: int = 50,
                     db_max_iter: int = 30, theta_source: int = 0):
    """Choose the batched class boundary by timing the caller's real batch (see
    logm_batched_autotune); returns (split, ms of the best run).  The choice holds for
    later batched calls on the device."""
    torch = _torch()
    if plan.complex or A_flat.dtype != torch.float64 or A_flat.numel() != plan.total:
        raise ValueError("autotune_batched takes a real packed batch of the plan's size")
    L_flat = torch.empty_like(A_flat)
    o = default_opts()
    o.k_max, o.max_sqrt, o.db_max_iter, o.theta_source = k_max, max_sqrt, db_max_iter, theta_source
    best = _i32(0)
    ms = _f64(0)
    rc = lib().logm_batched_autotune(len(plan.dims_host), plan.n_max, plan.total, _vp(plan.dims.data_ptr()),
                                     _vp(plan.offsets.data_ptr()), _vp(A_flat.data_ptr()), _vp(L_flat.data_ptr()),
                                     ctypes.byref(o), _vp(plan.status.data_ptr()), _vp(plan.ws.data_ptr()),
                                     plan.ws.numel(), _stream_ptr(A_flat), ctypes.byref(best), ctypes.byref(ms))
    _check(rc, "logm_batched_autotune")
    return best.value, ms.value


def set_batched_split(split: int) -> int:
    """Set the batched class boundary (1..64); returns the previous one."""
    old = lib().logm_batched_set_split(int(split))
    if old < 0:
        raise ValueError("split must be in 1..64")
    return old


def gemm(A, B, C=None, alpha: float = 1.0, beta: float = 0.0):
    torch = _torch()
    if A.stride(1) != 1:
        A = A.contiguous()
    if B.stride(1) != 1:
        B = B.contiguous()
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    if C is None:
        C = torch.zeros((m, n), dtype=torch.float64, device=A.device)
    rc = lib().logm_gemm_f64(m, n, k, alpha, _vp(A.data_ptr()), A.stride(0), _vp(B.data_ptr()), B.stride(0),
                             beta, _vp(C.data_ptr()), C.stride(0), _stream_ptr(A))
    _check(rc, "logm_gemm_f64")
    return C


def inverse(A, workspace=None):
    """(A^{-1}, log|det A|) by Gauss-Jordan with tournament pivoting."""
    torch = _torch()
    A = _as_matrix(A)
    n = A.shape[0]
    Ai = torch.empty_like(A)
    ld = _f64(0)
    ws = _workspace(n, A.device, workspace)
    rc = lib().logm_inverse_f64(n, _vp(A.data_ptr()), A.stride(0), _vp(Ai.data_ptr()), Ai.stride(0),
                                ctypes.byref(ld), _vp(ws.data_ptr()), ws.numel(), _stream_ptr(A))
    _check(rc, "logm_inverse_f64")
    return Ai, ld.value


def balance(A, workspace=None, permute: bool = True):
    """(T^{-1} P^T A P T, diag(T), sweeps, perm): the balancing of steps 1 and 14 on the
    GPU, perm[i] the index of A at position i (None without the permutation step)."""
    torch = _torch()
    A = _as_matrix(A)
    n = A.shape[0]
    B = torch.empty_like(A)
    d = torch.empty(n, dtype=torch.float64, device=A.device)
    perm = torch.empty(n, dtype=torch.int32, device=A.device) if permute else None
    sw = _i32(0)
    ws = _workspace(n, A.device, workspace)
    rc = lib().logm_balance_f64(n, _vp(A.data_ptr()), A.stride(0), _vp(B.data_ptr()), B.stride(0),
                                _vp(d.data_ptr()), _vp(perm.data_ptr()) if permute else None,
                                ctypes.byref(sw), _vp(ws.data_ptr()), ws.numel(), _stream_ptr(A))
    _check(rc, "logm_balance_f64")
    return B, d, sw.value, perm


def autotune(n: int, device=None, workspace=None):
    """Choose the trailing-update workgroup caps for size n by timing (see
    logm_autotune); returns ((cap with the pivot search, cap in a given row order),
    (ms per inversion pair in each mode))."""
    torch = _torch()
    device = device or torch.device("cuda:0")
    ws = workspace if workspace is not None else torch.empty(workspace_size(n), dtype=torch.uint8, device=device)
    best = (_i32 * 2)()
    ms = (_f64 * 2)()
    rc = lib().logm_autotune(n, _vp(ws.data_ptr()), ws.numel(),
                             _vp(torch.cuda.current_stream(device).cuda_stream), best, ms)
    _check(rc, "logm_autotune")
    return (best[0], best[1]), (ms[0], ms[1])


def sqrtm(A, db_max_iter: int = 30, workspace=None):
    """(A^{1/2}, iterations) by the scaled Denman-Beavers iteration."""
    torch = _torch()
    A = _as_matrix(A)
    n = A.shape[0]
    X = torch.empty_like(A)
    it = _i32(0)
    ws = _workspace(n, A.device, workspace)
    rc = lib().logm_sqrt_f64(n, _vp(A.data_ptr()), A.stride(0), _vp(X.data_ptr()), X.stride(0), db_max_iter,
                             ctypes.byref(it), _vp(ws.data_ptr()), ws.numel(), _stream_ptr(A))
    _check(rc, "logm_sqrt_f64")
    return X, it.value


def poly(B, B2, k: int, s: int = 0, workspace=None):
    """-2^s S_k(-B) with P_3 = B2."""
    torch = _torch()
    B = _as_matrix(B, "B")
    B2 = _as_matrix(B2, "B2")
    n = B.shape[0]
    L = torch.empty_like(B)
    ws = _workspace(n, B.device, workspace)
    rc = lib().logm_poly_f64(n, k, s, _vp(B.data_ptr()), B.stride(0), _vp(B2.data_ptr()), B2.stride(0),
                             _vp(L.data_ptr()), L.stride(0), _vp(ws.data_ptr()), ws.numel(), _stream_ptr(B))
    _check(rc, "logm_poly_f64")
    return L


def normest(B2, B, q: int, r: int, workspace=None):
    """(estimate of ||B2^q B^r||_1, matrix-vector products used)."""
    B = _as_matrix(B, "B")
    B2 = _as_matrix(B2, "B2")
    n = B.shape[0]
    est = _f64(0)
    nmv = _i32(0)
    ws = _workspace(n, B.device, workspace)
    rc = lib().logm_normest_f64(n, _vp(B2.data_ptr()), B2.stride(0), _vp(B.data_ptr()), B.stride(0), q, r,
                                ctypes.byref(est), ctypes.byref(nmv), _vp(ws.data_ptr()), ws.numel(),
                                _stream_ptr(B))
    _check(rc, "logm_normest_f64")
    return est.value, nmv.value
