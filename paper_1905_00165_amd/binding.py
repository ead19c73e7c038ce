"""Thin ctypes binding of libdpp.so (include/dpp.h). Argument marshalling only:
every step of the sampler runs in the library's HIP kernels.

Functions carry the C names. Matrices are torch CUDA tensors in column-major
layout (stride(0) == 1, stride(1) == lda >= n); `colmajor()` makes one.
Outputs are torch tensors allocated here when not given. Calls are issued on
torch's current stream of the tensor's device and are asynchronous.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpp.so")

DPP_F64, DPP_F32, DPP_C128 = 0, 1, 2
DPP_PREC_FP64, DPP_PREC_SPLIT_BF16, DPP_PREC_SPLIT_BF16X6, DPP_PREC_SPLIT_FP16 = 0, 1, 2, 3
DPP_OK = 0
DPP_NOALLOC_SCRATCH_BYTES = 64 << 20   # include/dpp.h
_STATUS = {0: "DPP_OK", 1: "DPP_ERR_INVALID_ARG", 2: "DPP_ERR_WORKSPACE", 3: "DPP_ERR_HIP",
           4: "DPP_ERR_UNSUPPORTED"}

_vp, _i64 = ctypes.c_void_p, ctypes.c_int64


class DppError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_STATUS.get(status, status)} ({dpp_status_string(status)})")


class dpp_problem(ctypes.Structure):
    _fields_ = [("A", _vp), ("n", _i64), ("lda", _i64), ("u", _vp), ("mask", _vp),
                ("pivots", _vp), ("loglik", _vp), ("info", _vp), ("K", _vp), ("ldk", _i64),
                ("npiv", _i64), ("stats", _vp)]


class dpp_lensemble(ctypes.Structure):
    _fields_ = [("L", _vp), ("n", _i64), ("ldl", _i64), ("K", _vp), ("ldk", _i64),
                ("logdet", _vp), ("info", _vp)]


class dpp_kernel_stats(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", _i64), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libdpp.so. Fails loudly when it has not been built: there is no
    other implementation to fall back to."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(or python -m paper_1905_00165_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    single = [_vp, ctypes.c_int, _i64, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp,
              ctypes.c_size_t, _vp]
    for name in ("dpp_sample_ldlh", "dpp_sample_lu"):
        f = getattr(L, name)
        f.argtypes, f.restype = single, ctypes.c_int
    for name in ("dpp_sample_ldlh_batched", "dpp_sample_lu_batched"):
        f = getattr(L, name)
        f.argtypes = [ctypes.POINTER(dpp_problem), _i64, ctypes.c_int, ctypes.c_int, _vp,
                      ctypes.c_size_t, _vp]
        f.restype = ctypes.c_int
    L.dpp_sample_ldlh_batched_noalloc.argtypes = [ctypes.POINTER(dpp_problem), _i64, ctypes.c_int,
                                                  ctypes.c_int, _vp]
    L.dpp_sample_ldlh_batched_noalloc.restype = ctypes.c_int
    L.dpp_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, _i64, ctypes.c_int]
    L.dpp_workspace_size.restype = ctypes.c_size_t
    L.dpp_workspace_size_batched.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_i64),
                                             _i64, ctypes.c_int]
    L.dpp_workspace_size_batched.restype = ctypes.c_size_t
    L.dpp_lensemble_to_marginal_batched.argtypes = [ctypes.POINTER(dpp_lensemble), _i64,
                                                    ctypes.c_int, _vp, ctypes.c_size_t, _vp]
    L.dpp_lensemble_to_marginal_batched.restype = ctypes.c_int
    L.dpp_lensemble_workspace_size.argtypes = [ctypes.POINTER(_i64), _i64]
    L.dpp_lensemble_workspace_size.restype = ctypes.c_size_t
    L.dpp_copy_lower.argtypes = [_vp, _vp, ctypes.c_int, _i64, _i64, _i64, _vp]
    L.dpp_copy_lower.restype = ctypes.c_int
    L.dpp_status_string.argtypes = [ctypes.c_int]
    L.dpp_status_string.restype = ctypes.c_char_p
    L.dpp_profile_begin.argtypes = []
    L.dpp_profile_begin.restype = ctypes.c_int
    L.dpp_profile_end.argtypes = [ctypes.POINTER(dpp_kernel_stats), ctypes.c_int]
    L.dpp_profile_end.restype = ctypes.c_int
    _lib = L
    return L


def dpp_status_string(status: int) -> str:
    return lib().dpp_status_string(int(status)).decode()


def dpp_copy_lower(dst, src):
    """Copy the lower triangle (with the diagonal) of src into dst: both
    column-major n x n device tensors of one dtype (a working copy for
    dpp_sample_ldlh). Asynchronous on the current stream."""
    n, ldd = _check_matrix(dst)
    m, lds = _check_matrix(src)
    if m != n or _dtype_code(src) != _dtype_code(dst):
        raise ValueError("dst and src must have the same size and dtype")
    st = lib().dpp_copy_lower(dst.data_ptr(), src.data_ptr(), _dtype_code(dst), n, ldd, lds,
                              _stream_handle(dst.device))
    if st != DPP_OK:
        raise DppError(st, "dpp_copy_lower")


def dpp_workspace_size(hermitian: bool, dtype: int, n: int, prec: int) -> int:
    return int(lib().dpp_workspace_size(int(bool(hermitian)), int(dtype), int(n), int(prec)))


def dpp_workspace_size_batched(hermitian: bool, dtype: int, ns, prec: int) -> int:
    arr = (_i64 * len(ns))(*[int(x) for x in ns])
    return int(lib().dpp_workspace_size_batched(int(bool(hermitian)), int(dtype), arr, len(ns),
                                                int(prec)))


def dpp_profile_begin() -> None:
    """Start recording the library's launches (hipEvents around each)."""
    lib().dpp_profile_begin()


def dpp_profile_end() -> dict:
    """Stop recording; {kernel: {launches, ms, flops, bytes}} of what ran."""
    buf = (dpp_kernel_stats * 16)()
    k = lib().dpp_profile_end(buf, 16)
    if k < 0:
        raise DppError(3, "dpp_profile_end")
    return {buf[i].name.decode(): {"launches": buf[i].launches, "ms": buf[i].ms,
                                   "flops": buf[i].flops, "bytes": buf[i].bytes}
            for i in range(k)}


# ----------------------------------------------------------------- torch glue

def _torch():
    import torch
    return torch


def colmajor(K, device=None, dtype=None):
    """A column-major (stride(0) == 1) copy of matrix K on `device`."""
    torch = _torch()
    t = torch.as_tensor(K)
    if dtype is not None:
        t = t.to(dtype)
    if device is not None:
        t = t.to(device)
    return t.t().contiguous().t()


def _dtype_code(A) -> int:
    torch = _torch()
    if A.dtype == torch.float64:
        return DPP_F64
    if A.dtype == torch.float32:
        return DPP_F32
    if A.dtype == torch.complex128:
        return DPP_C128
    raise TypeError(f"A must be float64, float32 or complex128, got {A.dtype}")


def _check_matrix(A):
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square 2-D tensor")
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    n = A.shape[0]
    if n > 1 and A.stride(0) != 1:
        raise ValueError("A must be column-major (stride(0) == 1); use colmajor()")
    lda = A.stride(1) if n > 1 else max(1, A.stride(1))
    return n, lda


# Output buffers of one problem: (dtype name, entries needed for n indices).
_OUTPUTS = {"mask": ("uint8", lambda n: n), "pivots": ("float64", lambda n: n),
            "loglik": ("float64", lambda n: 1), "info": ("int32", lambda n: 1),
            "stats": ("float64", lambda n: 3)}


def check_outputs(o, n, device):
    """Every supplied output buffer must live on `device`, with the dtype and at
    least the entries the library writes (a host tensor here would hand the
    kernels a host pointer). Raises ValueError otherwise."""
    torch = _torch()
    for key, t in o.items():
        if key not in _OUTPUTS:
            raise ValueError(f"unknown output {key!r}")
        dt, need = _OUTPUTS[key]
        if t.device != device:
            raise ValueError(f"output {key!r} is on {t.device}, the problem on {device}")
        if t.dtype != getattr(torch, dt):
            raise ValueError(f"output {key!r} must be {dt}, got {t.dtype}")
        if t.numel() < need(n) or not t.is_contiguous():
            raise ValueError(f"output {key!r} must be contiguous with >= {need(n)} entries")


def check_stream(u, n, device):
    """A uniform stream: contiguous float64 on `device` with >= n entries."""
    torch = _torch()
    if u.dtype != torch.float64 or u.device != device or u.numel() < n or not u.is_contiguous():
        raise ValueError("u must be a contiguous float64 tensor on the problem's device "
                         "with >= n entries")


def _outputs(n, device, out, stats=True):
    """The caller's output buffers (checked), the missing ones allocated. With
    `stats`, a problem whose outputs are all allocated here also gets the
    3-entry decision diagnostics buffer."""
    torch = _torch()
    o = dict(out) if out else {}
    check_outputs(o, n, device)
    o.setdefault("mask", torch.empty(n, dtype=torch.uint8, device=device))
    o.setdefault("pivots", torch.empty(n, dtype=torch.float64, device=device))
    o.setdefault("loglik", torch.empty(1, dtype=torch.float64, device=device))
    o.setdefault("info", torch.empty(1, dtype=torch.int32, device=device))
    if stats and not out:
        o["stats"] = torch.empty(3, dtype=torch.float64, device=device)
    return o


def _workspace(ws, need, device):
    """The caller's workspace (a contiguous uint8 tensor on `device`), or a new one."""
    torch = _torch()
    if ws is None:
        return torch.empty(max(need, 1), dtype=torch.uint8, device=device)
    if ws.device != device or ws.dtype != torch.uint8 or not ws.is_contiguous():
        raise ValueError("ws must be a contiguous uint8 tensor on the problem's device")
    return ws


def _stream_handle(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _single(name, hermitian, A, u, prec, ws, out):
    if out and "stats" in out:
        raise ValueError("the single-problem calls have no stats output; use the batched form")
    n, lda = _check_matrix(A)
    dt = _dtype_code(A)
    check_stream(u, n, A.device)
    ws = _workspace(ws, dpp_workspace_size(hermitian, dt, n, prec), A.device)
    o = _outputs(n, A.device, out, stats=False)
    st = getattr(lib(), name)(A.data_ptr(), dt, n, lda, u.data_ptr(), o["mask"].data_ptr(),
                              o["pivots"].data_ptr(), o["loglik"].data_ptr(),
                              o["info"].data_ptr(), int(prec), ws.data_ptr(), ws.numel(),
                              _stream_handle(A.device))
    if st != DPP_OK:
        raise DppError(st, name)
    return o


def dpp_sample_ldlh(A, u, prec=DPP_PREC_FP64, ws=None, out=None):
    """Sample DPP(K) for symmetric K given in the lower triangle of the
    column-major device tensor A (overwritten by L and D of K - 1_{Y^c}).
    Returns a dict of device tensors: mask, pivots, loglik, info."""
    return _single("dpp_sample_ldlh", True, A, u, prec, ws, out)


def dpp_sample_lu(A, u, prec=DPP_PREC_FP64, ws=None, out=None):
    """Sample DPP(K) for general K (all of A; overwritten by L and U)."""
    return _single("dpp_sample_lu", False, A, u, prec, ws, out)


def _batched(name, hermitian, As, us, prec, ws, outs, Ks=None, npivs=None, noalloc=False):
    if len(As) != len(us) or not As:
        raise ValueError("need matching, non-empty lists of matrices and streams")
    if Ks is not None and len(Ks) != len(As):
        raise ValueError("Ks needs one source matrix (or None) per problem")
    if npivs is not None and len(npivs) != len(As):
        raise ValueError("npivs needs one count (or 0 for all) per problem")
    if outs is not None and len(outs) != len(As):
        raise ValueError("outs needs one dict (or None) per problem")
    dt = _dtype_code(As[0])
    dev = As[0].device
    probs = (dpp_problem * len(As))()
    res = []
    ns = []
    for i, (A, u) in enumerate(zip(As, us)):
        n, lda = _check_matrix(A)
        if _dtype_code(A) != dt or A.device != dev:
            raise ValueError("all matrices of a batch share one dtype and one device")
        check_stream(u, n, dev)
        kp, ldk = None, 0
        K = Ks[i] if Ks is not None else None
        if K is not None:
            nk, ldk = _check_matrix(K)
            if nk != n or _dtype_code(K) != dt or K.device != dev:
                raise ValueError("each K must match its A in size, dtype and device")
            kp = K.data_ptr()
        o = _outputs(n, dev, outs[i] if outs else None)
        st = o.get("stats")
        probs[i] = dpp_problem(A.data_ptr(), n, lda, u.data_ptr(), o["mask"].data_ptr(),
                               o["pivots"].data_ptr(), o["loglik"].data_ptr(),
                               o["info"].data_ptr(), kp, ldk, int(npivs[i]) if npivs else 0,
                               st.data_ptr() if st is not None else None)
        res.append(o)
        ns.append(n)
    if noalloc:
        st = getattr(lib(), name)(probs, len(As), dt, int(prec), _stream_handle(dev))
    else:
        ws = _workspace(ws, dpp_workspace_size_batched(hermitian, dt, ns, prec), dev)
        st = getattr(lib(), name)(probs, len(As), dt, int(prec), ws.data_ptr(), ws.numel(),
                                  _stream_handle(dev))
    if st != DPP_OK:
        raise DppError(st, name)
    return res


def dpp_sample_ldlh_batched(As, us, prec=DPP_PREC_FP64, ws=None, outs=None, Ks=None, npivs=None):
    """Independent symmetric problems in one launch sequence. With Ks (one
    column-major source per problem, or None for in place), each K is read
    only and its A receives the factor (lower triangle). With npivs (0 = all),
    problem i decides only its first npivs[i] indices (a multiple of 64) and
    leaves the conditional marginal kernel of the rest in A's trailing block."""
    return _batched("dpp_sample_ldlh_batched", True, As, us, prec, ws, outs, Ks, npivs)


def dpp_sample_ldlh_batched_noalloc(As, us, prec=DPP_PREC_FP64, outs=None, Ks=None, npivs=None):
    """dpp_sample_ldlh_batched with the library's own per-device scratch as
    the workspace (at most DPP_NOALLOC_SCRATCH_BYTES): the library allocates
    nothing. Outputs not given in `outs` are allocated here, by the caller's
    side, as for the other calls. Calls that may overlap on one device race
    on the shared scratch."""
    return _batched("dpp_sample_ldlh_batched_noalloc", True, As, us, prec, None, outs, Ks, npivs,
                    noalloc=True)


def dpp_sample_lu_batched(As, us, prec=DPP_PREC_FP64, ws=None, outs=None, Ks=None, npivs=None):
    """Independent general problems in one launch sequence; Ks and npivs as for
    dpp_sample_ldlh_batched."""
    return _batched("dpp_sample_lu_batched", False, As, us, prec, ws, outs, Ks, npivs)


def dpp_lensemble_workspace_size(ns) -> int:
    arr = (_i64 * len(ns))(*[int(n) for n in ns])
    return int(lib().dpp_lensemble_workspace_size(arr, len(ns)))


def dpp_lensemble_to_marginal_batched(Ls, Ks=None, ws=None):
    """K_i = I - (L_i + I)^{-1} for symmetric positive semi-definite L_i
    (column-major device tensors, lower triangle read), on the device. Ks: one
    output per problem (None: allocated; it may be L_i itself). Returns a list
    of dicts with K, logdet (ln det(L + I), 1-element FP64 tensor) and info."""
    torch = _torch()
    if not Ls:
        raise ValueError("need a non-empty list of matrices")
    dt = _dtype_code(Ls[0])
    probs = (dpp_lensemble * len(Ls))()
    res = []
    for i, Lm in enumerate(Ls):
        n, ldl = _check_matrix(Lm)
        if _dtype_code(Lm) != dt:
            raise ValueError("all matrices of a batch share one dtype")
        if Lm.device != Ls[0].device:
            raise ValueError("all matrices of a batch live on one device")
        K = Ks[i] if Ks is not None and Ks[i] is not None else torch.empty_like(Lm)
        nk, ldk = _check_matrix(K)
        if nk != n or _dtype_code(K) != dt or K.device != Lm.device:
            raise ValueError("each K must match its L in size, dtype and device")
        o = {"K": K, "logdet": torch.empty(1, dtype=torch.float64, device=Lm.device),
             "info": torch.empty(1, dtype=torch.int32, device=Lm.device)}
        probs[i] = dpp_lensemble(Lm.data_ptr(), n, ldl, K.data_ptr(), ldk,
                                 o["logdet"].data_ptr(), o["info"].data_ptr())
        res.append(o)
    need = dpp_lensemble_workspace_size([Lm.shape[0] for Lm in Ls])
    if need == 0:
        raise ValueError("sizes out of range for the conversion")
    ws = _workspace(ws, need, Ls[0].device)
    st = lib().dpp_lensemble_to_marginal_batched(probs, len(Ls), dt, ws.data_ptr(), ws.numel(),
                                                 _stream_handle(Ls[0].device))
    if st != DPP_OK:
        raise DppError(st, "dpp_lensemble_to_marginal_batched")
    return res
