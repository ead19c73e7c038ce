"""ctypes front end of the FP64 oracle, plus the plain definitions used to check
results at sizes where the full oracle run is too slow.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Matrices are handled column-major (numpy order='F'), as the C oracle expects.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i32p = ctypes.POINTER(ctypes.c_int32)


def load_library():
    """Load liboracle.so (built by oracle/build.py); build it if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    common = [_dp, ctypes.c_int64, ctypes.c_int64, _dp, ctypes.c_int64, _u8p, _dp, _dp, _dp, _i32p]
    lib.dpp_oracle_lu.argtypes = common
    lib.dpp_oracle_lu.restype = ctypes.c_int
    lib.dpp_oracle_ldlh.argtypes = common + [_dp]
    lib.dpp_oracle_ldlh.restype = ctypes.c_int
    lib.dpp_oracle_zlu.argtypes = common
    lib.dpp_oracle_zlu.restype = ctypes.c_int
    lib.dpp_oracle_zldlh.argtypes = common + [_dp]
    lib.dpp_oracle_zldlh.restype = ctypes.c_int
    lib.dpp_oracle_threads.argtypes = []
    lib.dpp_oracle_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def omp_threads() -> int:
    return int(load_library().dpp_oracle_threads())


def _run(fn_name, K, u, npiv, inplace):
    lib = load_library()
    K = np.asarray(K)
    n = K.shape[0]
    assert K.shape == (n, n)
    cplx = fn_name.startswith("dpp_oracle_z")
    dt = np.complex128 if cplx else np.float64
    if inplace:
        assert K.dtype == dt and K.flags.f_contiguous
        A = K
    else:
        A = np.array(K, dtype=dt, order="F", copy=True)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.shape[0] >= n
    mask = np.zeros(n, dtype=np.uint8)
    piv = np.zeros(n, dtype=np.float64)
    pre = np.zeros(n, dtype=np.float64)
    ll = ctypes.c_double(0.0)
    info = ctypes.c_int32(0)
    args = [A.ctypes.data_as(_dp), n, max(n, 1), u.ctypes.data_as(_dp),
            int(npiv or 0), mask.ctypes.data_as(_u8p), piv.ctypes.data_as(_dp),
            pre.ctypes.data_as(_dp), ctypes.byref(ll), ctypes.byref(info)]
    if fn_name in ("dpp_oracle_ldlh", "dpp_oracle_zldlh"):
        row = np.zeros(max(n, 1), dtype=dt)
        args.append(row.ctypes.data_as(_dp))
    rc = getattr(lib, fn_name)(*args)
    if rc != 0:
        raise ValueError(f"{fn_name} rejected its arguments (rc={rc})")
    return {"mask": mask, "pivots": piv, "predec": pre, "loglik": ll.value,
            "info": info.value, "A": A}


def ldlh(K, u, npiv=None, inplace=False):
    """Hermitian sampler (lower triangle of K). Returns mask, pivots (d' after
    the decision), predec (d before it), loglik, info and the factored A."""
    return _run("dpp_oracle_ldlh", K, u, npiv, inplace)


def lu(K, u, npiv=None, inplace=False):
    """Non-Hermitian sampler (all of K); same outputs as ldlh."""
    return _run("dpp_oracle_lu", K, u, npiv, inplace)


def zldlh(K, u, npiv=None, inplace=False):
    """Complex Hermitian sampler (lower triangle of a complex128 K). Decisions,
    pivots, predec and loglik use the real parts of the diagonal entries (a
    conditional probability is real); A holds the complex L and the real D."""
    return _run("dpp_oracle_zldlh", K, u, npiv, inplace)


def zlu(K, u, npiv=None, inplace=False):
    """Complex non-Hermitian sampler (all of a complex128 K); outputs as zldlh,
    A holds the complex L and U (U's diagonal: the complex pivots)."""
    return _run("dpp_oracle_zlu", K, u, npiv, inplace)


def conditional_pivot(K, mask_prefix, j):
    """d_j given the decisions on indices 0..j-1, straight from Props. 3-5:
    the marginal kernel of the DPP on the remaining indices conditioned on the
    first j decisions is the Schur complement of K_A - 1_{A excluded} in K,
    A = [0, j), so
        d_j = K_jj - K_{j,A} (K_A - diag(1 - mask_A))^{-1} K_{A,j}.
    Uses a library solve; cost O(j^3)."""
    K = np.asarray(K)
    if not np.iscomplexobj(K):
        K = np.asarray(K, dtype=np.float64)
    if j == 0:
        return float(np.real(K[0, 0]))
    KA = K[:j, :j] - np.diag(1.0 - np.asarray(mask_prefix[:j], dtype=np.float64))
    x = np.linalg.solve(KA, K[:j, j])
    # a conditional probability is real; for complex K the imaginary part is rounding
    return float(np.real(K[j, j] - K[j, :j] @ x))


def conditional_kernel(K, mask_prefix):
    """Marginal kernel of the indices m.. given the decisions mask_prefix on
    0..m-1 (Props. 3-5): the Schur complement of K_A - 1_{A excluded} in K,
    A = [0, m),
        K_BB - K_BA (K_A - diag(1 - mask_A))^{-1} K_AB,   B = [m, n).
    Uses a library solve; cost O(n^3)."""
    K = np.asarray(K, dtype=np.float64)
    m = len(mask_prefix)
    if m == 0:
        return K.copy()
    KA = K[:m, :m] - np.diag(1.0 - np.asarray(mask_prefix, dtype=np.float64))
    return K[m:, m:] - K[m:, :m] @ np.linalg.solve(KA, K[:m, m:])


def lensemble_marginal(L):
    """Marginal kernel of the L-ensemble with kernel L: K = I - (L + I)^{-1}
    (equivalently L (L + I)^{-1}), by a library inverse."""
    L = np.asarray(L, dtype=np.float64)
    return np.eye(L.shape[0]) - np.linalg.inv(L + np.eye(L.shape[0]))


def reconstruct_ldlh(A):
    """L D L^H from a factored lower triangle (strict lower = L, diagonal = D;
    real or complex, D real)."""
    A = np.asarray(A)
    if not np.iscomplexobj(A):
        A = np.asarray(A, dtype=np.float64)
    L = np.tril(A, -1) + np.eye(A.shape[0])
    return (L * np.real(np.diag(A))) @ L.conj().T


def reconstruct_lu(A):
    """L U from an in-place unpivoted LU (strict lower = L, upper = U; real or
    complex)."""
    A = np.asarray(A)
    if not np.iscomplexobj(A):
        A = np.asarray(A, dtype=np.float64)
    L = np.tril(A, -1) + np.eye(A.shape[0])
    return L @ np.triu(A)
