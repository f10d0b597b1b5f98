"""Plain CPU FP64 oracle for the partition-method solver.

TEST INFRASTRUCTURE ONLY: the product package never imports this module.  It
is used by ``tests/``, by ``__graft_entry__.smoke()`` and by the CPU-baseline
leg of ``bench.py``.

The partition method of Amodio & Brugnano (Sec. 2, eqs. (syst), (parfact))
computes the unique solution ``x = A^{-1} f`` of a structured system up to
rounding.  The oracle therefore computes that plain definition: Gaussian
elimination with row partial pivoting over the whole matrix in its natural
ordering (``oracle.c``), plus the dense Schur complement onto a set of
separator rows, which is what the reduced matrix of eqs. (redmatr) and
(redmatr1) equals whatever local factorization is used.

Array conventions (numpy, not the GPU library's memory layout):
  * a block array has shape ``(count, m, m)`` and ``blk[k, i, j]`` is entry
    ``(i, j)`` of block ``k``;
  * BTRI: ``D[k] = A(k,k)``, ``Lo[j] = A(j+1,j)``, ``Up[j] = A(j,j+1)``;
  * BABD: ``D[k] = A(k,k)``, ``Lo[j] = A(j+1,j)``, ``C = A(0,nb-1)``;
  * right-hand sides / solutions have shape ``(n,)`` or ``(n, nrhs)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


def build() -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, -O2)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    vp = ctypes.c_void_p
    sig = {
        "orc_thomas": (ctypes.c_int, [_i64, vp, vp, vp, _i64, vp, _i64, vp, _i64]),
        "orc_dense_solve": (ctypes.c_int, [_i64, vp, _i64, vp, _i64, vp, _i64]),
        "orc_btri_solve": (ctypes.c_int, [_i64, _i64, vp, vp, vp, _i64, vp, _i64, vp, _i64]),
        "orc_babd_solve": (ctypes.c_int, [_i64, _i64, vp, vp, vp, _i64, vp, _i64, vp, _i64]),
        "orc_btri_solve_trans": (ctypes.c_int, [_i64, _i64, vp, vp, vp, _i64, vp, _i64, vp, _i64]),
        "orc_babd_solve_trans": (ctypes.c_int, [_i64, _i64, vp, vp, vp, _i64, vp, _i64, vp, _i64]),
        "orc_btri_residual": (None, [_i64, _i64, vp, vp, vp, _i64, vp, _i64, vp, _i64, vp, _i64]),
        "orc_babd_residual": (None, [_i64, _i64, vp, vp, vp, _i64, vp, _i64, vp, _i64, vp, _i64]),
        "orc_btri_norminf": (ctypes.c_double, [_i64, _i64, vp, vp, vp]),
        "orc_babd_norminf": (ctypes.c_double, [_i64, _i64, vp, vp, vp]),
        "orc_btri_condest": (ctypes.c_double, [_i64, _i64, vp, vp, vp]),
        "orc_babd_condest": (ctypes.c_double, [_i64, _i64, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _cm_blocks(a) -> np.ndarray:
    """(count, m, m) math-indexed blocks -> contiguous column-major blocks."""
    a = np.asarray(a, dtype=np.float64)
    return np.ascontiguousarray(a.transpose(0, 2, 1))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _rhs(f):
    f = np.asarray(f, dtype=np.float64)
    vec = f.ndim == 1
    f2 = f[:, None] if vec else f
    # (n, nrhs) -> column-major memory = C-contiguous (nrhs, n)
    return vec, np.ascontiguousarray(f2.T), f2.shape[0], f2.shape[1]


def _unrhs(vec, xt):
    x = xt.T
    return np.ascontiguousarray(x[:, 0]) if vec else np.ascontiguousarray(x)


class SingularError(ArithmeticError):
    pass


def _check(info, what):
    if info < 0:
        raise MemoryError(what)
    if info > 0:
        raise SingularError(f"{what}: zero pivot at step {info - 1}")


def thomas(lo, d, up, f):
    """Scalar tridiagonal solve without pivoting (Thomas algorithm)."""
    lib = _load()
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    up = np.ascontiguousarray(up, dtype=np.float64)
    vec, ft, n, k = _rhs(f)
    xt = np.empty_like(ft)
    _check(lib.orc_thomas(n, _ptr(lo), _ptr(d), _ptr(up), k, _ptr(ft), n, _ptr(xt), n), "thomas")
    return _unrhs(vec, xt)


def dense_solve(A, f):
    """Dense LU with row partial pivoting, then the two triangular solves."""
    lib = _load()
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    acm = np.ascontiguousarray(A.T)
    vec, ft, n2, k = _rhs(f)
    assert n2 == n
    xt = np.empty_like(ft)
    _check(lib.orc_dense_solve(n, _ptr(acm), k, _ptr(ft), n, _ptr(xt), n), "dense_solve")
    return _unrhs(vec, xt)


def btri_solve(D, Lo, Up, f):
    """BTRI solve: band LU with partial pivoting over the whole matrix."""
    lib = _load()
    nb, m, _ = np.shape(D)
    Dc, Lc, Uc = _cm_blocks(D), _cm_blocks(Lo if nb > 1 else np.zeros((1, m, m))), \
        _cm_blocks(Up if nb > 1 else np.zeros((1, m, m)))
    vec, ft, n, k = _rhs(f)
    assert n == m * nb
    xt = np.empty_like(ft)
    _check(lib.orc_btri_solve(m, nb, _ptr(Dc), _ptr(Lc), _ptr(Uc), k, _ptr(ft), n, _ptr(xt), n),
           "btri_solve")
    return _unrhs(vec, xt)


def babd_solve(D, Lo, C, f):
    """BABD solve: structured Gaussian elimination with row partial pivoting."""
    lib = _load()
    nb, m, _ = np.shape(D)
    Dc = _cm_blocks(D)
    Lc = _cm_blocks(Lo if nb > 1 else np.zeros((1, m, m)))
    Cc = _cm_blocks(np.asarray(C)[None])
    vec, ft, n, k = _rhs(f)
    assert n == m * nb
    xt = np.empty_like(ft)
    _check(lib.orc_babd_solve(m, nb, _ptr(Dc), _ptr(Lc), _ptr(Cc), k, _ptr(ft), n, _ptr(xt), n),
           "babd_solve")
    return _unrhs(vec, xt)


def btri_solve_trans(D, Lo, Up, f):
    """A^T x = f through the same band factors."""
    lib = _load()
    nb, m, _ = np.shape(D)
    Dc, Lc, Uc = _cm_blocks(D), _cm_blocks(Lo if nb > 1 else np.zeros((1, m, m))), \
        _cm_blocks(Up if nb > 1 else np.zeros((1, m, m)))
    vec, ft, n, k = _rhs(f)
    xt = np.empty_like(ft)
    _check(lib.orc_btri_solve_trans(m, nb, _ptr(Dc), _ptr(Lc), _ptr(Uc), k, _ptr(ft), n,
                                    _ptr(xt), n), "btri_solve_trans")
    return _unrhs(vec, xt)


def babd_solve_trans(D, Lo, C, f):
    """A^T x = f through the same structured factors."""
    lib = _load()
    nb, m, _ = np.shape(D)
    Dc = _cm_blocks(D)
    Lc = _cm_blocks(Lo if nb > 1 else np.zeros((1, m, m)))
    Cc = _cm_blocks(np.asarray(C)[None])
    vec, ft, n, k = _rhs(f)
    xt = np.empty_like(ft)
    _check(lib.orc_babd_solve_trans(m, nb, _ptr(Dc), _ptr(Lc), _ptr(Cc), k, _ptr(ft), n,
                                    _ptr(xt), n), "babd_solve_trans")
    return _unrhs(vec, xt)


def btri_residual(D, Lo, Up, f, x):
    """r = f - A x in FP64."""
    lib = _load()
    nb, m, _ = np.shape(D)
    Dc = _cm_blocks(D)
    Lc = _cm_blocks(Lo if nb > 1 else np.zeros((1, m, m)))
    Uc = _cm_blocks(Up if nb > 1 else np.zeros((1, m, m)))
    vec, ft, n, k = _rhs(f)
    _, xt, _, _ = _rhs(x)
    rt = np.empty_like(ft)
    lib.orc_btri_residual(m, nb, _ptr(Dc), _ptr(Lc), _ptr(Uc), k, _ptr(ft), n, _ptr(xt), n,
                          _ptr(rt), n)
    return _unrhs(vec, rt)


def babd_residual(D, Lo, C, f, x):
    lib = _load()
    nb, m, _ = np.shape(D)
    Dc = _cm_blocks(D)
    Lc = _cm_blocks(Lo if nb > 1 else np.zeros((1, m, m)))
    Cc = _cm_blocks(np.asarray(C)[None])
    vec, ft, n, k = _rhs(f)
    _, xt, _, _ = _rhs(x)
    rt = np.empty_like(ft)
    lib.orc_babd_residual(m, nb, _ptr(Dc), _ptr(Lc), _ptr(Cc), k, _ptr(ft), n, _ptr(xt), n,
                          _ptr(rt), n)
    return _unrhs(vec, rt)


def btri_norminf(D, Lo, Up) -> float:
    lib = _load()
    nb, m, _ = np.shape(D)
    Dc = _cm_blocks(D)
    Lc = _cm_blocks(Lo if nb > 1 else np.zeros((1, m, m)))
    Uc = _cm_blocks(Up if nb > 1 else np.zeros((1, m, m)))
    return float(lib.orc_btri_norminf(m, nb, _ptr(Dc), _ptr(Lc), _ptr(Uc)))


def babd_norminf(D, Lo, C) -> float:
    lib = _load()
    nb, m, _ = np.shape(D)
    Dc = _cm_blocks(D)
    Lc = _cm_blocks(Lo if nb > 1 else np.zeros((1, m, m)))
    Cc = _cm_blocks(np.asarray(C)[None])
    return float(lib.orc_babd_norminf(m, nb, _ptr(Dc), _ptr(Lc), _ptr(Cc)))


def btri_condest(D, Lo, Up) -> float:
    """Hager-Higham estimate of kappa_inf(A) from the band LU factors."""
    lib = _load()
    nb, m, _ = np.shape(D)
    Dc = _cm_blocks(D)
    Lc = _cm_blocks(Lo if nb > 1 else np.zeros((1, m, m)))
    Uc = _cm_blocks(Up if nb > 1 else np.zeros((1, m, m)))
    return float(lib.orc_btri_condest(m, nb, _ptr(Dc), _ptr(Lc), _ptr(Uc)))


def babd_condest(D, Lo, C) -> float:
    lib = _load()
    nb, m, _ = np.shape(D)
    Dc = _cm_blocks(D)
    Lc = _cm_blocks(Lo if nb > 1 else np.zeros((1, m, m)))
    Cc = _cm_blocks(np.asarray(C)[None])
    return float(lib.orc_babd_condest(m, nb, _ptr(Dc), _ptr(Lc), _ptr(Cc)))


def eta(norm_a: float, f, x, r) -> np.ndarray:
    """Normwise backward error per right-hand side,
    ||r||_inf / (||A||_inf ||x||_inf + ||f||_inf)."""
    f2 = np.atleast_2d(np.asarray(f).T).T if np.ndim(f) == 1 else np.asarray(f)
    x2 = np.atleast_2d(np.asarray(x).T).T if np.ndim(x) == 1 else np.asarray(x)
    r2 = np.atleast_2d(np.asarray(r).T).T if np.ndim(r) == 1 else np.asarray(r)
    num = np.abs(r2).max(axis=0)
    den = norm_a * np.abs(x2).max(axis=0) + np.abs(f2).max(axis=0)
    return num / den


# ---------------------------------------------------------------------------
# Dense forms and the Schur complement (tiny inputs only).

def btri_dense(D, Lo, Up) -> np.ndarray:
    nb, m, _ = np.shape(D)
    A = np.zeros((nb * m, nb * m))
    for k in range(nb):
        A[k * m:(k + 1) * m, k * m:(k + 1) * m] = D[k]
        if k + 1 < nb:
            A[(k + 1) * m:(k + 2) * m, k * m:(k + 1) * m] = Lo[k]
            A[k * m:(k + 1) * m, (k + 1) * m:(k + 2) * m] = Up[k]
    return A


def babd_dense(D, Lo, C) -> np.ndarray:
    nb, m, _ = np.shape(D)
    A = np.zeros((nb * m, nb * m))
    for k in range(nb):
        A[k * m:(k + 1) * m, k * m:(k + 1) * m] += D[k]
        if k + 1 < nb:
            A[(k + 1) * m:(k + 2) * m, k * m:(k + 1) * m] = Lo[k]
    A[0:m, (nb - 1) * m:nb * m] += C
    return A


def schur_complement(A: np.ndarray, m: int, sep_blocks, f=None):
    """Schur complement of the dense matrix A onto the block rows/columns
    listed in ``sep_blocks``: S = A_ss - A_sI A_II^{-1} A_Is, and the matching
    reduced right-hand side g = f_s - A_sI A_II^{-1} f_I.  By eq. (parfact) the
    reduced matrix of the partition method is exactly this S, whichever local
    factorization produced it."""
    n = A.shape[0]
    sep = np.concatenate([np.arange(b * m, (b + 1) * m) for b in sep_blocks]).astype(int)
    mask = np.ones(n, bool)
    mask[sep] = False
    interior = np.nonzero(mask)[0]
    Ass = A[np.ix_(sep, sep)]
    AsI = A[np.ix_(sep, interior)]
    AIs = A[np.ix_(interior, sep)]
    AII = A[np.ix_(interior, interior)]
    S = Ass - AsI @ np.linalg.solve(AII, AIs)
    if f is None:
        return S
    f = np.asarray(f, dtype=np.float64)
    g = f[sep] - AsI @ np.linalg.solve(AII, f[interior])
    return S, g


def ivp_trapezoid(L, h, g, y0):
    """The trapezoid discretization of y' = L y + g(t), y(t0) = y0, solved in
    the sequential fashion of Sec. 3 (before eq. (D)): one step at a time,
    y_0 = y0 and (I - h/2 L) y_n = (I + h/2 L) y_{n-1} + h/2 (g_{n-1} + g_n).
    L: (m, m); g: (steps+1, m) samples g(t0 + n h); y0: (m,).  Returns the
    (steps+1, m) array of y_n."""
    L = np.asarray(L, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = L.shape[0]
    eye = np.eye(m)
    left = eye - 0.5 * h * L
    right = eye + 0.5 * h * L
    y = np.empty_like(g)
    y[0] = np.asarray(y0, dtype=np.float64)
    for n in range(1, g.shape[0]):
        y[n] = np.linalg.solve(left, right @ y[n - 1] + 0.5 * h * (g[n - 1] + g[n]))
    return y
