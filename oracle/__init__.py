"""CPU oracle for the rank-k symmetric eigen-update (Oh & Hu, arXiv:1706.00773).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU product
path (``paper_1706_00773_amd``) never imports it, and the two share no code.

The arithmetic lives in ``eigref.c`` (plain FP64 C, OpenMP over independent
roots); this module only marshals numpy arrays through ctypes.  See the
header of ``eigref.c`` for the passages of the paper each routine follows and
for the readings taken where the paper is garbled.

Parity status: every routine here is pinned by ``tests/test_oracle_pins.py``
against LAPACK (numpy), exact-rational Sturm counts, closed forms and
invariants -- none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eigref.c")
_LIB_PATH = os.path.join(_HERE, "libeigref.so")
_lib = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i8p = ctypes.POINTER(ctypes.c_int8)


def build(force: bool = True) -> str:
    """Compile eigref.c with gcc (-O2, OpenMP, no fast-math) into libeigref.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
               "-ffp-contract=off", "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.eigref_qtk.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64, _dp]
    lib.eigref_count.argtypes = [_i64, _i64, _dp, _dp, _i8p, _i64, ctypes.c_double]
    lib.eigref_count.restype = _i64
    lib.eigref_pole_count.argtypes = [_i64, _i64, _dp, _dp, _i8p, _i64]
    lib.eigref_pole_count.restype = _i64
    lib.eigref_secular_det.argtypes = [_i64, _i64, _dp, _dp, _i8p, ctypes.c_double, _dp]
    lib.eigref_alpha.argtypes = [_i64, _i64, _dp, _dp, _i8p, _i64, _dp]
    lib.eigref_jacobi.argtypes = [_i64, _dp, _dp, _dp]
    lib.eigref_eigvals.argtypes = [_i64, _i64, _dp, _dp, _i8p, _i64, _i64p, _dp, _i64p, _dp,
                                   _i32p]
    lib.eigref_eigvecs.argtypes = [_i64, _i64, _dp, _dp, _i8p, _i64, _i64p, _dp, _i64p, _i64p,
                                   _dp, _i64]
    lib.eigref_gemm.argtypes = [_i64, _i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64]
    lib.eigref_update.argtypes = [_i64, _i64, _dp, _dp, _i64, _dp, _i64, _i8p, _i32, _dp, _dp,
                                  _i64, _dp]
    lib.eigref_set_threads.argtypes = [ctypes.c_int]
    lib.eigref_get_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _fortran(a):
    return np.asfortranarray(a, dtype=np.float64)


def _sig(sigma):
    s = np.ascontiguousarray(sigma, dtype=np.int8)
    return s, s.ctypes.data_as(_i8p)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def set_threads(t: int) -> None:
    _load().eigref_set_threads(int(t))


def get_threads() -> int:
    return int(_load().eigref_get_threads())


def qtk(Q, K):
    """U = Q^T K (Sec. 2.1), returned as an n-by-k array."""
    Q = _fortran(Q)
    K = _fortran(K.reshape(K.shape[0], -1))
    n, k = K.shape
    U = np.empty((n, k), dtype=np.float64)
    _check(_load().eigref_qtk(n, k, _d(Q), n, _d(K), n, _d(U)), "qtk")
    return U


def count(lam, U, sigma, x, origin: int = -1) -> int:
    """nu(x): eigenvalues of diag(lam) + U Sigma U^T strictly below x = lam[origin] + x
    (x absolute when origin < 0).  -1 means x is a pole."""
    lam = _f64(lam)
    U = _f64(U)
    s, sp = _sig(sigma)
    return int(_load().eigref_count(lam.size, U.shape[1], _d(lam), _d(U), sp, int(origin),
                                    float(x)))


def pole_count(lam, U, sigma, j: int) -> int:
    """nu(lam_j) from the bordered (k+1)-by-(k+1) inertia."""
    lam = _f64(lam)
    U = _f64(U)
    s, sp = _sig(sigma)
    r = int(_load().eigref_pole_count(lam.size, U.shape[1], _d(lam), _d(U), sp, int(j)))
    if r < -1:
        raise ValueError("pole_count: invalid arguments")
    return r


def secular_det(lam, U, sigma, x) -> float:
    """f(x) = det(I - Sigma U^T (xI - D)^{-1} U) (eq. (1))."""
    lam = _f64(lam)
    U = _f64(U)
    s, sp = _sig(sigma)
    out = np.zeros(1)
    _check(_load().eigref_secular_det(lam.size, U.shape[1], _d(lam), _d(U), sp, float(x),
                                      _d(out)), "secular_det")
    return float(out[0])


def alpha(lam, U, sigma, i: int) -> float:
    """alpha_i of eq. (2) (sign as read in eigref.c)."""
    lam = _f64(lam)
    U = _f64(U)
    s, sp = _sig(sigma)
    out = np.zeros(1)
    _check(_load().eigref_alpha(lam.size, U.shape[1], _d(lam), _d(U), sp, int(i), _d(out)),
           "alpha")
    return float(out[0])


def jacobi(A):
    """Brute-force cyclic Jacobi eigensolve of a symmetric matrix: (w ascending, V)."""
    A = _fortran(A)
    m = A.shape[0]
    w = np.empty(m)
    V = np.empty((m, m), order="F")
    _check(_load().eigref_jacobi(m, _d(A), _d(w), _d(V)), "jacobi")
    return w, V


def eigvals(lam, U, sigma, idx=None):
    """Eigenvalues (0-based indices idx, or all) by bisection on the count.

    Returns (values, origin, tau, evaluations) with value = lam[origin] + tau
    (origin == -1: value = tau)."""
    lam = _f64(lam)
    U = _f64(U)
    s, sp = _sig(sigma)
    n, k = U.shape
    if idx is None:
        m = n
        ip = None
    else:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        m = idx.size
        ip = idx.ctypes.data_as(_i64p)
    vals = np.empty(m)
    org = np.empty(m, dtype=np.int64)
    tau = np.empty(m)
    ev = np.empty(m, dtype=np.int32)
    _check(_load().eigref_eigvals(n, k, _d(lam), _d(U), sp, m, ip, _d(vals),
                                  org.ctypes.data_as(_i64p), _d(tau), ev.ctypes.data_as(_i32p)),
           "eigvals")
    return vals, org, tau, ev


def eigvecs(lam, U, sigma, origin, tau, cluster=None, mult=None):
    """Q-basis eigenvectors (eq. (10)) of the given roots, n-by-m column-major."""
    lam = _f64(lam)
    U = _f64(U)
    s, sp = _sig(sigma)
    n, k = U.shape
    origin = np.ascontiguousarray(origin, dtype=np.int64)
    tau = _f64(tau)
    m = origin.size
    cp = mp = None
    if cluster is not None:
        cluster = np.ascontiguousarray(cluster, dtype=np.int64)
        mult = np.ascontiguousarray(mult, dtype=np.int64)
        cp = cluster.ctypes.data_as(_i64p)
        mp = mult.ctypes.data_as(_i64p)
    W = np.empty((n, m), order="F")
    _check(_load().eigref_eigvecs(n, k, _d(lam), _d(U), sp, m, origin.ctypes.data_as(_i64p),
                                  _d(tau), cp, mp, _d(W), n), "eigvecs")
    return W


def gemm(A, B):
    A = _fortran(A)
    B = _fortran(B)
    m, kk = A.shape
    nn = B.shape[1]
    C = np.empty((m, nn), order="F")
    _check(_load().eigref_gemm(m, nn, kk, _d(A), m, _d(B), kk, _d(C), m), "gemm")
    return C


def update(lam, Q, K, sigma, values_only: bool = False):
    """The whole rank-k update: returns (lam', Q', W) (Q', W None if values_only)."""
    lam = _f64(lam)
    Q = _fortran(Q)
    K = _fortran(K.reshape(K.shape[0], -1))
    n, k = K.shape
    s, sp = _sig(sigma)
    lo = np.empty(n)
    if values_only:
        _check(_load().eigref_update(n, k, _d(lam), _d(Q), n, _d(K), n, sp, 1, _d(lo), None,
                                     n, None), "update")
        return lo, None, None
    Qo = np.empty((n, n), order="F")
    W = np.empty((n, n), order="F")
    _check(_load().eigref_update(n, k, _d(lam), _d(Q), n, _d(K), n, sp, 0, _d(lo), _d(Qo), n,
                                 _d(W)), "update")
    return lo, Qo, W
