"""MI355X rank-k symmetric eigen-update (Oh & Hu, arXiv:1706.00773).

Thin ctypes binding of ``libeigupd.so`` (include/eigupd.h).  The functions
keep the C names and only marshal arguments: every step of an update runs in
the library's HIP kernels.  Torch tensors on the GPU are passed by device
pointer (``data_ptr()``) together with torch's current HIP stream; numpy
arrays are passed as host pointers.  Matrices are column-major: pass a numpy
array in Fortran order or a torch tensor whose first stride is 1.

If the library has not been built, the first call raises ``RuntimeError`` --
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeigupd.so")

EIG_OK = 0
EIG_EINVAL = -1
EIG_ENOMEM = -2
EIG_EDEVICE = -3
EIG_ENOCONV = -4
EIG_ENOTSORTED = -5
EIG_EUNSUPPORTED = -6
EIG_EDEPENDENCY = -7
EIG_ESTATE = -8
EIG_ENONFINITE = -9
EIG_ECHECK = -10

EIG_GEMM_FP64 = 0
EIG_GEMM_FP32_CORR = 1
EIG_GEMM_BF16X3_CORR = 2
EIG_GEMM_MASK = 3
EIG_VALUES_ONLY = 1 << 4
EIG_DEBUG_CHECKS = 1 << 5
EIG_HOST_INPUT = 1 << 6
EIG_PHASE_TIMING = 1 << 7
EIG_LOCATE_RESIDUES = 1 << 8
EIG_QW_FARFIELD = 1 << 9
EIG_KMAX = 8
EIG_KMAX_GENERIC = 32
EIG_NOALLOC_NMAX = 16384

EIG_DBG_U = 1
EIG_DBG_POLE_COUNT = 2
EIG_DBG_SEG_START = 3
EIG_DBG_REDUCED_D = 4
EIG_DBG_REDUCED_ROW = 5
EIG_DBG_ROOT_ORIGIN = 6
EIG_DBG_ROOT_TAU = 7
EIG_DBG_ROOT_ITERS = 8
EIG_DBG_W = 9

EIG_KNOB_ROOTSOLVE = 1
EIG_KNOB_GEMM_TILE = 2
EIG_KNOB_GRAPHS = 3
EIG_STAT_GRAPH_LAUNCHES = 4
EIG_STAT_GRAPHS_CACHED = 5
EIG_KNOB_MAX_EVALS = 6
EIG_AUTO = 0
EIG_ROOTSOLVE_GROUPED = 1
EIG_ROOTSOLVE_PERSISTENT = 2

EXPORTED = ("eig_state_create", "eig_state_set", "eig_state_upload", "eig_update_rankk", "eig_update_interval",
            "eig_perturb_first_order", "eig_sturm_chain", "eig_query",
            "eig_state_destroy", "eig_status_str", "eig_debug_fetch", "eig_batch_create",
            "eig_update_batch", "eig_batch_set", "eig_batch_get", "eig_batch_destroy",
            "eig_server_create", "eig_server_add", "eig_server_submit", "eig_server_poll",
            "eig_server_drain", "eig_server_read", "eig_server_stats", "eig_server_destroy",
            "eig_eigvals_rankk_noalloc")


class eig_info(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("k", ctypes.c_int64),
        ("p", ctypes.c_int64),
        ("q", ctypes.c_int64),
        ("n_deflated_rows", ctypes.c_int64),
        ("n_deflated_groups", ctypes.c_int64),
        ("n_segments", ctypes.c_int64),
        ("iters_min", ctypes.c_int32),
        ("iters_max", ctypes.c_int32),
        ("iters_mean", ctypes.c_double),
        ("defl_backward_err", ctypes.c_double),
        ("anorm_bound", ctypes.c_double),
        ("generation", ctypes.c_int64),
        ("ms", ctypes.c_double * 8),
        ("located_by_residues", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: (list(getattr(self, f)) if f == "ms" else getattr(self, f))
                for f, _ in self._fields_}


class eig_chain_info(ctypes.Structure):
    _fields_ = [("n_poles", ctypes.c_int64), ("levels", ctypes.c_int64),
                ("lower_bound", ctypes.c_int64), ("n_deflated", ctypes.c_int64),
                ("complete", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class eig_batch_item(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_void_p),
        ("k", ctypes.c_int64),
        ("K", ctypes.c_void_p),
        ("ldk", ctypes.c_int64),
        ("sigma", ctypes.c_int8 * 8),
    ]


class eig_completion(ctypes.Structure):
    _fields_ = [
        ("request_id", ctypes.c_int64),
        ("matrix", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
        ("batch_size", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class eig_server_info(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("matrices", "submitted", "completed", "failed",
                                              "queued", "in_flight", "batches")] + [
        ("mean_batch", ctypes.c_double)] + [
        (f, ctypes.c_int64) for f in ("arena_bytes", "resident_bytes", "arena_used",
                                      "arena_peak", "compactions")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class EigError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {eig_status_str(code)} ({code})")


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libeigupd.so and declare its C signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_1706_00773_amd.build` "
            "(there is no non-HIP fallback)")
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.eig_state_create.argtypes = [ctypes.POINTER(vp), i64, i32]
    lib.eig_state_upload.argtypes = [vp, vp, vp, i64, i32, vp]
    lib.eig_state_set.argtypes = [vp, i32, i64]
    lib.eig_update_rankk.argtypes = [vp, i64, vp, i64, ctypes.POINTER(ctypes.c_int8),
                                     ctypes.c_uint32, vp]
    lib.eig_query.argtypes = [vp, vp, vp, i64, i32, ctypes.POINTER(eig_info), vp]
    lib.eig_perturb_first_order.argtypes = [vp, i64, vp, i64, ctypes.POINTER(ctypes.c_int8),
                                            ctypes.c_uint32, vp, vp, i64, vp]
    lib.eig_update_interval.argtypes = [vp, i64, vp, i64, ctypes.POINTER(ctypes.c_int8),
                                        ctypes.c_double, ctypes.c_double, ctypes.c_uint32, vp, vp,
                                        i64, i64, ctypes.POINTER(i64), vp]
    lib.eig_sturm_chain.argtypes = [vp, i64, vp, i64, ctypes.POINTER(ctypes.c_int8), vp, i64, vp,
                                    i64, vp, vp, i64, ctypes.POINTER(eig_chain_info), vp]
    lib.eig_state_destroy.argtypes = [vp]
    lib.eig_status_str.argtypes = [ctypes.c_int]
    lib.eig_status_str.restype = ctypes.c_char_p
    lib.eig_debug_fetch.argtypes = [vp, i32, vp, i64, vp]
    lib.eig_batch_create.argtypes = [ctypes.POINTER(vp), i32, i32]
    lib.eig_update_batch.argtypes = [vp, ctypes.POINTER(eig_batch_item), i32, ctypes.c_uint32, vp]
    lib.eig_batch_set.argtypes = [vp, i32, i32]
    lib.eig_batch_get.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.eig_batch_destroy.argtypes = [vp]
    lib.eig_server_create.argtypes = [ctypes.POINTER(vp), i32, i64, i32, i32, i64]
    lib.eig_server_add.argtypes = [vp, i64, vp, vp, i64, i32, ctypes.POINTER(i32)]
    lib.eig_server_submit.argtypes = [vp, i32, i64, vp, i64, ctypes.POINTER(ctypes.c_int8), i64]
    lib.eig_server_poll.argtypes = [vp, ctypes.POINTER(eig_completion), i32, i32,
                                    ctypes.POINTER(i32)]
    lib.eig_server_drain.argtypes = [vp]
    lib.eig_server_read.argtypes = [vp, i32, vp, vp, i64, i32]
    lib.eig_server_stats.argtypes = [vp, ctypes.POINTER(eig_server_info)]
    lib.eig_server_destroy.argtypes = [vp]
    lib.eig_eigvals_rankk_noalloc.argtypes = [i64, i64, vp, vp, i64, vp, i64,
                                              ctypes.POINTER(ctypes.c_int8), ctypes.c_uint32,
                                              vp, vp, i32, vp]
    for name in EXPORTED:
        getattr(lib, name).restype = (ctypes.c_char_p if name == "eig_status_str"
                                      else ctypes.c_int)
    _lib = lib
    return lib


def eig_status_str(code: int) -> str:
    return load_library().eig_status_str(int(code)).decode()


def _check(rc: int, where: str) -> None:
    if rc != EIG_OK:
        raise EigError(rc, where)


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _current_stream(stream):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch

    return torch.cuda.current_stream().cuda_stream


def _colmajor_ptr(a, n_rows: int):
    """(pointer, leading dimension, on_device, keepalive) of a column-major matrix."""
    if _is_torch(a):
        import torch

        if a.dtype != torch.float64:
            raise TypeError("expected float64")
        if a.dim() == 1:
            return a.data_ptr(), max(n_rows, a.shape[0]), 1, a
        if a.stride(0) != 1:
            a = a.t().contiguous().t()
        return a.data_ptr(), max(a.stride(1), n_rows), 1, a
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    a = np.asfortranarray(a)
    return a.ctypes.data, a.shape[0], 0, a


def eig_state_create(n: int, device: int = 0):
    h = ctypes.c_void_p()
    _check(load_library().eig_state_create(ctypes.byref(h), int(n), int(device)),
           "eig_state_create")
    return h


def eig_state_set(s, knob: int, value: int) -> None:
    _check(load_library().eig_state_set(s, int(knob), int(value)), "eig_state_set")


def eig_state_destroy(s) -> None:
    _check(load_library().eig_state_destroy(s), "eig_state_destroy")


def eig_state_upload(s, lam, Q, stream=None) -> None:
    """Load lambda (ascending) and Q (column-major); both torch-on-GPU or both numpy."""
    n = lam.shape[0]
    qp, ldq, qdev, qk = _colmajor_ptr(Q, n)
    if _is_torch(lam):
        lam_c = lam.contiguous()
        lp, ldev = lam_c.data_ptr(), 1
    else:
        lam_c = np.ascontiguousarray(lam, dtype=np.float64)
        lp, ldev = lam_c.ctypes.data, 0
    if ldev != qdev:
        raise ValueError("lambda and Q must both be device tensors or both host arrays")
    st = _current_stream(stream) if qdev else None
    _check(load_library().eig_state_upload(s, lp, qp, ldq, qdev, st), "eig_state_upload")


def eig_update_rankk(s, K, sigma, mode: int = EIG_GEMM_FP64, stream=None) -> None:
    """Enqueue A' = A + K diag(sigma) K^T.  K: n-by-k column-major (torch on the GPU, or
    numpy on the host, which sets EIG_HOST_INPUT); sigma: k values of +-1."""
    n = K.shape[0]
    k = 1 if K.ndim == 1 else K.shape[1]
    kp, ldk, kdev, keep = _colmajor_ptr(K, n)
    if not kdev:
        mode |= EIG_HOST_INPUT
    sig = (ctypes.c_int8 * k)(*[int(v) for v in np.asarray(sigma).ravel()[:k]])
    st = _current_stream(stream) if (kdev or stream is not None) else None
    _check(load_library().eig_update_rankk(s, k, kp, ldk, sig, int(mode), st),
           "eig_update_rankk")


def eig_update_interval(s, K, sigma, a: float, b: float, mode: int = 0, m_max: int = 0,
                        stream=None):
    """Eigenpairs of A' = A + K diag(sigma) K^T with eigenvalues in [a, b), without
    changing the state.  K: n-by-k torch tensor on the GPU (or numpy, copied).
    Returns (lam, V) as torch tensors on the GPU (V None with EIG_VALUES_ONLY); m_max
    is the initial capacity (grown once if the interval holds more)."""
    import torch

    n = K.shape[0]
    k = 1 if K.ndim == 1 else K.shape[1]
    kp, ldk, kdev, keep = _colmajor_ptr(K, n)
    if not kdev:
        mode |= EIG_HOST_INPUT
    sig = (ctypes.c_int8 * k)(*[int(v) for v in np.asarray(sigma).ravel()[:k]])
    st = _current_stream(stream)
    vo = bool(mode & EIG_VALUES_ONLY)
    cap = max(int(m_max), 1)
    lib = load_library()
    for _ in range(2):
        lam = torch.empty(cap, dtype=torch.float64, device="cuda")
        V = None if vo else torch.empty((cap, n), dtype=torch.float64, device="cuda").t()
        m = ctypes.c_int64()
        rc = lib.eig_update_interval(s, k, kp, ldk, sig, float(a), float(b), int(mode),
                                     lam.data_ptr(), None if vo else V.data_ptr(), n, cap,
                                     ctypes.byref(m), st)
        if rc == EIG_EINVAL and m.value > cap:
            cap = int(m.value)
            continue
        _check(rc, "eig_update_interval")
        mm = int(m.value)
        return lam[:mm], (None if vo else V[:, :mm])
    raise EigError(EIG_EINVAL, "eig_update_interval")


def eig_perturb_first_order(s, K, sigma, stream=None):
    """First-order perturbation estimate (eq. (11)) of the pairs of A + K diag(sigma) K^T:
    returns (lam, V) as torch tensors on the GPU, in the order of the resident pairs."""
    import torch

    n = K.shape[0]
    k = 1 if K.ndim == 1 else K.shape[1]
    kp, ldk, kdev, keep = _colmajor_ptr(K, n)
    mode = 0 if kdev else EIG_HOST_INPUT
    sig = (ctypes.c_int8 * k)(*[int(v) for v in np.asarray(sigma).ravel()[:k]])
    lam = torch.empty(n, dtype=torch.float64, device="cuda")
    V = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    _check(load_library().eig_perturb_first_order(s, k, kp, ldk, sig, mode, lam.data_ptr(),
                                                  V.data_ptr(), n, _current_stream(stream)),
           "eig_perturb_first_order")
    return lam, V


def eig_sturm_chain(s, K, sigma, x=None, xi=None, c_max: int = 0, stream=None):
    """Secular Sturm chain counter (Sec. 2.2, eqs. (4)-(9)) of A + K diag(sigma) K^T,
    without changing the state.  K: n-by-k torch tensor on the GPU; x: points (torch
    float64 on the GPU) to count the eigenvalues below; xi: known eigenvalues of the
    reduced problem, ascending, divided out first (eq. (9)).  Returns (counts as an
    int64 torch tensor or None, the first c_max leading constants or None, eig_chain_info)."""
    import torch

    n = K.shape[0]
    k = 1 if K.ndim == 1 else K.shape[1]
    kp, ldk, kdev, keep = _colmajor_ptr(K, n)
    if not kdev:
        raise ValueError("K must be a device tensor")
    sig = (ctypes.c_int8 * k)(*[int(v) for v in np.asarray(sigma).ravel()[:k]])
    xs = None if x is None else x.to(dtype=torch.float64).contiguous()
    xis = None if xi is None else xi.to(dtype=torch.float64).contiguous()
    n_x = 0 if xs is None else xs.numel()
    n_xi = 0 if xis is None else xis.numel()
    counts = torch.empty(max(n_x, 1), dtype=torch.int64, device="cuda")
    cbuf = torch.empty(max(int(c_max), 1), dtype=torch.float64, device="cuda")
    info = eig_chain_info()
    _check(load_library().eig_sturm_chain(
        s, k, kp, ldk, sig, None if xis is None else xis.data_ptr(), n_xi,
        None if xs is None else xs.data_ptr(), n_x, counts.data_ptr() if n_x else None,
        cbuf.data_ptr() if c_max > 0 else None, int(c_max), ctypes.byref(info),
        _current_stream(stream)), "eig_sturm_chain")
    c = cbuf[: min(int(c_max), int(info.levels))] if c_max > 0 else None
    return (counts[:n_x] if n_x else None), c, info


def eig_query(s, lambda_out=None, Q_out=None, stream=None, want_info: bool = True):
    """Synchronise, raise on a deferred error, copy out the committed decomposition.

    lambda_out / Q_out: torch tensors on the GPU (Q_out column-major) or numpy arrays
    (Q_out in Fortran order), or None.  Returns an eig_info (or None)."""
    lib = load_library()
    lp = qp = None
    ldq = 1
    dev = None
    if lambda_out is not None:
        if _is_torch(lambda_out):
            lp, dev = lambda_out.data_ptr(), 1
        else:
            if not (lambda_out.flags.c_contiguous and lambda_out.dtype == np.float64):
                raise ValueError("lambda_out must be a contiguous float64 array")
            lp, dev = lambda_out.ctypes.data, 0
    if Q_out is not None:
        if _is_torch(Q_out):
            if Q_out.stride(0) != 1:
                raise ValueError("Q_out must be column-major (stride(0) == 1)")
            qp, ldq, qdev = Q_out.data_ptr(), Q_out.stride(1), 1
        else:
            if not (Q_out.flags.f_contiguous and Q_out.dtype == np.float64):
                raise ValueError("Q_out must be a Fortran-ordered float64 array")
            qp, ldq, qdev = Q_out.ctypes.data, Q_out.shape[0], 0
        if dev is not None and dev != qdev:
            raise ValueError("outputs must both be on the device or both on the host")
        dev = qdev
    info = eig_info() if want_info else None
    st = _current_stream(stream) if (dev or stream is not None) else None
    rc = lib.eig_query(s, lp, qp, max(ldq, 1), int(bool(dev)),
                       ctypes.byref(info) if info is not None else None, st)
    _check(rc, "eig_query")
    return info


def eig_eigvals_rankk_noalloc(lam, Q, K, sigma, lam_out, status_out, mode: int = 0,
                              device: int = 0, stream=None) -> None:
    """Enqueue the eigenvalues of Q diag(lam) Q^T + K diag(sigma) K^T into lam_out with
    no device allocation (the library's static workspace).  lam, Q, K, lam_out: float64
    torch tensors on `device` (Q, K column-major); status_out: an int32 torch tensor
    of one element that receives the EIG_* status on the stream."""
    import torch

    n = lam.shape[0]
    k = 1 if K.ndim == 1 else K.shape[1]
    for t in (lam, Q, K, lam_out, status_out):
        if not _is_torch(t) or not t.is_cuda:
            raise TypeError("expected torch tensors on the GPU")
    if status_out.dtype != torch.int32 or lam_out.dtype != torch.float64:
        raise TypeError("lam_out must be float64 and status_out int32")
    if not (lam.is_contiguous() and lam_out.is_contiguous()):
        raise ValueError("lam and lam_out must be contiguous")
    qp, ldq, _, qk = _colmajor_ptr(Q, n)
    kp, ldk, _, kk = _colmajor_ptr(K, n)
    sig = (ctypes.c_int8 * k)(*[int(v) for v in np.asarray(sigma).ravel()[:k]])
    _check(load_library().eig_eigvals_rankk_noalloc(
        n, k, lam.data_ptr(), qp, ldq, kp, ldk, sig, int(mode), lam_out.data_ptr(),
        status_out.data_ptr(), int(device), _current_stream(stream)),
        "eig_eigvals_rankk_noalloc")


def eig_debug_fetch(s, what: int, count: int, dtype, stream=None) -> np.ndarray:
    out = np.empty(count, dtype=dtype)
    st = _current_stream(stream) if stream is not None else None
    _check(load_library().eig_debug_fetch(s, int(what), out.ctypes.data, out.nbytes, st),
           "eig_debug_fetch")
    return out


def eig_batch_create(max_items: int, device: int = 0):
    h = ctypes.c_void_p()
    _check(load_library().eig_batch_create(ctypes.byref(h), int(max_items), int(device)),
           "eig_batch_create")
    return h


def eig_batch_destroy(b) -> None:
    _check(load_library().eig_batch_destroy(b), "eig_batch_destroy")


def eig_update_batch(b, updates, mode: int = EIG_GEMM_FP64, stream=None) -> None:
    """updates: sequence of (state handle, K, sigma) with K an n-by-k column-major
    float64 torch tensor on the state's GPU."""
    items = (eig_batch_item * len(updates))()
    keep = []
    for i, (h, K, sigma) in enumerate(updates):
        if not _is_torch(K):
            raise TypeError("batched updates take device tensors for K")
        n = K.shape[0]
        k = 1 if K.dim() == 1 else K.shape[1]
        kp, ldk, _, kk = _colmajor_ptr(K, n)
        keep.append(kk)
        items[i].state = h.value if isinstance(h, ctypes.c_void_p) else h
        items[i].k = k
        items[i].K = kp
        items[i].ldk = ldk
        sig = np.asarray(sigma).ravel()
        for c in range(min(k, 8)):
            items[i].sigma[c] = int(sig[c])
    st = _current_stream(stream)
    _check(load_library().eig_update_batch(b, items, len(updates), int(mode), st),
           "eig_update_batch")


def eig_batch_set(b, knob: int, value: int) -> None:
    _check(load_library().eig_batch_set(b, int(knob), int(value)), "eig_batch_set")


def eig_batch_get(b, knob: int) -> int:
    v = ctypes.c_int64()
    _check(load_library().eig_batch_get(b, int(knob), ctypes.byref(v)), "eig_batch_get")
    return int(v.value)


class EigBatch:
    """A batch context: one update of each of several states per call."""

    def __init__(self, max_items: int, device: int = 0):
        self.handle = eig_batch_create(max_items, device)

    def update(self, updates, mode: int = EIG_GEMM_FP64, stream=None):
        """updates: sequence of (EigState, K, sigma)."""
        eig_update_batch(self.handle, [(s.handle, K, sig) for s, K, sig in updates], mode,
                         stream)

    def set(self, knob: int, value: int):
        eig_batch_set(self.handle, knob, value)

    def get(self, knob: int) -> int:
        return eig_batch_get(self.handle, knob)

    def close(self):
        if self.handle is not None:
            eig_batch_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EigServer:
    """Serving loop over many resident decompositions (owns an eig_server_t)."""

    def __init__(self, arena_bytes: int, max_batch: int = 32, streams: int = 2,
                 max_k_doubles: int = 1 << 22, device: int = 0):
        h = ctypes.c_void_p()
        _check(load_library().eig_server_create(ctypes.byref(h), int(device), int(arena_bytes),
                                                int(max_batch), int(streams),
                                                int(max_k_doubles)), "eig_server_create")
        self.handle = h
        self._sizes = []

    def add(self, lam, Q) -> int:
        """Register (lam, Q); torch tensors on the GPU (Q column-major) or numpy arrays."""
        n = lam.shape[0]
        qp, ldq, qdev, qk = _colmajor_ptr(Q, n)
        if _is_torch(lam):
            lam_c = lam.contiguous()
            lp = lam_c.data_ptr()
        else:
            lam_c = np.ascontiguousarray(lam, dtype=np.float64)
            lp = lam_c.ctypes.data
        mid = ctypes.c_int32()
        _check(load_library().eig_server_add(self.handle, n, lp, qp, ldq, qdev,
                                             ctypes.byref(mid)), "eig_server_add")
        self._sizes.append(n)
        return int(mid.value)

    def submit(self, matrix: int, K, sigma, request_id: int):
        """K: numpy n-by-k (host); copied before return."""
        Kf = np.asfortranarray(np.asarray(K, dtype=np.float64).reshape(K.shape[0], -1))
        k = Kf.shape[1]
        sig = (ctypes.c_int8 * k)(*[int(v) for v in np.asarray(sigma).ravel()[:k]])
        _check(load_library().eig_server_submit(self.handle, int(matrix), k, Kf.ctypes.data,
                                                Kf.shape[0], sig, int(request_id)),
               "eig_server_submit")

    def poll(self, max_items: int = 1024, timeout_ms: int = 0):
        buf = (eig_completion * max_items)()
        cnt = ctypes.c_int32()
        _check(load_library().eig_server_poll(self.handle, buf, max_items, int(timeout_ms),
                                              ctypes.byref(cnt)), "eig_server_poll")
        return [{f: getattr(buf[i], f) for f, _ in eig_completion._fields_}
                for i in range(cnt.value)]

    def drain(self):
        _check(load_library().eig_server_drain(self.handle), "eig_server_drain")

    def read(self, matrix: int):
        """(lam, Q) of a matrix as numpy arrays (waits for its queued updates)."""
        n = self._sizes[matrix]
        lam = np.empty(n)
        Q = np.empty((n, n), order="F")
        _check(load_library().eig_server_read(self.handle, int(matrix), lam.ctypes.data,
                                              Q.ctypes.data, n, 0), "eig_server_read")
        return lam, Q

    def stats(self):
        info = eig_server_info()
        _check(load_library().eig_server_stats(self.handle, ctypes.byref(info)),
               "eig_server_stats")
        return info.as_dict()

    def close(self):
        if self.handle is not None:
            _check(load_library().eig_server_destroy(self.handle), "eig_server_destroy")
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EigState:
    """A resident decomposition on one GPU (owns an eig_state_t)."""

    def __init__(self, n: int, device: int = 0):
        self.n = int(n)
        self.device = int(device)
        self.handle = eig_state_create(self.n, self.device)

    def upload(self, lam, Q, stream=None):
        eig_state_upload(self.handle, lam, Q, stream)

    def set(self, knob: int, value: int):
        eig_state_set(self.handle, knob, value)

    def update(self, K, sigma, mode: int = EIG_GEMM_FP64, stream=None):
        eig_update_rankk(self.handle, K, sigma, mode, stream)

    def query(self, lambda_out=None, Q_out=None, stream=None):
        return eig_query(self.handle, lambda_out, Q_out, stream)

    def interval(self, K, sigma, a, b, mode: int = 0, m_max: int = 0, stream=None):
        return eig_update_interval(self.handle, K, sigma, a, b, mode, m_max, stream)

    def sturm_chain(self, K, sigma, x=None, xi=None, c_max: int = 0, stream=None):
        return eig_sturm_chain(self.handle, K, sigma, x, xi, c_max, stream)

    def perturb_first_order(self, K, sigma, stream=None):
        return eig_perturb_first_order(self.handle, K, sigma, stream)

    def fetch(self, what: int, count: int, dtype=np.float64, stream=None):
        return eig_debug_fetch(self.handle, what, count, dtype, stream)

    def close(self):
        if self.handle is not None:
            eig_state_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
