"""The entry point that allocates nothing (eig_eigvals_rankk_noalloc): its
workspace is the library's static device array.  Each call is checked against
eig_update_rankk with EIG_VALUES_ONLY on the same input (the same kernels, so
bitwise equal) and against the oracle's bisection (within 1e-10 ||A'||_2), on
consecutive calls whose sizes shrink, so that a call that read the previous
call's leftovers would show."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1706_00773_amd as eu
from paper_1706_00773_amd import workloads as wl

from helpers import colmajor

pytestmark = pytest.mark.gpu

EVAL_TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eu.load_library()


def _state_values(lam_t, Q_t, K_t, sigma, mode=0):
    import torch

    n = lam_t.shape[0]
    with eu.EigState(n, 0) as s:
        s.upload(lam_t, Q_t)
        s.update(K_t, sigma, eu.EIG_VALUES_ONLY | mode)
        out = torch.empty(n, dtype=torch.float64, device="cuda:0")
        s.query(out)
    return out.cpu().numpy()


def _noalloc(lam_t, Q_t, K_t, sigma, mode=0):
    import torch

    n = lam_t.shape[0]
    out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
    st = torch.full((1,), 12345, dtype=torch.int32, device="cuda:0")
    eu.eig_eigvals_rankk_noalloc(lam_t, Q_t, K_t, sigma, out, st, mode)
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(st.item())


def _check_case(u, label, mode=0, sample=None, Q_t=None):
    import torch

    dev = "cuda:0"
    n = u.lam.size
    k = u.K.shape[1]
    print(f"case {label}: n={n} k={k} mode={mode}", flush=True)
    lam_t = torch.from_numpy(np.ascontiguousarray(u.lam)).to(dev)
    if Q_t is None:
        Q_t = u.Q if isinstance(u.Q, torch.Tensor) else colmajor(u.Q, dev)
    K_t = colmajor(u.K, dev)
    got, status = _noalloc(lam_t, Q_t, K_t, u.sigma, mode)
    assert status == eu.EIG_OK
    ref = _state_values(lam_t, Q_t, K_t, u.sigma, mode)
    assert np.array_equal(got, ref), np.abs(got - ref).max()
    Qh = np.asfortranarray(Q_t.cpu().numpy())
    U = oracle.qtk(Qh, np.asfortranarray(u.K))
    scale = np.abs(u.lam).max() + float(np.sum(U * U))
    idx = None if sample is None else np.unique(np.r_[sample, 0, n - 1])
    vals = oracle.eigvals(u.lam, U, u.sigma, idx)[0]
    sel = got if idx is None else got[idx]
    assert np.abs(sel - vals).max() <= EVAL_TOL * scale
    assert np.all(np.diff(got) >= 0.0)
    return got


def test_consecutive_calls_shrinking():
    """Two calls in a row, the second smaller (and of another rank): the second
    must not see the first one's workspace."""
    u1 = wl.general_rankk(4, n=1500, seed=31)
    _check_case(u1, "general rank-4 n=1500")
    u2 = wl.plain_rank2(301, seed=32)
    _check_case(u2, "plain rank-2 n=301 (after n=1500)")
    u3 = wl.plain_rank2(64, seed=33)
    _check_case(u3, "plain rank-2 n=64, residue location", mode=eu.EIG_LOCATE_RESIDUES)


def test_deflation_and_clusters():
    u = wl.clustered_rank2(1024, seed=34)
    _check_case(u, "clustered rank-2 n=1024 with tiny rows")


def test_leading_dimension_and_rank1():
    """Q given as the leading n x n block of a larger column-major matrix."""
    import torch

    dev = "cuda:0"
    u = wl.general_rankk(1, n=257, seed=35)
    n = u.lam.size
    big = torch.zeros((n + 3, n), dtype=torch.float64, device=dev)
    big[:n, :] = torch.from_numpy(np.asarray(u.Q)).to(dev)
    Qv = torch.as_strided(big.t().contiguous(), (n, n), (1, n + 3))
    assert Qv.stride() == (1, n + 3)
    _check_case(u, "rank-1 n=257, ldq = n + 3", Q_t=Qv)


def test_maximum_order():
    """n = EIG_NOALLOC_NMAX, rank 8, Q = I (U = K): the largest workspace."""
    import torch

    dev = "cuda:0"
    n, k = eu.EIG_NOALLOC_NMAX, 8
    rng = np.random.default_rng(36)
    lam = np.sort(rng.uniform(-10.0, 10.0, n))
    K = rng.normal(0.0, 1.0 / np.sqrt(n), (n, k))
    sigma = np.where(rng.random(k) < 0.5, 1, -1).astype(np.int8)
    Q_t = torch.eye(n, dtype=torch.float64, device=dev)

    class U:
        pass

    u = U()
    u.lam, u.K, u.sigma, u.Q = lam, K, sigma, Q_t
    got = _check_case(u, "rank-8 n=16384, Q = I", sample=rng.choice(n, 48, replace=False),
                      Q_t=Q_t)
    tr = float(np.sum(sigma * np.sum(K * K, axis=0)))
    assert abs((got.sum() - lam.sum()) - tr) <= 1e-12 * n * (np.abs(lam).max() + 1.0)


def test_device_error_is_reported_and_cleared():
    """A NaN in K gives EIG_ENONFINITE in the status word; the next call, on a
    valid input, starts from a cleared status."""
    import torch

    dev = "cuda:0"
    u = wl.plain_rank2(200, seed=37)
    lam_t = torch.from_numpy(u.lam).to(dev)
    Q_t = colmajor(u.Q, dev)
    K = np.array(u.K)
    K[17, 1] = np.nan
    _, status = _noalloc(lam_t, Q_t, colmajor(K, dev), u.sigma)
    assert status == eu.EIG_ENONFINITE
    _check_case(u, "plain rank-2 n=200 after a failed call")


def test_argument_errors():
    import torch

    dev = "cuda:0"
    lib = eu.load_library()
    n, k = 8, 2
    lam = torch.arange(n, dtype=torch.float64, device=dev)
    Q = torch.eye(n, dtype=torch.float64, device=dev)
    K = torch.ones((n, k), dtype=torch.float64, device=dev)
    out = torch.empty(n, dtype=torch.float64, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    sig = (ctypes.c_int8 * k)(1, -1)
    bad = (ctypes.c_int8 * k)(1, 0)
    p = lambda t: t.data_ptr()  # noqa: E731
    f = lib.eig_eigvals_rankk_noalloc
    assert f(n, k, p(lam), p(Q), n, p(K), n, sig, 0, p(out), None, 0, None) == eu.EIG_EINVAL
    assert f(n, k, p(lam), p(Q), n - 1, p(K), n, sig, 0, p(out), p(st), 0, None) == eu.EIG_EINVAL
    assert f(n, k, p(lam), p(Q), n, p(K), n, bad, 0, p(out), p(st), 0, None) == eu.EIG_EINVAL
    assert f(n, 9, p(lam), p(Q), n, p(K), n, sig, 0, p(out), p(st), 0, None) == \
        eu.EIG_EUNSUPPORTED
    assert f(eu.EIG_NOALLOC_NMAX + 1, k, p(lam), p(Q), eu.EIG_NOALLOC_NMAX + 1, p(K),
             eu.EIG_NOALLOC_NMAX + 1, sig, 0, p(out), p(st), 0, None) == eu.EIG_EUNSUPPORTED
    assert f(n, k, p(lam), p(Q), n, p(K), n, sig, eu.EIG_QW_FARFIELD, p(out), p(st), 0,
             None) == eu.EIG_EUNSUPPORTED
