"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Tolerances (FP64 form of the target): eigenvalues within 1e-10 ||A'||_2,
residual ||A' q - lambda q|| <= 1e-9 ||A'||_2, ||Q'^T Q' - I||_max <= 1e-9;
eigenvectors of eigenvalues separated by more than 1e-6 ||A'|| are compared
elementwise with the oracle's (up to sign) within 1e-8; pole counts are
integers and must match exactly.
"""
import numpy as np
import pytest

import oracle
import paper_1706_00773_amd as eu
from paper_1706_00773_amd import workloads as wl

from helpers import align_signs, colmajor, isolated_columns, run_update

pytestmark = pytest.mark.gpu

EVAL_TOL = 1e-10
RES_TOL = 1e-9
ORTH_TOL = 1e-9
VEC_TOL = 1e-8


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eu.load_library()


def _check_full(u, lo, Qo, ref_lam, ref_Q, vec_cols=None):
    A = wl.explicit_matrix(u.lam, u.Q, u.K, u.sigma)
    scale = max(np.abs(ref_lam).max(), 1e-300)
    n = lo.size
    assert np.all(np.diff(lo) >= 0.0)
    assert np.abs(lo - ref_lam).max() <= EVAL_TOL * scale
    if Qo is None:
        return
    res = np.abs(A @ Qo - Qo * lo).max()
    assert res <= RES_TOL * scale, res
    orth = np.abs(Qo.T @ Qo - np.eye(n)).max()
    assert orth <= ORTH_TOL, orth
    if ref_Q is not None:
        cols = isolated_columns(ref_lam, 1e-6, scale) if vec_cols is None else vec_cols
        if cols.size:
            Qa = align_signs(Qo[:, cols], ref_Q[:, cols])
            assert np.abs(Qa - ref_Q[:, cols]).max() <= VEC_TOL


@pytest.mark.parametrize("n,k", [(1, 1), (2, 1), (2, 2), (3, 2), (5, 3), (64, 1), (64, 2),
                                 (100, 4), (129, 2), (200, 8), (257, 5), (300, 3), (511, 2),
                                 (700, 6), (1000, 2)])
def test_update_matches_oracle(n, k):
    print(f"case n={n} k={k}", flush=True)
    u = wl.random_small(n, k, seed=1000 + 13 * n + k, knorm=1.5)
    lo, Qo, info, ex = run_update(u.lam, u.Q, u.K, u.sigma,
                                  fetch=(eu.EIG_DBG_U, eu.EIG_DBG_W))
    ref_lam, ref_Q, _ = oracle.update(u.lam, u.Q, u.K, u.sigma)
    # U = Q^T K
    Uo = oracle.qtk(u.Q, u.K)
    assert np.abs(ex[eu.EIG_DBG_U] - Uo).max() <= 1e-13 * max(1.0, np.abs(Uo).max())
    # Q' = Q W (isolates the GEMM)
    Wg = ex[eu.EIG_DBG_W]
    assert np.abs(np.asarray(u.Q) @ Wg - Qo).max() <= 1e-12
    _check_full(u, lo, Qo, ref_lam, ref_Q)
    assert info.generation == 1
    assert info.iters_max < 160


@pytest.mark.parametrize("n,k", [(40, 2), (150, 3), (400, 4), (333, 8)])
def test_pole_counts_match_oracle(n, k):
    print(f"case n={n} k={k}", flush=True)
    u = wl.random_small(n, k, seed=77 + n + k, knorm=2.0)
    lo, Qo, info, ex = run_update(u.lam, u.Q, u.K, u.sigma,
                                  fetch=(eu.EIG_DBG_POLE_COUNT, eu.EIG_DBG_SEG_START,
                                         eu.EIG_DBG_REDUCED_ROW))
    assert info.n_deflated_rows == 0 and info.n_segments == n
    U = oracle.qtk(u.Q, u.K)
    nu = ex[eu.EIG_DBG_POLE_COUNT]
    rows = ex[eu.EIG_DBG_REDUCED_ROW]
    ref = np.array([oracle.pole_count(u.lam, U, u.sigma, int(j)) for j in rows])
    assert np.array_equal(nu, ref)


def test_rank2_column_row_n200():
    """Plain rank-2 update e_j a^T + a e_j^T, n = 200 (Sec. 2.2, Steps 1-2)."""
    u = wl.plain_rank2(200, seed=1001)
    lo, Qo, info, _ = run_update(u.lam, u.Q, u.K, u.sigma)
    ref_lam, ref_Q, _ = oracle.update(u.lam, u.Q, u.K, u.sigma)
    _check_full(u, lo, Qo, ref_lam, ref_Q)
    assert info.p == 1 and info.q == 1


def test_values_only_mode():
    u = wl.random_small(300, 3, seed=5)
    lo, Qo, info, _ = run_update(u.lam, u.Q, u.K, u.sigma, values_only=True)
    ref_lam, _, _ = oracle.update(u.lam, u.Q, u.K, u.sigma, values_only=True)
    assert Qo is None
    assert np.abs(lo - ref_lam).max() <= EVAL_TOL * np.abs(ref_lam).max()
    assert info.generation == 0


def test_zero_perturbation_deflates_everything():
    n = 130
    u = wl.random_small(n, 2, seed=3)
    K = np.zeros((n, 2), order="F")
    lo, Qo, info, _ = run_update(u.lam, u.Q, K, u.sigma)
    assert info.n_deflated_rows == n
    assert np.array_equal(lo, u.lam)
    assert np.abs(Qo - np.asarray(u.Q)).max() <= 1e-15


def test_tiny_rows_deflate():
    n, k = 600, 2
    u = wl.random_small(n, k, seed=11)
    Qn = np.asarray(u.Q)
    U = Qn.T @ u.K
    rows = np.random.default_rng(1).choice(n, 30, replace=False)
    U[rows] *= (1e-14 / np.linalg.norm(U[rows], axis=1))[:, None]
    K = np.asfortranarray(Qn @ U)
    lo, Qo, info, _ = run_update(u.lam, Qn, K, u.sigma)
    assert info.n_deflated_rows == 30
    ref_lam, ref_Q, _ = oracle.update(u.lam, Qn, K, u.sigma)
    u2 = wl.Update(u.lam, Qn, K, u.sigma)
    _check_full(u2, lo, Qo, ref_lam, ref_Q)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_weakly_coupled_rows(k):
    """Rows of U with norms 1e-3 .. 1e-11, all above the deflation threshold: their
    roots lie within about ||u_j||^2 of their poles, where the evaluation of S
    loses relative accuracy in tau (the noise-floor stop of the root solver)."""
    print(f"case weakly coupled rows k={k}", flush=True)
    n = 400
    u = wl.random_small(n, k, seed=90 + k)
    Qn = np.asarray(u.Q)
    U = Qn.T @ u.K
    rng = np.random.default_rng(5 + k)
    rows = rng.choice(n, 50, replace=False)
    norms = 10.0 ** -rng.uniform(3.0, 11.0, rows.size)
    U[rows] *= (norms / np.linalg.norm(U[rows], axis=1))[:, None]
    K = np.asfortranarray(Qn @ U)
    lo, Qo, info, _ = run_update(u.lam, Qn, K, u.sigma)
    assert info.n_deflated_rows == 0
    ref_lam, ref_Q, _ = oracle.update(u.lam, Qn, K, u.sigma)
    _check_full(wl.Update(u.lam, Qn, K, u.sigma), lo, Qo, ref_lam, ref_Q)
    assert info.iters_max < 160


@pytest.mark.parametrize("e", [-300, 300])
@pytest.mark.parametrize("k", [2, 5])
def test_scale_invariance(e, k):
    """A' scaled by 2^e (lambda by 2^e, K by 2^(e/2)): powers of two scale exactly,
    so the update must return 2^e times the eigenvalues of the unscaled problem and
    the same eigenvectors, to the FP64 bar, with nothing overflowing or
    underflowing in the secular sums (u^2 ~ 2^e, 1/(x - d) ~ 2^-e, S' terms
    ~ 2^-e) -- and agree with the oracle on the scaled problem."""
    print(f"case scale 2^{e} k={k}", flush=True)
    n = 300
    u = wl.random_small(n, k, seed=700 + k, knorm=1.5)
    lam1, Q1, info1, _ = run_update(u.lam, u.Q, u.K, u.sigma)
    f = 2.0 ** e
    lam_s = u.lam * f
    K_s = np.asfortranarray(u.K * 2.0 ** (e // 2))
    lo, Qo, info, _ = run_update(lam_s, u.Q, K_s, u.sigma)
    assert info.n_deflated_rows == info1.n_deflated_rows
    scale = np.abs(lo).max()
    assert np.abs(lo - lam1 * f).max() <= EVAL_TOL * scale
    ref_lam, ref_Q, _ = oracle.update(lam_s, np.asarray(u.Q), K_s, u.sigma)
    _check_full(wl.Update(lam_s, u.Q, K_s, u.sigma), lo, Qo, ref_lam, ref_Q)
    cols = isolated_columns(lam1, 1e-6, np.abs(lam1).max())
    if cols.size:
        Qa = align_signs(Qo[:, cols], Q1[:, cols])
        assert np.abs(Qa - Q1[:, cols]).max() <= VEC_TOL


def test_equal_poles_group_deflation():
    """Groups of exactly equal poles: the m - k extra rows of each group deflate."""
    n, k = 200, 2
    rng = np.random.default_rng(17)
    lam = np.sort(rng.uniform(-1, 1, n))
    lam[50:55] = lam[50]          # group of 5
    lam[120:122] = lam[120]       # group of 2
    lam[190:] = lam[190]          # group of 10 at the top
    lam = np.sort(lam)
    Q = wl.orthogonal_from(rng.standard_normal((n, n)))
    K = np.asfortranarray(rng.standard_normal((n, k)) / np.sqrt(n))
    sig = np.array([1, -1], dtype=np.int8)
    lo, Qo, info, _ = run_update(lam, Q, K, sig)
    assert info.n_deflated_groups == 3
    assert info.n_deflated_rows == (5 - 2) + 0 + (10 - 2)
    A = wl.explicit_matrix(lam, Q, K, sig)
    ev = np.linalg.eigvalsh(A)
    scale = np.abs(ev).max()
    assert np.abs(lo - ev).max() <= EVAL_TOL * scale
    assert np.abs(A @ Qo - Qo * lo).max() <= RES_TOL * scale
    assert np.abs(Qo.T @ Qo - np.eye(n)).max() <= ORTH_TOL
    # the oracle's eigenvalues (it treats the ties without deflation)
    U = oracle.qtk(Q, K)
    vals, _, _, _ = oracle.eigvals(lam, U, sig)
    assert np.abs(lo - vals).max() <= EVAL_TOL * scale


@pytest.mark.parametrize("k", [1, 2, 4])
def test_zero_lambda_orthonormal_K(k):
    """Lambda = 0 (one group of n equal poles) and orthonormal K: eigenvalues
    {sigma_c} and n - k zeros."""
    n = 48
    rng = np.random.default_rng(k)
    Kq, _ = np.linalg.qr(rng.standard_normal((n, k)))
    sig = rng.choice(np.array([-1, 1], dtype=np.int8), k)
    Q = wl.orthogonal_from(rng.standard_normal((n, n)))
    K = np.asfortranarray(np.asarray(Q) @ Kq)
    lo, Qo, info, _ = run_update(np.zeros(n), Q, K, sig)
    expect = np.sort(np.concatenate([sig.astype(float), np.zeros(n - k)]))
    assert np.abs(lo - expect).max() <= 1e-13
    A = wl.explicit_matrix(np.zeros(n), Q, K, sig)
    assert np.abs(A @ Qo - Qo * lo).max() <= 1e-12
    assert np.abs(Qo.T @ Qo - np.eye(n)).max() <= 1e-12


def test_chained_updates_track_oracle():
    import torch

    n = 256
    rng = np.random.default_rng(99)
    u = wl.random_small(n, 2, seed=99)
    lam_r, Q_r = u.lam.copy(), np.asarray(u.Q).copy()
    dev = "cuda:0"
    with eu.EigState(n, 0) as s:
        s.upload(torch.as_tensor(u.lam, device=dev), colmajor(u.Q, dev))
        for step in range(12):
            k = [1, 2, 4, 8][step % 4]
            K = np.asfortranarray(rng.standard_normal((n, k)) / np.sqrt(n))
            sig = rng.choice(np.array([-1, 1], dtype=np.int8), k)
            s.update(colmajor(K, dev), sig)
            lam_r, Q_r, _ = oracle.update(lam_r, Q_r, K, sig)
        lo = torch.empty(n, dtype=torch.float64, device=dev)
        Qo = torch.empty((n, n), dtype=torch.float64, device=dev).t()
        info = s.query(lo, Qo)
    lo = lo.cpu().numpy()
    Qo = Qo.cpu().numpy()
    assert info.generation == 12
    scale = np.abs(lam_r).max()
    assert np.abs(lo - lam_r).max() <= EVAL_TOL * scale
    assert np.abs(Qo.T @ Qo - np.eye(n)).max() <= ORTH_TOL


def test_hundred_chained_updates_n512():
    """100 updates chained on one state (n = 512, ranks cycling through 1, 2, 4
    and 8, K ~ N(0, 1/n), random signs), against the oracle chained over the same
    updates, and against the explicit sum of all the perturbations: the drift of
    the committed decomposition stays at the FP64 bar after 100 commits."""
    import torch

    n, steps = 512, 100
    print(f"case 100 chained updates n={n}", flush=True)
    rng = np.random.default_rng(512)
    u = wl.random_small(n, 1, seed=512)
    lam_r, Q_r = u.lam.copy(), np.asarray(u.Q).copy()
    A = wl.explicit_matrix(u.lam, u.Q, np.zeros((n, 1)), np.array([1]))
    dev = "cuda:0"
    with eu.EigState(n, 0) as s:
        s.upload(torch.as_tensor(u.lam, device=dev), colmajor(u.Q, dev))
        for step in range(steps):
            k = [1, 2, 4, 8][step % 4]
            K = np.asfortranarray(rng.standard_normal((n, k)) / np.sqrt(n))
            sig = rng.choice(np.array([-1, 1], dtype=np.int8), k)
            s.update(colmajor(K, dev), sig)
            lam_r, Q_r, _ = oracle.update(lam_r, Q_r, K, sig)
            A += (K * sig.astype(float)) @ K.T
        lo = torch.empty(n, dtype=torch.float64, device=dev)
        Qo = torch.empty((n, n), dtype=torch.float64, device=dev).t()
        info = s.query(lo, Qo)
    lo, Qo = lo.cpu().numpy(), Qo.cpu().numpy()
    assert info.generation == steps
    A = (A + A.T) / 2.0
    scale = np.abs(lam_r).max()
    de = np.abs(lo - lam_r).max() / scale
    res = np.linalg.norm(A @ Qo - Qo * lo, axis=0).max() / scale
    orth = np.abs(Qo.T @ Qo - np.eye(n)).max()
    orth_ref = np.abs(Q_r.T @ Q_r - np.eye(n)).max()
    print(f"  after {steps} updates: eigenvalues vs oracle chain {de:.1e}, residual vs the "
          f"explicit A {res:.1e}, orthogonality {orth:.1e} (oracle chain {orth_ref:.1e})",
          flush=True)
    assert de <= EVAL_TOL
    assert res <= RES_TOL
    assert orth <= ORTH_TOL


def test_nonfinite_input_is_sticky_and_state_kept():
    import torch

    n = 80
    u = wl.random_small(n, 2, seed=21)
    dev = "cuda:0"
    with eu.EigState(n, 0) as s:
        s.upload(torch.as_tensor(u.lam, device=dev), colmajor(u.Q, dev))
        s.update(colmajor(u.K, dev), u.sigma)          # committed
        bad = np.array(u.K)
        bad[3, 1] = np.nan
        s.update(colmajor(bad, dev), u.sigma)          # fails on the device
        s.update(colmajor(u.K, dev), u.sigma)          # no-op after the failure
        lo = torch.empty(n, dtype=torch.float64, device=dev)
        with pytest.raises(eu.EigError) as e:
            s.query(lo)
        assert e.value.code == eu.EIG_ENONFINITE
        info = s.query(lo)                             # error cleared
        assert info.generation == 1
    ref_lam, _, _ = oracle.update(u.lam, u.Q, u.K, u.sigma, values_only=True)
    assert np.abs(lo.cpu().numpy() - ref_lam).max() <= EVAL_TOL * np.abs(ref_lam).max()


def test_argument_errors():
    import torch

    n = 16
    u = wl.random_small(n, 2, seed=2)
    dev = "cuda:0"
    with eu.EigState(n, 0) as s:
        with pytest.raises(eu.EigError) as e:
            s.update(colmajor(u.K, dev), u.sigma)
        assert e.value.code == eu.EIG_ESTATE
        with pytest.raises(eu.EigError) as e:
            s.upload(torch.as_tensor(u.lam[::-1].copy(), device=dev), colmajor(u.Q, dev))
        assert e.value.code == eu.EIG_ENOTSORTED
        s.upload(torch.as_tensor(u.lam, device=dev), colmajor(u.Q, dev))
        with pytest.raises(eu.EigError) as e:
            s.update(colmajor(u.K, dev), np.array([1, 0]))
        assert e.value.code == eu.EIG_EINVAL
        K33 = np.zeros((n, 33), order="F")
        with pytest.raises(eu.EigError) as e:
            s.update(colmajor(K33, dev), np.ones(33))
        assert e.value.code == eu.EIG_EUNSUPPORTED


def test_host_input_path():
    n = 90
    u = wl.random_small(n, 3, seed=8)
    import torch

    dev = "cuda:0"
    with eu.EigState(n, 0) as s:
        s.upload(u.lam, np.asfortranarray(u.Q))       # host upload
        s.update(np.asfortranarray(u.K), u.sigma)     # host K (EIG_HOST_INPUT)
        lo = np.empty(n)
        Qo = np.empty((n, n), order="F")
        s.query(lo, Qo)
    ref_lam, ref_Q, _ = oracle.update(u.lam, u.Q, u.K, u.sigma)
    _check_full(u, lo, Qo, ref_lam, ref_Q)


def test_double_root_away_from_poles():
    """Two decoupled rank-1 blocks sharing a root: an exact double eigenvalue inside
    one pole interval; the cluster branch must return orthonormal eigenvectors."""
    import math

    lam = np.array([0.0, 0.5, 1.0, 2.0])
    za = np.array([0.9, 0.3])
    f = lambda x: 1 + za[0] ** 2 / (0 - x) + za[1] ** 2 / (1 - x)
    lo_, hi_ = 1e-9, 1 - 1e-9
    for _ in range(200):
        mid = (lo_ + hi_) / 2
        if f(mid) < 0:
            lo_ = mid
        else:
            hi_ = mid
    r = (lo_ + hi_) / 2
    zb1 = 0.6
    zb3sq = -(1 + zb1 ** 2 / (0.5 - r)) * (2.0 - r)
    K = np.zeros((4, 2), order="F")
    K[0, 0], K[2, 0] = za
    K[1, 1], K[3, 1] = zb1, math.sqrt(zb3sq)
    sig = np.array([1, 1], dtype=np.int8)
    rng = np.random.default_rng(4)
    Q = wl.orthogonal_from(rng.standard_normal((4, 4)))
    Kq = np.asfortranarray(np.asarray(Q) @ K)
    lo, Qo, info, _ = run_update(lam, Q, Kq, sig)
    A = wl.explicit_matrix(lam, Q, Kq, sig)
    ev = np.linalg.eigvalsh(A)
    assert np.abs(lo - ev).max() <= 1e-14
    assert np.abs(Qo.T @ Qo - np.eye(4)).max() <= 1e-10
    assert np.abs(A @ Qo - Qo * lo).max() <= 1e-10


@pytest.mark.parametrize("k,m", [(3, 3), (6, 2), (6, 6), (7, 7), (8, 3), (8, 8)])
def test_multiple_root_cluster(k, m):
    """k decoupled rank-1 blocks, each with one pole at or below 0 and one at or
    above 1, m of them with their root at the same r in (0, 1): an m-fold
    eigenvalue inside one pole interval (the cluster branch for a group of m
    roots), next to k - m simple roots in the same interval.  Eigenvalues against
    LAPACK on the explicit matrix; residual and orthonormality of every column."""
    print(f"case multiple-root cluster k={k} m={m}", flush=True)
    r = 0.37
    lam = np.empty(2 * k)
    K = np.zeros((2 * k, k))
    for b in range(k):
        a, c = -0.1 * b, 1.0 + 0.1 * b
        rb = r if b < m else 0.05 + 0.9 * (b - m + 1) / (k - m + 1)
        za2 = 2.0 * (rb - a)  # 1 + za^2 / (a - rb) = -1
        lam[2 * b], lam[2 * b + 1] = a, c
        K[2 * b, b] = np.sqrt(za2)
        K[2 * b + 1, b] = np.sqrt(c - rb)  # f_b(rb) = -1 + zc^2 / (c - rb) = 0
    order = np.argsort(lam)
    lam, K = lam[order], K[order]
    sig = np.ones(k, dtype=np.int8)
    rng = np.random.default_rng(40 + k + m)
    Q = wl.orthogonal_from(rng.standard_normal((2 * k, 2 * k)))
    Kq = np.asfortranarray(np.asarray(Q) @ K)
    lo, Qo, info, _ = run_update(lam, Q, Kq, sig)
    A = wl.explicit_matrix(lam, Q, Kq, sig)
    ev = np.linalg.eigvalsh(A)
    assert np.sum(np.abs(ev - r) < 1e-12) == m
    assert np.abs(lo - ev).max() <= 1e-13
    assert np.abs(Qo.T @ Qo - np.eye(2 * k)).max() <= 1e-10
    assert np.abs(A @ Qo - Qo * lo).max() <= 1e-10
