"""GPU parity of updates of rank 9 to 32 (EIG_KMAX < k <= EIG_KMAX_GENERIC),
which the library applies as ceil(k / 8) chained updates of rank <= 8.

Against the oracle's single rank-k solve of the same A' (its count bisection on
the k-by-k secular matrix, eq. (1), and eq. (10) vectors): every eigenvalue
within 1e-10 ||A'||_2, isolated eigenvectors within 1e-8, residual within
1e-9 ||A'||_2 and ||Q'^T Q' - I||_max within 1e-9.  At n = 8192 (ranks 16 and
32, the far-field product) a seeded sample of eigenvalues against the oracle
and every column's residual and orthogonality on the device.  The chain's
contract: all or nothing (a device error in a later part leaves the state as
it was), values-only equal to the full update's values, and the far-field and
dense products agreeing.
"""
import math

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


@pytest.mark.parametrize("n,k,seed", [(257, 9, 1), (700, 12, 2), (1024, 16, 3), (513, 24, 4),
                                      (300, 32, 5), (64, 32, 6)])
def test_generic_rank_vs_oracle(n, k, seed):
    print(f"case generic rank n={n} k={k}", flush=True)
    u = wl.general_rankk(k, n=n, seed=900 + seed)
    Q = np.asfortranarray(u.Q)
    lo, Qo, info, _ = run_update(u.lam, Q, u.K, u.sigma)
    ref_lam, ref_Q, _ = oracle.update(u.lam, Q, u.K, u.sigma)
    U = oracle.qtk(Q, u.K)
    scale = np.abs(u.lam).max() + float(np.sum(U * U))
    de = np.abs(lo - ref_lam).max() / scale
    assert de <= EVAL_TOL, de
    assert np.all(np.diff(lo) >= 0.0)
    cols = isolated_columns(ref_lam, 1e-6, scale)
    dv = 0.0
    if cols.size:
        dv = np.abs(align_signs(Qo[:, cols], ref_Q[:, cols]) - ref_Q[:, cols]).max()
        assert dv <= VEC_TOL, dv
    A = wl.explicit_matrix(u.lam, Q, u.K, u.sigma)
    res = np.linalg.norm(A @ Qo - Qo * lo, axis=0).max() / scale
    orth = np.abs(Qo.T @ Qo - np.eye(n)).max()
    print(f"  eig {de:.1e}  vec {dv:.1e} ({cols.size} columns)  res {res:.1e}  orth {orth:.1e}",
          flush=True)
    assert res <= RES_TOL and orth <= ORTH_TOL
    sig = np.asarray(u.sigma)
    assert info.k == k and info.p == int(np.sum(sig > 0)) and info.q == int(np.sum(sig < 0))
    assert info.generation == 1


def test_generic_rank_values_only_and_reduced_precision():
    """Values-only gives the full update's eigenvalues bitwise; the BF16x3 mode
    (two chained parts) keeps the eigenvalues at the FP64 bar and Q' within the
    reduced products' bound, twice (one product per part)."""
    import torch

    n, k = 600, 12
    print(f"case generic rank values-only / bf16x3 n={n} k={k}", flush=True)
    u = wl.general_rankk(k, n=n, seed=911)
    Q = np.asfortranarray(u.Q)
    l_full, Q_full, _, _ = run_update(u.lam, Q, u.K, u.sigma)
    l_vo, _, info, _ = run_update(u.lam, Q, u.K, u.sigma, values_only=True)
    assert np.array_equal(l_full, l_vo) and info.generation == 0
    l_lp, Q_lp, _, _ = run_update(u.lam, Q, u.K, u.sigma, prec=eu.EIG_GEMM_BF16X3_CORR)
    U = oracle.qtk(Q, u.K)
    scale = np.abs(u.lam).max() + float(np.sum(U * U))
    assert np.abs(l_lp - l_full).max() <= EVAL_TOL * scale
    bound = 2 * 2.0 * math.sqrt(n) * 4e-6
    assert np.abs(Q_lp.T @ Q_lp - np.eye(n)).max() <= bound
    A = wl.explicit_matrix(u.lam, Q, u.K, u.sigma)
    assert np.linalg.norm(A @ Q_lp - Q_lp * l_lp, axis=0).max() <= bound * scale


def test_generic_rank_failure_keeps_the_state():
    """A NaN in the last part's columns: the earlier parts ran, but nothing is
    committed; the next update applies to the original decomposition."""
    import torch

    dev = "cuda:0"
    n, k = 400, 20
    print(f"case generic rank failure n={n} k={k}", flush=True)
    u = wl.general_rankk(k, n=n, seed=913)
    Kbad = np.array(u.K)
    Kbad[5, 18] = np.nan
    with eu.EigState(n, 0) as s:
        s.upload(torch.from_numpy(u.lam).to(dev), colmajor(u.Q, dev))
        s.update(colmajor(Kbad, dev), u.sigma)
        with pytest.raises(eu.EigError) as e:
            s.query()
        assert e.value.code == eu.EIG_ENONFINITE
        lo = torch.empty(n, dtype=torch.float64, device=dev)
        Qo = torch.empty((n, n), dtype=torch.float64, device=dev).t()
        info = s.query(lo, Qo)
        assert info.generation == 0
        assert np.array_equal(lo.cpu().numpy(), u.lam)
        assert np.array_equal(Qo.cpu().numpy(), np.asarray(u.Q))
        s.update(colmajor(u.K, dev), u.sigma)
        info = s.query(lo, Qo)
        assert info.generation == 1
    l_ref, _, _, _ = run_update(u.lam, np.asfortranarray(u.Q), u.K, u.sigma)
    assert np.array_equal(lo.cpu().numpy(), l_ref)


def test_generic_rank_arguments():
    import torch

    dev = "cuda:0"
    n = 40
    u = wl.random_small(n, 1, seed=914)
    with eu.EigState(n, 0) as s:
        s.upload(torch.from_numpy(u.lam).to(dev), colmajor(u.Q, dev))
        for k, code in [(33, eu.EIG_EUNSUPPORTED), (n + 1, eu.EIG_EUNSUPPORTED)]:
            K = torch.zeros((k, n), dtype=torch.float64, device=dev).t()
            with pytest.raises(eu.EigError) as e:
                s.update(K, np.ones(k, dtype=np.int8))
            assert e.value.code == code
    with eu.EigState(20, 0) as s:
        u = wl.random_small(20, 1, seed=915)
        s.upload(torch.from_numpy(u.lam).to(dev), colmajor(u.Q, dev))
        K = torch.zeros((21, 20), dtype=torch.float64, device=dev).t()
        with pytest.raises(eu.EigError) as e:
            s.update(K, np.ones(21, dtype=np.int8))
        assert e.value.code == eu.EIG_EINVAL  # k > n


@pytest.mark.parametrize("k", [16, 32])
def test_generic_rank_n8192(k):
    """The rank-k workload at n = 8192 (lambda uniform in [-10, 10], K ~ N(0, 1/n),
    random signs) through the far-field product with the debug checks on: 48
    sampled eigenvalues against the oracle, every eigenvalue in its window, the
    trace identity, and every column's residual and orthogonality."""
    import torch

    dev = "cuda:0"
    n = 8192
    print(f"case generic rank n={n} k={k}", flush=True)
    u = wl.general_rankk(k, n=n, device=dev)
    Kt = colmajor(u.K, dev)
    with eu.EigState(n, 0) as s:
        s.upload(torch.from_numpy(u.lam).to(dev), u.Q)
        s.update(Kt, u.sigma, eu.EIG_QW_FARFIELD | eu.EIG_DEBUG_CHECKS)
        lo = torch.empty(n, dtype=torch.float64, device=dev)
        Qo = torch.empty((n, n), dtype=torch.float64, device=dev).t()
        s.query(lo, Qo)
    lam_g = lo.cpu().numpy()
    Qh = np.asfortranarray(u.Q.cpu().numpy())
    U = oracle.qtk(Qh, np.asarray(u.K))
    del Qh
    scale = np.abs(u.lam).max() + float(np.sum(U * U))
    rng = np.random.default_rng(k)
    idx = np.unique(np.r_[rng.choice(n, 48, replace=False), 0, n - 1])
    vals = oracle.eigvals(u.lam, U, u.sigma, idx)[0]
    de = np.abs(lam_g[idx] - vals).max() / scale
    assert de <= EVAL_TOL, de
    sig = u.sigma.astype(float)
    tr = float(np.sum(sig * np.sum(np.asarray(u.K) ** 2, axis=0)))
    assert abs((lam_g.sum() - u.lam.sum()) - tr) <= 1e-12 * n * scale
    p, q = int(np.sum(sig > 0)), int(np.sum(sig < 0))
    i = np.arange(n)
    t = 1e-12 * scale
    assert np.all(lam_g[i[i - q >= 0]] >= u.lam[i[i - q >= 0] - q] - t)
    assert np.all(lam_g[i[i + p < n]] <= u.lam[i[i + p < n] + p] + t)
    lam_t = torch.from_numpy(u.lam).to(dev)
    sig_t = torch.from_numpy(sig).to(dev)
    R = u.Q @ (lam_t[:, None] * (u.Q.t() @ Qo))
    R += Kt @ (sig_t[:, None] * (Kt.t() @ Qo))
    R -= Qo * lo[None, :]
    res = float(torch.linalg.vector_norm(R, dim=0).max()) / scale
    del R
    G = Qo.t() @ Qo
    G.diagonal().sub_(1.0)
    orth = float(G.abs().max())
    print(f"  eig {de:.1e} (sample)  res {res:.1e}  orth {orth:.1e}", flush=True)
    assert res <= RES_TOL and orth <= ORTH_TOL
