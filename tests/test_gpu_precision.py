"""GPU parity of the reduced-precision modes EIG_GEMM_FP32_CORR and
EIG_GEMM_BF16X3_CORR against the oracle.

What each mode must deliver:
- U = Q^T K after the FP64 residual correction: within 1e-13 max|U| of the
  oracle's FP64 product, as in the FP64 mode.  U0 alone (FP32-level) would
  miss this by about six orders of magnitude, so the check pins the correction.
- Eigenvalues: the FP64 bar, 1e-10 ||A'||_2.  They depend only on U.
- Q' = Q W: elementwise within QW_TOL of the FP64 product of the same Q and W
  (W fetched from the device).  The bound comes from the arithmetic: every
  entry of a k-slice partial sum is rounded to FP32 at most 32 times (16 k-steps
  of 3 products, or 6 MFMAs of 32-deep dot products), each rounding at most
  2^-24 sum_k |Q_ik||W_kj| <= 2^-24 (unit rows of Q, unit columns of W), and
  the splitting residual and dropped products add about 2^-24 more:
  (32 + 2) 2^-24 ~ 2.0e-6, doubled for the FP64 promotion sums -> 4e-6.
- Eigenvectors vs the oracle's (isolated eigenvalues, up to sign): the same
  bound plus the FP64 vector tolerance.
- Residual and orthogonality: ||dq||_2 <= sqrt(n) QW_TOL per column gives
  ||A'q - lambda q|| <= 2 sqrt(n) QW_TOL ||A'|| and |q_i^T q_j - delta_ij| <=
  2 sqrt(n) QW_TOL.
The measured errors are printed for the record.  n a multiple of 32 (64, 544,
1056) runs the BF16X3 product through its LDS-ring kernel, with partial tiles
at 544 and 1056.
"""
import math

import numpy as np
import pytest

import oracle
import paper_1706_00773_amd as eu
from paper_1706_00773_amd import workloads as wl

from helpers import align_signs, isolated_columns, run_update

pytestmark = pytest.mark.gpu

MODES = {"fp32": eu.EIG_GEMM_FP32_CORR, "bf16x3": eu.EIG_GEMM_BF16X3_CORR}
EVAL_TOL = 1e-10
QW_TOL = 4e-6
VEC_TOL = 1e-8


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eu.load_library()


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("n,k,seed", [(300, 4, 11), (301, 2, 12), (257, 8, 13), (64, 1, 14),
                                      (515, 3, 15), (544, 4, 16), (1056, 2, 17)])
def test_reduced_precision_vs_oracle(mode, n, k, seed):
    print(f"case mode={mode} n={n} k={k} seed={seed}", flush=True)
    u = wl.logspread_rankk(k, n=n, seed=seed)
    lo, Qo, info, ex = run_update(u.lam, u.Q, u.K, u.sigma, prec=MODES[mode],
                                  fetch=(eu.EIG_DBG_U, eu.EIG_DBG_W))
    Q = np.asfortranarray(u.Q)
    U = oracle.qtk(Q, u.K)
    du = np.abs(ex[eu.EIG_DBG_U] - U).max() / np.abs(U).max()
    assert du <= 1e-13, du
    ref_lam, ref_Q, _ = oracle.update(u.lam, Q, u.K, u.sigma)
    scale = np.abs(u.lam).max() + float(np.sum(U * U))
    assert np.all(np.diff(lo) >= 0.0)
    de = np.abs(lo - ref_lam).max() / scale
    assert de <= EVAL_TOL, de
    # the product alone: same Q and W in FP64
    W = ex[eu.EIG_DBG_W]
    dqw = np.abs(Q @ W - Qo).max()
    assert dqw <= QW_TOL, dqw
    cols = isolated_columns(ref_lam, 1e-6, scale)
    dv = 0.0
    if cols.size:
        Qa = align_signs(Qo[:, cols], ref_Q[:, cols])
        dv = np.abs(Qa - ref_Q[:, cols]).max()
        assert dv <= QW_TOL + VEC_TOL, dv
    A = wl.explicit_matrix(u.lam, Q, u.K, u.sigma)
    res = np.abs(A @ Qo - Qo * lo).max() / scale
    orth = np.abs(Qo.T @ Qo - np.eye(n)).max()
    bound = 2.0 * math.sqrt(n) * QW_TOL
    print(f"  U {du:.1e}  eig {de:.1e}  QW {dqw:.1e}  vec {dv:.1e}  res {res:.1e}  "
          f"orth {orth:.1e}", flush=True)
    assert res <= bound and orth <= bound
    assert info.generation == 1


@pytest.mark.parametrize("mode", list(MODES))
def test_reduced_precision_chained_and_values_only(mode):
    """Three chained updates in a reduced mode, then a values-only one; the
    eigenvalues track the oracle applied to the committed decomposition."""
    import torch

    n, k = 400, 3
    u = wl.logspread_rankk(k, n=n, seed=21)
    dev = "cuda:0"
    rng = np.random.default_rng(5)
    lam = u.lam.copy()
    with eu.EigState(n, 0) as s:
        s.upload(torch.from_numpy(lam).to(dev),
                 torch.from_numpy(np.ascontiguousarray(np.asarray(u.Q).T)).to(dev).t())
        for step in range(4):
            K = np.asfortranarray(rng.standard_normal((n, k)) / math.sqrt(n))
            sig = wl.random_signs(k, rng)
            lq = torch.empty(n, dtype=torch.float64, device=dev)
            Qq = torch.empty((n, n), dtype=torch.float64, device=dev).t()
            s.query(lq, Qq)
            lam_c, Q_c = lq.cpu().numpy(), np.asfortranarray(Qq.cpu().numpy())
            vo = step == 3
            s.update(torch.from_numpy(np.ascontiguousarray(K.T)).to(dev).t(), sig,
                     MODES[mode] | (eu.EIG_VALUES_ONLY if vo else 0))
            lo = torch.empty(n, dtype=torch.float64, device=dev)
            info = s.query(lo)
            ref, _, _ = oracle.update(lam_c, Q_c, K, sig, values_only=True)
            U = oracle.qtk(Q_c, K)
            scale = np.abs(lam_c).max() + float(np.sum(U * U))
            assert np.abs(lo.cpu().numpy() - ref).max() <= EVAL_TOL * scale
            assert info.generation == (3 if vo else step + 1)


def test_unknown_precision_selector_rejected():
    import torch

    n = 16
    u = wl.random_small(n, 1, seed=2)
    dev = "cuda:0"
    with eu.EigState(n, 0) as s:
        s.upload(torch.from_numpy(u.lam).to(dev),
                 torch.from_numpy(np.ascontiguousarray(np.asarray(u.Q).T)).to(dev).t())
        K = torch.zeros((1, n), dtype=torch.float64, device=dev).t()
        with pytest.raises(eu.EigError) as e:
            s.update(K, np.array([1]), eu.EIG_GEMM_MASK)
        assert e.value.code == eu.EIG_EUNSUPPORTED


@pytest.fixture(scope="module")
def logspread_n16384():
    """The n = 16384, k = 4 log-spread workload on the device, with the oracle's
    U, a seeded sample of 512 eigenvalues, and eq. (10) vectors in the Q basis
    for 256 sampled columns with isolated eigenvalues."""
    print("case logspread rank-4 n=16384: oracle", flush=True)
    u = wl.logspread_rankk(4, n=16384, device="cuda:0")
    n = u.lam.size
    Qh = np.asfortranarray(u.Q.cpu().numpy())
    U = oracle.qtk(Qh, u.K)
    del Qh
    scale = np.abs(u.lam).max() + float(np.sum(U * U))
    rng = np.random.default_rng(16384)
    idx = np.unique(np.r_[rng.choice(n, 512, replace=False), 0, n - 1])
    vals, org, tau, _ = oracle.eigvals(u.lam, U, u.sigma, idx)
    d = np.diff(vals)
    gaps = np.minimum(np.r_[d, np.inf], np.r_[np.inf, d])
    # a sampled value is isolated when its neighbours in the sample are far; the
    # device's own neighbours are checked in the test
    iso = np.nonzero(gaps > 1e-6 * scale)[0][:256]
    Wv = oracle.eigvecs(u.lam, U, u.sigma, org[iso], tau[iso])
    return dict(u=u, U=U, scale=scale, idx=idx, vals=vals, iso=iso, Wv=Wv)


@pytest.mark.parametrize("mode", list(MODES))
def test_reduced_precision_n16384(logspread_n16384, mode):
    """The mixed-precision workload at its full size (n = 16384, k = 4): U and the
    eigenvalues at the FP64 bar, Q W within QW_TOL of the FP64 product of the same
    Q and W, W's columns against the oracle's eq. (10) vectors, and the residual
    and orthogonality of every column within 2 sqrt(n) QW_TOL."""
    import torch

    c = logspread_n16384
    u, scale, dev = c["u"], c["scale"], "cuda:0"
    n, k = u.lam.size, u.K.shape[1]
    print(f"case mode={mode} n={n} k={k}: update", flush=True)
    Kt = torch.from_numpy(np.ascontiguousarray(np.asarray(u.K).T)).to(dev).t()
    with eu.EigState(n, 0) as s:
        s.upload(torch.from_numpy(u.lam).to(dev), u.Q)
        s.update(Kt, u.sigma, MODES[mode])
        lo = torch.empty(n, dtype=torch.float64, device=dev)
        Qo = torch.empty((n, n), dtype=torch.float64, device=dev).t()
        s.query(lo, Qo)
        Ug = s.fetch(eu.EIG_DBG_U, n * k).reshape(n, k)
        Wh = s.fetch(eu.EIG_DBG_W, n * n).reshape(n, n, order="F")
    du = np.abs(Ug - c["U"]).max() / np.abs(c["U"]).max()
    assert du <= 1e-13, du
    lam_g = lo.cpu().numpy()
    assert np.all(np.diff(lam_g) >= 0.0)
    de = np.abs(lam_g[c["idx"]] - c["vals"]).max() / scale
    assert de <= EVAL_TOL, de
    sig = u.sigma.astype(float)
    tr = float(np.sum(sig * np.sum(np.asarray(u.K) ** 2, axis=0)))
    assert abs((lam_g.sum() - u.lam.sum()) - tr) <= 1e-12 * n * scale
    # W's sampled columns (isolated on the device too) against the oracle's vectors
    cols = c["idx"][c["iso"]]
    d = np.diff(lam_g)
    gaps = np.minimum(np.r_[d, np.inf], np.r_[np.inf, d])
    keep = gaps[cols] > 1e-6 * scale
    Wg = Wh[:, cols[keep]]
    Wr = c["Wv"][:, keep]
    sgn = np.sign(np.sum(Wg * Wr, axis=0))
    dv = np.abs(Wg * sgn - Wr).max()
    assert dv <= VEC_TOL, dv
    # the reduced product against the FP64 product of the same Q and W
    W_t = torch.from_numpy(np.ascontiguousarray(Wh.T)).to(dev).t()
    del Wh
    dqw = float((u.Q @ W_t - Qo).abs().max())
    del W_t
    assert dqw <= QW_TOL, dqw
    # residual of every column and orthogonality of the whole matrix
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
    del G
    bound = 2.0 * math.sqrt(n) * QW_TOL
    print(f"  U {du:.1e}  eig {de:.1e}  QW {dqw:.1e}  W-vec {dv:.1e} ({int(keep.sum())} cols)  "
          f"res {res:.1e}  orth {orth:.1e}", flush=True)
    assert res <= bound and orth <= bound
