"""GPU parity at the full sizes the benchmark runs (one update, same kernels and
launch configuration as bench.py), against the oracle on sampled outputs that it
computes one by one, plus invariants that hold at any size:

- eigenvalues: 64 seeded indices (and the extremes) vs the oracle's bisection,
  within 1e-10 ||A'||_2; all eigenvalues ascending, inside their Courant-Weyl
  windows, and summing to the trace identity;
- eigenvectors: 16 seeded columns vs the oracle's eq. (10) vectors times Q (up to
  sign, isolated eigenvalues), residual ||A' q - lambda q|| <= 1e-9 ||A'||_2 on 64
  columns, ||Q_S^T Q_S - I||_max <= 1e-9 on a 512-column sample.
"""
import numpy as np
import pytest

import oracle
import paper_1706_00773_amd as eu
from paper_1706_00773_amd import workloads as wl

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


def _run_fullsize(u, label):
    import torch

    dev = "cuda:0"
    n = u.lam.size
    k = u.K.shape[1]
    print(f"case {label}: n={n} k={k}", flush=True)
    Kt = torch.from_numpy(np.ascontiguousarray(np.asarray(u.K).T)).to(dev).t()
    with eu.EigState(n, 0) as s:
        s.upload(torch.from_numpy(u.lam).to(dev), u.Q)
        s.update(Kt, u.sigma)
        lo = torch.empty(n, dtype=torch.float64, device=dev)
        Qo = torch.empty((n, n), dtype=torch.float64, device=dev).t()
        info = s.query(lo, Qo)
    lam_g = lo.cpu().numpy()
    Qh = np.asfortranarray(u.Q.cpu().numpy())
    Kh = np.asfortranarray(np.asarray(u.K))
    U = oracle.qtk(Qh, Kh)
    scale = np.abs(u.lam).max() + float(np.sum(U * U))  # >= ||A'||_2
    rng = np.random.default_rng(n + k)
    # eigenvalues: sampled indices and the extremes
    idx = np.unique(np.concatenate([rng.choice(n, 64, replace=False), [0, n - 1]]))
    vals, org, tau, _ = oracle.eigvals(u.lam, U, u.sigma, idx)
    assert np.abs(lam_g[idx] - vals).max() <= EVAL_TOL * scale
    assert np.all(np.diff(lam_g) >= 0.0)
    sig = u.sigma.astype(float)
    tr = float(np.sum(sig * np.sum(Kh * Kh, axis=0)))
    assert abs((lam_g.sum() - u.lam.sum()) - tr) <= 1e-12 * n * scale
    p, q = int(np.sum(sig > 0)), int(np.sum(sig < 0))
    tol = 1e-12 * scale
    i = np.arange(n)
    assert np.all(lam_g[i[i - q >= 0]] >= u.lam[i[i - q >= 0] - q] - tol)
    assert np.all(lam_g[i[i + p < n]] <= u.lam[i[i + p < n] + p] + tol)
    # eigenvectors: oracle vectors (eq. (10)) for 16 isolated sampled columns
    d = np.diff(lam_g)
    gaps = np.minimum(np.r_[d, np.inf], np.r_[np.inf, d])
    iso = [t for t in range(idx.size) if gaps[idx[t]] > 1e-6 * scale][:16]
    cols = idx[iso]
    Wv = oracle.eigvecs(u.lam, U, u.sigma, org[iso], tau[iso])
    Qref = oracle.gemm(Qh, Wv)
    Qg = Qo[:, torch_index(cols)].cpu().numpy()
    sgn = np.sign(np.sum(Qg * Qref, axis=0))
    assert np.abs(Qg * sgn - Qref).max() <= VEC_TOL
    # residual on 64 columns, computed on the device in FP64
    import torch

    dev = "cuda:0"
    c64 = torch.as_tensor(idx[:64], device=dev)
    Qs = Qo[:, c64]
    lam_t = torch.from_numpy(u.lam).to(dev)
    sig_t = torch.from_numpy(sig).to(dev)
    AQs = u.Q @ (lam_t[:, None] * (u.Q.t() @ Qs)) + Kt @ (sig_t[:, None] * (Kt.t() @ Qs))
    res = float((AQs - Qs * lo[c64][None, :]).abs().max())
    assert res <= RES_TOL * scale, res
    # orthogonality on 512 columns
    c512 = torch.as_tensor(np.sort(rng.choice(n, 512, replace=False)), device=dev)
    Qb = Qo[:, c512]
    orth = float((Qb.t() @ Qb - torch.eye(512, dtype=torch.float64, device=dev)).abs().max())
    assert orth <= ORTH_TOL, orth
    return info


def torch_index(cols):
    import torch

    return torch.as_tensor(np.asarray(cols), device="cuda:0")


def test_headline_rank2_n8192():
    u = wl.headline(8192, device="cuda:0")
    info = _run_fullsize(u, "rank-2 column-row n=8192")
    assert info.p == 1 and info.q == 1


def test_clustered_rank2_n4096():
    u = wl.clustered_rank2(4096, device="cuda:0")
    info = _run_fullsize(u, "clustered rank-2 n=4096")
    # the rows rescaled to 1e-12 deflate
    assert info.n_deflated_rows >= u.tiny_rows.size


@pytest.mark.parametrize("k", [4, 8])
def test_general_rankk_n8192(k):
    u = wl.general_rankk(k, n=8192, device="cuda:0")
    _run_fullsize(u, f"rank-{k} n=8192")
