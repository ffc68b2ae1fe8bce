"""GPU parity at the full sizes the benchmark runs (one update, same kernels and
launch configuration as bench.py), against the oracle, complete where the
oracle and the device can afford it:

- eigenvalues: ALL n of them against the oracle's count bisection, within
  1e-10 ||A'||_2; ascending, inside their Courant-Weyl windows (Sec. 2.2), and
  summing to the trace identity;
- residual: ||A' q - lambda q||_2 <= 1e-9 ||A'||_2 for EVERY column, A' Q'
  formed on the device in FP64 as Q (Lambda (Q^T Q')) + K (Sigma (K^T Q'));
- orthogonality: ||Q'^T Q' - I||_max <= 1e-9 over the whole matrix;
- eigenvectors: 256 seeded columns with isolated eigenvalues against the
  oracle's eq. (10) vectors times Q (the oracle's own product), up to sign.

Each workload runs with the dense product and with the far-field product
(EIG_QW_FARFIELD, the benchmark's default), the oracle computed once for both.
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
NVEC = 256
MODES = {"dense": 0, "farfield": eu.EIG_QW_FARFIELD}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eu.load_library()


class Case:
    """A workload on the device plus the oracle's answers for it."""

    def __init__(self, u, label):
        import torch

        self.u = u
        self.label = label
        n = u.lam.size
        self.n, self.k = n, u.K.shape[1]
        print(f"case {label}: n={n} k={self.k}: oracle", flush=True)
        self.Kt = torch.from_numpy(np.ascontiguousarray(np.asarray(u.K).T)).to("cuda:0").t()
        self.Qh = np.asfortranarray(u.Q.cpu().numpy())
        self.Kh = np.asfortranarray(np.asarray(u.K))
        self.U = oracle.qtk(self.Qh, self.Kh)
        self.scale = np.abs(u.lam).max() + float(np.sum(self.U * self.U))  # >= ||A'||_2
        self.vals, self.org, self.tau, _ = oracle.eigvals(u.lam, self.U, u.sigma)
        d = np.diff(self.vals)
        gaps = np.minimum(np.r_[d, np.inf], np.r_[np.inf, d])
        iso = np.nonzero(gaps > 1e-6 * self.scale)[0]
        rng = np.random.default_rng(n + self.k)
        self.cols = np.sort(rng.choice(iso, min(NVEC, iso.size), replace=False))
        Wv = oracle.eigvecs(u.lam, self.U, u.sigma, self.org[self.cols], self.tau[self.cols])
        self.Qref = oracle.gemm(self.Qh, Wv)


def _run(case, mode_name):
    import torch

    u, n, dev = case.u, case.n, "cuda:0"
    print(f"case {case.label} {mode_name}: update", flush=True)
    with eu.EigState(n, 0) as s:
        s.upload(torch.from_numpy(u.lam).to(dev), u.Q)
        s.update(case.Kt, u.sigma, MODES[mode_name])
        lo = torch.empty(n, dtype=torch.float64, device=dev)
        Qo = torch.empty((n, n), dtype=torch.float64, device=dev).t()
        info = s.query(lo, Qo)
    lam_g = lo.cpu().numpy()
    scale = case.scale
    # every eigenvalue against the oracle
    de = np.abs(lam_g - case.vals).max()
    assert de <= EVAL_TOL * scale, de
    assert np.all(np.diff(lam_g) >= 0.0)
    sig = u.sigma.astype(float)
    tr = float(np.sum(sig * np.sum(case.Kh * case.Kh, axis=0)))
    assert abs((lam_g.sum() - u.lam.sum()) - tr) <= 1e-12 * n * scale
    p, q = int(np.sum(sig > 0)), int(np.sum(sig < 0))
    tol = 1e-12 * scale
    i = np.arange(n)
    assert np.all(lam_g[i[i - q >= 0]] >= u.lam[i[i - q >= 0] - q] - tol)
    assert np.all(lam_g[i[i + p < n]] <= u.lam[i[i + p < n] + p] + tol)
    # residual of every column, on the device in FP64
    lam_t = torch.from_numpy(u.lam).to(dev)
    sig_t = torch.from_numpy(sig).to(dev)
    AQ = u.Q @ (lam_t[:, None] * (u.Q.t() @ Qo))
    AQ += case.Kt @ (sig_t[:, None] * (case.Kt.t() @ Qo))
    AQ -= Qo * lo[None, :]
    res = float(torch.linalg.vector_norm(AQ, dim=0).max())
    del AQ
    assert res <= RES_TOL * scale, res
    # orthogonality of the whole matrix
    G = Qo.t() @ Qo
    G.diagonal().sub_(1.0)
    orth = float(G.abs().max())
    del G
    assert orth <= ORTH_TOL, orth
    # isolated eigenvectors against the oracle's eq. (10) vectors times Q
    Qg = Qo[:, torch.as_tensor(case.cols, device=dev)].cpu().numpy()
    sgn = np.sign(np.sum(Qg * case.Qref, axis=0))
    dv = np.abs(Qg * sgn - case.Qref).max()
    assert dv <= VEC_TOL, dv
    print(f"  {mode_name}: eig {de / scale:.1e}  res {res / scale:.1e}  orth {orth:.1e}  "
          f"vec {dv:.1e} ({case.cols.size} columns)", flush=True)
    return info


@pytest.fixture(scope="module")
def headline():
    return Case(wl.headline(8192, device="cuda:0"), "rank-2 column-row n=8192")


@pytest.fixture(scope="module")
def rank4():
    return Case(wl.general_rankk(4, n=8192, device="cuda:0"), "rank-4 n=8192")


@pytest.fixture(scope="module")
def rank8():
    return Case(wl.general_rankk(8, n=8192, device="cuda:0"), "rank-8 n=8192")


@pytest.mark.parametrize("mode", list(MODES))
def test_headline_rank2_n8192(headline, mode):
    info = _run(headline, mode)
    assert info.p == 1 and info.q == 1


@pytest.mark.parametrize("mode", list(MODES))
def test_general_rank4_n8192(rank4, mode):
    _run(rank4, mode)


@pytest.mark.parametrize("mode", list(MODES))
def test_general_rank8_n8192(rank8, mode):
    _run(rank8, mode)


def test_clustered_rank2_n4096():
    case = Case(wl.clustered_rank2(4096, device="cuda:0"), "clustered rank-2 n=4096")
    for mode in MODES:
        info = _run(case, mode)
        # the rows rescaled to 1e-12 deflate
        assert info.n_deflated_rows >= case.u.tiny_rows.size
