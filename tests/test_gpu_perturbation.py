"""GPU parity of the first-order perturbation estimate (eig_perturb_first_order,
Sec. 3 eq. (11) as read) against the oracle's plain implementation
(oracle/perturbation.py, pinned in test_oracle_perturbation.py): the
eigenvalue estimates to rounding (1e-14 relative), the eigenvector estimates to
the rounding of an FP64 GEMM (1e-12), ties getting no first-order term, and
the state left unchanged.
"""
import numpy as np
import pytest

import oracle  # noqa: F401  (builds/loads the oracle package)
import paper_1706_00773_amd as eu
from oracle import perturbation
from paper_1706_00773_amd import workloads as wl

from helpers import colmajor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eu.load_library()


@pytest.mark.parametrize("n,k,ties", [(300, 1, False), (257, 3, False), (200, 8, False),
                                      (128, 2, True)])
def test_perturbation_matches_oracle(n, k, ties):
    import torch

    print(f"case perturbation n={n} k={k} ties={ties}", flush=True)
    u = wl.random_small(n, k, seed=900 + n + k, knorm=0.2)
    lam = u.lam.copy()
    if ties:
        lam[10:14] = lam[10]
        lam[50:52] = lam[50]
    with eu.EigState(n, 0) as s:
        s.upload(torch.from_numpy(lam).to("cuda:0"), colmajor(u.Q, "cuda:0"))
        lp, V = s.perturb_first_order(colmajor(u.K, "cuda:0"), u.sigma)
        info = s.query()
        assert info.generation == 0
        lam_now = torch.empty(n, dtype=torch.float64, device="cuda:0")
        s.query(lam_now)
        assert np.array_equal(lam_now.cpu().numpy(), lam)
    ref_l, ref_V = perturbation.perturb_first_order(lam, np.asarray(u.Q), u.K, u.sigma)
    assert np.abs(lp.cpu().numpy() - ref_l).max() <= 1e-14 * np.abs(ref_l).max()
    assert np.abs(V.cpu().numpy() - ref_V).max() <= 1e-12 * max(1.0, np.abs(ref_V).max())
