"""Pins of the oracle's first-order perturbation estimate (Sec. 3, eq. (11),
reading G9; oracle/perturbation.py): an exact closed form, second-order
accuracy against LAPACK (numpy) as the perturbation shrinks, and a mutation
(the formula as printed) that the pins must reject.
"""
import numpy as np
import pytest

from oracle import perturbation
from paper_1706_00773_amd import workloads as wl


def test_diagonal_update_is_exact():
    n, j, kappa = 12, 5, 0.3
    lam = np.linspace(-1.0, 1.0, n)
    K = np.zeros((n, 1))
    K[j, 0] = kappa
    for s in (1, -1):
        lam_p, V = perturbation.perturb_first_order(lam, np.eye(n), K, [s])
        ref = lam.copy()
        ref[j] += s * kappa ** 2
        assert np.array_equal(lam_p, ref)
        assert np.array_equal(V, np.eye(n))


def _errors(lam, Q, K1, sig, delta):
    K = np.sqrt(delta) * K1
    lam_p, V = perturbation.perturb_first_order(lam, Q, K, sig)
    A = (Q * lam) @ Q.T + (K * sig) @ K.T
    w, X = np.linalg.eigh((A + A.T) / 2)
    # the spectrum is well separated: sorted order = original order
    e_val = np.abs(np.sort(lam_p) - w).max()
    order = np.argsort(lam_p)
    Vs = V[:, order]
    s = np.sign(np.sum(Vs * X, axis=0))
    e_vec = np.abs(Vs - X * s).max()
    return e_val, e_vec


@pytest.mark.parametrize("k,seed", [(1, 1), (2, 2), (4, 3)])
def test_second_order_accuracy(k, seed):
    n = 40
    rng = np.random.default_rng(seed)
    lam = np.sort(rng.uniform(-1.0, 1.0, n))
    lam = np.linspace(-1.0, 1.0, n) + 0.2 * (lam - lam.mean()) / n  # gaps ~ 0.05
    Q = wl.orthogonal_from(wl.gaussian_square(n, rng))
    K1 = rng.standard_normal((n, k)) / np.sqrt(n)
    sig = wl.random_signs(k, rng)
    e1 = _errors(lam, Q, K1, sig, 1e-3)
    e2 = _errors(lam, Q, K1, sig, 5e-4)
    # the neglected terms are second order in the perturbation size
    for a, b in zip(e1, e2):
        assert 3.0 < a / b < 5.0, (a, b)
        assert a < 1e-4


def _printed(lam, Q, K, sigma):
    """Eq. (11) exactly as printed: v_j^0 inside the sum, denominators lambda_i - lambda_j,
    no Sigma -- kept to show that the pins reject it."""
    U = Q.T @ np.asarray(K).reshape(lam.size, -1)
    n = lam.size
    lam_p = lam + np.sum(U * U, axis=1)
    V = Q.copy()
    for j in range(n):
        acc = 0.0
        for i in range(n):
            if i != j:
                acc += float(U[j] @ U[i]) / (lam[i] - lam[j])
        V[:, j] = Q[:, j] + acc * Q[:, j]
    return lam_p, V


def test_printed_form_is_rejected():
    n, k = 40, 2
    rng = np.random.default_rng(9)
    lam = np.linspace(-1.0, 1.0, n)
    Q = wl.orthogonal_from(wl.gaussian_square(n, rng))
    K = np.sqrt(1e-3) * rng.standard_normal((n, k)) / np.sqrt(n)
    sig = np.array([1, -1], dtype=np.int8)
    A = (Q * lam) @ Q.T + (K * sig) @ K.T
    w = np.linalg.eigvalsh((A + A.T) / 2)
    lam_ok, _ = perturbation.perturb_first_order(lam, Q, K, sig)
    lam_bad, _ = _printed(lam, Q, K, sig)
    assert np.abs(np.sort(lam_ok) - w).max() < 1e-6
    assert np.abs(np.sort(lam_bad) - w).max() > 1e-5
