"""Pins of the oracle's rank-2 location by residue signs (Sec. 2.2, Alg. 1a-1c,
oracle/location.py) against computations that do not use the signs: the
oracle's bordered-inertia pole counts (independent code), exact-rational Sturm
counts of A' on dyadic inputs, and the Courant-Weyl bounds.  A mutated rule
(the printed Alg. 1c threshold M + 2 <= t) must fail, so the pin
discriminates.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import location, sturm_exact
from paper_1706_00773_amd import workloads as wl

SIGNS = [(1, 1), (1, -1), (-1, 1), (-1, -1)]


def _instance(n, sig, seed, scale=1.0):
    u = wl.random_small(n, 2, seed=seed, knorm=scale)
    U = oracle.qtk(u.Q, u.K)
    return u.lam, U, np.array(sig, dtype=np.int8)


@pytest.mark.parametrize("sig", SIGNS)
@pytest.mark.parametrize("n,seed,scale", [(7, 1, 1.0), (20, 2, 1.5), (60, 3, 3.0), (120, 4, 0.5)])
def test_alg1_matches_pole_counts(sig, n, seed, scale):
    lam, U, s = _instance(n, sig, seed + 10 * SIGNS.index(sig), scale)
    L = location.location_alg1(lam, U, s)
    assert L.sum() == n and np.all((L >= 0) & (L <= 2))
    nu = location.counts_from_location(L)
    ref = np.array([oracle.pole_count(lam, U, s, j) for j in range(n)])
    assert np.array_equal(nu, ref)
    # Courant-Weyl: nu(lambda_j) in [j + 1 - p, j + q]
    p, q = int(np.sum(s > 0)), int(np.sum(s < 0))
    j = np.arange(n)
    assert np.all(nu >= np.maximum(j + 1 - p, 0)) and np.all(nu <= j + q)


def _dyadic(n, seed, sig):
    rng = np.random.default_rng(seed)
    lam = np.sort(rng.choice(np.arange(-40, 41), size=n, replace=False)) / 8.0
    U = rng.integers(-6, 7, size=(n, 2)) / 4.0
    for r in range(n):
        if not U[r].any():
            U[r, 0] = 0.25
    s = np.array(sig, dtype=np.int8)
    A = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        A[i][i] += Fraction(lam[i])
        for jj in range(n):
            A[i][jj] += sum(Fraction(U[i, c]) * int(s[c]) * Fraction(U[jj, c]) for c in range(2))
    return lam, U, s, A


@pytest.mark.parametrize("n,seed", [(4, 21), (5, 22), (6, 23), (6, 24)])
@pytest.mark.parametrize("sig", SIGNS)
def test_alg1_matches_exact_sturm(n, seed, sig):
    lam, U, s, A = _dyadic(n, seed, sig)
    if any(sturm_exact.is_root(A, lam[j]) for j in range(n)):
        pytest.skip("an eigenvalue of A' coincides with a pole")
    try:
        L = location.location_alg1(lam, U, s)
    except ValueError:
        pytest.skip("a residue is zero")
    nu = location.counts_from_location(L)
    for j in range(n):
        assert nu[j] == sturm_exact.count_below(A, lam[j]), j


def _printed_1c(lam, U, sig):
    """Alg. 1c with the threshold as printed (M + 2 <= t): kept only to show the pin
    catches it."""
    a = location.alphas(lam, U, sig)
    mu = np.concatenate([[-1.0], np.sign(a), [1.0]])
    n = lam.size
    L = np.zeros(n + 1, dtype=np.int64)
    M = 0
    for t in range(n + 1):
        if mu[t] * mu[t + 1] > 0:
            L[t] = 1
            M += 1
        elif M + 2 <= t:
            L[t] = 2
            M += 2
    return L


def test_printed_alg1c_threshold_is_caught():
    wrong = 0
    for seed in range(40):
        lam, U, s = _instance(30, (1, -1), 500 + seed, 2.0)
        ref = np.array([oracle.pole_count(lam, U, s, j) for j in range(lam.size)])
        if not np.array_equal(location.counts_from_location(_printed_1c(lam, U, s)), ref):
            wrong += 1
    assert wrong > 0


def test_alg1_rejects_other_ranks():
    lam, U, s = _instance(10, (1, 1), 5)
    with pytest.raises(ValueError):
        location.location_alg1(lam, np.hstack([U, U[:, :1]]), np.array([1, 1, 1], np.int8))
