"""Pins of the oracle's secular Sturm chain (Sec. 2.2, eqs. (4)-(9),
oracle/sturm_chain.py) against computations that do not use the secular form:

- the classical Sturm sequence of the polynomial prod (x - xi_i), built by exact
  rational polynomial division (oracle/sturm_exact.py); every secular member
  p_m = f_m pi_m must equal it exactly, as a polynomial;
- the characteristic polynomial of an explicit small A' = D + U Sigma U^T, whose
  quotient by prod (x - d_j) fixes the residues exactly (alpha_j = -p(d_j) / pi'(d_j)),
  and exact eigenvalue counts of that matrix;
- the fp64 oracle residues of eq. (2), through the identity
  det(I - Sigma U^T (xI - D)^{-1} U) = 1 - sum_j alpha_j / (x - d_j);
- exact found-root deflation (eq. (9)) on rational zeros.

A mutated division step (B_m with the printed sign) must fail the first pin.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import sturm_chain as sc
from oracle import sturm_exact as se
from paper_1706_00773_amd import workloads as wl


def _poly_from_roots(xi):
    p = [Fraction(1)]
    for r in xi:
        q = [Fraction(0)] * (len(p) + 1)
        for i, c in enumerate(p):
            q[i + 1] += c
            q[i] -= c * r
        p = q
    return p


def _peval(p, x):
    s = Fraction(0)
    for c in reversed(p):
        s = s * x + c
    return s


def _residues(p, d):
    """alpha_j of f = p / prod (x - d_j) = 1 - sum alpha_j / (x - d_j) (p monic, deg N)."""
    out = []
    for j, dj in enumerate(d):
        den = Fraction(1)
        for l, dl in enumerate(d):
            if l != j:
                den *= dj - dl
        out.append(-_peval(p, dj) / den)
    return out


def _member_value(ch, m, x):
    d = ch.d
    N = d.size
    f = ch.c[m] - sum((a / (x - dj) for a, dj in zip(ch.alpha[m], d[: N - m])), Fraction(0))
    pi = Fraction(1)
    for dj in d[: N - m]:
        pi *= x - dj
    return f * pi


def _rational_case(seed, N):
    rng = np.random.default_rng(seed)
    grid = np.sort(rng.choice(np.arange(-60, 61), size=2 * N + 1, replace=False))
    # interlaced-ish distinct poles and zeros on a grid of eighths
    d = [Fraction(int(v), 8) for v in grid[0::2][:N]]
    xi = [Fraction(int(v), 8) for v in grid[1::2][:N]]
    return d, xi


@pytest.mark.parametrize("seed,N", [(1, 3), (2, 5), (3, 6), (4, 8), (5, 9)])
def test_members_equal_classical_sturm_sequence(seed, N):
    d, xi = _rational_case(seed, N)
    p0 = _poly_from_roots(xi)
    ch = sc.build(d, _residues(p0, d), exact=True)
    seq = se.sturm_sequence(p0)
    assert ch.complete and ch.levels == N + 1 == len(seq)
    pts = [Fraction(2 * k + 1, 17) for k in range(-9, 9)]
    for m in range(N + 1):
        for x in pts:
            if x in d:
                continue
            assert _member_value(ch, m, x) == _peval(seq[m], x), (m, x)
    # every leading coefficient of a real-rooted p_0's sequence is positive
    assert all(c > 0 for c in ch.c)


def _printed_bm_chain(d, alpha):
    """The division step with B_m as printed (its sign flipped); exact."""
    d = [Fraction(v) for v in d]
    a = [Fraction(v) for v in alpha]
    ch = sc.build(d, a, exact=True, stop_nonpositive=False)
    N = len(d)
    cs, als = ch.c[:2], ch.alpha[:2]
    dd = np.array(d, dtype=object)
    for m in range(2, N + 1):
        e1, e2 = dd[N - m], dd[N - m + 1]
        am2, am1, c2, c1 = als[m - 2], als[m - 1], cs[m - 2], cs[m - 1]
        B = -(e2 + sum(am2, Fraction(0)) / c2 - sum(am1, Fraction(0)) / c1)
        A = c2 / c1
        dj = dd[: N - m]
        als.append(-am2[: N - m] * (dj - e1) * (dj - e2) + A * (dj - B) * am1[: N - m] * (dj - e1))
        s1_2, s1_1 = sum(am2, Fraction(0)), sum(am1, Fraction(0))
        s2_2 = sum(am2 * dd[: N - m + 2], Fraction(0))
        s2_1 = sum(am1 * dd[: N - m + 1], Fraction(0))
        cs.append(-(c2 * e1 * e2 + s1_2 * (e1 + e2) - s2_2) + A * (c1 * B * e1 + s1_1 * (B + e1) - s2_1))
    return sc.Chain(dd, cs, als, False)


def test_printed_division_sign_is_rejected():
    d, xi = _rational_case(4, 8)
    p0 = _poly_from_roots(xi)
    bad = _printed_bm_chain(d, _residues(p0, d))
    seq = se.sturm_sequence(p0)
    x = Fraction(3, 17)
    assert any(_member_value(bad, m, x) != _peval(seq[m], x) for m in range(2, 9))


def _dyadic_update(n, k, seed):
    rng = np.random.default_rng(seed)
    lam = np.sort(rng.choice(np.arange(-40, 41), size=n, replace=False)) / 8.0
    U = rng.integers(-6, 7, size=(n, k)) / 4.0
    U[np.all(U == 0, axis=1), 0] = 0.25
    sig = np.where(rng.random(k) < 0.5, 1, -1).astype(np.int8)
    A = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        A[i][i] += Fraction(lam[i])
        for j in range(n):
            A[i][j] += sum(Fraction(U[i, c]) * int(sig[c]) * Fraction(U[j, c]) for c in range(k))
    return lam, U, sig, A


@pytest.mark.parametrize("n,k,seed", [(5, 2, 1), (6, 3, 2), (7, 3, 3), (6, 4, 4)])
def test_counts_match_exact_counts_of_the_matrix(n, k, seed):
    lam, U, sig, A = _dyadic_update(n, k, seed)
    p0 = se.charpoly(A)
    d = [Fraction(v) for v in lam]
    alpha = _residues(p0, d)
    if any(a == 0 for a in alpha):
        pytest.skip("an eigenvalue of A' sits on a pole")
    # p_0 = det(xI - A') must have simple zeros for the classical count
    ch = sc.build(d, alpha, exact=True)
    if not ch.complete:
        pytest.skip("A' has a repeated eigenvalue")
    chf = sc.build(lam, [float(a) for a in alpha])
    assert chf.complete
    for x in [Fraction(2 * t + 1, 16) for t in range(-40, 40)]:
        if se.is_root(A, x) or x in d:
            continue
        ref = se.count_below(A, x)
        assert sc.count_below(ch, x) == ref
        assert sc.count_below(chf, float(x)) == ref
    # the fp64 chain follows the exact one closely at this size
    for ce, cf in zip(ch.c, chf.c):
        assert abs(float(ce) - cf) <= 1e-9 * abs(float(ce))


@pytest.mark.parametrize("k,seed", [(1, 1), (2, 2), (3, 3), (5, 4)])
def test_fp64_residues_reproduce_the_secular_determinant(k, seed):
    u = wl.random_small(30, k, seed=seed)
    U = oracle.qtk(u.Q, u.K)
    a = np.array([oracle.alpha(u.lam, U, u.sigma, i) for i in range(u.lam.size)])
    rng = np.random.default_rng(seed)
    for x in rng.uniform(-1.5, 1.5, 20):
        f = oracle.secular_det(u.lam, U, u.sigma, x)
        g = 1.0 - np.sum(a / (x - u.lam))
        scale = 1.0 + np.sum(np.abs(a / (x - u.lam)))
        assert abs(f - g) <= 1e-11 * scale


@pytest.mark.parametrize("k,seed", [(2, 5), (3, 6), (4, 7)])
def test_fp64_chain_counts_match_the_oracle_counts(k, seed):
    n = 24
    u = wl.random_small(n, k, seed=seed)
    U = oracle.qtk(u.Q, u.K)
    a = np.array([oracle.alpha(u.lam, U, u.sigma, i) for i in range(n)])
    ch = sc.build(u.lam, a)
    assert ch.complete
    ev = np.sort(oracle.eigvals(u.lam, U, u.sigma)[0])
    rng = np.random.default_rng(seed)
    for x in np.concatenate([rng.uniform(ev[0] - 0.5, ev[-1] + 0.5, 30), (ev[1:] + ev[:-1]) / 2]):
        if np.min(np.abs(ev - x)) < 1e-9 or np.min(np.abs(u.lam - x)) < 1e-12:
            continue
        assert sc.count_below(ch, x) == int(np.sum(ev < x))
        assert sc.count_below(ch, x) == oracle.count(u.lam, U, u.sigma, x)


def test_partial_chain_stops_at_first_nonpositive_c():
    # a large, badly scaled problem: the fp64 chain breaks down before m = N
    u = wl.random_small(160, 3, seed=11)
    U = oracle.qtk(u.Q, u.K)
    a = np.array([oracle.alpha(u.lam, U, u.sigma, i) for i in range(u.lam.size)])
    ch = sc.build(u.lam, a)
    if ch.complete:
        pytest.skip("the chain did not break down at this size")
    assert all(c > 0 for c in ch.c[:-1]) and not ch.c[-1] > 0
    assert sc.lower_bound(ch) == ch.levels - 2


@pytest.mark.parametrize("seed,N,s", [(1, 6, 2), (2, 8, 3), (3, 9, 5)])
def test_found_root_deflation_is_exact(seed, N, s):
    d, xi = _rational_case(seed, N)
    p0 = _poly_from_roots(xi)
    alpha = _residues(p0, d)
    found = xi[:s]
    d2, beta = sc.deflate_found(d, alpha, found, exact=True)
    assert list(d2) == d[s:]
    rest = _poly_from_roots(xi[s:])
    for x in [Fraction(2 * t + 1, 23) for t in range(-12, 12)]:
        if x in d:
            continue
        f2 = 1 - sum((b / (x - dj) for b, dj in zip(beta, d2)), Fraction(0))
        pi2 = Fraction(1)
        for dj in d2:
            pi2 *= x - dj
        assert f2 * pi2 == _peval(rest, x)
    # and the deflated chain counts the remaining zeros
    ch = sc.build(d2, beta, exact=True)
    assert ch.complete
    for x in [Fraction(t, 7) for t in range(-60, 61, 7)]:
        if x in d2 or x in xi:
            continue
        assert sc.count_below(ch, x) + sum(1 for r in found if r < x) == sum(1 for r in xi if r < x)
