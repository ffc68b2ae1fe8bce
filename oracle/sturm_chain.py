"""Secular Sturm chain (Sec. 2.2, eqs. (4)-(9)) -- TEST INFRASTRUCTURE ONLY
(see oracle/__init__.py).

The secular function of the update, f_0(x) = 1 - sum_j alpha_j / (x - d_j)
(eq. (4); alpha_j the residues of eq. (2), d_j distinct poles in ascending
order), times pi_0(x) = prod_j (x - d_j) is the degree-N polynomial p_0 whose
zeros are the eigenvalues.  Every member of its Sturm sequence is kept in the
same secular form,

    p_m(x) = f_m(x) pi_m(x),  f_m(x) = c_m - sum_{j < N-m} alpha^m_j / (x - d_j),
    pi_m(x) = prod_{j < N-m} (x - d_j)            (poles 0-based here),

so a member is N - m + 1 numbers and its sign at x needs no polynomial
coefficients.

  m = 1, p_1 = p_0' (eq. (6)): mu_j = 1 - sum_{i != j} (alpha_i + alpha_j) / (d_j - d_i),
         c_1 = sum_j mu_j, alpha^1_j = (d_{N-1} - d_j) mu_j (the last pole drops out).
  m >= 2, the secular long division p_m = -p_{m-2} + A_m (x - B_m) p_{m-1}:
         with e1 = d_{N-m} (dropped at this level) and e2 = d_{N-m+1} (dropped at the
         one before), and S1^l = sum_j alpha^l_j, S2^l = sum_j alpha^l_j d_j,
           A_m = c_{m-2} / c_{m-1},
           B_m = e2 + S1^{m-2} / c_{m-2} - S1^{m-1} / c_{m-1}        (reading G5),
           alpha^m_j = -alpha^{m-2}_j (d_j - e1)(d_j - e2)
                       + A_m (d_j - B_m) alpha^{m-1}_j (d_j - e1),
           c_m = -(c_{m-2} e1 e2 + S1^{m-2} (e1 + e2) - S2^{m-2})
                 + A_m (c_{m-1} B_m e1 + S1^{m-1} (B_m + e1) - S2^{m-1}).
         A_m and B_m cancel the x^2 and x terms of the right-hand side at infinity;
         the residues at d_j and the constant term follow from that expansion.  The
         printed B_m has the opposite sign throughout (a mutation the pins reject);
         the alpha^m and c_m recurrences are not printed and are derived here.

The number of zeros below x is V(-inf) - V(x), V the number of sign changes of
p_0(x), ..., p_N(x) (the classical theorem the section builds on).  At +inf the
signs are those of c_m, at -inf those of (-1)^(N-m) c_m.  The construction
stops at the first non-positive c_m, as the section prescribes; the chain is
then partial and its positive c's give only a lower bound on the zeros.

Found-root deflation (eqs. (7)-(9)): dividing p_0 by (x - xi_p) for zeros xi_p
already known and removing one pole d_p per zero gives again a secular
function, with residues beta_j = alpha_j prod_p (d_j - d_p) / (d_j - xi_p) on
the remaining poles.  The pairing of zeros with poles is not stated (reading
G6); here the s known zeros are paired in order with the s lowest poles.

The functions are written over generic numbers: numpy float64 arrays for the
oracle's floating-point chain, or object arrays of Fractions for exact pins.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


class Chain:
    """c[m] for m = 0..M and alpha[m] (N - m entries), the poles d, and whether
    the construction reached m = N with every c positive."""

    def __init__(self, d, c, alpha, complete):
        self.d = d
        self.c = c
        self.alpha = alpha
        self.complete = complete

    @property
    def levels(self) -> int:
        """M + 1: the number of members built (all with c_m > 0 except possibly
        the last, which is where the construction stopped)."""
        return len(self.c)


def _arr(v, exact):
    if exact:
        return np.array([Fraction(x) for x in v], dtype=object)
    return np.asarray(v, dtype=np.float64).copy()


def build(d, alpha, exact: bool = False, stop_nonpositive: bool = True) -> Chain:
    """The secular Sturm chain of f_0 = 1 - sum alpha_j / (x - d_j)."""
    d = _arr(d, exact)
    a0 = _arr(alpha, exact)
    N = d.size
    if N == 0:
        return Chain(d, [1], [a0], True)
    if np.any(d[1:] <= d[:-1]):
        raise ValueError("the poles must be distinct and ascending")
    one = Fraction(1) if exact else 1.0
    cs = [one]
    als = [a0]
    # m = 1: p_1 = p_0'
    mu = np.empty(N, dtype=object if exact else np.float64)
    for j in range(N):
        acc = one
        for i in range(N):
            if i != j:
                acc = acc - (a0[i] + a0[j]) / (d[j] - d[i])
        mu[j] = acc
    c1 = sum(mu, Fraction(0) if exact else 0.0)
    a1 = (d[N - 1] - d[: N - 1]) * mu[: N - 1]
    cs.append(c1)
    als.append(a1)
    if stop_nonpositive and not c1 > 0:
        return Chain(d, cs, als, False)
    for m in range(2, N + 1):
        e1, e2 = d[N - m], d[N - m + 1]
        am2, am1 = als[m - 2], als[m - 1]
        c2, c1 = cs[m - 2], cs[m - 1]
        s1_2 = sum(am2, Fraction(0) if exact else 0.0)
        s2_2 = sum(am2 * d[: N - m + 2], Fraction(0) if exact else 0.0)
        s1_1 = sum(am1, Fraction(0) if exact else 0.0)
        s2_1 = sum(am1 * d[: N - m + 1], Fraction(0) if exact else 0.0)
        A = c2 / c1
        B = e2 + s1_2 / c2 - s1_1 / c1
        dj = d[: N - m]
        am = -am2[: N - m] * (dj - e1) * (dj - e2) + A * (dj - B) * am1[: N - m] * (dj - e1)
        cm = -(c2 * e1 * e2 + s1_2 * (e1 + e2) - s2_2) + A * (c1 * B * e1 + s1_1 * (B + e1) - s2_1)
        cs.append(cm)
        als.append(am)
        if stop_nonpositive and not cm > 0:
            return Chain(d, cs, als, False)
    return Chain(d, cs, als, all(c > 0 for c in cs))


def _sign(v) -> int:
    return int(v > 0) - int(v < 0)


def member_signs(ch: Chain, x):
    """sign(p_m(x)) for every member built (x must not be a pole)."""
    d = ch.d
    N = d.size
    below = int(np.sum(d < x))
    if np.any(d == x):
        raise ValueError("x is a pole")
    out = []
    for m, (c, a) in enumerate(zip(ch.c, ch.alpha)):
        f = c - sum(a / (x - d[: N - m]), Fraction(0) if isinstance(c, Fraction) else 0.0)
        above = max(0, (N - m) - below)  # poles of pi_m above x
        out.append(_sign(f) * (-1 if above % 2 else 1))
    return out


def sign_changes(signs) -> int:
    s = [v for v in signs if v != 0]
    return sum(1 for a, b in zip(s, s[1:]) if a != b)


def changes_at_infinity(ch: Chain, plus: bool) -> int:
    N = ch.d.size
    sg = []
    for m, c in enumerate(ch.c):
        v = _sign(c)
        sg.append(v if plus else v * (-1 if (N - m) % 2 else 1))
    return sign_changes(sg)


def count_below(ch: Chain, x) -> int:
    """Zeros of p_0 below x, V(-inf) - V(x) over the members built."""
    return changes_at_infinity(ch, False) - sign_changes(member_signs(ch, x))


def lower_bound(ch: Chain) -> int:
    """Zeros guaranteed by a chain stopped at its first non-positive c: the
    number of leading positive c's, less one."""
    k = 0
    for c in ch.c:
        if not c > 0:
            break
        k += 1
    return k - 1


def deflate_found(d, alpha, xi, exact: bool = False):
    """Eq. (9): residues beta on the poles that remain after removing the known
    zeros xi (ascending), each paired with one of the lowest poles in order.
    Returns (remaining poles, beta)."""
    d = _arr(d, exact)
    a = _arr(alpha, exact)
    xi = _arr(sorted(xi), exact)
    s = xi.size
    if s > d.size:
        raise ValueError("more zeros than poles")
    beta = a.copy()
    for p in range(s):
        beta = beta * (d - d[p]) / (d - xi[p])
    return d[s:], beta[s:]
