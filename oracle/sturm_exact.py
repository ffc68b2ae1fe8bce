"""Exact-rational eigenvalue counts for tiny matrices (test infrastructure only).

The modified Sturm chain of Sec. 2.2 is justified by the classical Sturm
theorem for polynomials (the four properties listed there).  This module
applies that classical theorem, in exact rational arithmetic, to the
characteristic polynomial det(xI - A') of an explicit small matrix, which
pins the oracle's floating-point count nu(x) independently of the secular
form: for x not an eigenvalue, nu(x) = V(-inf) - V(x), where V counts sign
changes along the Sturm sequence p0 = p, p1 = p', p_{m+1} = -rem(p_{m-1}, p_m).

Characteristic polynomial by the Faddeev-LeVerrier recurrence (exact over Q).
Polynomials are lists of Fractions, lowest degree first.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence


def _trim(p):
    while len(p) > 1 and p[-1] == 0:
        p = p[:-1]
    return p


def charpoly(A: Sequence[Sequence[Fraction]]) -> List[Fraction]:
    """Coefficients (lowest degree first) of det(xI - A) for a square rational A."""
    n = len(A)
    A = [[Fraction(v) for v in row] for row in A]
    c = [Fraction(0)] * (n + 1)
    c[n] = Fraction(1)
    M = [[Fraction(0)] * n for _ in range(n)]
    for k in range(1, n + 1):
        # M_k = A M_{k-1} + c_{n-k+1} I
        AM = [[sum(A[i][t] * M[t][j] for t in range(n)) for j in range(n)] for i in range(n)]
        for i in range(n):
            AM[i][i] += c[n - k + 1]
        M = AM
        AMk = [[sum(A[i][t] * M[t][j] for t in range(n)) for j in range(n)] for i in range(n)]
        tr = sum(AMk[i][i] for i in range(n))
        c[n - k] = -tr / k
    return c


def _deriv(p):
    return _trim([p[i] * i for i in range(1, len(p))] or [Fraction(0)])


def _rem(a, b):
    a = list(a)
    b = _trim(b)
    while len(_trim(a)) >= len(b) and any(v != 0 for v in a):
        a = _trim(a)
        if len(a) < len(b):
            break
        f = a[-1] / b[-1]
        shift = len(a) - len(b)
        for i in range(len(b)):
            a[i + shift] -= f * b[i]
        a = a[:-1]
    return _trim(a) if a else [Fraction(0)]


def sturm_sequence(p):
    seq = [_trim(p), _deriv(p)]
    while len(seq[-1]) > 1 or seq[-1][0] != 0:
        r = _rem(seq[-2], seq[-1])
        r = [-v for v in r]
        if all(v == 0 for v in r):
            break
        seq.append(r)
        if len(r) == 1:
            break
    return seq


def _eval(p, x):
    s = Fraction(0)
    for c in reversed(p):
        s = s * x + c
    return s


def _changes(vals):
    signs = [v for v in vals if v != 0]
    return sum(1 for a, b in zip(signs, signs[1:]) if (a > 0) != (b > 0))


def count_below(A, x) -> int:
    """Number of distinct eigenvalues of the rational symmetric A strictly below x
    (x must not be an eigenvalue)."""
    seq = sturm_sequence(charpoly(A))
    x = Fraction(x)
    at_minus_inf = [(-1) ** (len(p) - 1) * p[-1] for p in seq]
    return _changes(at_minus_inf) - _changes([_eval(p, x) for p in seq])


def is_root(A, x) -> bool:
    return _eval(charpoly(A), Fraction(x)) == 0
