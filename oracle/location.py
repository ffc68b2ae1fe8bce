"""Location vector of a rank-2 update from the signs of the residues alpha_i
(Sec. 2.2, Alg. 1a, 1b, 1c) -- TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For k = 2 the secular function f(x) = 1 + sum_j alpha_j / (lambda_j - x)
(eq. (3), alpha_j of eq. (2) as read in eigref.c) runs from -sign(alpha_t) inf
just right of lambda_t to sign(alpha_{t+1}) inf just left of lambda_{t+1}, so
the interval (lambda_t, lambda_{t+1}) holds an odd number of roots (one) when
alpha_t and alpha_{t+1} have the same sign and an even number (zero or two)
otherwise.  The two outer intervals are covered by virtual signs mu_0 = -1 and
mu_{n+1} = +1 (f tends to 1 at +-infinity).  Which of zero or two is taken
follows from the Courant-Weyl bounds, counted while scanning the intervals in
order: with p of the two signs positive and q = 2 - p negative, an even
interval t (t old eigenvalues below it) receives two roots exactly when the M
roots already placed plus two do not exceed t + q.  This is Alg. 1a (q = 0)
and Alg. 1c (q = 1) with the threshold read as M + 2 <= t + q; for q = 2 the
printed Alg. 1b scans from the last interval with M counting roots above, and
the same rule reads M + 2 <= (n - t).

Interval t here is 0-based: t = 0 is (-inf, lambda_1), t = n is (lambda_n, inf).
Requires distinct lambda and nonzero alpha (no deflation), as the paper does.
"""
from __future__ import annotations

import numpy as np

from . import alpha as _alpha


def alphas(lam, U, sigma):
    """alpha_i of eq. (2) for every pole (0-based)."""
    return np.array([_alpha(lam, U, sigma, i) for i in range(len(lam))])


def location_alg1(lam, U, sigma):
    """The location vector L (n + 1 counts) of a rank-2 update (Alg. 1a/1b/1c)."""
    lam = np.asarray(lam, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64).reshape(lam.size, -1)
    sig = np.asarray(sigma).ravel()
    if U.shape[1] != 2 or sig.size != 2:
        raise ValueError("Alg. 1 locates the roots of rank-2 updates only")
    n = lam.size
    a = alphas(lam, U, sig)
    if np.any(a == 0.0):
        raise ValueError("a residue alpha_i is zero: the signs do not locate the roots")
    mu = np.concatenate([[-1.0], np.sign(a), [1.0]])
    odd = [mu[t] * mu[t + 1] > 0 for t in range(n + 1)]
    q = int(np.sum(sig < 0))
    L = np.zeros(n + 1, dtype=np.int64)
    M = 0
    if q < 2:
        # Alg. 1a (q = 0) and Alg. 1c (q = 1): intervals left to right
        for t in range(n + 1):
            if odd[t]:
                L[t] = 1
                M += 1
            elif M + 2 <= t + q:
                L[t] = 2
                M += 2
    else:
        # Alg. 1b: intervals right to left, M = roots above
        for t in range(n, -1, -1):
            if odd[t]:
                L[t] = 1
                M += 1
            elif M + 2 <= n - t:
                L[t] = 2
                M += 2
    return L


def counts_from_location(L):
    """nu(lambda_s) = roots below pole s (0-based), from the location vector."""
    return np.cumsum(np.asarray(L))[:-1]
