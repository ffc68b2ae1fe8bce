"""First-order perturbation estimate of the eigenpairs of A + K Sigma K^T
(Sec. 3, eq. (11)) -- TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Eq. (11) as read (G9): with U = Q^T K (row u_j belongs to eigenpair j),
    lambda_j ~ lambda_j + u_j^T Sigma u_j,
    v_j      ~ v_j + sum_{i != j} (u_i^T Sigma u_j) / (lambda_j - lambda_i) v_i.
The printed formula repeats v_j^0 where the sum needs v_i^0, has the
denominator the other way round and no Sigma (it treats K K^T).  Pairs with
equal eigenvalues have no first-order term here (the estimate does not hold
for a degenerate spectrum).  The estimate keeps the original ordering.
"""
from __future__ import annotations

import numpy as np


def perturb_first_order(lam, Q, K, sigma):
    """(lambda estimate, V estimate) of eq. (11), in the order of lam."""
    lam = np.asarray(lam, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64).reshape(lam.size, -1)
    sig = np.asarray(sigma, dtype=np.float64).ravel()
    n = lam.size
    U = Q.T @ K
    lam_p = np.empty(n)
    for j in range(n):
        lam_p[j] = lam[j] + float(np.sum(sig * U[j] * U[j]))
    W = np.eye(n)
    for j in range(n):
        for i in range(n):
            if i != j and lam[i] != lam[j]:
                W[i, j] = float(np.sum(U[i] * sig * U[j])) / (lam[j] - lam[i])
    return lam_p, Q @ W
