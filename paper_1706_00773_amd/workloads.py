"""Seeded synthetic inputs for the rank-k symmetric eigen-update.

This module only draws inputs; it holds none of the update's arithmetic.  It
is the one module shared by the GPU path's tests and benchmark and by the
oracle's tests.  The paper measures on randomly generated matrices only
(Sec. 3: random rank-3 updates, N = 100 comparisons), so these generators are
the workload itself; no dataset stands behind them.

Every generator returns ``(lam, Q, K, sigma)``: ``lam`` ascending (n,),
``Q`` n-by-n orthogonal (Fortran order for numpy, column-major storage),
``K`` n-by-k, ``sigma`` int8 (k,) of +-1, so that the updated matrix is
``Q diag(lam) Q^T + K diag(sigma) K^T``.

Seeds: workload ``c`` uses ``numpy.random.default_rng(1000 + c)``; draws are
taken in a fixed order (lam, Q's Gaussian matrix, then the perturbation).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np


@dataclass
class Update:
    lam: np.ndarray
    Q: object  # numpy array (Fortran order) or torch tensor (column-major storage)
    K: np.ndarray
    sigma: np.ndarray
    name: str = ""


def distinct_uniform(n: int, lo: float, hi: float, min_gap: float, rng) -> np.ndarray:
    """n sorted values uniform in [lo, hi] whose neighbours differ by at least min_gap
    (offenders are redrawn)."""
    v = np.sort(rng.uniform(lo, hi, n))
    for _ in range(1000):
        bad = np.nonzero(np.diff(v) < min_gap)[0]
        if bad.size == 0:
            return v
        v[bad + 1] = rng.uniform(lo, hi, bad.size)
        v.sort()
    raise RuntimeError("could not draw distinct values")


def gaussian_square(n: int, rng) -> np.ndarray:
    return rng.standard_normal((n, n))


def orthogonal_from(G, device: Optional[str] = None):
    """Q factor of the Householder QR of G with columns signed so that diag(R) > 0.

    With ``device`` set (e.g. "cuda:0") the QR runs there through torch (input
    preparation only) and a torch tensor holding Q in column-major storage is
    returned; otherwise a Fortran-ordered numpy array."""
    if device is None:
        Qm, R = np.linalg.qr(G)
        s = np.sign(np.diag(R))
        s[s == 0] = 1.0
        return np.asfortranarray(Qm * s)
    import torch

    Gt = torch.as_tensor(G, dtype=torch.float64, device=device)
    Qt, Rt = torch.linalg.qr(Gt)
    s = torch.sign(torch.diagonal(Rt))
    s[s == 0] = 1.0
    Qt = Qt * s
    # column-major storage: the transpose of a contiguous row-major tensor
    return Qt.t().contiguous().t()


def rank2_column_row(n: int, j: int, a: np.ndarray):
    """The one-column-one-row update e_j a^T + a e_j^T written as K Sigma K^T
    with K = [(e_j + a)/sqrt2, (e_j - a)/sqrt2], Sigma = diag(1, -1) (Sec. 2.2,
    Steps 1-2)."""
    e = np.zeros(n)
    e[j] = 1.0
    K = np.empty((n, 2), order="F")
    K[:, 0] = (e + a) / math.sqrt(2.0)
    K[:, 1] = (e - a) / math.sqrt(2.0)
    return K, np.array([1, -1], dtype=np.int8)


def random_signs(k: int, rng) -> np.ndarray:
    return rng.choice(np.array([-1, 1], dtype=np.int8), size=k)


def plain_rank2(n: int = 200, seed: int = 1001, device: Optional[str] = None,
                min_gap: float = 1e-6) -> Update:
    """Plain rank-2 update: lam uniform in [-1, 1] with min gap, Q from the QR of a
    seeded N(0,1) matrix, perturbation e_j a^T + a e_j^T with j uniform, a ~ N(0, 1/n)."""
    rng = np.random.default_rng(seed)
    lam = distinct_uniform(n, -1.0, 1.0, min_gap, rng)
    Q = orthogonal_from(gaussian_square(n, rng), device)
    j = int(rng.integers(0, n))
    a = rng.standard_normal(n) / math.sqrt(n)
    K, sig = rank2_column_row(n, j, a)
    return Update(lam, Q, K, sig, f"rank2-n{n}")


def headline(n: int = 8192, device: Optional[str] = None) -> Update:
    """Rank-2 e_j a^T + a e_j^T at n = 8192 (seed 1000), min gap 1e-12."""
    u = plain_rank2(n, seed=1000, device=device, min_gap=1e-12)
    u.name = f"rank2-n{n}"
    return u


def clustered_rank2(n: int = 4096, seed: int = 1002, device: Optional[str] = None) -> Update:
    """Rank-2 update with 10% of lam in clusters of 8 (relative gaps 1e-9) and 5% of
    the rows of U = Q^T K rescaled to 2-norm 1e-12 (then K := Q U)."""
    rng = np.random.default_rng(seed)
    lam = rng.uniform(-1.0, 1.0, n)
    ncl = (n // 10) // 8
    pos = rng.choice(n, size=ncl * 8, replace=False)
    centers = rng.uniform(-1.0, 1.0, ncl)
    vals = (centers[:, None] * (1.0 + 1e-9 * np.arange(8)[None, :])).ravel()
    lam[pos] = vals
    lam.sort()
    # keep values distinct (clusters use relative steps 1e-9; the rest are random)
    for _ in range(100):
        bad = np.nonzero(np.diff(lam) <= 0.0)[0]
        if bad.size == 0:
            break
        lam[bad + 1] = np.nextafter(lam[bad + 1], np.inf)
        lam.sort()
    G = gaussian_square(n, rng)
    j = int(rng.integers(0, n))
    a = rng.standard_normal(n) / math.sqrt(n)
    K, sig = rank2_column_row(n, j, a)
    rows = rng.choice(n, size=max(1, n // 20), replace=False)
    Q = orthogonal_from(G, device)
    if device is None:
        U = Q.T @ K
        U[rows] *= (1e-12 / np.linalg.norm(U[rows], axis=1))[:, None]
        K = np.asfortranarray(Q @ U)
    else:
        import torch

        Kt = torch.as_tensor(np.asarray(K), dtype=torch.float64, device=Q.device)
        U = Q.t() @ Kt
        r = torch.as_tensor(rows, device=Q.device)
        U[r] *= (1e-12 / torch.linalg.norm(U[r], dim=1))[:, None]
        K = np.asfortranarray((Q @ U).cpu().numpy())
    u = Update(lam, Q, K, sig, f"clustered-rank2-n{n}")
    u.tiny_rows = np.sort(rows)
    return u


def general_rankk(k: int, n: int = 8192, seed: int = 1003,
                  device: Optional[str] = None) -> Update:
    """Rank-k update: lam uniform in [-10, 10] distinct, Q random orthogonal,
    K ~ N(0, 1/n), sigma random +-1."""
    rng = np.random.default_rng(seed + 17 * k)
    lam = distinct_uniform(n, -10.0, 10.0, 1e-12, rng)
    Q = orthogonal_from(gaussian_square(n, rng), device)
    K = np.asfortranarray(rng.standard_normal((n, k)) / math.sqrt(n))
    sig = random_signs(k, rng)
    return Update(lam, Q, K, sig, f"rank{k}-n{n}")


def logspread_rankk(k: int = 4, n: int = 16384, seed: int = 1004,
                    device: Optional[str] = None) -> Update:
    """lam = +-10^{U[-3,3]} with random signs (sorted), Q random orthogonal,
    K ~ N(0, 1/n), sigma random +-1."""
    rng = np.random.default_rng(seed)
    mag = 10.0 ** rng.uniform(-3.0, 3.0, n)
    lam = np.sort(mag * rng.choice([-1.0, 1.0], n))
    Q = orthogonal_from(gaussian_square(n, rng), device)
    K = np.asfortranarray(rng.standard_normal((n, k)) / math.sqrt(n))
    sig = random_signs(k, rng)
    return Update(lam, Q, K, sig, f"logspread-rank{k}-n{n}")


def random_small(n: int, k: int, seed: int, lam_range=(-1.0, 1.0), knorm: float = 1.0,
                 min_gap: float = 1e-6) -> Update:
    """Small random instance for tests: distinct lam, Haar Q, K ~ N(0, knorm^2/n)."""
    rng = np.random.default_rng(seed)
    lam = distinct_uniform(n, lam_range[0], lam_range[1], min_gap, rng)
    Q = orthogonal_from(gaussian_square(n, rng))
    K = np.asfortranarray(knorm * rng.standard_normal((n, k)) / math.sqrt(n))
    sig = random_signs(k, rng)
    return Update(lam, Q, K, sig, f"random-n{n}-k{k}")


def serving_sizes(count: int = 64, lo: int = 256, hi: int = 8192, seed: int = 1005) -> List[int]:
    """Sizes log-uniform in [lo, hi] for the resident decompositions of a serving run."""
    rng = np.random.default_rng(seed)
    return [int(math.floor(math.exp(v))) for v in rng.uniform(math.log(lo), math.log(hi), count)]


def explicit_matrix(lam, Q, K, sigma) -> np.ndarray:
    """Q diag(lam) Q^T + K diag(sigma) K^T as a dense numpy array (test helper)."""
    Q = np.asarray(Q)
    K = np.asarray(K).reshape(Q.shape[0], -1)
    A = (Q * lam) @ Q.T + (K * np.asarray(sigma, dtype=np.float64)) @ K.T
    return (A + A.T) / 2.0
