"""Shared helpers for the GPU tests: moving seeded inputs to the device and
running one update through the C ABI."""
import numpy as np

import paper_1706_00773_amd as eu


def colmajor(a, dev):
    """numpy (any order) -> torch float64 tensor on dev with column-major storage."""
    import torch

    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(dev).t()


def run_update(lam, Q, K, sigma, dev="cuda:0", values_only=False, fetch=(), prec=0):
    """Upload (lam, Q), apply K diag(sigma) K^T, return (lam', Q', info, extras)."""
    import torch

    n = lam.shape[0]
    Qt = Q if isinstance(Q, torch.Tensor) else colmajor(Q, dev)
    mode = (eu.EIG_VALUES_ONLY if values_only else 0) | prec
    extras = {}
    with eu.EigState(n, 0) as s:
        s.upload(torch.as_tensor(np.asarray(lam), device=dev), Qt)
        s.update(colmajor(K, dev), sigma, mode)
        lo = torch.empty(n, dtype=torch.float64, device=dev)
        Qo = None if values_only else torch.empty((n, n), dtype=torch.float64, device=dev).t()
        info = s.query(lo, Qo)
        for what in fetch:
            extras[what] = fetch_item(s, what, info, n, K.shape[1] if K.ndim > 1 else 1)
    return lo.cpu().numpy(), (None if Qo is None else Qo.cpu().numpy()), info, extras


def fetch_item(s, what, info, n, k):
    nd = n - info.n_deflated_rows
    ns = info.n_segments
    if what == eu.EIG_DBG_U:
        return s.fetch(what, n * k).reshape(n, k)
    if what == eu.EIG_DBG_POLE_COUNT:
        return s.fetch(what, ns, np.int32)
    if what == eu.EIG_DBG_SEG_START:
        return s.fetch(what, ns + 1, np.int32)
    if what in (eu.EIG_DBG_REDUCED_D, eu.EIG_DBG_ROOT_TAU):
        return s.fetch(what, nd)
    if what in (eu.EIG_DBG_REDUCED_ROW, eu.EIG_DBG_ROOT_ORIGIN, eu.EIG_DBG_ROOT_ITERS):
        return s.fetch(what, nd, np.int32)
    if what == eu.EIG_DBG_W:
        return s.fetch(what, n * n).reshape(n, n, order="F")
    raise ValueError(what)


def align_signs(Qa, Qb):
    """Flip columns of Qa to agree in sign with Qb."""
    s = np.sign(np.sum(Qa * Qb, axis=0))
    s[s == 0] = 1.0
    return Qa * s


def isolated_columns(vals, rel_gap, scale):
    n = vals.size
    gaps = np.full(n, np.inf)
    if n > 1:
        d = np.diff(vals)
        gaps[:-1] = d
        gaps[1:] = np.minimum(gaps[1:], d)
    return np.nonzero(gaps > rel_gap * scale)[0]
