"""GPU parity of the far-field product Q' = Q W (EIG_QW_FARFIELD).

The mode changes only how Q W is formed, so:
- its eigenvalues must be bitwise those of the dense path;
- its Q' must agree with the dense product entrywise within 1e-12 (the
  Chebyshev interpolation of 1/(x - y) on far block pairs errs by at most
  about 3e-13 relative, and far entries of W are small next to near ones; the
  margin covers sums over n = 8192 terms of entries below 1);
- on block pairs placed at the plan's acceptance limits, with Q = I (so that Q'
  is the effective W entry by entry), every entry of a far pair has a relative
  error within the interpolant's bound at that limit: up to rank 2 (row blocks
  of 128) below 6e-13 at the column-side limit and 1.5e-13 at the row-side one,
  from rank 3 (row blocks of 256) below 1.5e-13 (6e-14 expected);
- against the oracle's matrix A' it must meet the tolerances of every update
  (eigenvalues 1e-10 ||A'||, residual 1e-9 ||A'||, ||Q'^T Q' - I||_max 1e-9).
Where the plan must fall back (merged equal poles, or half or more of the
column blocks too close to too many row blocks for the expansions) or the mode
does not apply (n < 2048), the result must be bitwise the dense one.
"""
import numpy as np
import pytest

import oracle
import paper_1706_00773_amd as eu
from paper_1706_00773_amd import workloads as wl

from helpers import colmajor, run_update

pytestmark = pytest.mark.gpu

DIFF_TOL = 1e-12
EVAL_TOL = 1e-10
RES_TOL = 1e-9
ORTH_TOL = 1e-9
FF = eu.EIG_QW_FARFIELD


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eu.load_library()


def _both(u):
    lam, Q, K, sig = np.asarray(u.lam), np.asarray(u.Q), np.asarray(u.K), u.sigma
    ld, Qd, _, _ = run_update(lam, Q, K, sig)
    lf, Qf, info, _ = run_update(lam, Q, K, sig, prec=FF)
    return ld, Qd, lf, Qf, info


def _check_oracle(u, lo, Qo):
    A = wl.explicit_matrix(u.lam, u.Q, u.K, u.sigma)
    U = oracle.qtk(np.asfortranarray(np.asarray(u.Q)), np.asarray(u.K))
    ref = np.sort(oracle.eigvals(np.asarray(u.lam), U, u.sigma)[0])
    scale = np.abs(ref).max()
    n = lo.size
    assert np.abs(lo - ref).max() <= EVAL_TOL * scale
    assert np.abs(A @ Qo - Qo * lo).max() <= RES_TOL * scale
    assert np.abs(Qo.T @ Qo - np.eye(n)).max() <= ORTH_TOL


def _outlying_poles(n, t, seed):
    """t poles uniform in [-1.4, -1.05] and t in [1.05, 1.4] around a bulk uniform in
    [-1, 1] (the spectrum's ends after a chain of rank-2 updates), Haar Q, rank-2 K
    of norm about 0.3."""
    rng = np.random.default_rng(seed)
    lo, hi = np.sort(rng.uniform(-1.4, -1.05, t)), np.sort(rng.uniform(1.05, 1.4, t))
    lam = np.concatenate([lo, wl.distinct_uniform(n - 2 * t, -1.0, 1.0, 1e-6, rng), hi])
    Q = wl.orthogonal_from(wl.gaussian_square(n, rng))
    K = np.asfortranarray(0.3 * rng.standard_normal((n, 2)) / np.sqrt(n))
    return wl.Update(lam, Q, K, wl.random_signs(2, rng), f"outlying-poles-n{n}")


CASES = [
    ("rank2 e_j a^T + a e_j^T, n=2048", lambda: wl.plain_rank2(2048, seed=31, min_gap=1e-12)),
    ("ragged n=2500 (last block 452), k=3", lambda: wl.random_small(2500, 3, seed=32)),
    ("odd n=2049 (no 16-byte accesses), k=2", lambda: wl.random_small(2049, 2, seed=37)),
    ("k=1, n=2304", lambda: wl.general_rankk(1, n=2304, seed=33)),
    ("k=5, n=2304", lambda: wl.general_rankk(5, n=2304, seed=34)),
    ("k=8, n=2048", lambda: wl.general_rankk(8, n=2048, seed=35)),
    ("clusters and tiny rows, n=4096", lambda: wl.clustered_rank2(4096, seed=36)),
    # the top root lies far above the spectrum: the last column block is close to
    # every row block, so its band widens over all rows and its product is
    # launched first
    ("strong perturbation (||K|| ~ 10: outlying eigenvalues), n=2048",
     lambda: wl.random_small(2048, 2, seed=38, knorm=10.0)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_farfield_matches_dense_and_oracle(name, make):
    print(f"case farfield {name}", flush=True)
    u = make()
    ld, Qd, lf, Qf, info = _both(u)
    assert np.array_equal(ld, lf)
    # the far-field path ran (its fallback, the dense product, is bitwise Qd)
    assert not np.array_equal(Qf, Qd)
    assert np.abs(Qf - Qd).max() <= DIFF_TOL
    _check_oracle(u, lf, Qf)


def _further_ranges(lam, x, k):
    """Ranges of near row blocks apart from each column block's band, from the
    plan's rules (a band is the run of near row blocks around its column block)."""
    pairs, _, _ = _far_pairs(lam, x, k)
    rb = _rules(k)[0]
    n = lam.size
    nb, nr = n // 256, n // rb
    far = {(I, h) for I, h, _, _ in pairs}
    out = []
    for I in range(nb):
        near = [h for h in range(nr) if (I, h) not in far]
        out.append(sum(1 for a, b in zip(near, near[1:]) if b != a + 1))
    return out


def test_outlying_poles_give_further_near_ranges():
    """Poles spread beyond both ends of the bulk (the spectrum's ends after a chain
    of rank-2 updates) widen the end row blocks, and column blocks two blocks in
    multiply them exactly as ranges apart from their bands: the product's extra
    segments."""
    print("case farfield outlying poles at both ends, n=4096", flush=True)
    u = _outlying_poles(4096, 30, seed=39)
    ld, Qd, lf, Qf, info = _both(u)
    assert np.array_equal(ld, lf)
    ranges = _further_ranges(np.asarray(u.lam), lf, 2)
    print(f"  further near ranges per column block: {ranges}", flush=True)
    assert sum(ranges) >= 2 and max(ranges) <= 4
    assert not np.array_equal(Qf, Qd)
    assert np.abs(Qf - Qd).max() <= DIFF_TOL
    _check_oracle(u, lf, Qf)


def test_farfield_chained_updates():
    import torch

    print("case farfield chained n=2048 k=2", flush=True)
    n, dev = 2048, "cuda:0"
    u = wl.random_small(n, 2, seed=40)
    rng = np.random.default_rng(41)
    Ks = [rng.standard_normal((n, 2)) / np.sqrt(n) for _ in range(3)]
    outs = []
    for mode in (0, FF):
        with eu.EigState(n, 0) as s:
            s.upload(torch.as_tensor(u.lam, device=dev), colmajor(u.Q, dev))
            for K in Ks:
                s.update(colmajor(K, dev), np.array([1, -1]), mode)
            lo = torch.empty(n, dtype=torch.float64, device=dev)
            Qo = torch.empty((n, n), dtype=torch.float64, device=dev).t()
            s.query(lo, Qo)
            outs.append((lo.cpu().numpy(), Qo.cpu().numpy()))
    (ld, Qd), (lf, Qf) = outs
    assert not np.array_equal(Qf, Qd)  # the far-field path ran
    assert np.abs(lf - ld).max() <= 1e-13 * np.abs(ld).max()
    assert np.abs(Qf - Qd).max() <= DIFF_TOL
    assert np.abs(Qf.T @ Qf - np.eye(n)).max() <= ORTH_TOL


def test_nonfinite_perturbation_fails_and_keeps_the_state():
    """A NaN in K fails the update on the device in the far-field mode as in the
    dense one: both products are skipped, the state keeps the last committed
    decomposition, and the next update is a no-op until the error is read."""
    import torch

    print("case farfield non-finite K n=2048", flush=True)
    n, dev = 2048, "cuda:0"
    u = wl.random_small(n, 2, seed=46)
    bad = np.array(u.K)
    bad[5, 1] = np.nan
    outs = []
    for mode in (0, FF):
        with eu.EigState(n, 0) as s:
            s.upload(torch.as_tensor(u.lam, device=dev), colmajor(u.Q, dev))
            s.update(colmajor(u.K, dev), u.sigma, mode)    # committed
            s.update(colmajor(bad, dev), u.sigma, mode)    # fails on the device
            s.update(colmajor(u.K, dev), u.sigma, mode)    # no-op after the failure
            lo = torch.empty(n, dtype=torch.float64, device=dev)
            Qo = torch.empty((n, n), dtype=torch.float64, device=dev).t()
            with pytest.raises(eu.EigError) as e:
                s.query(lo, Qo)
            assert e.value.code == eu.EIG_ENONFINITE
            info = s.query(lo, Qo)                         # error cleared
            assert info.generation == 1
            outs.append((lo.cpu().numpy(), Qo.cpu().numpy()))
    (ld, Qd), (lf, Qf) = outs
    assert np.array_equal(ld, lf)
    assert not np.array_equal(Qf, Qd)  # the committed update took the far-field path
    assert np.abs(Qf - Qd).max() <= DIFF_TOL
    _check_oracle(u, lf, Qf)


def test_equal_poles_fall_back_to_the_dense_product():
    print("case farfield fallback with equal-pole groups n=2048", flush=True)
    n, k = 2048, 2
    rng = np.random.default_rng(42)
    lam = np.sort(rng.uniform(-1, 1, n))
    lam[700:704] = lam[700]
    lam = np.sort(lam)
    Q = wl.orthogonal_from(rng.standard_normal((n, n)))
    K = np.asfortranarray(rng.standard_normal((n, k)) / np.sqrt(n))
    sig = np.array([1, -1], dtype=np.int8)
    ld, Qd, info, _ = run_update(lam, Q, K, sig)
    lf, Qf, info_f, _ = run_update(lam, Q, K, sig, prec=FF)
    assert info_f.n_deflated_groups == 1
    assert np.array_equal(ld, lf) and np.array_equal(Qd, Qf)


def test_widely_spread_spectrum_falls_back_to_the_dense_product():
    """lambda = +-10^U[-3, 3]: blocks of 256 consecutive eigenvalues span decades,
    so every column block has more close row blocks than extra near products; with
    half or more of them over all rows the plan takes the dense product."""
    print("case farfield fallback with a log-spread spectrum n=2048 k=4", flush=True)
    u = wl.logspread_rankk(4, n=2048, seed=50)
    ld, Qd, lf, Qf, _ = _both(u)
    assert np.array_equal(ld, lf) and np.array_equal(Qd, Qf)


def test_small_order_ignores_the_mode():
    print("case farfield below the size threshold n=600", flush=True)
    u = wl.random_small(600, 3, seed=43)
    ld, Qd, lf, Qf, _ = _both(u)
    assert np.array_equal(ld, lf) and np.array_equal(Qd, Qf)


def test_values_only_and_reduced_precision_ignore_the_mode():
    print("case farfield with values-only and FP32 modes n=2048", flush=True)
    u = wl.random_small(2048, 2, seed=44)
    lam, Q, K, sig = np.asarray(u.lam), np.asarray(u.Q), np.asarray(u.K), u.sigma
    lv, _, _, _ = run_update(lam, Q, K, sig, values_only=True)
    lvf, _, _, _ = run_update(lam, Q, K, sig, values_only=True, prec=FF)
    assert np.array_equal(lv, lvf)
    l32, Q32, _, _ = run_update(lam, Q, K, sig, prec=eu.EIG_GEMM_FP32_CORR)
    l32f, Q32f, _, _ = run_update(lam, Q, K, sig, prec=eu.EIG_GEMM_FP32_CORR | FF)
    assert np.array_equal(l32, l32f) and np.array_equal(Q32, Q32f)


FULL = [
    ("rank-2 e_j a^T + a e_j^T, n=8192", lambda dev: wl.headline(8192, device=dev)),
    ("rank 4, n=8192", lambda dev: wl.general_rankk(4, n=8192, device=dev)),
    ("rank 8, n=8192", lambda dev: wl.general_rankk(8, n=8192, device=dev)),
]


@pytest.mark.parametrize("name,make", FULL, ids=[c[0] for c in FULL])
def test_full_size_n8192(name, make):
    """n = 8192 in the benchmark's workloads: entrywise against the dense product,
    and residual and orthogonality against A' on 256 sampled columns."""
    import torch

    print(f"case farfield {name}", flush=True)
    n, dev = 8192, "cuda:0"
    u = make(dev)
    Kh = u.K.cpu().numpy() if isinstance(u.K, torch.Tensor) else np.asarray(u.K)
    outs = []
    for mode in (0, FF):
        with eu.EigState(n, 0) as s:
            s.upload(torch.as_tensor(np.asarray(u.lam), device=dev), u.Q)
            s.update(colmajor(Kh, dev), u.sigma, mode)
            lo = torch.empty(n, dtype=torch.float64, device=dev)
            Qo = torch.empty((n, n), dtype=torch.float64, device=dev).t()
            s.query(lo, Qo)
            outs.append((lo, Qo))
    (ld, Qd), (lf, Qf) = outs
    assert torch.equal(ld, lf)
    assert not torch.equal(Qf, Qd)  # the far-field path ran
    assert float((Qf - Qd).abs().max()) <= DIFF_TOL
    cols = np.random.default_rng(45).choice(n, 256, replace=False)
    Qs = Qf[:, cols].cpu().numpy()
    Qh = u.Q.cpu().numpy() if isinstance(u.Q, torch.Tensor) else np.asarray(u.Q)
    lam = np.asarray(u.lam.cpu() if isinstance(u.lam, torch.Tensor) else u.lam)
    lv = lf.cpu().numpy()[cols]
    Aq = Qh @ (lam[:, None] * (Qh.T @ Qs)) + Kh @ (np.asarray(u.sigma, float)[:, None] * (Kh.T @ Qs))
    scale = np.abs(lf.cpu().numpy()).max()
    assert np.abs(Aq - Qs * lv).max() <= RES_TOL * scale
    G = (Qf.t() @ Qf[:, cols]).cpu().numpy()
    G[cols, np.arange(cols.size)] -= 1.0
    assert np.abs(G).max() <= ORTH_TOL


@pytest.mark.parametrize("k", [2, 4])
def test_full_size_n16384(k):
    """n = 16384: at k = 2 the benchmark's rank-2 workload at twice the order (128
    row blocks of 128, 64 column blocks: the largest interaction product the tests
    run), at k = 4 the general rank-k workload (row blocks of 256, 20 nodes each
    side).  Q' entrywise against the dense product, eigenvalues bitwise equal,
    residual against A' and orthogonality on 128 sampled columns (on the GPU)."""
    import torch

    print(f"case farfield rank {k}, n=16384", flush=True)
    n, dev = 16384, "cuda:0"
    if k == 2:
        u = wl.plain_rank2(n, seed=1006, device=dev, min_gap=1e-12)
    else:
        u = wl.general_rankk(k, n=n, seed=1007, device=dev)
    K = colmajor(np.asarray(u.K), dev)
    lam = torch.as_tensor(np.asarray(u.lam), device=dev)
    outs = []
    for mode in (0, FF):
        with eu.EigState(n, 0) as s:
            s.upload(lam, u.Q)
            s.update(K, u.sigma, mode)
            lo = torch.empty(n, dtype=torch.float64, device=dev)
            Qo = torch.empty((n, n), dtype=torch.float64, device=dev).t()
            s.query(lo, Qo)
            outs.append((lo, Qo))
    (ld, Qd), (lf, Qf) = outs
    assert torch.equal(ld, lf)
    assert not torch.equal(Qf, Qd)  # the far-field path ran
    diff = float((Qf - Qd).abs().max())
    del Qd
    cols = torch.as_tensor(np.sort(np.random.default_rng(46).choice(n, 128, replace=False)),
                           device=dev)
    Qs = Qf[:, cols].contiguous()
    sig = torch.as_tensor(np.asarray(u.sigma, dtype=np.float64), device=dev)
    Aq = u.Q @ (lam[:, None] * (u.Q.t().contiguous() @ Qs)) + K @ (sig[:, None] * (K.t() @ Qs))
    scale = float(lf.abs().max())
    res = float((Aq - Qs * lf[cols][None, :]).abs().max()) / scale
    G = Qf.t().contiguous() @ Qs
    G[cols, torch.arange(cols.numel(), device=dev)] -= 1.0
    orth = float(G.abs().max())
    print(f"  max |Q'_far - Q'_dense| {diff:.2e}, residual {res:.2e}, orthogonality {orth:.2e}",
          flush=True)
    assert diff <= DIFF_TOL
    assert res <= RES_TOL
    assert orth <= ORTH_TOL


def _rules(k):
    """Rows per row block and the row / column separation factors of the plan."""
    return (128, 0.85, 0.45) if k <= 2 else (256, 0.78, 0.78)


def _far_pairs(lam, x, k):
    """The plan's far (column block, row block) pairs for poles lam and column
    points x, each with its distance over the column-side and the row-side limit
    (far: both at least 1), and the rows of each row block."""
    rb, etar, etac = _rules(k)
    n = lam.size
    nb, nr, rpc = n // 256, n // rb, 256 // rb

    def rows(h):
        return h * rb, (n if h + 1 >= nr else (h + 1) * rb)

    def cols(I):
        return 256 * I, (n if I + 1 == nb else 256 * I + 256)

    ivr = np.array([(lam[rows(h)[0]], lam[rows(h)[1] - 1]) for h in range(nr)])
    ivc = np.array([(x[slice(*cols(I))].min(), x[slice(*cols(I))].max()) for I in range(nb)])

    def ratios(I, h):
        d = max(ivc[I, 0] - ivr[h, 1], ivr[h, 0] - ivc[I, 1])
        return d / (etac * (ivc[I, 1] - ivc[I, 0])), d / (etar * (ivr[h, 1] - ivr[h, 0]))

    def far(I, h):
        return min(ratios(I, h)) >= 1.0

    out = []
    for I in range(nb):
        lo = max(0, I * rpc - 1)
        hi = nr - 1 if I + 1 == nb else min(nr - 1, (I + 1) * rpc)
        while lo > 0 and not far(I, lo - 1):
            lo -= 1
        while hi < nr - 1 and not far(I, hi + 1):
            hi += 1
        out += [(I, h) + ratios(I, h) for h in range(nr) if (h < lo or h > hi) and far(I, h)]
    return out, rows, cols


def _entry_scale(lam, x, U, W):
    """|u_j| |c_p| / |x_p - lambda_j|: the size of entry (j, p) of W without the
    cancellation of its sum over the rank (c_p solved from W(:, p) =
    (x_p - D)^-1 U c_p)."""
    R = (x[None, :] - lam[:, None]) * W
    C = np.linalg.solve(U.T @ U, U.T @ R)
    return (np.linalg.norm(U, axis=1)[:, None] * np.linalg.norm(C, axis=0)[None, :]
            / np.abs(x[None, :] - lam[:, None]))


def _identity_updates(lam, K, sig):
    """The dense and the far-field update of diag(lam) (Q = I, so that Q' is W)."""
    import torch

    dev = "cuda:0"
    n = lam.size
    outs = []
    for mode in (0, FF):
        with eu.EigState(n, 0) as s:
            s.upload(torch.from_numpy(lam).to(dev), torch.eye(n, dtype=torch.float64, device=dev))
            s.update(colmajor(K, dev), sig, mode)
            lo = torch.empty(n, dtype=torch.float64, device=dev)
            Qo = torch.empty((n, n), dtype=torch.float64, device=dev).t()
            info = s.query(lo, Qo)
            assert info.n_deflated_rows == 0
        outs.append((lo.cpu().numpy(), Qo.cpu().numpy()))
    (ld, Wd), (lf, Wf) = outs
    assert np.array_equal(ld, lf)
    assert not np.array_equal(Wd, Wf)  # the far-field path ran
    return ld, Wd, Wf


def _far_errors(lam, ld, K, Wd, Wf, pairs, rows, cols):
    """Largest scaled error of the entries of each far pair."""
    scale = _entry_scale(lam, ld, K, Wd)
    err = np.abs(Wf - Wd) / scale
    return np.array([err[slice(*rows(h)), slice(*cols(I))].max() for I, h, _, _ in pairs])


def _limit_spectrum_rank2(margin, rng):
    """16 row blocks of 128 poles in periods of four (a, b, c, d): a, b and c 0.3
    wide, d one unit wide.  d starts 0.85 (1 + margin) after b, so column block
    (a, b) and row block d are just far on the row side.  The next period's b
    starts 0.45 (1 + margin) widths of column block (c, d) after d, so that pair
    is just far on the column side.  Blocks whose column points end a block are
    0.3 wide or more, so the perturbation moves those points by about 1e-5 of
    the distances only."""
    halves = []

    def put(lo, w):
        v = lo + np.sort(rng.uniform(0.0, w, 128))
        v[0], v[-1] = lo, lo + w
        halves.append(v)
        return lo + w

    d_end = c_lo = 0.0
    for t in range(4):
        if t == 0:
            b_end = put(put(0.0, 0.3) + 0.01, 0.3)
        else:
            put(d_end + 0.01, 0.3)
            b_end = put(d_end + 0.45 * (d_end - c_lo) * (1.0 + margin), 0.3)
        c_lo = b_end + 0.1
        put(c_lo, 0.3)
        d_end = put(b_end + 0.85 * (1.0 + margin), 1.0)
    return np.concatenate(halves)


def test_far_pairs_at_the_acceptance_limits_up_to_rank_2():
    """Up to rank 2 the row blocks hold 128 poles; a pair is far when its distance
    is at least 0.45 of the column block's width and 0.85 of the row block's.
    Pairs placed at (1 + 2e-4) times either limit: with Q = I and k = 1, Q' is W
    itself, W(j, p) = u_j c_p / (x_p - lambda_j) with no cancellation, so the
    far-field result against the dense one measures the error of the Chebyshev
    expansion entry by entry: about 3e-13 at the column-side limit (24 nodes,
    rho = 3.52), 2e-14 at the row-side one (20 nodes, rho = 5.21)."""
    rng = np.random.default_rng(2026)
    lam = _limit_spectrum_rank2(2e-4, rng)
    n = lam.size
    print(f"case far pairs at the acceptance limits, rank 1: n={n}", flush=True)
    K = rng.normal(0.0, np.sqrt(0.01 / n), (n, 1))
    ld, Wd, Wf = _identity_updates(lam, K, np.array([1], dtype=np.int8))
    pairs, rows, cols = _far_pairs(lam, ld, 1)
    rc = np.array([p[2] for p in pairs])
    rr = np.array([p[3] for p in pairs])
    assert rc.min() >= 1.0 and rr.min() >= 1.0
    at_c, at_r = rc <= 1.0003, rr <= 1.0003
    assert at_c.sum() >= 3 and at_r.sum() >= 4, (at_c.sum(), at_r.sum())
    e = _far_errors(lam, ld, K, Wd, Wf, pairs, rows, cols)
    print(f"  {len(pairs)} far pairs; largest relative error at the column-side limit "
          f"{e[at_c].max():.2e}, at the row-side limit {e[at_r].max():.2e}, overall "
          f"{e.max():.2e}", flush=True)
    assert e[at_r].max() <= 1.5e-13
    assert e.max() <= 6e-13


def _boundary_spectrum(eta, margin, rng):
    """8 blocks of 256 poles: even blocks span exactly one unit, odd blocks are
    1e-3 wide and sit in the gaps; block b + 2 starts eta (1 + margin) after the
    end of block b, so that every pair of even blocks two apart is just far."""
    lam, s, end = [], 0.0, 0.0
    for b in range(8):
        if b % 2 == 0:
            v = s + np.sort(rng.uniform(0.0, 1.0, 256))
            v[0], v[-1] = s, s + 1.0
            lam.append(v)
            end = s + 1.0
            s = end + eta * (1.0 + margin)
        else:
            lam.append(end + 0.5 * eta + np.sort(rng.uniform(-5e-4, 5e-4, 256)))
    return np.concatenate(lam)


def test_far_pair_at_the_acceptance_boundary_from_rank_3():
    """From rank 3 the row blocks hold 256 poles; a pair is far when its distance
    is at least 0.78 of both widths (20 nodes each side).  Pairs placed at
    0.78 (1 + 2e-4) widths, Q = I and k = 3: each entry of W is
    (u_j . c_p) / (x_p - lambda_j), so its error is measured against
    |u_j| |c_p| / |x_p - lambda_j| (the sum over the rank may cancel); about
    6e-14 is expected from the interpolant at the limit (rho = 4.92)."""
    rng = np.random.default_rng(2026)
    lam = _boundary_spectrum(0.78, 2e-4, rng)
    n = lam.size
    print(f"case far pair at the acceptance boundary, rank 3: n={n}", flush=True)
    K = rng.normal(0.0, np.sqrt(0.01 / n), (n, 3))
    ld, Wd, Wf = _identity_updates(lam, K, np.array([1, 1, 1], dtype=np.int8))
    pairs, rows, cols = _far_pairs(lam, ld, 3)
    r = np.array([min(p[2], p[3]) for p in pairs])
    assert r.min() >= 1.0 and r.min() <= 1.0006, r.min()
    assert np.sum(r <= 1.0006) >= 6
    e = _far_errors(lam, ld, K, Wd, Wf, pairs, rows, cols)
    print(f"  closest far pair {r.min():.5f} of the limit; largest relative error of the "
          f"{len(pairs)} far pairs {e.max():.2e}", flush=True)
    assert e.max() <= 1.5e-13, e.max()
