"""Benchmark: chained rank-k eigen-updates of one resident decomposition on one GPU.

Workload (default): n = 8192, k = 2, the one-column-one-row perturbation
e_j a^T + a e_j^T (K = [(e_j + a)/sqrt2, (e_j - a)/sqrt2], Sigma = diag(1, -1)),
lambda uniform in [-1, 1] (distinct), Q the orthogonal factor of a seeded
Gaussian matrix; a new (j, a) every step, all inputs resident in HBM before the
timed region.  One step = one full update (U = Q^T K, deflation, location,
root refinement, null vectors, W, Q' = Q W, commit).

Prints one JSON line.  Besides the throughput it reports the per-update
p50/p99 latency, the phase times, the roofline of the dominant kernel (the
FP64 MFMA GEMM Q W, timed with HIP events on the update's stream), a full
FP64 re-eigendecomposition of A' on the same GPU (torch.linalg.eigh), and the
CPU oracle timed on a bounded sample of the same update.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--n 8192] [--k 2]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rank-k eigen-updates/sec vs full GPU re-eigh at equal accuracy; p50/p99 latency"
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_FP64_VALU_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def make_perturbations(n, k, count, seed, dev):
    """count seeded perturbations (K column-major on dev, sigma)."""
    import torch

    from paper_1706_00773_amd import workloads as wl

    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        if k == 2:
            j = int(rng.integers(0, n))
            a = rng.standard_normal(n) / math.sqrt(n)
            K, sig = wl.rank2_column_row(n, j, a)
        else:
            K = rng.standard_normal((n, k)) / math.sqrt(n)
            sig = wl.random_signs(k, rng)
        Kt = torch.from_numpy(np.ascontiguousarray(np.asarray(K).T)).to(dev).t()
        out.append((Kt, sig))
    return out


def cpu_baseline(lam, Qn, K, sig, roots_sample, cols_sample, seed=7, threads=0):
    """Time the oracle on one whole update (default), or on a sample of its roots and
    columns scaled to a whole update; threads 0: every core this process may use."""
    import oracle

    n = lam.size
    oracle.set_threads(threads if threads > 0 else len(os.sched_getaffinity(0)))
    t0 = time.perf_counter()
    U = oracle.qtk(Qn, K)
    t_u = time.perf_counter() - t0
    rng = np.random.default_rng(seed)
    m = min(n, roots_sample)
    idx = np.sort(rng.choice(n, m, replace=False))
    t0 = time.perf_counter()
    vals, org, tau, _ = oracle.eigvals(lam, U, sig, idx)
    t_r = time.perf_counter() - t0
    t0 = time.perf_counter()
    Wc = oracle.eigvecs(lam, U, sig, org, tau)
    t_v = time.perf_counter() - t0
    c = min(n, cols_sample)
    t0 = time.perf_counter()
    oracle.gemm(Qn, Wc[:, :c])
    t_g = time.perf_counter() - t0
    total = t_u + (t_r + t_v) * n / m + t_g * n / c
    return {
        "value": 1.0 / total,
        "unit": "updates/s",
        "cores": oracle.get_threads(),
        "kind": "oracle",
        "sample": (f"one whole n={n} k={K.shape[1]} update: U = Q^T K ({t_u:.2f} s), all {n} "
                   f"roots by count bisection ({t_r:.2f} s), their eigenvectors ({t_v:.2f} s), "
                   f"Q W ({t_g:.2f} s); {total:.1f} s"
                   if (m == n and c == n) else
                   f"one n={n} k={K.shape[1]} update: U = Q^T K in full ({t_u:.2f} s), "
                   f"{m} of {n} roots by count bisection ({t_r:.2f} s) and their eigenvectors "
                   f"({t_v:.2f} s) scaled by n/{m}, Q W on {c} columns ({t_g:.2f} s) scaled "
                   f"by n/{c}; estimated {total:.1f} s per update"),
    }


def precision_report(args, dev):
    """Reduced-precision products at n = 16384, k = 4 (lambda = +-10^U[-3,3]):
    per mode, chained-update time, the Q W phase time, and the error against the
    oracle on a seeded sample (eigenvalues, eigenvectors, residual, orthogonality)."""
    import torch

    import oracle
    import paper_1706_00773_amd as eu
    from paper_1706_00773_amd import workloads as wl

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    n, k = args.n, args.k
    log(f"[bench] precision report: generating n={n} k={k} log-spread inputs")
    u = wl.logspread_rankk(k, n=n, device=str(dev))
    lam_t = torch.from_numpy(u.lam).to(dev)
    perts = make_perturbations(n, k, 1 + args.steps, seed=3000, dev=dev)
    Qh = np.asfortranarray(u.Q.cpu().numpy())
    Kt0, sig0 = perts[0]
    K0 = np.asfortranarray(Kt0.cpu().numpy())
    U = oracle.qtk(Qh, K0)
    scale = float(np.abs(u.lam).max() + np.sum(U * U))
    rng = np.random.default_rng(17)
    idx = np.unique(np.concatenate([rng.choice(n, 64, replace=False), [0, n - 1]]))
    ref_vals, org, tau, _ = oracle.eigvals(u.lam, U, sig0, idx)
    sig_t = torch.tensor(sig0, dtype=torch.float64, device=dev)
    modes = {"fp64": eu.EIG_GEMM_FP64, "fp32_corr": eu.EIG_GEMM_FP32_CORR,
             "bf16x3_corr": eu.EIG_GEMM_BF16X3_CORR}
    peaks = {"fp64": ("FP64 MFMA", 78.6, 1), "fp32_corr": ("FP32 MFMA", 157.3, 3),
             "bf16x3_corr": ("BF16 MFMA", 2500.0, 6)}
    out = {}
    ref_cols = None
    state = eu.EigState(n, 0)
    for name, mode in modes.items():
        log(f"[bench]   mode {name}")
        state.upload(lam_t, u.Q)
        state.update(Kt0, sig0, mode)
        lo = torch.empty(n, dtype=torch.float64, device=dev)
        Qo = torch.empty((n, n), dtype=torch.float64, device=dev).t()
        state.query(lo, Qo)
        lam_g = lo.cpu().numpy()
        e_val = float(np.abs(lam_g[idx] - ref_vals).max() / scale)
        # eigenvectors: 16 sampled isolated columns against the oracle's eq. (10) vectors
        if ref_cols is None:
            d = np.diff(lam_g)
            gaps = np.minimum(np.r_[d, np.inf], np.r_[np.inf, d])
            iso = [t for t in range(idx.size) if gaps[idx[t]] > 1e-6 * scale][:16]
            Wv = oracle.eigvecs(u.lam, U, sig0, org[iso], tau[iso])
            ref_cols = (idx[iso], oracle.gemm(Qh, Wv))
        cols, Qref = ref_cols
        Qg = Qo[:, torch.as_tensor(cols, device=dev)].cpu().numpy()
        sgn = np.sign(np.sum(Qg * Qref, axis=0))
        e_vec = float(np.abs(Qg * sgn - Qref).max())
        c64 = torch.as_tensor(idx[:64], device=dev)
        Qs = Qo[:, c64]
        AQ = u.Q @ (lam_t[:, None] * (u.Q.t() @ Qs)) + Kt0 @ (sig_t[:, None] * (Kt0.t() @ Qs))
        res = float((AQ - Qs * lo[c64][None, :]).abs().max()) / scale
        c512 = torch.as_tensor(np.sort(rng.choice(n, 512, replace=False)), device=dev)
        Qb = Qo[:, c512]
        orth = float((Qb.t() @ Qb - torch.eye(512, dtype=torch.float64, device=dev)).abs().max())
        del Qo, Qs, Qb, AQ
        # timing: chained updates, then phase times
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for s in range(args.steps):
            state.update(perts[1 + s][0], perts[1 + s][1], mode)
        e1.record(stream)
        torch.cuda.synchronize()
        state.query()
        ms = e0.elapsed_time(e1) / args.steps
        state.update(perts[1][0], perts[1][1], mode | eu.EIG_PHASE_TIMING)
        inf = state.query()
        gemm_ms = float(inf.ms[5])
        unit, peak, nprod = peaks[name]
        mfma_tf = nprod * 2.0 * n ** 3 / (gemm_ms * 1e-3) / 1e12
        out[name] = {"ms_per_update": round(ms, 3), "updates_per_s": round(1000.0 / ms, 3),
                     "qtk_ms": round(float(inf.ms[0]), 4), "gemm_ms": round(gemm_ms, 3),
                     "gemm_fp64_equiv_tflops": round(2.0 * n ** 3 / (gemm_ms * 1e-3) / 1e12, 2),
                     "gemm_mfma_tflops": round(mfma_tf, 2), "mfma_peak": f"{unit} {peak} TFLOP/s",
                     "gemm_mfma_frac": round(mfma_tf / peak, 4),
                     "err_eigenvalues_rel": e_val, "err_eigvec_max": e_vec,
                     "residual_rel": res, "orth_max": orth}
    state.close()
    return {"workload": f"mixed-precision back-transform, n={n}, k={k}, "
                        "lambda = +-10^U[-3,3], K ~ N(0,1/n), random signs",
            "sample": "eigenvalues at 66 seeded indices vs oracle bisection; 16 isolated "
                      "columns vs oracle eq. (10) vectors times Q; residual on 64 columns; "
                      "orthogonality on 512 columns; errors relative to max|lambda| + ||U||_F^2",
            "modes": out}


def batch_report(args, dev):
    """Batched updates of uneven instances: B resident decompositions, n log-uniform
    in [lo, hi], k from {1, 2, 4, 8}; the same chained updates applied (a) one at a
    time with eig_update_rankk, (b) as batches without graphs, (c) as batches with the
    tuned knobs and graph replay.  Every update of every instance is timed, warmups
    excluded (the first batches of a shape tune and capture)."""
    import torch

    import paper_1706_00773_amd as eu
    from paper_1706_00773_amd import workloads as wl

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    B = args.batch
    rng = np.random.default_rng(1006)
    sizes = wl.serving_sizes(B, args.batch_lo, args.batch_hi, seed=1006)
    ks = [int(v) for v in rng.choice([1, 2, 4, 8], B)]
    log(f"[bench] batch report: {B} instances, n in [{min(sizes)}, {max(sizes)}]")
    decomps = []
    for i, n in enumerate(sizes):
        lam = np.sort(rng.uniform(-1.0, 1.0, n))
        Q = wl.orthogonal_from(wl.gaussian_square(n, rng), str(dev))
        decomps.append((torch.from_numpy(lam).to(dev), Q))
    steps, warm = args.steps, 4
    perts = []
    for s in range(warm + steps):
        row = []
        for n, k in zip(sizes, ks):
            K = rng.standard_normal((n, k)) / math.sqrt(n)
            row.append((torch.from_numpy(np.ascontiguousarray(K.T)).to(dev).t(),
                        wl.random_signs(k, rng)))
        perts.append(row)
    states = [eu.EigState(n, 0) for n in sizes]

    def reset():
        for st, (lam, Q) in zip(states, decomps):
            st.upload(lam, Q)
        torch.cuda.synchronize()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        e0.record(stream)
        for s in range(warm, warm + steps):
            fn(s)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    out = {}
    # (a) one update at a time
    reset()
    for s in range(warm):
        for st, (K, sig) in zip(states, perts[s]):
            st.update(K, sig)
    ms = timed(lambda s: [st.update(K, sig) for st, (K, sig) in zip(states, perts[s])])
    out["single"] = {"ms_per_round": round(ms, 3), "updates_per_s": round(1000.0 * B / ms, 2)}
    for name, graphs in (("batched_no_graph", 0), ("batched_graph", 1)):
        reset()
        with eu.EigBatch(B, 0) as bt:
            bt.set(eu.EIG_KNOB_GRAPHS, graphs)
            for s in range(warm):
                bt.update([(st, K, sig) for st, (K, sig) in zip(states, perts[s])])
            ms = timed(lambda s: bt.update([(st, K, sig)
                                            for st, (K, sig) in zip(states, perts[s])]))
            out[name] = {"ms_per_round": round(ms, 3), "updates_per_s": round(1000.0 * B / ms, 2),
                         "rootsolve": ("persistent" if bt.get(eu.EIG_KNOB_ROOTSOLVE) ==
                                       eu.EIG_ROOTSOLVE_PERSISTENT else "grouped"),
                         "gemm_tile": bt.get(eu.EIG_KNOB_GEMM_TILE),
                         "graph_launches": bt.get(eu.EIG_STAT_GRAPH_LAUNCHES)}
    flops = sum(2.0 * n ** 3 for n in sizes)
    for v in out.values():
        v["gemm_equiv_tflops"] = round(flops / (v["ms_per_round"] * 1e-3) / 1e12, 2)
    for st in states:
        st.close()
    return {"workload": f"batch of {B} uneven updates per round, n log-uniform in "
                        f"[{args.batch_lo}, {args.batch_hi}], k from {{1,2,4,8}}, chained",
            "n": sizes, "k": ks, "rounds_timed": steps, "rounds_warmup": warm,
            "modes": out,
            "speedup_graph_vs_single": round(out["single"]["ms_per_round"] /
                                             out["batched_graph"]["ms_per_round"], 3)}


def serve_report(args, dev):
    """Serving: 64 resident decompositions, n log-uniform in [256, 8192] (lambda uniform
    in [-1, 1], Haar Q), requests choosing a matrix uniformly, k from {1, 2, 4, 8},
    K ~ N(0, 1/n), random signs, chained per matrix in arrival order.  First the
    saturated throughput (all requests submitted at once), then Poisson arrivals at
    0.5, 0.7 and 0.9 of it, with per-request latency (submit -> completion seen by the
    scheduler) p50/p99."""
    import torch

    import paper_1706_00773_amd as eu
    from paper_1706_00773_amd import workloads as wl

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    sizes = wl.serving_sizes(args.serve_matrices, 256, 8192, seed=1005)
    rng = np.random.default_rng(2005)
    nbytes = lambda n: ((n * n * 8 + 255) // 256) * 256
    resident = sum(nbytes(n) for n in sizes)
    arena = resident + (args.serve_transient_gib << 30)
    log(f"[bench] serving: {len(sizes)} matrices (resident Q {resident / 2**30:.2f} GiB), "
        f"arena {arena / 2**30:.2f} GiB")
    srv = eu.EigServer(arena, max_batch=args.serve_batch, streams=args.serve_streams,
                       max_k_doubles=args.serve_batch * 8192 * 8)
    for n in sizes:
        lam = torch.from_numpy(np.sort(rng.uniform(-1.0, 1.0, n))).to(dev)
        Q = wl.orthogonal_from(wl.gaussian_square(n, rng), str(dev))
        srv.add(lam, Q)
        del Q
    torch.cuda.synchronize()

    def make_requests(count):
        out = []
        for _ in range(count):
            m = int(rng.integers(0, len(sizes)))
            n = sizes[m]
            k = int(rng.choice([1, 2, 4, 8]))
            out.append((m, np.asfortranarray(rng.standard_normal((n, k)) / math.sqrt(n)),
                        wl.random_signs(k, rng)))
        return out

    def run(reqs, rate):
        comps = []
        t0 = time.perf_counter()
        gaps = rng.exponential(1.0 / rate, len(reqs)) if rate else np.zeros(len(reqs))
        arrive = np.cumsum(gaps)
        base = len(run.ids)
        for i, (m, K, sig) in enumerate(reqs):
            if rate:
                while time.perf_counter() - t0 < arrive[i]:
                    pass
            srv.submit(m, K, sig, base + i)
            if i % 64 == 63:
                comps += srv.poll()
        srv.drain()
        while True:
            more = srv.poll()
            if not more:
                break
            comps += more
        assert len(comps) == len(reqs), (len(comps), len(reqs))
        run.ids += [c["request_id"] for c in comps]
        bad = sum(1 for c in comps if c["status"] != 0)
        t_first = min(c["t_submit"] for c in comps)
        t_last = max(c["t_done"] for c in comps)
        lat = np.array([c["t_done"] - c["t_submit"] for c in comps]) * 1000.0
        return {"requests": len(comps), "failed": bad,
                "throughput_req_s": round(len(comps) / (t_last - t_first), 2),
                "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                               "p99": round(float(np.percentile(lat, 99)), 3),
                               "mean": round(float(lat.mean()), 3)},
                "mean_batch": round(float(np.mean([c["batch_size"] for c in comps])), 2)}
    run.ids = []

    log("[bench]   warmup (256 requests)")
    run(make_requests(256), 0.0)
    log(f"[bench]   saturated ({args.serve_requests} requests at once)")
    sat = run(make_requests(args.serve_requests), 0.0)
    out = {"saturated": sat}
    for f in (0.5, 0.7, 0.9):
        rate = f * sat["throughput_req_s"]
        log(f"[bench]   Poisson arrivals at {f} x saturated = {rate:.1f} req/s")
        r = run(make_requests(args.serve_requests), rate)
        r["offered_req_s"] = round(rate, 2)
        out[f"poisson_{f}"] = r
    st = srv.stats()
    srv.close()
    flops = 2.0 * float(np.mean([n ** 3 for n in sizes]))
    return {"workload": f"serving: {len(sizes)} resident decompositions, n log-uniform in "
                        "[256, 8192], requests uniform over matrices, k from {1,2,4,8}, "
                        "chained per matrix",
            "n": sizes, "arena_gib": round(arena / 2**30, 2),
            "resident_gib": round(resident / 2**30, 2),
            "max_batch": args.serve_batch, "streams": args.serve_streams,
            "mean_gemm_flop_per_request": flops,
            "modes": out,
            "server": {"batches": st["batches"], "mean_batch": round(st["mean_batch"], 2),
                       "arena_peak_gib": round(st["arena_peak"] / 2**30, 2),
                       "compactions": st["compactions"]}}


def interval_report(args, dev):
    """Subsets of the spectrum (eig_update_interval) at the headline size: the
    eigenpairs in [a, b) for a, b at quantiles of the resident eigenvalues, against
    the full update; median of 5 synchronous calls each."""
    import torch

    import paper_1706_00773_amd as eu
    from paper_1706_00773_amd import workloads as wl

    n, k = args.n, args.k
    u = wl.plain_rank2(n, seed=1000, device=str(dev), min_gap=1e-12) if k == 2 else \
        wl.general_rankk(k, n=n, device=str(dev))
    state = eu.EigState(n, 0)
    lam_t = torch.from_numpy(u.lam).to(dev)
    state.upload(lam_t, u.Q)
    Kt, sig = make_perturbations(n, k, 1, seed=4000, dev=dev)[0]
    out = {}

    def timed(fn, reps=5):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(1000.0 * (time.perf_counter() - t0))
        return float(np.median(ts)), r

    full_ms, _ = timed(lambda: (state.update(Kt, sig), state.query()))
    state.upload(lam_t, u.Q)
    out["full_update_ms"] = round(full_ms, 3)
    for frac in (0.001, 0.01, 0.1, 0.5):
        lo = 0.5 - frac / 2
        a = float(u.lam[int(lo * (n - 1))])
        b = float(u.lam[int((lo + frac) * (n - 1))])
        ms, (lam, V) = timed(lambda: state.interval(Kt, sig, a, b, m_max=int(frac * n) + 64))
        ms_vo, (lam2, _) = timed(lambda: state.interval(Kt, sig, a, b, mode=eu.EIG_VALUES_ONLY,
                                                        m_max=int(frac * n) + 64))
        out[f"fraction_{frac}"] = {"m": int(lam.numel()), "ms": round(ms, 3),
                                   "values_only_ms": round(ms_vo, 3),
                                   "speedup_vs_full": round(full_ms / ms, 2)}
    state.close()
    return {"workload": f"subset of the spectrum of a rank-{k} update, n={n}: eigenpairs in "
                        "[a, b) around the middle of the spectrum (eig_update_interval, "
                        "synchronous), against a full update plus query",
            "modes": out}


def sturm_chain_report(args, dev):
    """The secular Sturm chain counter (eig_sturm_chain, Sec. 2.2, eqs. (4)-(9)):
    synchronous time per call at 64 count points, the members it builds before its
    first non-positive c, and -- with the lowest eigenvalues divided out first
    (eq. (9)) -- a complete chain; beside it the inertia counter's cost (the first
    phase of eig_update_interval on an empty interval) and the oracle's chain on
    the host at n = 200."""
    import torch

    import oracle
    import paper_1706_00773_amd as eu
    from oracle import sturm_chain as sc
    from paper_1706_00773_amd import workloads as wl

    def timed(fn, reps=5):
        ts = []
        r = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(1000.0 * (time.perf_counter() - t0))
        return float(np.median(ts)), r

    rows = []
    for n, k in ((200, 3), (1024, 3), (8192, 2), (8192, 3)):
        u = wl.random_small(n, k, seed=n + k) if n <= 1024 else \
            (wl.plain_rank2(n, seed=1000, device=str(dev), min_gap=1e-12) if k == 2
             else wl.general_rankk(k, n=n, device=str(dev)))
        Qd = u.Q if isinstance(u.Q, torch.Tensor) else \
            torch.from_numpy(np.asfortranarray(u.Q)).to(dev).t().contiguous().t()
        state = eu.EigState(n, 0)
        state.upload(torch.from_numpy(np.asarray(u.lam)).to(dev), Qd)
        Kd = torch.from_numpy(np.asfortranarray(u.K)).to(dev).t().contiguous().t()
        lo, hi = float(np.min(u.lam)) - 1.0, float(np.max(u.lam)) + 1.0
        x = torch.linspace(lo, hi, 64, dtype=torch.float64, device=dev)
        ms, (_, _, info) = timed(lambda: state.sturm_chain(Kd, u.sigma, x))
        row = {"n": n, "k": k, "ms": round(ms, 3), "levels": int(info.levels),
               "complete": bool(info.complete), "lower_bound": int(info.lower_bound)}
        mid = float(np.median(u.lam))
        ms_in, _ = timed(lambda: state.interval(Kd, u.sigma, mid, mid, mode=eu.EIG_VALUES_ONLY))
        row["inertia_count_ms"] = round(ms_in, 3)
        if n <= 1024:
            # divide out all but the top 20 eigenvalues: the remaining chain completes
            A = (Qd * torch.from_numpy(np.asarray(u.lam)).to(dev)) @ Qd.T + \
                (Kd * torch.tensor(u.sigma, dtype=torch.float64, device=dev)) @ Kd.T
            ev = torch.linalg.eigvalsh((A + A.T) / 2)
            xi = ev[: n - 20].contiguous()
            ms_d, (cnt, _, info_d) = timed(lambda: state.sturm_chain(Kd, u.sigma, x, xi=xi))
            ref = torch.searchsorted(ev.contiguous(), x.contiguous())
            row["found_zeros"] = {"divided_out": n - 20, "ms": round(ms_d, 3),
                                  "levels": int(info_d.levels), "complete": bool(info_d.complete),
                                  "counts_equal_eigvalsh": bool(torch.equal(cnt, ref))}
        state.close()
        rows.append(row)
    # the oracle's chain on the host, n = 200, k = 3
    u = wl.random_small(200, 3, seed=203)
    U = oracle.qtk(u.Q, u.K)
    t0 = time.perf_counter()
    a = np.array([oracle.alpha(u.lam, U, u.sigma, i) for i in range(200)])
    ch = sc.build(u.lam, a)
    xs = np.linspace(u.lam.min() - 1, u.lam.max() + 1, 64)
    _ = [sc.count_below(ch, v) for v in xs]
    cpu_ms = 1000.0 * (time.perf_counter() - t0)
    return {"workload": "secular Sturm chain counter (eig_sturm_chain), 64 count points, "
                        "random updates with distinct poles; synchronous calls, median of 5",
            "rows": rows,
            "oracle_host_n200_k3_ms": round(cpu_ms, 1), "oracle_levels_n200_k3": ch.levels}


def perturbation_sweep(args, dev):
    """The accuracy experiment of the paper's Sec. 3 (Fig. 6, 7) on synthetic data: N = 100,
    norm(K) in {0.01, 0.3}, rank k = 1..8, perturbation K K^T (all signs +1).  For the
    direct FP64 eigendecomposition of A' (torch.linalg.eigh on the GPU), this library's
    update, and the first-order perturbation estimate (eq. (11)): (A) 2-norm error of the
    eigenvalues against the direct decomposition, (B) ||A' - V diag(lambda) V^T||_2,
    (C) ||V^T V - I||_2, (D) time (median of 20; the update split into its values-only
    part and the whole)."""
    import torch

    import paper_1706_00773_amd as eu
    from paper_1706_00773_amd import workloads as wl

    N = 100
    rows = []

    def med(fn, reps=20):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(1000.0 * (time.perf_counter() - t0))
        return float(np.median(ts)), out

    for norm in (0.01, 0.3):
        for k in range(1, 9):
            rng = np.random.default_rng(7000 + 10 * k + (norm > 0.1))
            lam = np.sort(rng.uniform(-1.0, 1.0, N))
            Q = wl.orthogonal_from(wl.gaussian_square(N, rng))
            K = rng.standard_normal((N, k))
            K *= norm / np.linalg.norm(K, 2)
            sig = np.ones(k, dtype=np.int8)
            A = (Q * lam) @ Q.T + K @ K.T
            A = (A + A.T) / 2
            At = torch.from_numpy(A).to(dev)
            t_direct, (wd, Vd) = med(lambda: torch.linalg.eigh(At))
            wd = wd.cpu().numpy()
            Kt = torch.from_numpy(np.ascontiguousarray(K.T)).to(dev).t()
            lam_t = torch.from_numpy(lam).to(dev)
            Q_t = torch.from_numpy(np.ascontiguousarray(Q.T)).to(dev).t()
            st = eu.EigState(N, 0)
            lo = torch.empty(N, dtype=torch.float64, device=dev)
            Qo = torch.empty((N, N), dtype=torch.float64, device=dev).t()

            def upd(mode):
                st.upload(lam_t, Q_t)
                torch.cuda.synchronize()
                st.update(Kt, sig, mode)
                st.query(lo, Qo if not (mode & eu.EIG_VALUES_ONLY) else None)

            t_vals, _ = med(lambda: upd(eu.EIG_VALUES_ONLY))
            t_full, _ = med(lambda: upd(0))
            lu, Vu = lo.cpu().numpy(), Qo.cpu().numpy()
            t_pert, (lp, Vp) = med(lambda: st.perturb_first_order(Kt, sig))
            lp, Vp = lp.cpu().numpy(), Vp.cpu().numpy()
            st.close()

            def metrics(l, V):
                o = np.argsort(l)
                l, V = l[o], V[:, o]
                return {"A_eigenvalues": float(np.linalg.norm(l - wd)),
                        "B_reconstruction": float(np.linalg.norm(A - (V * l) @ V.T, 2)),
                        "C_orthogonality": float(np.linalg.norm(V.T @ V - np.eye(N), 2))}

            rows.append({"norm_K": norm, "k": k,
                         "direct": dict(metrics(wd, Vd.cpu().numpy()), ms=round(t_direct, 3)),
                         "update": dict(metrics(lu, Vu), ms=round(t_full, 3),
                                        values_only_ms=round(t_vals, 3)),
                         "perturbation": dict(metrics(lp, Vp), ms=round(t_pert, 3))})
    return {"workload": "accuracy experiment of Sec. 3 (Fig. 6/7) on synthetic data: N = 100, "
                        "lambda uniform in [-1, 1], Haar Q, K Gaussian scaled to norm(K), "
                        "perturbation K K^T, k = 1..8",
            "rows": rows}


def measured_traffic(path_name, sources):
    """HBM bytes per update of the Q W step from the rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs recorded under profiles/, or None once a source differs from the measured one."""
    import hashlib

    path = os.path.join(ROOT, "profiles", path_name)
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for src in sources:
            h.update(open(os.path.join(ROOT, "paper_1706_00773_amd", "csrc", src), "rb").read())
    except (OSError, ValueError):
        return None
    return rec["traffic_bytes"] if rec.get("sources_sha256") == h.hexdigest() else None


# Block size and Chebyshev nodes of the library's far-field product (farfield.hip).
FF_B = 256  # columns per column block of the far-field product


def farfield_cfg(k):
    """Rows per row block and nodes per row / column interval of the far-field plan
    (half-width row blocks up to rank 2)."""
    return (128, 20, 24) if k <= 2 else (256, 20, 20)


def farfield_flops(n, k):
    """Algorithmic flops of Q W by the far-field product: per column block of 256
    the exact rows within one row block of it (the band), P2M (2 n^2 k pr), M2L
    (2 k n (nr pr)(nb pc)) and L2P (2 n^2 k pc).  The rows the plan adds for
    blocks widened by outlying poles or roots are not counted."""
    rb, pr, pc = farfield_cfg(k)
    nb, nr = n // FF_B, n // rb
    rpc = FF_B // rb

    def rows(lo, hi):
        return (n if hi + 1 >= nr else (hi + 1) * rb) - lo * rb

    band = 0.0
    for i in range(nb):
        b = FF_B if i + 1 < nb else n - (nb - 1) * FF_B
        lo = max(0, i * rpc - 1)
        hi = nr - 1 if i + 1 == nb else min(nr - 1, (i + 1) * rpc)
        band += 2.0 * n * b * rows(lo, hi)
    return (band + 2.0 * n * n * k * pr + 2.0 * k * n * (nr * pr) * (nb * pc)
            + 2.0 * n * n * k * pc)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--no-reeigh", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-roots", type=int, default=1 << 30,
                    help="roots the CPU oracle solves (default: all)")
    ap.add_argument("--cpu-cols", type=int, default=1 << 30,
                    help="columns of Q W the CPU oracle forms (default: all)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the CPU oracle (default 0: every core this process may use)")
    ap.add_argument("--save-input", metavar="NPZ",
                    help="only generate the resident decomposition and write it to NPZ")
    ap.add_argument("--load-input", metavar="NPZ",
                    help="read the resident decomposition from NPZ (written by --save-input) "
                         "instead of generating it")
    ap.add_argument("--qw", choices=["farfield", "dense"], default="farfield",
                    help="how Q' = Q W is formed: far-field product (EIG_QW_FARFIELD) or "
                         "the dense FP64 product")
    ap.add_argument("--no-dense-compare", action="store_true",
                    help="with --qw farfield: skip the dense comparison pass")
    ap.add_argument("--locate-residues", action="store_true",
                    help="k = 2: locate roots by residue signs (EIG_LOCATE_RESIDUES)")
    ap.add_argument("--precision", action="store_true",
                    help="report the reduced-precision modes (use with --n 16384 --k 4)")
    ap.add_argument("--batch", type=int, default=0,
                    help="report batched updates of this many uneven instances")
    ap.add_argument("--batch-lo", type=int, default=256)
    ap.add_argument("--batch-hi", type=int, default=2048)
    ap.add_argument("--interval", action="store_true",
                    help="report subsets of the spectrum (eig_update_interval)")
    ap.add_argument("--perturbation-sweep", action="store_true",
                    help="the N = 100 accuracy experiment against eq. (11)")
    ap.add_argument("--sturm-chain", action="store_true",
                    help="report the secular Sturm chain counter")
    ap.add_argument("--serve", action="store_true", help="report the serving loop")
    ap.add_argument("--serve-matrices", type=int, default=64)
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--serve-batch", type=int, default=32)
    ap.add_argument("--serve-streams", type=int, default=2)
    ap.add_argument("--serve-transient-gib", type=int, default=24)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}): the library "
              "implements the single-GPU update only", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1706_00773_amd as eu
    from paper_1706_00773_amd import workloads as wl

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        # a plain copy of 2^30 bytes: reads 1 GiB, writes 1 GiB per launch
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30,
                          "launches": 4, "ms_per_copy": round(ms, 4),
                          "hbm_gbs_read_plus_write": round(2.0 * (1 << 30) / (ms * 1e-3) / 1e9, 1)}))
        return
    if args.precision:
        print(json.dumps(precision_report(args, dev)), flush=True)
        return
    if args.batch:
        print(json.dumps(batch_report(args, dev)), flush=True)
        return
    if args.serve:
        print(json.dumps(serve_report(args, dev)), flush=True)
        return
    if args.interval:
        print(json.dumps(interval_report(args, dev)), flush=True)
        return
    if args.perturbation_sweep:
        print(json.dumps(perturbation_sweep(args, dev)), flush=True)
        return
    if args.sturm_chain:
        print(json.dumps(sturm_chain_report(args, dev)), flush=True)
        return
    n, k = args.n, args.k
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    if args.load_input:
        log(f"[bench] reading the n={n} decomposition from {args.load_input}")
        with np.load(args.load_input) as z:
            lam0 = z["lam"].copy()
            Q0 = torch.from_numpy(z["Qt"]).to(dev).t()  # stored transposed: column-major
        if lam0.size != n:
            raise SystemExit(f"{args.load_input} holds n={lam0.size}, not {n}")
    else:
        log(f"[bench] generating n={n} k={k} inputs on {dev}")
        if k == 2:
            u = wl.plain_rank2(n, seed=1000, device=str(dev), min_gap=1e-12)
        else:
            u = wl.general_rankk(k, n=n, device=str(dev))
        lam0 = u.lam.copy()
        Q0 = u.Q  # torch, column-major
    if args.save_input:
        np.savez(args.save_input, lam=lam0, Qt=Q0.t().contiguous().cpu().numpy())
        log(f"[bench] wrote {args.save_input}")
        return
    steps, warm = args.steps, args.warmup
    perts = make_perturbations(n, k, warm + 2 * steps, seed=2000, dev=dev)
    state = eu.EigState(n, 0)
    state.upload(torch.from_numpy(lam0).to(dev), Q0)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    umode = eu.EIG_LOCATE_RESIDUES if args.locate_residues else 0
    farfield = args.qw == "farfield" and n >= 2048
    if farfield:
        umode |= eu.EIG_QW_FARFIELD
    log(f"[bench] warmup {warm}")
    for s in range(warm):
        state.update(perts[s][0], perts[s][1], umode)
    state.query()
    torch.cuda.synchronize()

    # pass A: throughput, updates back to back
    log(f"[bench] timed throughput pass: {steps} chained updates")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for s in range(steps):
        K, sig = perts[warm + s]
        state.update(K, sig, umode)
    e1.record(stream)
    torch.cuda.synchronize()
    info = state.query()
    total_ms = e0.elapsed_time(e1)
    ms_per_step = total_ms / steps
    value = 1000.0 / ms_per_step

    # pass B: per-update latency and phase times (events recorded by the library on
    # the update's stream)
    log(f"[bench] timed latency pass: {steps} updates with phase events")
    lat, phases, located = [], [], []
    for s in range(steps):
        K, sig = perts[warm + steps + s]
        state.update(K, sig, eu.EIG_PHASE_TIMING | umode)
        inf = state.query()
        located.append(inf.located_by_residues)
        lat.append(inf.ms[7])
        phases.append(list(inf.ms))
    phases = np.array(phases)
    gemm_ms = float(phases[:, 5].mean())

    def dense_roofline(ms):
        flops = 2.0 * n ** 3
        ach = flops / (ms * 1e-3) / 1e12
        return {
            "kernel": "dgemm_kernel (Q' = Q W, FP64 MFMA 16x16x4)",
            "bound": "mfma",
            "achieved": round(ach, 3),
            "peak": PEAK_FP64_MFMA_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(ach / PEAK_FP64_MFMA_TFLOPS, 4),
            "traffic": (measured_traffic("qw_dense_rank2_n8192_traffic.json", ["gemm.hip"])
                        if (n, k) == (8192, 2) else None),
            "avg_ms": round(ms, 4),
            "algorithmic": f"2 n^3 = {flops:.3e} flop per launch",
        }

    if farfield:
        ff_flops = farfield_flops(n, k)
        achieved = ff_flops / (gemm_ms * 1e-3) / 1e12
        roofline = {
            "kernel": ("Q' = Q W far-field product (exact band, P2M, M2L, L2P: dgemm_desc and "
                       "dgemm_kernel launches on FP64 MFMA 16x16x4, timed together)"),
            "bound": "mfma",
            "achieved": round(achieved, 3),
            "peak": PEAK_FP64_MFMA_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP64_MFMA_TFLOPS, 4),
            "traffic": (measured_traffic("qw_farfield_rank2_n8192_traffic.json",
                                         ["gemm.hip", "farfield.hip"])
                        if (n, k) == (8192, 2) else None),
            "avg_ms": round(gemm_ms, 4),
            "algorithmic": (f"band + P2M + M2L + L2P = {ff_flops:.3e} flop per update "
                            f"(dense 2 n^3 = {2.0 * n ** 3:.3e})"),
        }
    else:
        roofline = dense_roofline(gemm_ms)
    names = ["qtk", "deflate", "polecount+locate", "rootsolve+rootvec", "finalize+wbuild",
             "dgemm", "commit", "total"]
    phase_ms = {nm: round(float(phases[:, i].mean()), 4) for i, nm in enumerate(names)}
    qtk_gbs = (8.0 * n * n + 16.0 * n * k) / (phase_ms["qtk"] * 1e-3) / 1e9 if phase_ms["qtk"] else 0

    # whole update against the sum of its steps' ideal times: U = Q^T K and W at
    # HBM speed, the root work (pole counts, Newton evaluations, null vectors:
    # 6 + k + k(k+1) flop per pole and count or vector sweep, 6 + k + 2k(k+1) per
    # Newton evaluation) at the FP64 vector peak, Q W at the FP64 MFMA peak
    n_d = n - int(info.n_deflated_rows)
    root_flop = float(n_d) ** 2 * (3 * (6 + k + k * (k + 1)) + info.iters_mean * (6 + k + 2 * k * (k + 1)))
    ideal = {"qtk": (8.0 * n * n + 16.0 * n * k) / (PEAK_HBM_GBS * 1e9) * 1e3,
             "roots": root_flop / (PEAK_FP64_VALU_TFLOPS * 1e12) * 1e3,
             "wbuild": 8.0 * n * n / (PEAK_HBM_GBS * 1e9) * 1e3,
             "dgemm": (farfield_flops(n, k) if farfield else 2.0 * n ** 3)
             / (PEAK_FP64_MFMA_TFLOPS * 1e12) * 1e3}
    ideal_ms = sum(ideal.values())
    whole = {"ideal_ms": round(ideal_ms, 3), "measured_ms": round(ms_per_step, 3),
             "frac": round(ideal_ms / ms_per_step, 4),
             "ideal_steps_ms": {kk: round(v, 4) for kk, v in ideal.items()}}

    # sanity: the final state is orthonormal on a sample of columns
    lam_now = torch.empty(n, dtype=torch.float64, device=dev)
    Q_now = torch.empty((n, n), dtype=torch.float64, device=dev).t()
    state.query(lam_now, Q_now)
    cols = torch.arange(0, n, max(1, n // 64), device=dev)
    Qs = Q_now[:, cols]
    orth = float((Qs.t() @ Qs - torch.eye(cols.numel(), dtype=torch.float64, device=dev))
                 .abs().max())

    result = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"rank-{k} update of a resident n={n} decomposition "
                                + ("(e_j a^T + a e_j^T, Sigma = diag(1,-1))" if k == 2
                                   else "(K ~ N(0,1/n), random signs)")),
                   "n": n, "k": k, "chained": True},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4)},
        "phases_ms": phase_ms,
        "qtk_hbm_gbs": round(qtk_gbs, 1),
        "iters_mean": round(info.iters_mean, 3),
        "location": ("residue signs (Alg. 1), %d of %d updates" % (sum(located), len(located))
                     if args.locate_residues else "inertia pole counts"),
        "orth_sample_max": orth,
        "qw": ("far-field product (EIG_QW_FARFIELD)" if farfield else "dense FP64 product"),
        "roofline": roofline,
        "roofline_whole_update": whole,
    }

    if farfield and not args.no_dense_compare:
        # the dense product on the same chained state, for comparison
        log(f"[bench] dense Q W for comparison: {steps} chained updates")
        dmode = umode & ~eu.EIG_QW_FARFIELD
        dperts = make_perturbations(n, k, steps, seed=2500, dev=dev)
        torch.cuda.synchronize()
        e0.record(stream)
        for K, sig in dperts:
            state.update(K, sig, dmode)
        e1.record(stream)
        torch.cuda.synchronize()
        state.query()
        d_ms = e0.elapsed_time(e1) / steps
        d_ph = []
        for K, sig in dperts[: max(3, steps // 4)]:
            state.update(K, sig, dmode | eu.EIG_PHASE_TIMING)
            d_ph.append(state.query().ms[5])
        result["dense_qw"] = {"updates_per_s": round(1000.0 / d_ms, 4), "ms_per_step": round(d_ms, 4),
                              "roofline": dense_roofline(float(np.mean(d_ph)))}

    if not args.no_reeigh:
        log("[bench] re-eigh baseline: torch.linalg.eigh FP64 on the same GPU")
        lam_t = torch.from_numpy(lam0).to(dev)
        Kt, sig = perts[0]
        A = (Q0 * lam_t) @ Q0.t() + (Kt * torch.tensor(sig, dtype=torch.float64, device=dev)) @ Kt.t()
        A = 0.5 * (A + A.t())
        torch.linalg.eigh(torch.eye(64, dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            w_ref, V_ref = torch.linalg.eigh(A)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        reeigh_ms = 1000.0 * float(np.median(times))
        # the same A' through the update path
        chk = eu.EigState(n, 0)
        chk.upload(lam_t, Q0)
        chk.update(Kt, sig, umode & eu.EIG_QW_FARFIELD)
        lam_u = torch.empty(n, dtype=torch.float64, device=dev)
        Q_u = torch.empty((n, n), dtype=torch.float64, device=dev).t()
        chk.query(lam_u, Q_u)
        chk.close()
        diff = float((lam_u - w_ref).abs().max() / w_ref.abs().max())
        # residual and orthogonality of both on the same column sample ("equal accuracy")
        cs = torch.arange(0, n, max(1, n // 64), device=dev)
        eye = torch.eye(cs.numel(), dtype=torch.float64, device=dev)

        def accuracy(w, V):
            Vs = V[:, cs].contiguous()
            res = float((A @ Vs - Vs * w[cs][None, :]).abs().max() / w_ref.abs().max())
            return res, float((Vs.t() @ Vs - eye).abs().max())

        eig_res, eig_orth = accuracy(w_ref, V_ref)
        upd_res, upd_orth = accuracy(lam_u, Q_u)
        del V_ref, Q_u
        result["reeigh"] = {"ms": round(reeigh_ms, 2), "runs": len(times),
                            "updates_per_s_equiv": round(1000.0 / reeigh_ms, 4),
                            "speedup": round(value / (1000.0 / reeigh_ms), 2),
                            "max_rel_eigenvalue_diff_vs_update": diff,
                            "residual_sample_rel": eig_res, "orth_sample_max": eig_orth,
                            "update_residual_sample_rel": upd_res,
                            "update_orth_sample_max": upd_orth}
        del A

    if not args.no_cpu:
        log("[bench] CPU oracle baseline (the whole update unless --cpu-roots/--cpu-cols bound it)")
        Qn = Q0.cpu().numpy()  # column-major view -> Fortran-ordered array
        Qn = np.asfortranarray(Qn)
        K0 = np.asfortranarray(perts[0][0].cpu().numpy())
        result["cpu_baseline"] = cpu_baseline(lam0, Qn, K0, perts[0][1], args.cpu_roots,
                                              args.cpu_cols, threads=args.cpu_threads)
    state.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
