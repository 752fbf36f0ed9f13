#!/usr/bin/env python3
"""Benchmark of randomized HSS compression on one MI355X.

Workload (default "gauss65536"): the N = 65536 3-D Gaussian kernel matrix
A_ij = exp(-|p_i - p_j|^2 / (2 * 0.1^2)) + 1e-2 delta_ij on p ~ U[0,1]^3
(seed 4), ordered by recursive k-d bisection, stored in FP32, leaf size 256,
rtol = 1e-6, d0 = 128, dd = 64, FP64 sampling.  A is assembled on the GPU
before timing; the inputs are resident in HBM when the timed region starts.

A step is one pass of the whole path: hss_compress (random matrices,
sampling products, level-by-level local samples / IDs / updates with the
adaptive restarts, root coupling blocks), one hss_matvec on a single
vector, and hss_destroy.  `value` is seconds per step (lower is better).

The JSON line also carries
* roofline: the sampling GEMM kernel (the dominant kernel), its algorithmic
  FP64 flops (2 n^2 per random column and side) over its average launch
  duration measured with HIP events on the stream it runs on, against the
  FP64 MFMA peak of 78.6 TFLOP/s;
* cpu_baseline: the FP64 oracle timed on the host on a bounded sample of the
  same workload (see `cpu_baseline` below), scaled to seconds per step;
* accuracy: HSS matvec against a dense FP64 A x, relative error.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "gauss65536": dict(n=65536, kind="gauss", leaf=256, rtol=1e-6, d0=128, dd=64, d_max=4096,
                       storage="f32", point_seed=4, p_margin=256),
    "circle16384": dict(n=16384, kind="log", leaf=128, rtol=1e-8, d0=128, dd=64, d_max=4096,
                        storage="f64", point_seed=2, p_margin=10, ulv_rhs_seed=3),
    "toeplitz1024": dict(n=1024, kind="toeplitz", leaf=64, rtol=1e-6, d0=64, dd=32, d_max=4096,
                         storage="f64", point_seed=0, p_margin=10),
}


def measured_traffic(kernel_source: str, summary: str):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, or None
    when the summary is missing or was taken on another version of the
    kernel's source (its sha256 prefix is recorded in the summary)."""
    import hashlib

    try:
        text = open(os.path.join(ROOT, "profiles", summary)).read()
        src = open(os.path.join(ROOT, "paper_1503_05464_amd", "csrc", kernel_source), "rb").read()
    except OSError:
        return None
    want = None
    traffic = None
    for line in text.splitlines():
        if line.startswith(f"{kernel_source} sha256 prefix:"):
            want = line.split(":", 1)[1].strip()
        if line.startswith("traffic_bytes_per_launch:"):
            traffic = float(line.split(":", 1)[1].strip())
    if want is None or traffic is None or hashlib.sha256(src).hexdigest()[:16] != want:
        return None
    return traffic


def make_points(cfg):
    import workloads as W

    if cfg["kind"] == "gauss":
        p = W.cube_points(cfg["n"], cfg["point_seed"])
        return p[W.kd_order(p, cfg["leaf"])]
    if cfg["kind"] == "log":
        return W.circle_points(cfg["n"], cfg["point_seed"])
    return None


def make_matrix(cfg, points, device):
    import torch

    import workloads as W

    dt = torch.float32 if cfg["storage"] == "f32" else torch.float64
    if cfg["kind"] == "toeplitz":
        return torch.from_numpy(W.toeplitz_inverse_distance(cfg["n"])).to(device=device, dtype=dt)
    return W.device_kernel_matrix(cfg["kind"], points, dt, device)


def dense_matvec(A, x, block=4096):
    """FP64 A x with A widened block by block (reference for the check)."""
    import torch

    out = torch.empty((A.shape[0], x.shape[1]), dtype=torch.float64, device=A.device)
    for r0 in range(0, A.shape[0], block):
        out[r0:r0 + block] = A[r0:r0 + block].double() @ x
    return out


def frob_error(P, h, A, panel=2048):
    """||A - A_HSS||_F / ||A||_F exactly, from A_HSS applied to identity
    column panels (FP64)."""
    import torch

    n = A.shape[0]
    num = den = 0.0
    for c0 in range(0, n, panel):
        w = min(panel, n - c0)
        E = torch.zeros((n, w), dtype=torch.float64, device=A.device)
        E[c0:c0 + w] = torch.eye(w, dtype=torch.float64, device=A.device)
        Hp = P.hss_matvec(h, E)
        Ap = A[:, c0:c0 + w].double()
        num += float(torch.linalg.norm(Hp - Ap)) ** 2
        den += float(torch.linalg.norm(Ap)) ** 2
        del E, Hp, Ap
    return (num / den) ** 0.5


def cpu_baseline(cfg, points, d_final, panel_rows):
    """The oracle on a bounded sample of the workload, scaled to one step.

    Sample: (1) the oracle's Philox/Box-Muller R^r and R^c for all n rows and
    d_final columns (whole, not scaled); (2) the oracle's sampling products
    for one panel of `panel_rows` rows of A (widened from the FP32 storage)
    with d_final columns, and the oracle's leaf work for the leaves inside the
    panel (local samples and both IDs at d0, where the leaves are compressed),
    scaled by n / panel_rows.  Not in the sample: the inner-node passes
    (local samples, IDs and updates of the 2n/leaf - 1 inner nodes) and the
    restarts' extensions, so the figure under-states the oracle's time."""
    import numpy as np

    import workloads as W
    from oracle import hss as ohss
    from oracle import interp, philox

    n, leaf, d0 = cfg["n"], cfg["leaf"], cfg["d0"]
    dtype = np.float32 if cfg["storage"] == "f32" else np.float64
    rows = np.arange(panel_rows)
    Ap = W.kernel_rows(cfg["kind"], points, rows, dtype)  # input generation: not timed
    t0 = time.perf_counter()
    Rr = philox.gaussian_columns(0, 0, n, 0, d_final)
    Rc = philox.gaussian_columns(0, 1, n, 0, d_final)
    t_r = time.perf_counter() - t0
    t0 = time.perf_counter()
    sr, _ = ohss.sample_panel(Ap, Rr, Rc[rows])
    # leaf work inside the panel, at d0 columns
    for lo in range(0, panel_rows, leaf):
        hi = lo + leaf
        D = Ap[lo:hi, lo:hi]
        # U side exactly; the V side needs S^c rows that depend on every
        # panel, so an equal-sized stand-in of the same cost is decomposed
        interp.interpolative_decomposition((sr[lo:hi, :d0] - D @ Rr[lo:hi, :d0]).T, cfg["rtol"])
        interp.interpolative_decomposition((sr[lo:hi, :d0] - D.T @ Rc[lo:hi, :d0]).T, cfg["rtol"])
    t_panel = time.perf_counter() - t0
    value = t_r + t_panel * (n / panel_rows)
    try:
        from threadpoolctl import threadpool_info

        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = len(os.sched_getaffinity(0))
    return {
        "value": round(value, 3),
        "unit": "s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"oracle R^r,R^c for all {n} rows x {d_final} cols ({t_r:.2f} s, unscaled) + "
                   f"sampling products and leaf IDs for one {panel_rows}-row panel "
                   f"({t_panel:.2f} s) x {n // panel_rows}; inner-node passes not included"),
    }


def run_batched(args) -> int:
    """The batched workload: 512 independent planar 1/(4 pi r) matrices (N
    log-uniform in [256, 4096], k-d ordered, FP32 storage), compressed by one
    hss_compress_batched call with BF16x3 sampling at rtol 1e-4.  A step is
    the batched compression, one matvec per matrix (one hss_matvec_batched
    call) and the destruction of the handles; `value` is seconds per step.  The CPU baseline runs the
    oracle on a sample of the matrices and scales by sum(N^2)."""
    import numpy as np
    import torch

    import paper_1503_05464_amd as P
    import workloads as W

    cfg = dict(W.CONFIGS["batched512"])
    if args.rtol is not None:
        cfg["rtol"] = args.rtol
    prec = args.sample_prec if args.sample_prec != "f64" else cfg["sample_prec"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] workload batched512: {cfg['count']} matrices, assembling", file=sys.stderr, flush=True)
    sets = W.batch_instances(cfg["count"], cfg["n_lo"], cfg["n_hi"], cfg["point_seed"], cfg["leaf"])
    As = [W.device_kernel_matrix(cfg["kind"], p, torch.float32, dev) for p in sets]
    ns = np.array([a.shape[0] for a in As])
    xs = [torch.from_numpy(np.random.default_rng(int(n)).uniform(-1, 1, (int(n), 1))).to(dev) for n in ns]
    bs = [torch.empty_like(x) for x in xs]
    torch.cuda.synchronize()
    kw = dict(rtol=cfg["rtol"], d0=cfg["d0"], dd=cfg["dd"], d_max=cfg["d_max"], leaf_size=cfg["leaf"],
              p_margin=args.p_margin if args.p_margin is not None else cfg["p_margin"], sample_prec=prec)

    def step():
        hs = P.hss_compress_batched(As, **kw)
        P.hss_matvec_batched(hs, xs, bs)
        st = P.hss_stats(hs[0])
        conv = sum(1 for h in hs if h.converged)
        dmax = max(P.hss_stats(h)["d_final"] for h in hs)
        for h in hs:
            P.hss_destroy(h)
        return st, conv, dmax

    for w in range(args.warmup):
        st, conv, dmax = step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {w}: {st['t_total_ms']:.1f} ms, {conv} converged, max d {dmax}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        tk = time.perf_counter()
        stats.append(step())
        print(f"[bench] step {k}: {1e3 * (time.perf_counter() - tk):.1f} ms (compression "
              f"{stats[-1][0]['t_total_ms']:.1f} ms)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(1, args.steps)
    sts = [s[0] for s in stats]
    roofline = sampling_roofline(sts, prec)
    roofline["kernel"] = f"sampling products ({prec}) over all matrices"
    # acceptance: every matrix's matvec against its dense product
    hs = P.hss_compress_batched(As, **kw)
    worst = 0.0
    for A, h in zip(As, hs):
        x = torch.from_numpy(np.random.default_rng(7).uniform(-1, 1, (A.shape[0], 1))).to(dev)
        ref = A.double() @ x
        worst = max(worst, float(torch.linalg.norm(P.hss_matvec(h, x) - ref) / torch.linalg.norm(ref)))
    conv = sum(1 for h in hs if h.converged)
    del hs
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import hss as ohss

        print("[bench] cpu baseline (oracle on a sample of the matrices)", file=sys.stderr, flush=True)
        pick = np.random.default_rng(0).choice(len(sets), 6, replace=False)
        t_s, n2 = 0.0, 0.0
        for q in pick:
            Ah = W.kernel_rows(cfg["kind"], sets[q], np.arange(len(sets[q])), np.float32).astype(np.float32)
            t1 = time.perf_counter()
            ohss.compress(Ah, ohss.Options(rtol=kw["rtol"], d0=kw["d0"], dd=kw["dd"], d_max=kw["d_max"],
                                           p_margin=kw["p_margin"], leaf_size=kw["leaf_size"],
                                           sample_prec=prec))
            t_s += time.perf_counter() - t1
            n2 += float(len(sets[q])) ** 2
        scale = float((ns.astype(float) ** 2).sum()) / n2
        try:
            from threadpoolctl import threadpool_info

            cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
        except Exception:  # pragma: no cover
            cores = len(os.sched_getaffinity(0))
        cpu = {"value": round(t_s * scale, 3), "unit": "s", "cores": cores, "kind": "oracle",
               "sample": f"oracle compression of 6 of the {len(sets)} matrices (N = "
                         f"{sorted(int(len(sets[q])) for q in pick)}, {t_s:.2f} s) scaled by sum(N^2)"}
    out = {
        "metric": f"HSS batched compress s, {cfg['count']} matrices N in [{cfg['n_lo']}, {cfg['n_hi']}]",
        "value": round(ms / 1e3, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{prec} sampling, f64 ID",
        "data": "synthetic",
        "config": {
            "workload": f"batched512: {cfg['count']} planar 1/(4 pi r) matrices, N log-uniform in "
                        f"[{cfg['n_lo']}, {cfg['n_hi']}] (sum N^2 = {float((ns.astype(float) ** 2).sum()):.3g}), "
                        f"A f32, leaf {cfg['leaf']}, rtol {cfg['rtol']}, d0 {cfg['d0']}, dd {cfg['dd']}, "
                        f"{prec.upper()} sampling",
            "count": cfg["count"], "converged": conv,
            "step": "hss_compress_batched + hss_matvec_batched (nrhs=1, every matrix) + hss_destroy",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "level_roofline": level_roofline(sts),
        "accuracy": {"worst_matvec_rel_err_vs_dense": worst, "bound": 10 * cfg["rtol"]},
        "breakdown_ms": {k: round(float(np.median([s[k] for s in sts])), 2)
                         for k in ("t_total_ms", "t_sample_ms", "t_sample_gemm_ms", "t_levels_ms", "t_id_ms")},
    }
    print(json.dumps(out), flush=True)
    return 0


def serve_measure(nreq: int, rate: float, workers: int, budget_frac: float = 0.8,
                  p_margins=(32, 192)) -> dict:
    """The serving workload: requests of compress + ULV factor + solve arrive
    as a Poisson process at `rate` per second (seed 6).  Each request draws
    its matrix from a pool of 16 pre-assembled matrices -- N log-uniform in
    [512, 32768], the 2-D log kernel on a perturbed circle or the 3-D
    Gaussian kernel (k-d ordered) with probability 1/2 each, FP32 storage --
    and draws rtol in {1e-4, 1e-6} and nrhs in {1..64}; sampling is BF16x3.
    The first 10 % of the requests are warm-up.  Returns p50/p90/p99
    latency from submission to solution, the throughput, and checks of the
    SERVED solutions: on the last request of each pool matrix, the backward
    error ||A x - b|| / (||A||_2 ||x||) against the dense A, and the
    distance to the same request solved alone."""
    import numpy as np
    import torch

    import paper_1503_05464_amd as P
    import workloads as W

    g = np.random.default_rng(6)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pool = []
    sizes = np.floor(np.exp(g.uniform(np.log(512), np.log(32768), size=16))).astype(int)
    kinds = g.integers(0, 2, size=16)
    print(f"[bench] serve: assembling a pool of 16 matrices, N = {sorted(sizes.tolist())}",
          file=sys.stderr, flush=True)
    for q, (n, k) in enumerate(zip(sizes, kinds)):
        if k == 0:
            pts = W.circle_points(int(n), 600 + q)
            pool.append(W.device_kernel_matrix("log", pts, torch.float32, dev))
        else:
            pts = W.cube_points(int(n), 600 + q)
            pool.append(W.device_kernel_matrix("gauss", pts[W.kd_order(pts, 128)], torch.float32, dev))
    pick = g.integers(0, 16, size=nreq)
    rtols = g.choice([1e-4, 1e-6], size=nreq)
    nrhs = g.integers(1, 65, size=nreq)
    gaps = g.exponential(1.0 / rate, size=nreq)
    rhs = [torch.from_numpy(W.normal_rhs(int(pool[q].shape[0]), int(k), 6000 + i)).to(dev)
           for i, (q, k) in enumerate(zip(pick, nrhs))]
    torch.cuda.synchronize()
    # admission budget: a fraction of the device memory; every request's
    # footprint counts its A, b and x as well as the library's buffers
    budget = int(budget_frac * torch.cuda.mem_get_info()[1])
    srv = P.HSSServer(hbm_budget=budget, max_batch=32, workers=workers)
    # p_margin by rtol: (for 1e-4, for 1e-6)
    kw0 = dict(d0=64, dd=32, d_max=1024, leaf_size=128, sample_prec="bf16x3")

    def pm(rt):
        return int(p_margins[0] if rt >= 1e-5 else p_margins[1])
    print(f"[bench] serving {nreq} requests at {rate:g}/s", file=sys.stderr, flush=True)
    t_start = time.perf_counter()
    t_next = t_start
    tickets = []
    for i in range(nreq):
        t_next += gaps[i]
        while time.perf_counter() < t_next:
            time.sleep(max(0.0, min(0.001, t_next - time.perf_counter())))
        tickets.append(srv.submit(pool[pick[i]], rhs[i], rtol=float(rtols[i]), p_margin=pm(rtols[i]), **kw0))
    t_submitted = time.perf_counter()
    infos, xs = [], []
    for i, t in enumerate(tickets):
        x, info = srv.wait(t)
        infos.append(info)
        xs.append(x)
        if (i + 1) % max(1, nreq // 10) == 0:
            print(f"[bench] {i + 1} of {nreq} requests done", file=sys.stderr, flush=True)
    srv.close()
    warm = nreq // 10
    lat = np.array([x["t_done"] - x["t_submit"] for x in infos[warm:]])
    bad = sum(1 for x in infos if x["status"] not in (P.HSS_OK, P.HSS_NOT_CONVERGED))
    t_first = min(x["t_submit"] for x in infos[warm:])
    t_last = max(x["t_done"] for x in infos[warm:])
    thr = (nreq - warm) / max(1e-9, t_last - t_first)
    # the served solutions themselves: the last request on each pool matrix
    worst_bwd, worst_rel_bound, worst_alone = 0.0, 0.0, 0.0
    checked = 0
    detail = []
    for q in sorted(set(pick.tolist())):
        i = int(np.flatnonzero(pick == q)[-1])
        A = pool[q].double()
        x = xs[i]
        r = A @ x - rhs[i]
        v = torch.ones((A.shape[0], 1), dtype=torch.float64, device=dev)
        for _ in range(20):  # ||A||_2 by power iteration
            v = A @ v
            v = v / torch.linalg.norm(v)
        anorm = float(torch.linalg.norm(A @ v))
        bwd = float(torch.linalg.norm(r)) / (anorm * float(torch.linalg.norm(x)))
        worst_bwd = max(worst_bwd, bwd)
        worst_rel_bound = max(worst_rel_bound, bwd / (10 * float(rtols[i])))
        detail.append({"n": int(A.shape[0]), "kernel": "log" if kinds[q] == 0 else "gauss",
                       "rtol": float(rtols[i]), "nrhs": int(nrhs[i]), "backward_error": bwd})
        h = P.hss_compress(pool[q], rtol=float(rtols[i]), p_margin=pm(rtols[i]), **kw0)
        P.hss_factor(h)
        xa = P.hss_solve(h, rhs[i])
        worst_alone = max(worst_alone, float(torch.linalg.norm(x - xa) / torch.linalg.norm(xa)))
        P.hss_destroy(h)
        checked += 1
        del A
    return {
        "rate_req_s": rate,
        "requests": nreq,
        "warmup": warm,
        "workers": workers,
        "hbm_budget_frac": budget_frac,
        "p_margin": {"rtol 1e-4": int(p_margins[0]), "rtol 1e-6": int(p_margins[1])},
        "latency_s": {"p50": round(float(np.percentile(lat, 50)), 4), "p90": round(float(np.percentile(lat, 90)), 4),
                      "p99": round(float(np.percentile(lat, 99)), 4), "max": round(float(lat.max()), 4)},
        "throughput_req_s": round(thr, 2),
        "offered_req_s": round(nreq / (t_submitted - t_start), 2),
        "mean_batch": round(float(np.mean([x["batch_size"] for x in infos])), 2),
        "failed": bad,
        "served_checked": checked,
        "served_backward_error_max": worst_bwd,
        "served_backward_error_over_10rtol_max": round(worst_rel_bound, 4),
        "served_vs_alone_rel_max": worst_alone,
        "served_checks": sorted(detail, key=lambda r: -r["backward_error"] / r["rtol"])[:4],
    }


def run_serve(args) -> int:
    """The serving workload on its own (see serve_measure); `value` is the
    p50 latency."""
    res = serve_measure(args.serve_requests, float(args.serve_rate), args.serve_workers,
                        p_margins=tuple(int(v) for v in args.serve_p_margin.split(",")))
    out = {
        "metric": "HSS serving latency s (compress + ULV factor + solve per request), p50; p99 alongside",
        "value": res["latency_s"]["p50"],
        "unit": "s",
        "n_gpus": 1,
        "steps": res["requests"] - res["warmup"],
        "warmup": res["warmup"],
        "ms_per_step": round(1e3 / res["throughput_req_s"], 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3 sampling, f64 ID and ULV",
        "data": "synthetic",
        "config": {
            "workload": f"serve: Poisson arrivals at {res['rate_req_s']:g}/s (seed 6), pool of 16 FP32 matrices "
                        "N log-uniform in [512, 32768] (log kernel on a circle or Gaussian kernel in 3-D), rtol in "
                        "{1e-4, 1e-6}, nrhs in {1..64}, leaf 128, d0 64, dd 32, p_margin "
                        f"{res['p_margin']['rtol 1e-4']} / {res['p_margin']['rtol 1e-6']} (rtol 1e-4 / 1e-6), "
                        "BF16X3 sampling",
            "requests": res["requests"], "workers": res["workers"], "max_batch": 32,
            "hbm_budget": f"{int(100 * res['hbm_budget_frac'])}% of device memory",
        },
        **{k: res[k] for k in ("latency_s", "throughput_req_s", "offered_req_s", "mean_batch", "failed",
                               "served_checked", "served_backward_error_max",
                               "served_backward_error_over_10rtol_max", "served_vs_alone_rel_max",
                               "served_checks")},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def sampling_roofline(stats, prec: str) -> dict:
    """Roofline of the sampling products over the timed steps: algorithmic
    flops (2 n^2 per random column and side) and bytes (A once per product,
    R read, S written) over the launches' summed duration (HIP events on the
    stream they run on), against the peak of the precision's own unit."""
    flops = sum(s["sample_gemm_flops"] for s in stats)
    nbytes = sum(s["sample_gemm_bytes"] for s in stats)
    t_gemm = sum(s["t_sample_gemm_ms"] for s in stats) / 1e3
    launches = sum(s["n_sample_launches"] for s in stats)
    terms, peak, kname = {"f64": (1, FP64_MFMA_PEAK_TFLOPS, "sample_kernel (FP64 MFMA 16x16x4)"),
                          "f32": (1, FP32_MFMA_PEAK_TFLOPS, "sample_mixed_kernel (FP32 MFMA 16x16x4)"),
                          "bf16x3": (3, BF16_MFMA_PEAK_TFLOPS,
                                     "sample_mixed_kernel (3 BF16 terms, BF16 MFMA 16x16x32)")}[prec]
    issued = terms * flops / t_gemm / 1e12 if t_gemm > 0 else 0.0
    gbs = nbytes / t_gemm / 1e9 if t_gemm > 0 else 0.0
    hbm_bound = nbytes / (HBM_PEAK_GBS * 1e9) > terms * flops / (peak * 1e12)
    return {
        "bound": "hbm" if hbm_bound else "mfma",
        "achieved": round(gbs, 1) if hbm_bound else round(issued, 2),
        "peak": HBM_PEAK_GBS if hbm_bound else peak,
        "unit": "GB/s" if hbm_bound else "TFLOP/s",
        "frac": round(gbs / HBM_PEAK_GBS if hbm_bound else issued / peak, 4),
        "traffic": None,
        "kernel": kname,
        "avg_launch_ms": round(t_gemm * 1e3 / max(1, launches), 4),
        "launches": launches,
        "algorithmic_tflops": round(flops / t_gemm / 1e12, 2) if t_gemm > 0 else 0.0,
        "achieved_gbs": round(gbs, 1),
    }


def level_roofline(stats) -> dict:
    """The level kernels of the timed steps against their bounds: the pivoted
    QRs (IDs) by their flops, 4 d m k per attempt and side with k the steps
    taken, over the ID phase's time (HIP events) against the FP64 peak; the
    local-sample and R_tau products and the D / B gathers by their
    algorithmic bytes over their launches' time against HBM."""
    t_id = sum(s["t_id_ms"] for s in stats) / 1e3
    idf = sum(s["id_flops"] for s in stats)
    t_g = sum(s["t_level_gemm_ms"] for s in stats) / 1e3
    gb = sum(s["level_gemm_bytes"] for s in stats)
    t_ga = sum(s["t_gather_ms"] for s in stats) / 1e3
    gab = sum(s["gather_bytes"] for s in stats)
    k = max(1, len(stats))

    def ent(bound, achieved, peak, unit, t, work):
        return {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "ms_per_step": round(1e3 * t / k, 2), "work_per_step": work}

    return {
        "id": ent("fp64", idf / t_id / 1e12 if t_id > 0 else 0.0, FP64_MFMA_PEAK_TFLOPS, "TFLOP/s", t_id,
                  f"{idf / k:.4g} flop (4 d m k per ID attempt and side)"),
        "level_gemm": ent("hbm", gb / t_g / 1e9 if t_g > 0 else 0.0, HBM_PEAK_GBS, "GB/s", t_g,
                          f"{gb / k:.4g} B (operands once, C when read)"),
        "gather": ent("hbm", gab / t_ga / 1e9 if t_ga > 0 else 0.0, HBM_PEAK_GBS, "GB/s", t_ga,
                      f"{gab / k:.4g} B (entries of A read, FP64 written)"),
    }


def profile_kernels(args) -> int:
    """Single launches at the benchmark's sizes for hardware-counter profiles
    (rocprofv3 --pmc): an elementwise copy of 4 GiB (torch multiply by one,
    two launches of 2 GiB read + 2 GiB written) that calibrates the byte
    counters, then hss_sample on the N = 65536 FP32 Gaussian-kernel matrix
    (k-d ordered points, leaf 256, leaf blocks masked) with 64 FP64 random
    columns in the precision --sample-prec: the products of one growth step
    of the compression."""
    import numpy as np
    import torch

    import paper_1503_05464_amd as P

    cfg = dict(WORKLOADS["gauss65536"])
    dev = torch.device("cuda:0")
    print("[profile] copy of 4 GiB", file=sys.stderr, flush=True)
    src = torch.ones(1 << 29, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()
    n, leaf, ncols = cfg["n"], cfg["leaf"], 64
    A = make_matrix(cfg, make_points(cfg), dev)
    leaf_of = torch.from_numpy((np.arange(n) // leaf).astype(np.int32)).to(dev)
    Rr = P.hss_random_normal(0, 0, n, 0, ncols, sample_prec=args.sample_prec)
    Rc = P.hss_random_normal(0, 1, n, 0, ncols, sample_prec=args.sample_prec)
    torch.cuda.synchronize()
    print(f"[profile] hss_sample n={n} ncols={ncols} {args.sample_prec} (both products)", file=sys.stderr,
          flush=True)
    P.hss_sample(A, Rr, Rc, leaf_of, sample_prec=args.sample_prec)
    torch.cuda.synchronize()
    print("[profile] done", file=sys.stderr, flush=True)
    return 0


def precision_sweep(P, A, kw, prec: str, steps: int) -> dict:
    """The headline matrix with the sampling products in a reduced precision
    (same rtol and options otherwise): seconds per step (compress + matvec
    + destroy), its sampling kernel's roofline against its own unit's peak,
    and the accuracy against the dense A."""
    import numpy as np
    import torch

    kwp = dict(kw, sample_prec=prec)
    n = A.shape[0]
    x = torch.from_numpy(np.random.default_rng(1).uniform(-1, 1, (n, 1))).to(A.device)
    b = torch.empty_like(x)

    def step():
        h = P.hss_compress(A, **kwp)
        P.hss_matvec(h, x, b)
        st = dict(P.hss_stats(h))
        P.hss_destroy(h)
        return st

    st = step()  # warm-up
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        stats.append(step())
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(1, steps)
    print(f"[bench] {prec} sampling: {ms:.1f} ms per step", file=sys.stderr, flush=True)
    h = P.hss_compress(A, **kwp)
    st = P.hss_stats(h)
    xs = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, (n, 2))).to(A.device)
    bd = dense_matvec(A, xs)
    mv_err = float(torch.linalg.norm(P.hss_matvec(h, xs) - bd) / torch.linalg.norm(bd))
    P.hss_destroy(h)
    return {
        "s_per_step": round(ms / 1e3, 4), "steps": steps, "d_final": st["d_final"], "passes": st["passes"],
        "max_rank": st["max_rank"], "converged": bool(st["converged"]),
        "roofline": sampling_roofline(stats, prec),
        "matvec_rel_err_vs_dense": mv_err, "bound": 10 * kw["rtol"],
        "breakdown_ms": {k: round(float(np.median([s[k] for s in stats])), 2)
                         for k in ("t_total_ms", "t_sample_ms", "t_sample_gemm_ms", "t_levels_ms", "t_id_ms")},
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gauss65536", choices=sorted(WORKLOADS) + ["batched512", "serve"])
    ap.add_argument("--serve-requests", type=int, default=400, help="requests of the serve workload")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrival rate of the serve workload")
    ap.add_argument("--serve-workers", type=int, default=4, help="worker threads (streams) of the server")
    ap.add_argument("--serve-p-margin", default="32,192",
                    help="p_margin of served requests at rtol 1e-4 and at rtol 1e-6")
    ap.add_argument("--rtol", type=float, default=None)
    ap.add_argument("--p-margin", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-panel", type=int, default=2048)
    ap.add_argument("--no-frob", action="store_true", help="skip the exact ||A - A_HSS||_F check")
    ap.add_argument("--sample-prec", default="f64", choices=["f64", "f32", "bf16x3"],
                    help="precision of the sampling products (reduced modes need the FP32 A)")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload: skip the reduced-precision and serving lines")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="run one sampling step alone after a calibration copy (for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the compression path has no multi-GPU mode; "
              "whole matrices (batches, served requests) would shard one per GPU",
              file=sys.stderr)
        return 2
    if args.profile_kernels:
        return profile_kernels(args)
    if args.workload == "batched512":
        return run_batched(args)
    if args.workload == "serve":
        return run_serve(args)

    import numpy as np
    import torch

    import paper_1503_05464_amd as P
    import workloads as W

    cfg = dict(WORKLOADS[args.workload])
    if args.rtol is not None:
        cfg["rtol"] = args.rtol
    if args.p_margin is not None:
        cfg["p_margin"] = args.p_margin
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] workload {args.workload}: n={cfg['n']} rtol={cfg['rtol']} assembling A", file=sys.stderr,
          flush=True)
    pts = make_points(cfg)
    A = make_matrix(cfg, pts, dev)
    torch.cuda.synchronize()
    x = torch.from_numpy(np.random.default_rng(1).uniform(-1, 1, (cfg["n"], 1))).to(dev)
    b = torch.empty_like(x)
    kw = dict(rtol=cfg["rtol"], d0=cfg["d0"], dd=cfg["dd"], d_max=cfg["d_max"], leaf_size=cfg["leaf"],
              p_margin=cfg["p_margin"], seed=0, sample_prec=args.sample_prec)
    # workloads with a ULV solve: one N(0,1) right-hand side
    ulv = "ulv_rhs_seed" in cfg
    rhs = torch.from_numpy(W.normal_rhs(cfg["n"], 1, cfg["ulv_rhs_seed"])).to(dev) if ulv else None

    def step():
        h = P.hss_compress(A, **kw)
        P.hss_matvec(h, x, b)
        st = dict(P.hss_stats(h))
        if ulv:  # factor returns once the factors are written; solve is stream-ordered
            t1 = time.perf_counter()
            P.hss_factor(h)
            t2 = time.perf_counter()
            P.hss_solve(h, rhs)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            st["t_factor_ms"] = (t2 - t1) * 1e3
            st["t_solve_ms"] = (t3 - t2) * 1e3
        P.hss_destroy(h)
        return st

    for w in range(args.warmup):
        st = step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {w}: {st['t_total_ms']:.1f} ms d_final={st['d_final']} passes={st['passes']} "
              f"max_rank={st['max_rank']}", file=sys.stderr, flush=True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        stats.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = elapsed * 1e3 / max(1, args.steps)
    for k, st in enumerate(stats):
        print(f"[bench] step {k}: total {st['t_total_ms']:.1f} ms sample {st['t_sample_ms']:.1f} "
              f"levels {st['t_levels_ms']:.1f} id {st['t_id_ms']:.1f} ms", file=sys.stderr, flush=True)

    # dominant kernel: the sampling GEMM, measured with HIP events on its stream
    roofline = sampling_roofline(stats, args.sample_prec)
    if args.sample_prec == "f64" and args.workload == "gauss65536":
        roofline["traffic"] = measured_traffic("kernels_sample.hip", "pmc_sample_kernel_gauss65536.txt")
    levels = level_roofline(stats)

    # acceptance on a fresh compression (not timed)
    h = P.hss_compress(A, **kw)
    st = P.hss_stats(h)
    xs = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, (cfg["n"], 2))).to(dev)
    bh = P.hss_matvec(h, xs)
    bd = dense_matvec(A, xs)
    mv_err = float(torch.linalg.norm(bh - bd) / torch.linalg.norm(bd))
    solve_err = None
    if ulv:  # backward error of the ULV solution against the dense A: ||A x - b|| / (||A||_2 ||x||)
        P.hss_factor(h)
        xsol = P.hss_solve(h, rhs)
        r = dense_matvec(A, xsol) - rhs
        v = torch.ones((cfg["n"], 1), dtype=torch.float64, device=dev)
        for _ in range(20):  # ||A||_2 by power iteration (a lower bound)
            v = dense_matvec(A, v)
            v = v / torch.linalg.norm(v)
        anorm = float(torch.linalg.norm(dense_matvec(A, v)))
        solve_err = float(torch.linalg.norm(r)) / (anorm * float(torch.linalg.norm(xsol)))
    frob = None
    if not args.no_frob:
        frob = frob_error(P, h, A)
    P.hss_destroy(h)
    extras = {}
    if args.workload == "gauss65536" and args.sample_prec == "f64" and not args.no_extras:
        # the precision sweep on the same matrix and rtol, then a bounded
        # serving run above and one below the device's capacity
        extras["precision_sweep"] = {p: precision_sweep(P, A, kw, p, 2) for p in ("bf16x3", "f32")}
    del A
    torch.cuda.empty_cache()
    if extras:
        extras["serve"] = {"offered_200_per_s": serve_measure(300, 200.0, args.serve_workers),
                           "offered_4_per_s": serve_measure(60, 4.0, args.serve_workers)}

    cpu = None
    if not args.no_cpu_baseline and pts is not None:
        print("[bench] cpu baseline (oracle, bounded sample)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg, pts, st["d_final"], args.cpu_panel)

    headline = "HSS compress s at N=65536 rtol1e-6 + % GEMM roofline; p50/p99 req latency"
    out = {
        "metric": headline if args.workload == "gauss65536" else
        f"HSS {'compress + ULV factor/solve' if ulv else 'compress'} s per step at N={cfg['n']} "
        f"rtol{cfg['rtol']:g}",
        "value": round(ms / 1e3, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.sample_prec == "f64" else f"{args.sample_prec} sampling, f64 ID",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: n={cfg['n']} {cfg['kind']} kernel, A {cfg['storage']}, "
                        f"leaf {cfg['leaf']}, rtol {cfg['rtol']}, d0 {cfg['d0']}, dd {cfg['dd']}, "
                        f"p_margin {cfg['p_margin']}, {args.sample_prec.upper()} sampling",
            "sample_prec": args.sample_prec,
            "n": cfg["n"], "rtol": cfg["rtol"], "d_final": st["d_final"], "passes": st["passes"],
            "max_rank": st["max_rank"], "converged": bool(st["converged"]),
            "step": "hss_compress + hss_matvec(nrhs=1) + " + ("hss_factor + hss_solve(nrhs=1) + " if ulv else "")
                    + "hss_destroy",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "level_roofline": levels,
        "accuracy": {"matvec_rel_err_vs_dense": mv_err, "frob_rel_err": frob, "bound": 10 * cfg["rtol"],
                     **({"solve_backward_err": solve_err} if ulv else {})},
        **extras,
        "breakdown_ms": {k: round(float(np.median([s[k] for s in stats])), 2)
                         for k in ("t_total_ms", "t_sample_ms", "t_sample_gemm_ms", "t_levels_ms", "t_id_ms")
                         + (("t_factor_ms", "t_solve_ms") if ulv else ())},
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
