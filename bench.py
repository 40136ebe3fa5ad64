"""Benchmark of the lattice-sum library on one MI355X.

Workload (default, `--workload mix`): the served mixed workload -- the first requests of a seeded
stream of 10,000 lattice sums with Poisson arrivals: per request L uniform in [8, 96] per axis
(rectangular), N in {257, ..., 4097} for the longest axis, kernel Newton / Yukawa (kappa 0.5) /
Slater (lambda 1), 0-500 vacancies or impurities, eps in {1e-4, 1e-6}, each a Tucker result
(RHOSVD) with the potential sampled at 1000 points resident in HBM.  One step is one request:
quadrature, collocation, shift-sums, defect assembly, side matrices, certified truncated SVD,
projections, core, and the values at its points.  `--warmup W` requests run untimed, then
`--steps K` are timed.

Two paths on the same GPU:
  * served: all K requests submitted to a context with several slots (continuous batching,
    admission by the HBM budget), reference vectors shared through the cache, FP32 contractions
    where eps = 1e-4 (their arithmetic error, a few 1e-7, is far below eps);
  * plain FP64: one request at a time, one slot, no batching, no reference cache, FP64 everywhere.
`value` is the served throughput (lattice sums/s); `latency_ms` is p50/p99 from submission to
completion with the stream's own Poisson gaps scaled to 0.8 x the served capacity.  Beside it:
the plain throughput and latency, each request's error against the oracle's direct sum, the
roofline of the dominant stage (event-timed inside the library), the oracle's same method on the
host cores, and the config-2 stream (the 64^3 canonical lattice with 1e5 points per sum, where
the sampling and shift-sum kernels are HBM-bound) as `secondary_cfg2`.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload mix|cfg2|cfg3|cfg4|timesL|extras]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# One hardware queue per stream: the library runs several slot streams plus three per-mode SVD
# streams per slot, and HIP's default of 4 queues per process makes some of them share a queue
# (the three concurrent SVDs of the first context then take 1.6x longer).  An environment that
# already exports the default is raised too.  Must be set before the HIP runtime starts.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16x3": 2500.0 / 3}
METRIC = "lattice sums/s served vs plain FP64 at 1e-6 rel err; p50/p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed requests (default: 20 for the served mix, 2048 for the config-2 stream)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed requests before them (5 / 128)")
    ap.add_argument("--workload", default="mix", choices=["cfg2", "cfg3", "cfg4", "mix", "timesL", "extras", "shiftrect"])
    ap.add_argument("--inflight", type=int, default=64)
    ap.add_argument("--slots", type=int, default=3)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--chunk", type=int, default=32,
                    help="requests per submit call of the served stream (one batch each)")
    ap.add_argument("--plain-steps", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy (for scaling HBM counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain device-to-device copy of known size: 512 MiB read + 512 MiB written per launch."""
    import torch
    a = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": a.numel() * 8, "launches": 5}))


def percentile(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def run_stream(L, ctx, problem, points, outs, steps, inflight, chunk=1):
    """Submit `steps` requests keeping at most `inflight` in flight, `chunk` at a time: each chunk
    is a RequestSet (one lsum_submit_many call), submitted once that many have finished and
    harvested with one lsum_finish_many call; returns (seconds, latencies).  `problem` is
    marshalled once (L.prepare); the library copies it at every submit."""
    import torch
    from collections import deque
    q = deque()
    lat = []
    n_in = 0

    def harvest():
        nonlocal n_in
        rs = q.popleft()
        status, infos = rs.finish()
        for k in range(rs.n):
            if status[k] != 0:
                raise RuntimeError(f"request failed: {status[k]}")
            lat.append(infos[k].t_queue_ms + infos[k].t_run_ms)
        n_in -= rs.n

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i = 0
    while i < steps:
        k = min(chunk, steps - i, inflight)
        while n_in + k > inflight:
            harvest()
        q.append(ctx.submit_set(problem, k, points=points, values=[outs[(i + j) % len(outs)] for j in range(k)]))
        n_in += k
        i += k
    while q:
        harvest()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, lat


def dominant_roofline(prof: dict, dtype_peak: str):
    """The stage with the largest GPU time: achieved = algorithmic work per launch / mean launch time."""
    # stages with an algorithmic byte or flop count (the iterative SVD has its own limit: time only)
    prof = {k: v for k, v in (prof or {}).items() if v["bytes"] > 0 or v["flops"] > 0}
    if not prof:
        return None, None
    name, st = max(prof.items(), key=lambda kv: kv[1]["ms"])
    n = max(1, st["launches"])
    ms = st["ms"] / n
    if st["flops"] > 0 and st["bytes"] == 0 or name in ("core", "tile", "projection", "norm"):
        achieved = st["flops"] / n / (ms * 1e-3) / 1e12
        # the SVD and the norm are FP64 at every precision; the contractions take the request's
        peak = PEAK_TFLOPS["f64" if name in ("svd", "norm") else dtype_peak]
        return name, {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                      "frac": achieved / peak, "traffic": None, "kernel_stage": name,
                      "avg_launch_ms": ms, "launches": st["launches"],
                      "work_per_launch": st["flops"] / n}
    achieved = st["bytes"] / n / (ms * 1e-3) / 1e9
    return name, {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel_stage": name,
                  "avg_launch_ms": ms, "launches": st["launches"], "bytes_per_launch": st["bytes"] / n}


def traffic_from_profiles(name: str, units_per_launch: float):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries: FETCH_SIZE and WRITE_SIZE
    per unit of work (a request's points, a shift-sum job), each scaled by what the counter reads
    for a plain copy of known size, times the units one launch of this run processes.  None
    unless the counters were taken on the current kernel source (the recorded hash matches)."""
    path = os.path.join(ROOT, "profiles", f"pmc_{name}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        src = os.path.join(ROOT, rec["source"])
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if sha != rec.get("source_sha256"):
            return None
        return rec["hbm_bytes_per_unit"] * units_per_launch
    except Exception:
        return None


def cpu_baseline(problem, xyz, seconds):
    """The oracle (plain numpy FP64, same method) on the host cores: lattice sums/s."""
    import oracle as O
    try:
        import psutil
        proc = psutil.Process()
    except Exception:
        proc = None
    n = 0
    c0 = proc.cpu_times() if proc else None
    t0 = time.perf_counter()
    while True:
        O.canonical_pipeline(problem, xyz)
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    wall = time.perf_counter() - t0
    cores = None
    if proc:
        c1 = proc.cpu_times()
        cores = round(((c1.user - c0.user) + (c1.system - c0.system)) / wall, 2)
    # the oracle's direct sum (every charge at every point, no factorisation over the axes)
    t, _ = O.quadrature_of(problem)
    n_charges = len(O.charges(problem)[0])
    cells = O.points_to_cells(xyz[:8], problem.h, problem.N)
    d0 = time.perf_counter()
    O.brute_force_points(problem, cells)
    dwall = time.perf_counter() - d0
    return {"value": n / wall, "unit": "lattice sums/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} full lattice sums of the same workload (nodes, collocation, 1D shift-sums, "
                      f"{len(xyz)} sampled points) in {wall:.1f} s", "host_cpus": os.cpu_count(),
            "direct_sum": {"value": len(cells) * n_charges * len(t) / dwall, "unit": "point-charge-node terms/s",
                           "sample": f"{len(cells)} points x {n_charges} charges x {len(t)} nodes in {dwall:.2f} s"}}


def _oracle_request(p):
    """One request by the oracle's same method: canonical terms, LAPACK SVD of the literal side
    matrices with the certified truncation, the core by canonical projection, values at 3 cells."""
    import oracle as O
    t0 = time.perf_counter()
    xi, A = O.canonical_terms(p)
    res = O.rhosvd(xi, A, eps=p.eps)
    cells = np.stack([np.array([(n - 1) // 2, n // 3, (2 * n) // 3]) for n in p.N], axis=1)
    O.tucker_points(res.core, res.Z, cells)
    return time.perf_counter() - t0


def mix_cpu_baseline(probs, seconds):
    """The oracle's same method on the host cores: one worker process per core (at most 16, one
    BLAS thread each) takes requests smallest first (by literal side-matrix size, those under
    about 1.5 GB of side matrices and Grams) until `seconds` have passed; unfinished ones are
    abandoned.  `probs` are the timed requests followed by later ones of the same stream (so that
    every worker has work); the indices of the finished ones are returned in "finished"."""
    import multiprocessing as mp
    try:
        import psutil
        proc = psutil.Process()
    except Exception:
        proc = None
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    workers = max(1, min(16, ncpu))
    def mem(p):
        rhat = p.M * (1 + len(p.defects))
        return 8.0 * rhat * (sum(p.N) + 3 * rhat)
    cand = sorted((k for k in range(len(probs)) if mem(probs[k]) < 1.5e9), key=lambda k: mem(probs[k]))
    old = {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for v in old:
        os.environ[v] = "1"
    c0 = proc.cpu_times() if proc else None
    t0 = time.perf_counter()
    pool = mp.get_context("spawn").Pool(workers)
    for v, x in old.items():
        if x is None:
            os.environ.pop(v, None)
        else:
            os.environ[v] = x
    jobs = {k: pool.apply_async(_oracle_request, (probs[k],)) for k in cand}
    done = {}
    while time.perf_counter() - t0 < seconds and len(done) < len(jobs):
        for k, j in jobs.items():
            if k not in done and j.ready():
                done[k] = j.get()
        time.sleep(0.05)
    wall = time.perf_counter() - t0
    pool.terminate()
    pool.join()
    cores = None
    if proc:
        c1 = proc.cpu_times()
        used = sum(getattr(c1, f) - getattr(c0, f) for f in ("user", "system", "children_user", "children_system"))
        cores = round(used / wall, 2)
    ks = sorted(done)
    return {"value": len(ks) / wall, "unit": "lattice sums/s", "cores": cores, "kind": "oracle",
            "workers": workers, "host_cpus": ncpu,
            "sample": f"{len(ks)} of {len(probs)} served-mix requests (the timed ones and the next ones of the same "
                      f"stream) finished in {wall:.1f} s by {workers} worker processes (one BLAS thread each), "
                      f"smallest first; each: canonical terms, LAPACK SVD of the literal side matrices with the "
                      f"certified truncation, core by canonical projection, values at 3 cells",
            "seconds_per_request": {str(k): round(done[k], 2) for k in ks},
            "finished": ks}


def run_shift_rect(n_req=1024):
    """The batched shift-sum on config-5-shaped lattices: n_req canonical requests (no defects,
    FP64 point-major rows) with the served mix's rectangular L in [8, 96] per axis, grids of
    257..4097 cells, the three kernels -- every axis a job of its own (no two axes alike) --
    submitted together as one batch, so that all their shift-sums run as one launch."""
    import paper_1411_1994_amd as L
    import workloads as W
    rng = np.random.default_rng(W.SEED_BASE + 77)
    probs = [W.Problem(**{**W.served_request(rng, i).__dict__, "defects": [], "eps": 0.0, "precision": W.FP64})
             for i in range(n_req)]
    ctx = L.Context(0, n_slots=1)
    ctx.set_option(L.OPT_MAX_BATCH, n_req)
    ctx.set_option(L.OPT_AUTOTUNE, 0)      # the fixed tile rule (48 nodes per workgroup at this size)
    prepared = [L.prepare(p) for p in probs]
    for attempt in range(2):               # the first run fills the reference and window caches
        ctx.reset_profile()
        reqs = ctx.submit_many(prepared)
        for r in reqs:
            if r.wait() != 0:
                raise RuntimeError(f"rectangular shift-sum request failed: {r.stats().get('error')}")
        jobs = sum(sum(1 for l in range(3) if r.stats()["axis_src"][l] == l) for r in reqs)
        for r in reqs:
            r.release()
    prof = ctx.profile()
    ctx.close()
    _, roof = dominant_roofline({"shift_sum": prof["shift_sum"]}, "f64")
    if roof is not None:
        roof["jobs_per_launch"] = jobs / max(1, prof["shift_sum"]["launches"])
        roof["requests_per_launch"] = n_req / max(1, prof["shift_sum"]["launches"])
        roof["traffic"] = traffic_from_profiles("shift_sum_rect", roof["jobs_per_launch"])
        roof["workload"] = (f"{n_req} canonical requests of the served mix's shapes (L in [8, 96] per axis, "
                            f"N 257..4097, Newton/Yukawa/Slater, FP64 rows), one batch")
    return roof


def run_mix(args):
    """The served mixed workload: requests of the seeded 10,000-request stream (uneven lattice,
    grid, kernel, defect count and eps); `warmup` requests untimed, then `steps` requests served
    on several slots (continuous batching, admission by the HBM budget) against the plain FP64
    path on the same requests one at a time, then again under Poisson arrivals at 0.8 x the
    served capacity for latency."""
    import torch
    import oracle as O
    import paper_1411_1994_amd as L
    import workloads as W

    steps, warmup = args.steps, args.warmup
    stream = W.served_mix_stream(warmup + steps)
    gaps = [g for g, _ in stream]
    probs = [p for _, p in stream]
    n_pts = 1000
    pts = [torch.from_numpy(W.sample_points(5, n_pts, W.half_widths(p)) * 0.999).cuda() for p in probs]
    outs = [torch.zeros(n_pts, dtype=torch.float64, device="cuda") for _ in probs]
    torch.cuda.synchronize()

    probe, sweeps = {}, {}

    def closed(ctx, idx, inflight):
        """Submit the requests idx keeping at most `inflight` in flight; (seconds, latencies)."""
        from collections import deque
        q, lat = deque(), {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        i = 0
        while i < len(idx) or q:
            while i < len(idx) and len(q) < inflight:
                k = idx[i]
                q.append((k, ctx.submit(L.prepare(probs[k]), points=pts[k], values=outs[k])))
                i += 1
            k, r = q.popleft()
            rc = r.wait()
            if rc != 0:
                raise RuntimeError(f"request {k} failed: {rc} {r.stats().get('error')}")
            inf = r.info()
            lat[k] = inf.t_queue_ms + inf.t_run_ms
            probe[k] = (inf.probe_err, inf.rel_bound)
            st = r.stats()
            sweeps[k] = (sum(st["sweeps"]), sum(st["jacobi_persistent"]), sum(st["jacobi_aborted"]))
            r.release()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, lat

    warm_idx = list(range(warmup))
    timed_idx = list(range(warmup, warmup + steps))

    # ---- served: continuous batching on several slots ----------------------------------
    sctx = L.Context(0, n_slots=args.slots)
    sctx.set_option(L.OPT_MAX_BATCH, args.batch)
    if warm_idx:
        closed(sctx, warm_idx, 2 * args.slots)
    sctx.reset_profile()
    s_secs, s_lat = closed(sctx, timed_idx, 2 * args.slots)
    prof = sctx.profile()
    tuning = sctx.tuning()
    served = steps / s_secs
    served_vals = {k: outs[k].cpu().numpy().copy() for k in timed_idx}
    infos = {}

    # ---- plain FP64: one request at a time, one slot, no batching, no reference cache ----
    pctx = L.Context(0, n_slots=1)
    pctx.set_option(L.OPT_MAX_BATCH, 1)
    pctx.set_option(L.OPT_REF_CACHE_BYTES, 0)
    pctx.set_option(L.OPT_AUTOTUNE, 0)       # fixed launches: round-by-round sweeps, no graphs
    plain_probs = [W.Problem(**{**p.__dict__, "precision": W.FP64}) for p in probs]
    plain_s, p_lat, plain_vals = {}, {}, {}
    for k in ([warm_idx[0]] if warm_idx else []) + timed_idx:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = pctx.submit(L.prepare(plain_probs[k]), points=pts[k], values=outs[k])
        if r.wait() != 0:
            raise RuntimeError(f"plain request {k} failed: {r.stats().get('error')}")
        torch.cuda.synchronize()
        plain_s[k] = time.perf_counter() - t0
        inf = r.info()
        p_lat[k] = inf.t_queue_ms + inf.t_run_ms
        infos[k] = {"r": list(inf.r), "bound": inf.bound, "norm_A": inf.norm_A}
        r.release()
        plain_vals[k] = outs[k].cpu().numpy().copy()
    pctx.close()
    plain = steps / sum(plain_s[k] for k in timed_idx)

    # ---- open loop: the stream's own Poisson gaps at 0.8 x the served capacity ---------
    rate = 0.8 * served
    arrivals = np.cumsum([gaps[k] for k in timed_idx]) / rate
    pending, o_lat = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, k in zip(arrivals, timed_idx):
        while time.perf_counter() - t0 < a:
            time.sleep(0.0002)
        pending.append(sctx.submit(L.prepare(probs[k]), points=pts[k], values=outs[k]))
    for r in pending:
        if r.wait() != 0:
            raise RuntimeError("open-loop request failed")
        inf = r.info()
        o_lat.append(inf.t_queue_ms + inf.t_run_ms)
        r.release()
    o_secs = time.perf_counter() - t0
    sctx.close()

    # ---- accuracy: every timed request against the oracle's direct sum at 3 points ------
    errs, devs = [], []
    for k in timed_idx:
        p = probs[k]
        xyz = pts[k][:3].cpu().numpy()
        cells = O.points_to_cells(xyz, p.h, p.N)
        ref = O.brute_force_points(p, cells)
        scale = np.max(np.abs(ref))
        errs.append(float(np.max(np.abs(served_vals[k][:3] - ref)) / scale))
        devs.append(float(np.max(np.abs(served_vals[k] - plain_vals[k])) / np.max(np.abs(plain_vals[k]))))
    eps_of = [probs[k].eps for k in timed_idx]

    stage, roof = dominant_roofline(prof, "f64")
    mfma = {}
    for st_name in ("svd", "core", "projection", "sample"):
        if st_name in prof and prof[st_name]["flops"] > 0 and prof[st_name]["ms"] > 0:
            v = prof[st_name]
            tf = v["flops"] / (v["ms"] * 1e-3) / 1e12
            pk = PEAK_TFLOPS["f64"] if st_name == "svd" else None
            mfma[st_name] = {"tflops": tf, "ms_per_launch": v["ms"] / max(1, v["launches"]),
                             "launches": v["launches"], "frac_of_f64_peak": tf / PEAK_TFLOPS["f64"],
                             "frac_of_f32_peak": tf / PEAK_TFLOPS["f32"]}
    out = {
        "metric": METRIC,
        "value": served,
        "unit": "lattice sums/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1000.0 / served,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "served-mix", "stream": "first requests of the seeded 10,000-request stream "
                   "(numpy default_rng(1411_1994 + 5))", "requests_timed": steps,
                   "requests_warmup": warmup, "timed_request_indices": [warmup, warmup + steps - 1],
                   "slots": args.slots, "sample_points_per_request": n_pts,
                   "L_max": max(max(probs[k].blocks[0].L) for k in timed_idx),
                   "N_max": max(max(probs[k].N) for k in timed_idx),
                   "defects_max": max(len(probs[k].defects) for k in timed_idx),
                   "eps": sorted(set(eps_of)),
                   "precision": "FP32 contractions at eps 1e-4, FP64 at 1e-6; Gram/SVD/truncation FP64"},
        "latency_ms": {"p50": percentile(o_lat, 50), "p99": percentile(o_lat, 99),
                       "arrivals": f"Poisson at {rate:.2f}/s (0.8 x served capacity), {steps} requests in {o_secs:.2f} s"},
        "latency_closed_loop_ms": {"p50": percentile(list(s_lat.values()), 50),
                                   "p99": percentile(list(s_lat.values()), 99)},
        "plain_fp64": {"value": plain, "unit": "lattice sums/s",
                       "latency_ms": {"p50": percentile([p_lat[k] for k in timed_idx], 50),
                                      "p99": percentile([p_lat[k] for k in timed_idx], 99)}},
        "served_over_plain": served / plain,
        "max_rel_err_vs_oracle": max(errs),
        "rel_err_vs_oracle_per_request": errs,
        "all_within_eps": bool(all(e <= ep for e, ep in zip(errs, eps_of))),
        "max_rel_dev_served_vs_plain": max(devs),
        "stated_error": {"what": "each result's own statement (lsum_info.probe_err): max-norm relative deviation "
                                 "from the untruncated FP64 canonical sum at 32 seeded cells, and its certified "
                                 "Frobenius bound relative to ||A|| (rel_bound)",
                         "probe_err_max": max(probe[k][0] for k in timed_idx),
                         "probe_err_per_request": [probe[k][0] for k in timed_idx],
                         "rel_bound_per_request": [probe[k][1] for k in timed_idx]},
        "roofline": roof,
        "mfma_stages": mfma,
        "autotuner": tuning,
        "jacobi_sweeps": {"total": sum(sweeps[k][0] for k in timed_idx),
                          "persistent": sum(sweeps[k][1] for k in timed_idx),
                          "persistent_aborted": sum(sweeps[k][2] for k in timed_idx)},
        "stages": {k: {"ms_per_launch": v["ms"] / max(1, v["launches"]), "launches": v["launches"]}
                   for k, v in prof.items()},
    }
    if not args.no_cpu:
        extra = [p for _, p in W.served_mix_stream(warmup + steps + 200)[warmup + steps:]]
        cprobs = [probs[k] for k in timed_idx] + extra
        cb = mix_cpu_baseline(cprobs, args.cpu_seconds)
        # the plain FP64 GPU path on exactly the requests the oracle finished
        done = cb.pop("finished")
        if done:
            gctx = L.Context(0, n_slots=1)
            gctx.set_option(L.OPT_MAX_BATCH, 1)
            gctx.set_option(L.OPT_REF_CACHE_BYTES, 0)
            gctx.set_option(L.OPT_AUTOTUNE, 0)
            gs = 0.0
            for k in done:
                p = W.Problem(**{**cprobs[k].__dict__, "precision": W.FP64})
                t0 = time.perf_counter()
                r = gctx.submit(L.prepare(p))
                if r.wait() != 0:
                    raise RuntimeError("plain request for the CPU comparison failed")
                gs += time.perf_counter() - t0
                r.release()
            gctx.close()
            cb["plain_fp64_gpu_on_same_requests"] = {"value": len(done) / gs, "unit": "lattice sums/s",
                                                     "requests": len(done)}
        out["cpu_baseline"] = cb
    return out


# The sizes of Table Table_timesL: L^3 unit charges on an L x L x L lattice, grid N_L per axis
# (N_L / L cells per lattice spacing), mesh size 0.0034, Tucker output at eps = 1e-6.
TIMES_L = [(16, 5632), (32, 9728), (64, 17920), (128, 34304)]


def run_times_l(args):
    """Time per lattice sum in Tucker format for the lattice sizes of Table Table_timesL, by the
    Tucker-reference sum (Thm thm:sumCaseE (B)) and by canonical assembly + RHOSVD, with M the
    smallest meeting 1e-6 in the max norm; values checked against the plain sum at a few cells."""
    import oracle as O
    import paper_1411_1994_amd as L
    import workloads as W

    h, eps = 0.0034, 1e-6
    steps = max(1, min(args.steps, 5))
    rows = []
    with L.Context(0, n_slots=1) as ctx:
        for Lsz, NL in TIMES_L:
            N = (NL + 1,) * 3
            M, m_err = L.lsum_choose_M(W.NEWTON, 0.0, N, h, 1e-6, 128)
            blk = W.Block((Lsz,) * 3, ((NL // Lsz) * h,) * 3, (0.0, 0.0, 0.0))
            rng = np.random.default_rng(W.SEED_BASE + Lsz)
            cells = np.stack([rng.integers(0, n, 4) for n in N], axis=1)
            xyz = np.stack([(cells[:, a] - (N[a] - 1) // 2) * h for a in range(3)], axis=1)
            row = {"L": Lsz, "sites": Lsz ** 3, "N": N[0], "M": M, "sinc_max_norm_err": m_err}
            for name, method in (("tucker_ref", 1), ("canonical_rhosvd", 0)):
                p = W.Problem("timesL", W.NEWTON, 0.0, M, N, h, [blk], eps=eps, method=method)
                prepared = L.prepare(p)
                r = ctx.submit(prepared)                       # warm-up (reference caches)
                if r.wait() != 0:
                    raise RuntimeError(f"{name} L={Lsz} failed: {r.stats()}")
                r.release()
                t = []
                for _ in range(steps):
                    t0 = time.perf_counter()
                    r = ctx.submit(prepared)
                    rc = r.wait()
                    t.append(time.perf_counter() - t0)
                    if rc != 0:
                        raise RuntimeError(f"{name} L={Lsz} failed")
                    vals = r.sample(xyz)
                    ranks = tuple(r.info().r)
                    stages = r.stats().get("t_ms", {})
                    r.release()
                row[name] = {"s_per_sum": float(np.median(t)), "ranks": ranks, "vals": vals,
                             "stages_ms": stages}
            ref = O.brute_force_points(W.Problem("timesL", W.NEWTON, 0.0, M, N, h, [blk]), cells)
            for name in ("tucker_ref", "canonical_rhosvd"):
                v = row[name].pop("vals")
                row[name]["max_rel_err_vs_oracle"] = float(np.max(np.abs(v - ref)) / np.max(np.abs(ref)))
            rows.append(row)
            print(json.dumps({"progress": "timesL", "L": Lsz, "tucker_ref_s": row["tucker_ref"]["s_per_sum"],
                              "canonical_rhosvd_s": row["canonical_rhosvd"]["s_per_sum"]}), file=sys.stderr,
                  flush=True)
    last = rows[-1]["tucker_ref"]["s_per_sum"]
    out = {
        "metric": "time per Tucker lattice sum vs L^3 (Table Table_timesL)",
        "value": 1.0 / last,
        "unit": "lattice sums/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 1,
        "ms_per_step": 1000.0 * last,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "timesL", "largest": "128^3 sites, N = 34305, h = 0.0034", "eps": eps,
                   "method": "tucker_ref"},
        "sizes": rows,
        "paper_seconds_matlab_cpu": [1.8, 0.8, 3.1, 15.8],
    }
    print(json.dumps(out))


def _timed(fn, reps=3):
    best = None
    out = None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return best, out


def run_extras(args):
    """Timings of the paths beyond the served lattice sum, each with an accuracy check: the choice
    of M, a parallelogram lattice (Sec. 4.4 case (B)), ALS after the RHOSVD (Thm thm:C2Tucker (b)),
    the canonical form of a Tucker result (Can -> Tuck -> Can) and the Galerkin matrix (eq.
    nuc_pot)."""
    import oracle as O
    import paper_1411_1994_amd as L
    import workloads as W

    out = {"metric": "extra paths: time per call", "n_gpus": 1, "data": "synthetic", "dtype": "f64",
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "warmup": 1}
    rng = np.random.default_rng(W.SEED_BASE + 900)
    # choice of M (host): N = 4097, eps = 1e-6
    t, (M, err) = _timed(lambda: L.lsum_choose_M(W.NEWTON, 0.0, (4097,) * 3, 5 / 256, 1e-6, 128))
    out["choose_M"] = {"ms": 1e3 * t, "M": M, "max_norm_err": err, "N": 4097}
    with L.Context(0, n_slots=1) as ctx:
        # parallelogram lattice: 32 x 32 x 8 sites, x moving 0.4 per step along y, N = 1025
        base = W.Block((32, 32, 8), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
        blocks = [W.Block(b.L, b.b, b.center, b.charge) for b in L.lsum_shear_blocks(base, 0, 1, 0.4)]
        p = W.Problem("shear", W.NEWTON, 0.0, 36, (1025, 1025, 513), 1 / 16, blocks)
        pts = np.stack([rng.integers(0, n, 100_000) for n in p.N], axis=1)
        xyz = np.stack([(pts[:, a] - (p.N[a] - 1) // 2) * p.h for a in range(3)], axis=1)
        prep = L.prepare(p)

        def shear_run():
            r = ctx.submit(prep, points=xyz, values=np.zeros(len(xyz)))
            assert r.wait() == 0
            v = r.values.copy()
            r.release()
            return v
        t, v = _timed(shear_run)
        pos = O.shear_sites(base, 0, 1, 0.4)
        ref = O.brute_force_points_at(p, pts[:4], pos, np.ones(len(pos)))
        out["parallelogram"] = {"ms_per_sum": 1e3 * t, "sites": len(pos), "sub_blocks": len(blocks),
                                "sample_points": len(xyz),
                                "max_rel_err_vs_oracle": float(np.max(np.abs(v[:4] - ref)) / np.max(np.abs(ref)))}
        # ALS after the RHOSVD: 12^3 lattice with 10 defects, eps = 1e-3, N = 129 (ranks about 60,
        # inside the ALS limit r_a r_b <= 4096 and the 128 x 128 core slices of Can -> Tuck -> Can)
        blk = W.Block((12, 12, 12), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
        defects = W.draw_defects(np.random.default_rng(5), [blk], 5, 5)
        res = {}
        for sweeps in (0, 2):
            q = W.Problem("als", W.NEWTON, 0.0, 32, (129, 129, 129), 1 / 4, [blk], defects, eps=1e-3,
                          als_sweeps=sweeps)
            prep = L.prepare(q)

            def tucker_run():
                r = ctx.submit(prep)
                assert r.wait() == 0
                return r
            t, r = _timed(tucker_run, 2)
            st = r.stats()
            cells = np.stack([rng.integers(0, n, 4) for n in q.N], axis=1)
            vals = r.sample(np.stack([(cells[:, a] - 64) * q.h for a in range(3)], axis=1))
            ref = O.brute_force_points(q, cells)
            res[sweeps] = {"ms": 1e3 * t, "ranks": list(r.info().r), "als_ms": st["t_ms"].get("als", 0.0),
                           "als_core_norm": st["als_core_norm"],
                           "max_rel_err_vs_oracle": float(np.max(np.abs(vals - ref)) / np.max(np.abs(ref)))}
            if sweeps == 2:
                # the same Tucker result in canonical form at eps = 1e-6
                tc, (xi, U, e) = _timed(lambda: r.tucker_to_canonical(1e-6), 2)
                out["tucker_to_canonical"] = {"ms": 1e3 * tc, "rank": len(xi), "frobenius_err": e}
                # Galerkin matrix in 64 Gaussians
                alpha = rng.uniform(0.5, 2.0, 64)
                A = rng.uniform(-6.0, 6.0, (64, 3))
                x = (np.arange(129) - 64) * q.h
                G = [np.exp(-alpha[:, None] * (x[None, :] - A[:, l][:, None]) ** 2) for l in range(3)]
                tg, V = _timed(lambda: r.galerkin(G), 2)
                out["galerkin"] = {"ms": 1e3 * tg, "basis": 64, "N": 129, "symmetric_dev":
                                   float(np.max(np.abs(V - V.T)) / np.max(np.abs(V)))}
            r.release()
        out["rhosvd"] = res[0]
        out["rhosvd_als2"] = res[2]
    out["value"] = out["parallelogram"]["ms_per_sum"]
    out["unit"] = "ms per parallelogram lattice sum"
    out["steps"] = 3
    out["ms_per_step"] = out["value"]
    out["config"] = {"workload": "extras"}
    print(json.dumps(out))


def per_precision(L, W, problem, xyz):
    """The reduction request in FP64, FP32 and split-BF16x3: MFMA rate of the core and of the
    tile's mode products (event-timed stage time, algorithmic flops), and each result's deviation
    from the FP64 one (the tile if the request has one, else the values at the sample points)."""
    res, ref = {}, None
    for name, prec in (("f64", W.FP64), ("f32", W.FP32), ("bf16x3", W.BF16X3)):
        ctx = L.Context(0, n_slots=1)
        r = ctx.submit(W.Problem(**{**problem.__dict__, "precision": prec}), points=xyz)
        if r.wait() != 0:
            raise RuntimeError(f"{name} request failed")
        prof = ctx.profile()
        vals = r.tile().astype(np.float64) if problem.tile_T[0] > 0 else r.values.copy()
        st = r.stats()
        svd = {"ranks": list(r.info().r), "range_basis": st["range_k"], "jacobi_sweeps": st["sweeps"]}
        r.release()
        ctx.close()
        if ref is None:
            ref = vals
        entry = {"max_rel_dev_vs_f64": float(np.max(np.abs(vals - ref)) / np.max(np.abs(ref))), "svd": svd}
        peak = PEAK_TFLOPS[name]
        for stage in ("core", "tile", "projection"):
            if stage in prof and prof[stage]["ms"] > 0:
                tf = prof[stage]["flops"] / (prof[stage]["ms"] * 1e-3) / 1e12
                entry[stage] = {"ms": prof[stage]["ms"], "tflops": tf, "peak": peak, "frac": tf / peak}
        res[name] = entry
        del vals
    return res


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (--gpus 1); it has no multi-GPU path",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "mix":
        if args.steps is None:
            args.steps = 20
        if args.warmup is None:
            args.warmup = 5
        out = run_mix(args)
        # the 64^3 canonical stream (config 2) beside it: the HBM-bound sampling and shift-sum.
        # It starts from a settled process: the mix's Python garbage collected (a collection
        # inside its timed stream of 2048 short requests would stall it) and the device idle.
        import gc
        import torch
        gc.collect()
        torch.cuda.synchronize()
        sec = argparse.Namespace(**{**vars(args), "steps": 2048, "warmup": 128, "no_cpu": True})
        c2 = run_cfg(sec, 2)
        out["secondary_cfg2"] = {k: c2[k] for k in ("value", "unit", "steps", "config", "latency_ms", "plain_fp64",
                                                    "served_over_plain", "served_fp64_rows", "served_exact_sites",
                                                    "max_rel_err_vs_oracle", "roofline", "roofline_shift_sum",
                                                    "roofline_shift_sum_batched", "dtype")}
        out["roofline_shift_sum_rect"] = run_shift_rect()
        print(json.dumps(out))
        return
    if args.workload == "shiftrect":
        print(json.dumps({"roofline_shift_sum_rect": run_shift_rect()}))
        return
    if args.steps is None:
        args.steps = 2048
    if args.warmup is None:
        args.warmup = 128
    if args.workload == "timesL":
        run_times_l(args)
        return
    if args.workload == "extras":
        run_extras(args)
        return
    cfg = {"cfg2": 2, "cfg3": 3, "cfg4": 4}[args.workload]
    print(json.dumps(run_cfg(args, cfg)))


def run_cfg(args, cfg):
    """A named configuration served as a stream of identical requests (config 2: the 64^3
    canonical stream; configs 3 and 4: reduction requests, a few steps), against the plain FP64
    path; returns the bench record."""
    import torch
    import oracle as O
    import paper_1411_1994_amd as L
    import workloads as W

    problem = W.config(cfg)
    fp64_rows = None
    if cfg == 2:
        # served policy for canonical output: FP32 factor rows (FP64 products and sums), whose
        # error (<= 3 roundings of 2^-24 per term for these positive sums) is far below 1e-6;
        # the same stream with FP64 rows is measured beside it
        fp64_rows = problem
        problem = W.Problem(**{**problem.__dict__, "precision": W.FP32})
    n_pts = 100_000 if cfg == 2 else 4096
    xyz = W.sample_points(cfg, n_pts, W.half_widths(problem))
    xyz_d = torch.from_numpy(xyz).cuda()
    steps, warmup = args.steps, args.warmup
    if cfg != 2:                     # reduction workloads take seconds per request
        steps, warmup = min(steps, 3), min(warmup, 1)
    n_out = min(args.inflight, steps) + 2
    outs = [torch.zeros(n_pts, dtype=torch.float64, device="cuda") for _ in range(n_out)]
    torch.cuda.synchronize()

    # ---- served path --------------------------------------------------------------------
    ctx = L.Context(0, n_slots=args.slots if cfg == 2 else 1)
    ctx.set_option(L.OPT_MAX_BATCH, args.batch)
    prepared = L.prepare(problem)
    run_stream(L, ctx, prepared, xyz_d, outs, warmup, args.inflight, args.chunk)
    ctx.reset_profile()
    secs, lat = run_stream(L, ctx, prepared, xyz_d, outs, steps, args.inflight, args.chunk)
    prof = ctx.profile()
    served = steps / secs
    served64 = None
    if fp64_rows is not None:
        vals32 = outs[(steps - 1) % len(outs)].cpu().numpy()
        p64 = L.prepare(fp64_rows)
        run_stream(L, ctx, p64, xyz_d, outs, warmup, args.inflight, args.chunk)
        s64, lat64 = run_stream(L, ctx, p64, xyz_d, outs, steps, args.inflight, args.chunk)
        vals64 = outs[(steps - 1) % len(outs)].cpu().numpy()
        served64 = {"value": steps / s64, "unit": "lattice sums/s",
                    "latency_ms": {"p50": percentile(lat64, 50), "p99": percentile(lat64, 99)}}
    # the same stream with the sites at their exact positions (b/h = 51.2: five sub-cell classes
    # per axis, each with its own cached rows) instead of snapped to cell centres
    served_x = None
    if fp64_rows is not None:
        exact_problem = W.Problem(**{**problem.__dict__, "exact_sites": True})
        px = L.prepare(exact_problem)
        run_stream(L, ctx, px, xyz_d, outs, warmup, args.inflight, args.chunk)
        sx, latx = run_stream(L, ctx, px, xyz_d, outs, steps, args.inflight, args.chunk)
        valsx = outs[(steps - 1) % len(outs)].cpu().numpy()
        served_x = {"value": steps / sx, "unit": "lattice sums/s",
                    "latency_ms": {"p50": percentile(latx, 50), "p99": percentile(latx, 99)}}
    ctx.close()

    # ---- plain FP64 path: one at a time, no batching, no reference cache ----------------
    pctx = L.Context(0, n_slots=1)
    pctx.set_option(L.OPT_MAX_BATCH, 1)
    pctx.set_option(L.OPT_REF_CACHE_BYTES, 0)
    plain_problem = W.Problem(**{**problem.__dict__, "precision": W.FP64})
    psteps = min(args.plain_steps, steps) if cfg == 2 else 1
    plain_prepared = L.prepare(plain_problem)
    run_stream(L, pctx, plain_prepared, xyz_d, outs, min(8, psteps), 1)
    psecs, plat = run_stream(L, pctx, plain_prepared, xyz_d, outs, psteps, 1)
    plain = psteps / psecs
    pctx.close()

    # ---- the shift-sum over one batched launch of >= 1000 jobs (submitted together) ------
    ss_batched = None
    if cfg == 2:
        bctx = L.Context(0, n_slots=1)
        bctx.set_option(L.OPT_MAX_BATCH, 1024)
        ss_prob = L.prepare(fp64_rows)                        # FP64 point-major output
        reqs = bctx.submit_many([ss_prob] * 8)                # warm the reference and window cache
        for r in reqs:
            r.wait()
            r.release()
        bctx.reset_profile()
        reqs = bctx.submit_many([ss_prob] * 1024)
        for r in reqs:
            if r.wait() != 0:
                raise RuntimeError("batched shift-sum request failed")
        jobs = sum(1 for l in range(3) if reqs[0].stats()["axis_src"][l] == l) * len(reqs)
        for r in reqs:
            r.release()
        bprof = bctx.profile()
        bctx.close()
        _, ss_batched = dominant_roofline({"shift_sum": bprof["shift_sum"]}, "f64")
        if ss_batched is not None:
            ss_batched["jobs_per_launch"] = jobs / max(1, bprof["shift_sum"]["launches"])
            ss_batched["traffic"] = traffic_from_profiles("shift_sum_batched", ss_batched["jobs_per_launch"])

    # ---- accuracy of the served result against the oracle's brute-force sum ------------
    vals = vals32 if fp64_rows is not None else outs[(steps - 1) % len(outs)].cpu().numpy()
    sel = np.random.default_rng(7).choice(n_pts, 32, replace=False)
    cells = O.points_to_cells(xyz[sel], problem.h, problem.N)
    ref = O.brute_force_points(problem, cells)
    rel_err = float(np.max(np.abs(vals[sel] - ref)) / np.max(np.abs(ref)))
    if served64 is not None:
        served64["max_rel_err_vs_oracle"] = float(np.max(np.abs(vals64[sel] - ref)) / np.max(np.abs(ref)))
        served64["max_rel_dev_f32_rows"] = float(np.max(np.abs(vals - vals64)) / np.max(np.abs(vals64)))
    if served_x is not None:
        # the oracle's charge-by-charge sum at the exact positions, at 12 of the points; beside it
        # the distance of the snapped served result from that sum (the snapping error)
        sx_sel = sel[:12]
        refx = O.brute_force_points_exact(exact_problem, cells[:12])
        scale = np.max(np.abs(refx))
        served_x["max_rel_err_vs_oracle"] = float(np.max(np.abs(valsx[sx_sel] - refx)) / scale)
        served_x["snapped_rel_dev_from_exact"] = float(np.max(np.abs(vals[sx_sel] - refx)) / scale)

    # canonical output at FP32 precision: FP32-rounded factor rows, FP64 products and sums
    dtype = "f64" if problem.precision == W.FP64 else ("f32" if problem.precision == W.FP32 or cfg == 2 else "bf16x3")
    stage, roof = dominant_roofline(prof, dtype)
    if roof is not None and cfg == 2 and stage == "sample":
        # the counters were taken per request of 1e5 points on FP32 rows (the served policy)
        roof["traffic"] = traffic_from_profiles("sample", steps / max(1, prof["sample"]["launches"]))
    # the shift-sum kernel's own roofline beside the dominant one (small served batches: the
    # per-launch table reads make a per-job traffic figure meaningless, so none is given)
    roof_ss = None
    if "shift_sum" in prof and prof["shift_sum"]["launches"] > 0:
        _, roof_ss = dominant_roofline({"shift_sum": prof["shift_sum"]}, dtype)
    out = {
        "metric": METRIC,
        "value": served,
        "unit": "lattice sums/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1000.0 / served,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": problem.name, "kernel": "newton" if problem.kind == 0 else "yukawa",
                   "lattice_sites": problem.n_sites, "N": list(problem.N), "M": problem.M,
                   "sample_points": n_pts, "defects": len(problem.defects), "eps": problem.eps,
                   "slots": args.slots, "max_batch": args.batch, "inflight": args.inflight,
                   "submit_chunk": args.chunk},
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
        "plain_fp64": {"value": plain, "unit": "lattice sums/s",
                       "latency_ms": {"p50": percentile(plat, 50), "p99": percentile(plat, 99)}},
        "served_over_plain": served / plain,
        "served_fp64_rows": served64,
        "served_exact_sites": served_x,
        "max_rel_err_vs_oracle": rel_err,
        "roofline": roof,
        "roofline_shift_sum": roof_ss,
        "roofline_shift_sum_batched": ss_batched,
        "stages": {k: {"ms_per_launch": v["ms"] / max(1, v["launches"]), "launches": v["launches"]}
                   for k, v in prof.items()},
    }
    if cfg in (3, 4):
        out["precisions"] = per_precision(L, W, problem, xyz)
    if not args.no_cpu:
        cxyz = xyz if cfg == 2 else xyz[:1000]
        out["cpu_baseline"] = cpu_baseline(problem if cfg == 2 else W.Problem(**{**problem.__dict__, "defects": [], "eps": 0.0}),
                                           cxyz, args.cpu_seconds)
    return out


if __name__ == "__main__":
    main()
