"""Benchmark of one robust rotation solve on one MI355X.

A step is one whole solve (clear grid, vote, top-K, rescore, mask, readback of
q and the count) on the large workload: N = 1e6 correspondences at 99 %
outliers, G = 256 (64 MiB int32 grid), J = 2048 samples per circle, eps = 1.5
deg, K = 64.  Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  ``value`` is circle-sample votes per second of the whole
solve (N * J / seconds per solve); solves/s, the per-stage device times (HIP
events recorded on the solve stream inside the timed region), the roofline of
the dominant kernel and the CPU oracle's rate ride along, and so does the
metric's served half: after the timed solves, ``--serve-duration`` seconds (20
by default, 0 skips it) of the serve workload below, whose p99 latency is
``served_p99_ms``.

``--workload serve`` drives the request server with Poisson arrivals (2000
requests/s; N log-uniform on [1e3, 1e6]; G = 64 / 128 / 256 for N below 1e4 /
below 1e5 / above; J = 8G; outliers U[0.8, 0.99]; sigma 1 deg) and reports
throughput and latency percentiles; the requests are drawn from a resident
pool of seeded instances.

``--workload multi`` times a several-rotations solve (9 rotations in one scene);
``--workload rigid`` a rigid-pose solve from point correspondences (Sec. 4.5).

``--workload batch`` times the batched solve instead: a step is one
rot_vote_solve_batch over 4096 instances (N log-uniform on [100, 20000], G =
64, J = 512), reported with the same fields plus the one-solve-per-call loop
over the same instances.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "circle-sample votes/s + solves/s at N=1e6, 99% outliers; p99 latency served"

# Peak rates of one MI355X used for the roofline fractions.
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: one 32-bit vector operation per lane
# per clock (the 157.3 TFLOP/s fp32 figure counts an FMA as 2 and packed dual
# issue as 2 more, and packed fp32 is not used here).
ALU_PEAK_GOPS = 256 * 64 * 2.4

# Algorithmic 32-bit operations per circle sample, counted from the binary32
# rule (one IEEE operation each): sampling 4 mul + 4 fma; sign test 1;
# chart 1 add + 1 reciprocal + 1 mul; cell 3 fma + 3 floor + 6 clamp
# compares + 2 index multiply-adds; vote 1 integer add.
OPS_PER_SAMPLE = 27


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--strategy", default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-runs", type=int, default=5,
                    help="whole-workload oracle solves on all host threads (median reported)")
    ap.add_argument("--cpu-single-fraction", type=int, default=64,
                    help="the one-thread oracle leg times this fraction 1/F of the workload")
    ap.add_argument("--cpu-single-runs", type=int, default=3,
                    help="one-thread oracle solves (median reported)")
    ap.add_argument("--cpu-instances", type=int, default=1000,
                    help="batch workload: instances the CPU oracle times")
    ap.add_argument("--duration", type=float, default=60.0,
                    help="serve workload: seconds of arrivals")
    ap.add_argument("--serve-duration", type=float, default=20.0,
                    help="large workload: seconds of the served leg after the timed solves "
                         "(0 skips it)")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve workload: requests/s")
    ap.add_argument("--workers", type=int, default=8, help="serve workload: server lanes")
    ap.add_argument("--hbm-budget-gib", type=float, default=8.0,
                    help="serve workload: the server's scratch arena (admission by footprint)")
    ap.add_argument("--tuning-cache", default=os.environ.get(
        "ROTVOTE_TUNING", str(Path.home() / ".cache" / "rotvote" / "tuning.json")),
                    help="batch workload: tuning file (JSON) read if present, else written")
    ap.add_argument("--no-loop", action="store_true",
                    help="batch workload: skip the one-solve-per-call comparison")
    ap.add_argument("--ceilings", action="store_true",
                    help="only measure the GPU's ceilings (VALU issue, LDS and device atomics, "
                         "copy bandwidth) with the probe library's micro-benchmarks and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run plain device-to-device copies of MIB MiB (profiler "
                         "calibration of the HBM byte counters) and exit")
    return ap.parse_args()


def copy_calibration(mib: int):
    """Plain copies of a known size: a profiler's byte counters for these
    dispatches give the scale factor for the solve's kernels."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "dispatches": 5}), flush=True)


_CEILINGS = {}


def measured_ceilings(full: bool = False) -> dict:
    """Ceilings measured on this GPU by the probe library's micro-benchmarks:
    32-bit FMA lane-operations/s (independent chains); with ``full`` also LDS
    atomic adds/s (random and bank-distinct cells, 128 KiB array), relaxed
    device-scope atomic adds/s into random cells of 1, 8 and 64 MiB int32
    grids (random cells, and a wave at a time into 64 consecutive cells), and
    device copy bandwidth (read + write bytes/s of a 1 GiB copy)."""
    key = "full" if full else "valu"
    if key in _CEILINGS:
        return _CEILINGS[key]
    from paper_2506_11547_amd import rotvote
    p = rotvote.Probe()
    out = {"valu_top_s": p.ceiling_valu() / 1e12}
    if full:
        out["lds_atomic_random_per_s"] = p.ceiling_lds_atomic(True)
        out["lds_atomic_distinct_per_s"] = p.ceiling_lds_atomic(False)
        out["global_atomic_per_s"] = {f"{mib}MiB": p.ceiling_global_atomic(mib << 18)
                                      for mib in (1, 8, 64)}
        out["global_atomic_contiguous_per_s"] = {
            f"{mib}MiB": p.ceiling_global_atomic(mib << 18, contiguous=True) for mib in (1, 64)}
        out["copy_gb_s"] = p.ceiling_copy() / 1e9
        out["read_gb_s"] = p.ceiling_read() / 1e9
    _CEILINGS[key] = out
    return out


def alu_roofline(kernel: str, achieved_gops: float, traffic, **extra) -> dict:
    """The roofline object of an ALU-bound vote kernel: against the published
    issue peak (``frac``) and against the FMA issue rate measured here
    (``frac_measured``)."""
    valu = measured_ceilings()["valu_top_s"]
    return {"bound": "alu", "kernel": kernel, "achieved": achieved_gops / 1e3,
            "peak": ALU_PEAK_GOPS / 1e3, "unit": "TOP/s", "frac": achieved_gops / ALU_PEAK_GOPS,
            "traffic": traffic, "measured_peak": valu, "frac_measured": achieved_gops / 1e3 / valu,
            **extra}


# committed HBM-byte records of a workload's vote kernel, one per profiled
# strategy (profiles/vote_bin__*, vote_keys__*)
TRAFFIC_RECORDS = {w: [ROOT / "profiles" / f"vote_{k}__{w}_traffic.json" for k in ("bin", "keys")]
                   for w in ("large", "batch", "paper_default", "rigid")}


KEY_VOTE_KERNEL = "rv::k_vote_keys<rv::KeyPack<16, 32, 1> >"


def vote_kernel_name(grid: int, edge: int = 0, strategy: str = "brick") -> str:
    """The vote kernel instance a binned solve launches: for runs, brick edge
    2^5 or 2^4 (a single solve takes 16 up to grid 128, else 32; a batch its
    tuned edge) and the wide run layout above grid 256; for keys, the key
    kernel."""
    if strategy == "keys":
        return KEY_VOTE_KERNEL
    if edge == 0:
        edge = 16 if grid <= 128 else 32
    return f"rv::k_vote_bin<{5 if edge == 32 else 4}, {'true' if grid > 256 else 'false'}>"


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of the vote kernel from the committed FETCH_SIZE /
    WRITE_SIZE profile (scaled by the copy calibration), or None when the
    profile is of another workload or kernel instance, or the kernel's sources
    changed since."""
    import hashlib
    rec = None
    for path in TRAFFIC_RECORDS.get(workload, []):
        try:
            r = json.loads(path.read_text())
        except (OSError, ValueError):
            continue
        if r.get("workload") == workload and r.get("kernel") == kernel:
            rec = r
    if rec is None:
        return None
    for path, digest in rec["sources_sha256"].items():
        try:
            if hashlib.sha256((ROOT / path).read_bytes()).hexdigest() != digest:
                return None
        except OSError:
            return None
    return float(rec["traffic_bytes_per_launch"])


def host_cpu() -> dict:
    """The host the CPU baseline ran on: processors online (nproc), the ones
    this process may use, and the CPU model."""
    model = "unknown"
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable": usable, "cpu_model": model}


def cpu_baseline(w, inst, runs: int, single_fraction: int, single_runs: int) -> dict:
    """The oracle, as it is, on the whole workload: the median wall time of
    ``runs`` whole solves on every usable host thread (OpenMP vote loop; the
    top-K scan and the rescoring are single-threaded in the oracle), and the
    median of ``single_runs`` whole solves on one thread over the first
    1/single_fraction of the correspondences.  Data generation is outside
    every timing."""
    import statistics

    import oracle
    o = oracle.get()
    threads = oracle.threads()
    x, y = inst.x, inst.y
    eps = float(__import__("ctypes").c_float(w.eps_deg * math.pi / 180.0).value)
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        o.solve(x, y, w.grid, w.samples, eps, w.topk, nthreads=threads)
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    n1 = max(1, inst.n // single_fraction)
    x1, y1 = x[:, :n1].copy(), y[:, :n1].copy()
    times1 = []
    for _ in range(single_runs):
        t1 = time.perf_counter()
        o.solve(x1, y1, w.grid, w.samples, eps, w.topk, nthreads=1)
        times1.append(time.perf_counter() - t1)
    med1 = statistics.median(times1)
    return {"value": inst.n * w.samples / med, "unit": "votes/s", "cores": threads,
            "kind": "oracle", "n": inst.n, "runs": runs, "median_s": med,
            "times_s": times, **host_cpu(),
            "sample": f"the whole workload ({inst.n} correspondences; G={w.grid}, J={w.samples}, "
                      f"K={w.topk}), median of {runs} whole solves; vote loop on {threads} "
                      f"OpenMP threads, top-K and rescoring single-threaded",
            "single_thread": {"value": n1 * w.samples / med1, "unit": "votes/s", "cores": 1,
                              "n": n1, "runs": single_runs, "median_s": med1,
                              "sample": f"first {n1} correspondences (1/{single_fraction} of "
                                        f"the workload), whole solve on one thread, median of "
                                        f"{single_runs}"}}


def cpu_baseline_batch(w, bt, max_instances: int) -> dict:
    """The oracle, as it is, on the first instances of the batch."""
    import oracle
    o = oracle.get()
    threads = oracle.threads()
    eps = float(__import__("ctypes").c_float(w.eps_deg * math.pi / 180.0).value)
    m = min(max_instances, bt.B)
    t0 = time.perf_counter()
    for b in range(m):
        xb, yb = bt.instance(b)
        o.solve(xb, yb, w.grid, w.samples, eps, w.topk, nthreads=threads)
    dt = time.perf_counter() - t0
    n = int(bt.offsets[m])
    return {"value": n * w.samples / dt, "unit": "votes/s", "cores": threads, "kind": "oracle",
            "solves_per_s": m / dt,
            "sample": f"first {m} of the {bt.B} instances ({n} correspondences), one oracle "
                      f"solve each; vote loop on {threads} OpenMP threads; {dt:.2f} s"}


def loop_baseline(args, w, bt, x, y, mask, stream, q, cnt) -> dict:
    """The same instances, one rot_vote_solve call each (one timed pass after
    an untimed pass over the first 64), on a handle made for single solves."""
    import numpy as np
    import torch

    from paper_2506_11547_amd import rotvote
    offs = bt.offsets
    single = rotvote.Solver(device=0, max_n=int(np.diff(bt.offsets).max()), max_grid=w.grid,
                            topk=w.topk, samples_per_circle=w.samples, stream=stream)
    views = [(x[:, offs[b]:offs[b + 1]], y[:, offs[b]:offs[b + 1]], mask[offs[b]:offs[b + 1]])
             for b in range(bt.B)]
    for xb, yb, mb in views[:64]:
        single.solve(xb, yb, w.grid, w.eps_deg, mask=mb)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    same = 0
    for b, (xb, yb, mb) in enumerate(views):
        qb, cb, _ = single.solve(xb, yb, w.grid, w.eps_deg, mask=mb)
        same += int(qb == q[b].tolist() and cb == cnt[b])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    plan = single.plan()
    single.close()
    samples = int(bt.offsets[-1]) * w.samples
    return {"solves_per_s": bt.B / dt, "votes_per_s": samples / dt, "ms": dt * 1e3,
            "vote_strategy": plan["strategy"], "identical_results": same}


def serve_pool(per_tier: int, seed: int):
    """Resident request pool: per tier, per_tier seeded instances whose N are
    the midpoint quantiles of the log-uniform law over the tier's decade (so
    the pool's mean load is the law's)."""
    import numpy as np

    from paper_2506_11547_amd import datagen
    rng = np.random.default_rng(seed)
    pool = []
    for lo, hi, G in ((1_000, 10_000, 64), (10_000, 100_000, 128), (100_000, 1_000_000, 256)):
        for k in range(per_tier):
            n = int(round(np.exp(np.log(lo) + (k + 0.5) / per_tier * np.log(hi / lo))))
            inst = datagen.make_instance(n, float(rng.uniform(0.8, 0.99)), 1.0,
                                         int(rng.integers(0, 2**62)))
            pool.append((G, inst))
    return pool


def serve_measure(rate: float, duration: float, workers: int, hbm_budget_gib: float) -> dict:
    """Poisson arrivals of the seeded request pool at `rate` requests/s for
    `duration` s into a Server; the serving statistics, the run's
    configuration and the throughput figures."""
    import numpy as np
    import torch

    from paper_2506_11547_amd import rotvote
    seed = 4
    eps_deg = 1.5
    pool = serve_pool(24, seed)
    dev = torch.device("cuda", 0)
    res = []
    for G, inst in pool:
        x = torch.from_numpy(inst.x).to(dev)
        y = torch.from_numpy(inst.y).to(dev)
        masks = [torch.empty(inst.n, dtype=torch.uint8, device=dev) for _ in range(4)]
        res.append((G, inst.n, x, y, masks))
    rng = np.random.default_rng(seed + 1)
    n_req = int(rng.poisson(rate * duration))
    arrivals = np.sort(rng.uniform(0.0, duration, n_req))
    picks = rng.integers(0, len(res), n_req)
    srv = rotvote.Server(workers=workers, max_n=1_000_000, max_grid=256, topk=16,
                         max_batch=64, batch_max_n=65536, max_queue=1 << 22,
                         hbm_budget=int(hbm_budget_gib * (1 << 30)))
    # warm-up: one request of every pool entry
    for k, (G, n, x, y, masks) in enumerate(res):
        srv.wait(srv.submit(x, y, G, eps_deg, masks[0]))
    torch.cuda.synchronize()
    tickets = [None] * n_req
    use = [0] * len(res)
    t0 = time.monotonic() + 0.05
    next_note = 10.0
    for i in range(n_req):
        k = int(picks[i])
        G, n, x, y, masks = res[k]
        m = masks[use[k] % len(masks)]
        use[k] += 1
        ta = t0 + arrivals[i]
        while True:
            d = ta - time.monotonic()
            if d <= 0:
                break
            if d > 2e-4:
                time.sleep(d - 1e-4)
        tickets[i] = srv.submit(x, y, G, eps_deg, m)
        if arrivals[i] >= next_note:
            print(f"serve: {i + 1} of {n_req} requests submitted at {arrivals[i]:.0f} s",
                  file=sys.stderr, flush=True)
            next_note += 10.0
    replies = [srv.wait(t) for t in tickets]
    torch.cuda.synchronize()
    st = srv.stats()
    mem = srv.memory()
    srv.close()
    lat = np.array([r["t_end"] - (t0 + a) for r, a in zip(replies, arrivals)])
    wait = np.array([r["t_start"] - r["t_submit"] for r in replies])
    end = max(r["t_end"] for r in replies)
    span = end - t0
    samples = np.array([res[int(k)][1] * 8 * res[int(k)][0] for k in picks], np.float64)
    offered = samples.sum() / duration
    achieved = samples.sum() / span
    tier = np.array([res[int(k)][0] for k in picks])
    return {
        "requests": n_req, "warmup": len(res), "span_s": span, "achieved_votes_per_s": achieved,
        "config": {"workload": "serve", "rate_rps": rate, "duration_s": duration,
                   "n_range": [1_000, 1_000_000], "grids": [64, 128, 256], "outlier_ratio": [0.8, 0.99],
                   "sigma_deg": 1.0, "eps_deg": eps_deg, "topk": 16, "seed": seed,
                   "pool_per_tier": 24, "workers": st["workers"], "max_batch": 64,
                   "hbm_budget_bytes": mem["arena_bytes"]},
        "serving": {
            "requests": n_req, "offered_rps": n_req / duration, "achieved_rps": n_req / span,
            "offered_votes_per_s": offered, "achieved_votes_per_s": achieved,
            "saturated": bool(achieved < 0.97 * offered),
            "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                           "p90": float(np.percentile(lat, 90) * 1e3),
                           "p99": float(np.percentile(lat, 99) * 1e3)},
            "latency_p99_ms_by_grid": {int(g): float(np.percentile(lat[tier == g], 99) * 1e3)
                                       for g in (64, 128, 256) if (tier == g).any()},
            "queue_wait_ms_p50": float(np.percentile(wait, 50) * 1e3),
            "batched_fraction": float(np.mean([r["batched"] > 1 for r in replies])),
            "mean_batch": float(np.mean([r["batched"] for r in replies])),
            "server_device_bytes": st["device_bytes"],
            "arena_peak_in_use_bytes": mem["peak_in_use"],
            "peak_in_flight": mem["peak_in_flight"],
            "scratch_mib_p50_by_grid": {
                int(g): float(np.percentile([r["scratch_bytes"] for r, t in zip(replies, tier)
                                             if t == g and r["batched"] == 1], 50) / (1 << 20))
                for g in (64, 128, 256)
                if any(t == g and r["batched"] == 1 for r, t in zip(replies, tier))},
        },
    }


def run_serve(args):
    m = serve_measure(args.rate, args.duration, args.workers, args.hbm_budget_gib)
    out = {
        "metric": METRIC,
        "value": m["achieved_votes_per_s"],
        "unit": "votes/s",
        "n_gpus": 1,
        "steps": m["requests"],
        "warmup": m["warmup"],
        "ms_per_step": m["span_s"] / m["requests"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": m["config"],
        "serving": m["serving"],
    }
    print(json.dumps(out), flush=True)


def run_multi(args):
    """Several rotations in one scene (the paper's multiple-rotation setting:
    9 rotations x 3000 correspondences, delta 0.01, J = 540) plus 27 000
    uniform outliers; G = 128, K = 64, eps 2 deg, at most 12 models."""
    import numpy as np
    import torch

    from paper_2506_11547_amd import datagen, rotvote
    models, per_model, G, J, K, eps_deg = 9, 3000, 128, 540, 64, 2.0
    inst = datagen.make_multi_instance(models, per_model, models * per_model, 0.01, 6)
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(inst.x).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    n = x.shape[1]
    labels = torch.empty(n, dtype=torch.uint8, device=dev)
    solver = rotvote.Solver(device=0, max_n=n, max_grid=G, topk=K, samples_per_circle=J)
    for _ in range(args.warmup):
        solver.solve_multi(x, y, G, eps_deg, models + 3, 10.0, 50, labels=labels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        q, cnt, _ = solver.solve_multi(x, y, G, eps_deg, models + 3, 10.0, 50, labels=labels)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    solver.close()
    errs = [min(datagen.rotation_error_deg(np.array(qm), qg) for qm in q) for qg in inst.q_gt]
    lab = labels.cpu().numpy()
    out = {"metric": METRIC, "value": n * J / dt, "unit": "votes/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "multi", "models": models, "per_model": per_model,
                      "outliers": models * per_model, "delta": 0.01, "grid": G,
                      "samples_per_circle": J, "topk": K, "eps_deg": eps_deg, "sep_deg": 10.0,
                      "min_inliers": 50, "seed": 6},
           "result": {"models_found": len(q), "counts": cnt, "max_err_deg": max(errs),
                      "mean_err_deg": float(np.mean(errs)),
                      "labelled_fraction": float((lab > 0).mean())}}
    print(json.dumps(out), flush=True)


def run_rigid(args):
    """Rigid pose from point correspondences (the paper's 6-DoF synthetic
    experiment, Sec. 5.4.1: N = 5000, 90 % outliers, delta 0.01, translation
    domain [-5, 5]^3 with step 0.025) at the paper's default rotation
    resolution (G = 360, J = 180); length tolerance 0.05, rotation inlier
    angle 2 deg, 8 least-squares rounds, inlier distance 0.06."""
    import numpy as np
    import torch

    from paper_2506_11547_amd import datagen, rotvote
    n, rho, delta, seed = 5000, 0.9, 0.01, 7
    mu, G, J, K, eps_deg, rounds = 0.05, 360, 180, 16, 2.0, 8
    t_min, t_step, t_cells, tau = -5.0, 0.025, 400, 0.06
    inst = datagen.make_rigid_instance(n, rho, delta, seed)
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(inst.x).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    mask = torch.empty(n, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    solver = rotvote.Solver(device=0, max_n=1 << 21, max_grid=G, topk=K, samples_per_circle=J,
                            max_pairs=1 << 21, timing=True, stream=stream)
    args_r = (x, y, mu, G, eps_deg, t_min, t_step, t_cells, tau)
    for _ in range(args.warmup):
        solver.solve_rigid(*args_r, refine_rounds=rounds, mask=mask)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = solver.solve_rigid(*args_r, refine_rounds=rounds, mask=mask)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # the stages one by one (events on the solve stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    ev[0].record(stream)
    m, nn, _ = solver.pairs(x, y, mu, capacity=r["pairs"])
    ev[1].record(stream)
    pm = torch.empty(m.shape[1], dtype=torch.uint8, device=dev)
    q, c, _ = solver.solve(m, nn, G, eps_deg, mask=pm)
    vote_ms = solver.timings()["vote"]
    strategy = solver.plan()["strategy"]
    ev[2].record(stream)
    q, c, ran = solver.refine(m, nn, q, pm, eps_deg, max_rounds=rounds)
    ev[3].record(stream)
    solver.translation(x, y, q, t_min, t_step, t_cells, tau, mask=mask)
    ev[4].record(stream)
    torch.cuda.synchronize()
    stage_ms = {"pairs": ev[0].elapsed_time(ev[1]), "rotation": ev[1].elapsed_time(ev[2]),
                "refine": ev[2].elapsed_time(ev[3]), "translation": ev[3].elapsed_time(ev[4])}
    solver.close()
    P = r["pairs"]
    lab = mask.cpu().numpy().astype(bool)
    achieved = OPS_PER_SAMPLE * P * J / (vote_ms * 1e-3) / 1e9
    out = {"metric": METRIC, "value": P * J / dt, "unit": "votes/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "rigid", "n": n, "outlier_ratio": rho, "delta": delta,
                      "seed": seed, "mu": mu, "grid": G, "samples_per_circle": J, "topk": K,
                      "eps_deg": eps_deg, "refine_rounds": rounds,
                      "t_domain": [t_min, t_min + t_cells * t_step], "t_step": t_step,
                      "t_inlier": tau, "vote_strategy": strategy},
           "solves_per_s": 1.0 / dt,
           "pair_tests_per_s": n * (n - 1) / 2 / (stage_ms["pairs"] * 1e-3),
           "stage_ms": stage_ms, "vote_ms": vote_ms,
           "roofline": alu_roofline("vote (pairs)", achieved,
                                    measured_traffic("rigid", vote_kernel_name(G, strategy=strategy)),
                                    ops_per_sample=OPS_PER_SAMPLE, samples_per_launch=P * J,
                                    vote_ms=vote_ms),
           "result": {"pairs": P, "rot_inliers": r["rot_inliers"],
                      "refine_rounds_run": r["refine_rounds_run"],
                      "e_R_deg": datagen.rotation_error_deg(np.float64(r["q"]), inst.q_gt),
                      "e_t": float(np.linalg.norm(np.float64(r["t"]) - inst.t_gt)),
                      "t_votes": r["t_votes"], "inliers": r["inliers"],
                      "true_positives": int((lab & inst.inlier).sum()),
                      "true_inliers": int(inst.inlier.sum())}}
    if not args.no_cpu_baseline:
        import oracle
        from oracle import rigid as RG
        import math
        orc = oracle.get()
        th = oracle.threads()
        t1 = time.perf_counter()
        RG.solve_rigid(orc, inst.x, inst.y, mu, G, J, float(np.float32(math.radians(eps_deg))), K,
                       rounds, t_min, t_step, t_cells, tau, nthreads=th)
        ct = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": P * J / ct, "unit": "votes/s", "cores": th,
                               "kind": "oracle", "sample": "the whole workload, one solve",
                               "solves_per_s": 1.0 / ct}
    print(json.dumps(out), flush=True)


def run_batch(args):
    import numpy as np
    import torch

    from paper_2506_11547_amd import datagen, rotvote

    w = datagen.BATCH_WORKLOADS[args.workload]
    bt = w.batch()
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(bt.x).to(dev)
    y = torch.from_numpy(bt.y).to(dev)
    n = int(bt.offsets[-1])
    mask = torch.empty(n, dtype=torch.bool, device=dev)
    stream = torch.cuda.current_stream(dev)
    offs = bt.offsets
    solver = rotvote.Solver(device=0, max_n=n, max_grid=w.grid, topk=w.topk,
                            samples_per_circle=w.samples, timing=True, stream=stream,
                            max_batch=bt.B)
    # the batch schedule (brick edge per instance-size bucket): from the tuning
    # file when it holds one for this GPU, grid and J, else by measurement
    cache = Path(args.tuning_cache)
    tuning = {"file": str(cache)}
    if cache.exists() and solver.load_tuning(cache) > 0:
        tuning["source"] = "loaded"
    else:
        edges, ms = solver.tune_batch(x, y, offs, w.grid, w.eps_deg, reps=2)
        tuning.update(source="measured", ms_all32=ms[0],
                      ms_bucket_at16=[ms[k + 1] for k in range(rotvote.BATCH_BUCKETS)])
        cache.parent.mkdir(parents=True, exist_ok=True)
        solver.save_tuning(cache)
    sched = solver.batch_schedule(w.grid)
    tuning["schedule"] = dict(zip(["n<512", "512<=n<2048", "2048<=n<8192", "n>=8192"], sched))
    # the brick edge that votes most of the samples (its vote kernel is the profiled one)
    sizes = np.diff(offs)
    bucket = np.searchsorted(np.array(rotvote.BATCH_BUCKET_BOUNDS), sizes, side="right")
    edge = sched[int(np.argmax(np.bincount(bucket, weights=sizes, minlength=4)))]
    for _ in range(args.warmup):
        solver.solve_batch(x, y, offs, w.grid, w.eps_deg, mask=mask)
    stage = {k: 0.0 for k in rotvote.STAGE_NAMES}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        q, cnt, _ = solver.solve_batch(x, y, offs, w.grid, w.eps_deg, mask=mask)
        for k, v in solver.timings().items():
            stage[k] += v
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    graph = graph_batch_leg(sched, x, y, offs, w, bt.B, args.steps, q, cnt)
    loop = None
    if not args.no_loop:
        loop = loop_baseline(args, w, bt, x, y, mask, stream, q, cnt)
    solver.close()

    steps = args.steps
    samples = n * w.samples
    stage_ms = {k: v / steps for k, v in stage.items()}
    vote_s = stage_ms["vote"] * 1e-3
    achieved = OPS_PER_SAMPLE * samples / vote_s / 1e9
    err = [datagen.rotation_error_deg(q[b], bt.q_gt[b]) for b in range(bt.B)]
    out = {
        "metric": METRIC,
        "value": samples / (dt / steps),
        "unit": "votes/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": dt / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "instances": bt.B, "n_total": n, "n_lo": w.n_lo,
                   "n_hi": w.n_hi, "outlier_ratio": [w.rho_lo, w.rho_hi],
                   "sigma_deg": w.sigma_deg, "grid": w.grid, "samples_per_circle": w.samples,
                   "eps_deg": w.eps_deg, "topk": w.topk, "seed": w.seed,
                   "vote_strategy": "brick (batched)", "brick_edge": edge},
        "batch_schedule": tuning,
        "graph": graph,
        "solves_per_s": bt.B * steps / dt,
        "stage_ms": stage_ms,
        "loop": loop if loop is None else dict(loop, speedup_of_batch=(bt.B * steps / dt) /
                                                  loop["solves_per_s"]),
        "roofline": alu_roofline("vote (batched)", achieved,
                                 measured_traffic(w.name, vote_kernel_name(w.grid, edge)),
                                 ops_per_sample=OPS_PER_SAMPLE, samples_per_launch=samples,
                                 vote_ms=stage_ms["vote"]),
        "result": {"median_e_R_deg": float(np.median(err)), "p99_e_R_deg": float(np.percentile(err, 99)),
                   "inliers_total": int(sum(cnt))},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(w, bt, args.cpu_instances)
    print(json.dumps(out), flush=True)


def graph_batch_leg(sched, x, y, offs, w, B: int, reps: int, q, cnt) -> dict:
    """The device-planned batch (offsets in device memory) captured once into
    a HIP graph on a side stream (a handle without timing events, with the
    same batch schedule) and replayed ``reps`` times; wall time per replay,
    and whether every instance's rotation and count equal the synchronous
    batch's."""
    import numpy as np
    import torch

    from paper_2506_11547_amd import rotvote
    side = torch.cuda.Stream()
    ob = torch.from_numpy(np.ascontiguousarray(offs, np.int64)).cuda()
    res = torch.zeros(B, rotvote.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    mask = torch.empty(x.shape[1], dtype=torch.bool, device="cuda")
    solver = rotvote.Solver(device=0, max_n=x.shape[1], max_grid=w.grid, topk=w.topk,
                            samples_per_circle=w.samples, stream=side, max_batch=B)
    solver.set_batch_schedule(w.grid, sched)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        solver.solve_batch_async(x, y, ob, w.grid, w.eps_deg, results=res, mask=mask)
    side.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        solver.solve_batch_async(x, y, ob, w.grid, w.eps_deg, results=res, mask=mask)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    raw = res.cpu().numpy()
    gq = raw[:, :16].copy().view(np.float32).reshape(B, 4)
    gc = raw[:, 16:24].copy().view(np.int64).reshape(B)
    same = bool(np.array_equal(gq.view(np.uint32), np.float32(q).view(np.uint32)) and
                np.array_equal(gc, cnt))
    del g
    solver.close()
    return {"replays": reps, "ms_per_batch": dt * 1e3, "solves_per_s": B / dt,
            "identical_to_sync": same}


def refine_leg(solver, x, y, q, mask, w, inst, reps: int = 5) -> dict:
    """Least-squares refinement (up to 8 rounds) from the last solve's rotation
    and inlier mask; wall time per call (synchronous) after one untimed call."""
    import torch

    from paper_2506_11547_amd import datagen
    m = mask.clone()
    solver.refine(x, y, q, m, w.eps_deg, max_rounds=8)
    times = []
    for _ in range(reps):
        m = mask.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        qr, cr, rounds = solver.refine(x, y, q, m, w.eps_deg, max_rounds=8)
        times.append(time.perf_counter() - t0)
    return {"ms": sorted(times)[len(times) // 2] * 1e3, "rounds": rounds, "inliers": cr,
            "q": qr, "e_R_deg": datagen.rotation_error_deg(qr, inst.q_gt)}


def async_leg(w, inst, x, y, q_sync, cnt_sync, steps: int) -> dict:
    """The same solve enqueued without waiting (rot_vote_solve_async): ms per
    solve for `steps` solves back to back on one stream with one wait at the
    end, and for `steps` replays of one solve captured in a HIP graph.  Uses a
    handle of its own (no timing events); the last result of each mode is
    checked against the synchronous solve."""
    import torch

    from paper_2506_11547_amd import rotvote
    stream = torch.cuda.Stream()
    res = torch.zeros(rotvote.RESULT_BYTES, dtype=torch.uint8, device=x.device)
    mask = torch.empty(inst.n, dtype=torch.bool, device=x.device)
    out = {"solves": steps}
    with rotvote.Solver(device=0, max_n=inst.n, max_grid=w.grid, topk=w.topk,
                        samples_per_circle=w.samples, stream=stream) as s:
        s.solve_async(x, y, w.grid, w.eps_deg, result=res, mask=mask)   # sample table
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.solve_async(x, y, w.grid, w.eps_deg, result=res, mask=mask)
        stream.synchronize()
        out["ms_per_solve"] = (time.perf_counter() - t0) / steps * 1e3
        r = rotvote.decode_result(res)
        out["identical"] = r["q"] == list(q_sync) and r["count"] == cnt_sync
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream, capture_error_mode="relaxed"):
            s.solve_async(x, y, w.grid, w.eps_deg, result=res, mask=mask)
        res.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        out["graph_ms_per_solve"] = (time.perf_counter() - t0) / steps * 1e3
        r = rotvote.decode_result(res)
        out["graph_identical"] = r["q"] == list(q_sync) and r["count"] == cnt_sync
        del g
    return out


def main():
    args = parse()
    if args.ceilings:
        print(json.dumps({"ceilings": measured_ceilings(full=True),
                          "published": {"alu_top_s": ALU_PEAK_GOPS / 1e3,
                                        "hbm_gb_s": HBM_PEAK_GBS}}), flush=True)
        return
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)
    from paper_2506_11547_amd import datagen
    if args.workload in datagen.BATCH_WORKLOADS:
        run_batch(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "multi":
        run_multi(args)
        return
    if args.workload == "rigid":
        run_rigid(args)
        return
    import numpy as np
    import torch

    from paper_2506_11547_amd import rotvote

    w, inst = datagen.make_workload(args.workload)
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(inst.x).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    mask = torch.empty(inst.n, dtype=torch.bool, device=dev)
    stream = torch.cuda.current_stream(dev)
    solver = rotvote.Solver(device=0, max_n=inst.n, max_grid=w.grid, topk=w.topk,
                            samples_per_circle=w.samples, strategy=args.strategy, timing=True,
                            stream=stream)
    tuned = None
    if args.strategy == "auto":
        best, ms = solver.tune(x, y, w.grid, w.eps_deg, reps=3)
        tuned = {"chosen": best, "ms_global": ms["global"], "ms_brick": ms["brick"],
                 "ms_keys": ms["keys"]}
    for _ in range(args.warmup):
        solver.solve(x, y, w.grid, w.eps_deg, mask=mask)
    stage = {k: 0.0 for k in rotvote.STAGE_NAMES}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        q, cnt, _ = solver.solve(x, y, w.grid, w.eps_deg, mask=mask)
        for k, v in solver.timings().items():
            stage[k] += v
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan = solver.plan()
    top = solver.topk()
    refine = refine_leg(solver, x, y, q, mask, w, inst)
    solver.close()
    pipelined = async_leg(w, inst, x, y, q, cnt, args.steps)

    steps = args.steps
    samples = inst.n * w.samples
    ms_step = dt / steps * 1e3
    stage_ms = {k: v / steps for k, v in stage.items()}
    vote_s = stage_ms["vote"] * 1e-3
    achieved = OPS_PER_SAMPLE * samples / vote_s / 1e9
    out = {
        "metric": METRIC,
        "value": samples / (dt / steps),
        "unit": "votes/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "outlier_ratio": w.outlier_ratio,
                   "sigma_deg": w.sigma_deg, "grid": w.grid, "samples_per_circle": w.samples,
                   "eps_deg": w.eps_deg, "topk": w.topk, "seed": w.seed,
                   "vote_strategy": plan["strategy"]},
        "solves_per_s": steps / dt,
        "stage_ms": stage_ms,
        "strategy_tuning": tuned,
        "roofline": alu_roofline("vote", achieved,
                                 (measured_traffic(w.name, vote_kernel_name(
                                     w.grid, strategy=plan["strategy"]))
                                  if plan["strategy"] in ("brick", "keys") else None),
                                 ops_per_sample=OPS_PER_SAMPLE, samples_per_launch=samples,
                                 vote_ms=stage_ms["vote"]),
        "result": {"q": q, "inliers": cnt, "e_R_deg": datagen.rotation_error_deg(q, inst.q_gt),
                   "winner": top["winner"], "true_inliers": int(inst.inlier.sum())},
        "refine": refine,
        "async": pipelined,
    }
    if args.serve_duration > 0 and w.name == "large":
        # the metric's served half: the request server under Poisson arrivals
        # (the same leg as --workload serve, shorter), after the timed solves
        m = serve_measure(args.rate, args.serve_duration, args.workers, args.hbm_budget_gib)
        out["served_p99_ms"] = m["serving"]["latency_ms"]["p99"]
        out["serving"] = dict(m["serving"], config=m["config"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, inst, args.cpu_runs, args.cpu_single_fraction,
                                           args.cpu_single_runs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
