"""Benchmark of the hot path: one step = Wilson loop-erased-walk sampling
(omega trees rooted at the max-degree node), omega uniform-start and omega
stationary-start absorbed walks, and the FP64 assembly of diag(L^dagger),
closeness and Kemeny's constant, on a Barabasi-Albert graph n = 100,000,
m = 5 with omega = 4096 (synthetic input, resident in HBM before timing).

Prints one JSON line.  `value` is walk steps per second (Wilson draws plus
absorbed-walk draws) of the whole job.
"""
import argparse
import json

import numpy as np
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WILSON_BYTES_PER_STEP = 33.0     # offsets 16 + column 4 + draw count 8 + next 4 + tree flag 1
RETRACE_BYTES_PER_NODE = 5.0
LOADS_PER_WILSON_STEP = 3        # dependent random loads per draw: column, target state, target offsets
CHASE_BYTES_PER_LOAD = 128       # FETCH_SIZE per 4 GiB pointer-chase load, measured on the gather benchmark


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "wilson_wave_traffic.json")
KERNEL_SOURCES = ["paper_2311_10290_amd/csrc/" + f for f in
                  ("wave_sample.h", "wilson.hip", "lap_device.h")]


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(part="bytes_per_launch"):
    """HBM bytes per Wilson launch (or its FETCH_SIZE part) from the committed
    counter summary, if it was taken on the current kernel sources; otherwise
    null."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t["bytes_per_launch"] if part == "bytes_per_launch" else t["FETCH_SIZE"]["bytes"]


def write_traffic(pmc_dir):
    """Reduce the counter runs under pmc_dir to the traffic summary for the
    current kernel sources.  Expects the databases of four one-counter runs:
    copy_FETCH_SIZE/ and copy_WRITE_SIZE/ (``--copy-calibration``: a 1 GiB
    device copy), pmc_FETCH_SIZE/ and pmc_WRITE_SIZE/ (one plain step).  Each
    counter is scaled by copy bytes / what it read for the copy."""
    import glob
    import sqlite3

    def per_dispatch(sub, counter, kernel):
        db, = glob.glob(os.path.join(pmc_dir, sub, "*_results.db"))
        con = sqlite3.connect(db)
        rows = con.execute("select dispatch_id, sum(value) from counters_collection where counter_name=? and "
                           "kernel_name like ? group by dispatch_id order by dispatch_id",
                           (counter, f"%{kernel}%")).fetchall()
        con.close()
        return [r[1] for r in rows]

    copy_kib = 1 << 20
    res = {"kernel": "wilson_wave_kernel", "workload": "Barabasi-Albert n=100000 m=5, omega=4096, one launch",
           "kernel_hash": kernel_hash()}
    total = 0.0
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        cal = copy_kib / per_dispatch(f"copy_{c}", c, "copyBuffer")[0]
        raw = per_dispatch(f"pmc_{c}", c, "wilson_wave")
        res[c] = {"raw_kib_per_dispatch": raw, "calibration": cal, "bytes": raw[0] * 1024 * cal}
        total += raw[0] * 1024 * cal
    res["bytes_per_launch"] = total
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(og, root, omega_full, seed, budget_s=15.0):
    """The oracle (C, OpenMP over samples) on a bounded sample of the same workload."""
    from oracle import native
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t = time.perf_counter()
    w = native.wilson(og, root, omega_full, seed, n_samples=64, want_y1=True, threads=threads)
    dt = time.perf_counter() - t
    n_s = int(min(omega_full, max(64, 64 * budget_s / max(dt, 1e-3))))
    # when the whole workload is shorter than the budget, it is repeated
    reps, steps, t = 0, 0, time.perf_counter()
    while True:
        w = native.wilson(og, root, omega_full, seed, n_samples=n_s, threads=threads)
        a1 = native.absorbed(og, root, n_s, seed, 1, omega_total=omega_full, threads=threads)
        a2 = native.absorbed(og, root, n_s, seed, 2, omega_total=omega_full, want_y2=False, threads=threads)
        steps += int(w["y1"].sum() + a1["len"].sum() + a2["len"].sum())
        reps += 1
        dt = time.perf_counter() - t
        if n_s < omega_full or dt >= 0.7 * budget_s:
            break
    # one thread on a smaller sample: the per-core rate
    n1 = max(8, n_s // (2 * threads))
    t1 = time.perf_counter()
    w = native.wilson(og, root, omega_full, seed, n_samples=n1, threads=1)
    a1 = native.absorbed(og, root, n1, seed, 1, omega_total=omega_full, threads=1)
    a2 = native.absorbed(og, root, n1, seed, 2, omega_total=omega_full, want_y2=False, threads=1)
    steps1 = int(w["y1"].sum() + a1["len"].sum() + a2["len"].sum())
    dt1 = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": steps / dt, "unit": "walk steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_s} of {omega_full} samples (Wilson + both absorbed-walk kinds), "
                      f"{reps} pass(es), {dt:.1f} s",
            "trees_per_s": reps * n_s / dt,
            "single_thread": {"value": steps1 / dt1, "unit": "walk steps/s",
                              "sample": f"first {n1} samples, {dt1:.1f} s"},
            "host_cpu": model, "host_cpus": os.cpu_count()}


def bench_batch(lap, gg, n_jobs):
    """Many-graph batch: 512 jobs (half ER with average degree in [8, 20],
    half BA with m in 2..8, n log-uniform in [1000, 200000], omega uniform in
    [256, 4096], job list seed 2), each estimating closeness and Kemeny's
    constant, in one persistent launch; against the same jobs run one by one
    through the plain path (identical counts, so equal accuracy)."""
    import torch
    t0 = time.perf_counter()
    specs = gg.batch_jobs(n_jobs, seed=2)
    jobs = []
    for sp in specs:
        s, d = gg.job_edges(sp)
        jobs.append(dict(n=sp["n"], src=s, dst=d, keep_lcc=True, root=-1, omega=sp["omega"], seed=1))
    log(f"batch: generated {n_jobs} graphs in {time.perf_counter() - t0:.1f} s")
    # autotune on the whole batch (a probe subset of the jobs favours smaller
    # pools than the whole batch runs best with), then time the tuned batch
    b = lap.Batch(jobs)
    t_tune = time.perf_counter()
    tuning, tune_ms = b.autotune()
    log(f"batch: autotuned pool={tuning.pool} chunk={tuning.chunk_nodes} ({tune_ms:.1f} ms per run, "
        f"{time.perf_counter() - t_tune:.1f} s of tuning)")
    b.run(tuning)
    torch.cuda.synchronize()
    reps = 3
    t = time.perf_counter()
    for _ in range(reps):
        b.run(tuning)
    torch.cuda.synchronize()
    bt = (time.perf_counter() - t) / reps
    st = b.stats()
    steps = st["wilson_steps"] + st["absorbed_steps"]
    # plain path, one job after another (graph preparation untimed)
    plain_s = 0.0
    dev = torch.device("cuda:0")
    for j, job in enumerate(jobs):
        g = lap.Graph(job["n"], job["src"], job["dst"], keep_lcc=True)
        out = {k: torch.empty(g.n, dtype=torch.float64, device=dev) for k in ("diag", "closeness")}
        out.update({k: torch.empty(1, dtype=torch.float64, device=dev) for k in ("trace", "kemeny", "kemeny_se")})
        g.estimate(job["omega"], 1, -1, B=1, se=False, out=out)         # warm the workspace
        torch.cuda.synchronize()
        t = time.perf_counter()
        g.estimate(job["omega"], 1, -1, B=1, se=False, out=out)
        torch.cuda.synchronize()
        plain_s += time.perf_counter() - t
        g.close()
        if (j + 1) % 128 == 0:
            log(f"batch: plain path {j + 1}/{len(jobs)}")
    return {"workload": f"{n_jobs} graphs (ER/BA mix, n log-uniform 1e3..2e5, omega 256..4096), one launch",
            "jobs": n_jobs, "total_nodes": int(sum(i["n"] for i in b.info)),
            "total_trees": st["trees"], "walk_steps": steps,
            "batched_s": bt, "batched_steps_per_s": steps / bt, "batched_trees_per_s": st["trees"] / bt,
            "plain_s": plain_s, "plain_steps_per_s": steps / plain_s, "plain_trees_per_s": st["trees"] / plain_s,
            "speedup_batched_vs_plain": plain_s / bt,
            "tuning": {"pool": tuning.pool, "chunk_nodes": tuning.chunk_nodes, "use_graph": tuning.use_graph}}


def _replay(lap, srv, qs, qid0):
    """Submit each query at its arrival time (seconds from start), drive the
    loop, return per-query latencies (completion - submission)."""
    kinds = {0: lap.Server.CLOSENESS, 1: lap.Server.RESISTANCE, 2: lap.Server.KEMENY}
    t0 = time.perf_counter()
    i, out = 0, []
    while len(out) < len(qs):
        now = time.perf_counter() - t0
        while i < len(qs) and qs[i]["t"] <= now:
            q = qs[i]
            srv.submit(qid0 + q["qid"], kinds[q["kind"]], q["budget"], q["u"], q["w"])
            i += 1
        srv.step(wait=False)
        out += srv.poll()
        if i < len(qs) and not srv.pending()["inflight"]:
            time.sleep(min(0.001, max(0.0, qs[i]["t"] - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    lat = np.array([r["t_done"] - r["t_submit"] for r in out])
    bad = sum(r["status"] != 0 for r in out)
    return lat, wall, bad


def bench_spantree(lap, g, root, omega):
    """SpanTree estimators (Alg. 1 + Alg. 3) on the mid workload: the same
    Wilson trees as the plain LEWalk step, plus the per-tree pass; the
    LEWalk estimate at the same omega is timed beside it."""
    import torch
    g.estimate(omega, 1, root, B=64)
    t = time.perf_counter()
    g.estimate(omega, 1, root, B=64)
    lewalk_s = time.perf_counter() - t
    g.spantree_estimate(omega, 1, root, B=64)
    torch.cuda.synchronize()
    lap.prof_reset()
    lap.prof_enable(True)
    t = time.perf_counter()
    e = g.spantree_estimate(omega, 1, root, B=64)
    dt = time.perf_counter() - t
    lap.prof_enable(False)
    ms_t, n_t = lap.prof_read("spantree")
    ms_w = lap.prof_read("wilson_wave")[0] + lap.prof_read("wilson_group")[0]
    return {"workload": f"SpanTree closeness + Kemeny (Alg. 1, Alg. 3), same graph and trees, omega={omega}",
            "s_per_step": dt, "trees_per_s": omega / dt, "spantree_kernel_ms": ms_t,
            "wilson_kernel_ms": ms_w, "kemeny": float(e["kemeny"][0]), "kemeny_se": float(e["kemeny_se"][0]),
            "lewalk_s_per_step_same_omega": lewalk_s, "spantree_over_lewalk_time": dt / lewalk_s}


def bench_loop_paths(lap, g, root, omega):
    """Loop-included paths (Sec. 3.4) on the mid workload: per Wilson sample,
    the path from where absorbed walk i starts, read from the sample's
    stacks, for both start laws; the fresh absorbed walks they stand in for
    are timed beside them (their Wilson trees included)."""
    out = {"workload": f"loop-included paths, Barabasi-Albert n=100000 m=5, omega={omega}"}
    for tag, name in ((1, "uniform"), (2, "stationary")):
        g.loop_included(omega, 1, tag, root, B=64)
        lap.prof_reset()
        lap.prof_enable(True)
        t = time.perf_counter()
        r = g.loop_included(omega, 1, tag, root, B=64)
        dt = time.perf_counter() - t
        lap.prof_enable(False)
        ms, _ = lap.prof_read("loop_included")
        out[name] = {"s": dt, "path_kernel_ms": ms, "path_steps": int(r["len"].sum()),
                     "mean_len": float(r["len"].mean())}
    g.sample_forests(omega, 1, root, y1=False, per_sample=False, y2=True, y2_pi=True, B=64)
    lap.prof_reset()
    lap.prof_enable(True)
    g.sample_forests(omega, 1, root, y1=False, per_sample=False, y2=True, y2_pi=True, B=64)
    lap.prof_enable(False)
    ms_a, n_a = lap.prof_read("absorbed")
    out["fresh_absorbed_kernel_ms_per_kind"] = ms_a / max(n_a, 1)
    return out


def bench_pairs(lap, g, root, n, omega=1024, n_pairs=256):
    """Resistances and grounded-inverse entries of node pairs from
    loop-included paths (Sec. 3.4) on the mid workload: 256 random pairs
    (seed 3), 1024 samples, B = 64; the entries read without the sampler
    (check 0), then with the Wilson run that checks them (check 1); then
    whole rows of L_v^{-1} for 64 of the sources."""
    rng = np.random.default_rng(3)
    s = rng.integers(0, n, n_pairs).astype(np.int32)
    t = rng.integers(0, n, n_pairs).astype(np.int32)
    out = {"workload": f"node pairs, Barabasi-Albert n=100000 m=5, {n_pairs} random pairs, omega={omega}",
           "paths": 2 * n_pairs * omega}
    for check in (0, 1):
        g.pair_paths(s, t, omega, 1, root, B=64, check=check)
        lap.prof_reset()
        lap.prof_enable(True)
        t0 = time.perf_counter()
        r = g.pair_paths(s, t, omega, 1, root, B=64, check=check)
        dt = time.perf_counter() - t0
        lap.prof_enable(False)
        ms, _ = lap.prof_read("pair_paths")
        st = g.last_stats()
        out[f"check{check}"] = {"s": dt, "path_kernel_ms": ms, "path_steps": st["absorbed_steps"],
                                "wilson_steps": st["wilson_steps"],
                                "path_steps_per_s": st["absorbed_steps"] / (ms * 1e-3)}
    ok = r["r"] > 0
    out["median_rel_se_r"] = float(np.median(r["r_se"][ok] / r["r"][ok]))
    out["mean_path_len"] = out["check0"]["path_steps"] / out["paths"]
    # whole rows of L_v^{-1} for 64 of the sources, same samples
    src = s[:64]
    g.lv_rows(src, omega, 1, root, check=0)
    lap.prof_reset()
    lap.prof_enable(True)
    t0 = time.perf_counter()
    g.lv_rows(src, omega, 1, root, check=0)
    dt = time.perf_counter() - t0
    lap.prof_enable(False)
    ms, _ = lap.prof_read("pair_paths")
    st = g.last_stats()
    out["rows"] = {"sources": len(src), "s": dt, "path_kernel_ms": ms, "path_steps": st["absorbed_steps"],
                   "path_steps_per_s": st["absorbed_steps"] / (ms * 1e-3)}
    return out


def bench_landmark(lap, gg):
    """Landmark study: Tr((I - P_v)^{-1}) for every node v of a
    Barabasi-Albert graph n = 10,000, m = 5 as the candidate root, 32 Wilson
    samples per root, all roots in one persistent launch."""
    n, omega = 10_000, 32
    src, dst = gg.barabasi_albert(n, 5, 0)
    g = lap.Graph(n, src, dst)
    roots = np.arange(n, dtype=np.int32)
    g.landmark_traces(roots[:64], omega, 1)
    t = time.perf_counter()
    tr, se = g.landmark_traces(roots, omega, 1)
    dt = time.perf_counter() - t
    deg = np.diff(g.csr()[0])
    order = np.argsort(tr)
    res = {"workload": f"Barabasi-Albert n={n} m=5, every node as the root, {omega} trees per root, one launch",
           "roots": n, "trees": n * omega, "s": dt, "trees_per_s": n * omega / dt,
           "trace_over_n_max_degree_root": float(tr[int(np.argmax(deg))] / n),
           "trace_over_n_median": float(np.median(tr) / n),
           "trace_over_n_best": float(tr[order[0]] / n), "best_root_degree": int(deg[order[0]]),
           "max_degree": int(deg.max())}
    g.close()
    return res


def bench_kc_families(lap, gg, n):
    """Kemeny's constant of synthetic families (the paper's Sec. 6 study on
    BA, ER and hyperbolic graphs): BA with m = 2..6; ER with average degree
    200..1000 (p = 2..10 x 1e-4 at 1e6 nodes); hyperbolic with gamma =
    2.2..3.0 and average degree 10 (largest component); 256 samples each,
    all 15 graphs in one batched launch."""
    import torch
    t0 = time.perf_counter()
    jobs, labels = [], []
    for m in (2, 3, 4, 5, 6):
        s, d = gg.barabasi_albert(n, m, 100 + m)
        jobs.append(dict(n=n, src=s, dst=d, keep_lcc=True, root=-1, omega=256, seed=1))
        labels.append(f"BA m={m}")
    for k in (200, 400, 600, 800, 1000):
        s, d = gg.erdos_renyi(n, k / (n - 1), 200 + k)
        jobs.append(dict(n=n, src=s, dst=d, keep_lcc=True, root=-1, omega=256, seed=1))
        labels.append(f"ER avg degree {k}")
    for gamma in (2.2, 2.4, 2.6, 2.8, 3.0):
        s, d = gg.hyperbolic(n, 10.0, gamma, 300 + int(round(gamma * 10)))
        jobs.append(dict(n=n, src=s, dst=d, keep_lcc=True, root=-1, omega=256, seed=1))
        labels.append(f"hyperbolic gamma={gamma}")
    log(f"kc families: {len(jobs)} graphs generated in {time.perf_counter() - t0:.1f} s "
        f"({sum(len(j['src']) for j in jobs) / 1e6:.0f} M edges)")
    b = lap.Batch(jobs)
    del jobs
    gen_s = time.perf_counter() - t0
    log(f"kc families: batch built in {gen_s:.1f} s")
    tuning = lap.Batch.tuning()
    b.run(tuning)
    torch.cuda.synchronize()
    log("kc families: warm-up run done")
    t = time.perf_counter()
    b.run(tuning)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    rows = []
    for j, lab in enumerate(labels):
        r = b.result(j)
        rows.append({"graph": lab, "n_lcc": int(b.info[j]["n"]), "kemeny": float(r["kemeny"][0]),
                     "kemeny_se": float(r["kemeny_se"][0]),
                     "kemeny_over_n": float(r["kemeny"][0]) / b.info[j]["n"]})
    st = b.stats()
    b.close()
    return {"workload": f"15 synthetic graphs, n={n}, 256 samples each, one batched launch", "s": dt,
            "prepare_s": gen_s, "walk_steps_per_s": (st["wilson_steps"] + st["absorbed_steps"]) / dt,
            "graphs": rows}


def _serial(lap, srv, qs, qid0):
    """The same queries one at a time: each is submitted when the previous
    one has completed (no batching across queries).  Returns the wall time."""
    kinds = {0: lap.Server.CLOSENESS, 1: lap.Server.RESISTANCE, 2: lap.Server.KEMENY}
    t0 = time.perf_counter()
    bad = 0
    for q in qs:
        srv.submit(qid0 + q["qid"], kinds[q["kind"]], q["budget"], q["u"], q["w"])
        done = []
        while not done:
            srv.step(wait=True)
            done = srv.poll()
        bad += sum(r["status"] != 0 for r in done)
    return time.perf_counter() - t0, bad


def bench_large(lap, gg, peaks):
    """Large plain run: R-MAT scale 22 (edge factor 16, a/b/c/d = .57/.19/.19/.05),
    symmetrised, self-loops and duplicates dropped, largest component kept;
    root = max degree; 512 trees plus 512 walks of each kind per step."""
    import torch
    t = time.perf_counter()
    src, dst = gg.rmat(22, 16, seed=0)
    g = lap.Graph(1 << 22, src, dst, keep_lcc=True)
    del src, dst
    log(f"large: R-MAT 22 LCC n={g.n} 2m={g.nnz} prepared in {time.perf_counter() - t:.1f} s")
    dev = torch.device("cuda:0")
    out = {k: torch.empty(g.n, dtype=torch.float64, device=dev) for k in ("diag", "diag_se", "closeness")}
    out.update({k: torch.empty(1, dtype=torch.float64, device=dev) for k in ("trace", "kemeny", "kemeny_se")})
    omega = 512
    g.estimate(omega, 1, -1, B=64, out=out)
    torch.cuda.synchronize()
    lap.prof_reset()
    lap.prof_enable(True)
    reps = 2
    t = time.perf_counter()
    for _ in range(reps):
        g.estimate(omega, 1, -1, B=64, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    lap.prof_enable(False)
    st = g.last_stats()
    kern = "wilson_group" if lap.prof_read("wilson_group")[1] else "wilson_wave"
    ms_w, n_w = lap.prof_read(kern)
    wave_s = ms_w / max(n_w, 1) * 1e-3
    loads = LOADS_PER_WILSON_STEP * st["wilson_steps"] / wave_s
    res = {"workload": "R-MAT scale 22 LCC, root = max degree, 512 trees + 512 walks of each kind",
           "n": g.n, "nnz": g.nnz, "omega": omega, "s_per_step": dt, "kernel": kern,
           "walk_steps_per_s": (st["wilson_steps"] + st["absorbed_steps"]) / dt,
           "trees_per_s": omega / dt, "wilson_steps_per_tree": st["wilson_steps"] / omega,
           "wilson_kernel_s": wave_s, "wilson_loads_per_s": loads,
           "state_bytes": 8 * g.n * omega,
           "kemeny": float(out["kemeny"].item()), "kemeny_se": float(out["kemeny_se"].item())}
    if peaks:
        res["frac_of_chase_peak_4GiB"] = loads / peaks["4GiB"]["chase"]
    g.close()
    return res


def bench_serve(lap, gg, n_queries):
    """Serving: resident R-MAT scale-21 graph (edge factor 16, a/b/c/d =
    .57/.19/.19/.05, symmetrised, self-loops and duplicates dropped, largest
    component); Poisson arrivals mixing single-node closeness (64..1024 walks,
    log-uniform), pairwise resistance (1024 walk pairs) and Kemeny (256
    samples) in proportions 45/45/10.  Saturation throughput is measured with
    every query submitted at once; latency percentiles at 50% and 80% of it."""
    t = time.perf_counter()
    src, dst = gg.rmat(21, 16, seed=0)
    g = lap.Graph(1 << 21, src, dst, keep_lcc=True)
    del src, dst
    log(f"serve: R-MAT 21 LCC n={g.n} 2m={g.nnz} prepared in {time.perf_counter() - t:.1f} s")
    srv = lap.Server(g, seed=1, global_samples=256)
    qs = gg.query_stream(g.n, n_queries, qps=1.0, seed=3)
    for q in qs:
        q["t"] = 0.0
    lat, wall, bad = _replay(lap, srv, qs, 0)
    sat = n_queries / wall
    log(f"serve: saturation {sat:.1f} queries/s")
    n_serial = min(n_queries, 100)
    wall_serial, bad_serial = _serial(lap, srv, qs[:n_serial], 10_000_000)
    log(f"serve: one query at a time {n_serial / wall_serial:.1f} queries/s")
    out = {"workload": "R-MAT scale 21 LCC resident; Poisson mix 45% closeness (64-1024 walks), "
                       "45% resistance (1024 walk pairs), 10% Kemeny (256 samples)",
           "n": g.n, "nnz": g.nnz, "queries": n_queries, "saturation_qps": sat,
           "closed_loop_p50_ms": float(np.percentile(lat, 50) * 1e3), "errors": int(bad) + int(bad_serial),
           "one_at_a_time_qps": n_serial / wall_serial,
           "speedup_served_vs_one_at_a_time": sat / (n_serial / wall_serial), "runs": []}
    for k, frac in enumerate((0.5, 0.8)):
        qs = gg.query_stream(g.n, n_queries, qps=frac * sat, seed=4 + k)
        lat, wall, bad = _replay(lap, srv, qs, (k + 1) * 1_000_000)
        out["runs"].append({"offered_qps": frac * sat, "achieved_qps": n_queries / wall,
                            "p50_ms": float(np.percentile(lat, 50) * 1e3),
                            "p99_ms": float(np.percentile(lat, 99) * 1e3), "errors": int(bad)})
        log(f"serve: {frac:.0%} load p50 {out['runs'][-1]['p50_ms']:.1f} ms p99 {out['runs'][-1]['p99_ms']:.1f} ms")
    srv.close()
    g.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--omega", type=int, default=4096)
    ap.add_argument("--no-gather", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-jobs", type=int, default=512)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-spantree", action="store_true")
    ap.add_argument("--no-landmark", action="store_true")
    ap.add_argument("--no-loop-paths", action="store_true")
    ap.add_argument("--no-pairs", action="store_true")
    ap.add_argument("--no-kc-families", action="store_true")
    ap.add_argument("--kc-n", type=int, default=100_000)
    ap.add_argument("--serve-queries", type=int, default=2000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of 1 GiB (counter calibration) and exit")
    ap.add_argument("--write-traffic", metavar="DIR",
                    help="only reduce the counter databases under DIR to the traffic summary and exit")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args.write_traffic)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen as gg
    import paper_2311_10290_amd as lap

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)     # 1 GiB
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 8}), flush=True)
        return
    n, m, omega, seed = 100_000, 5, args.omega, 1
    log("generating BA(100000, 5)")
    src, dst = gg.barabasi_albert(n, m, 0)
    g = lap.Graph(n, src, dst)
    root = g.max_deg_node
    out = {k: torch.empty(g.n, dtype=torch.float64, device=dev) for k in ("diag", "diag_se", "closeness")}
    out.update({k: torch.empty(1, dtype=torch.float64, device=dev) for k in ("trace", "kemeny", "kemeny_se")})
    stream = torch.cuda.current_stream()

    def step():
        g.estimate(omega, seed, root, B=64, out=out, stream=stream)

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    st = g.last_stats()
    lap.prof_reset()
    lap.prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        log(f"step {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lap.prof_enable(False)
    st = g.last_stats()
    steps_per = st["wilson_steps"] + st["absorbed_steps"]
    value = steps_per * args.steps / dt
    ms_w, n_w = lap.prof_read("wilson_wave")
    ms_a, n_a = lap.prof_read("absorbed")
    ms_s, n_s = lap.prof_read("assemble")
    wave_ms = ms_w / max(n_w, 1)
    alg_bytes = WILSON_BYTES_PER_STEP * st["wilson_steps"] + RETRACE_BYTES_PER_NODE * g.n * st["trees"]
    achieved = alg_bytes / (wave_ms * 1e-3) / 1e9
    res = {
        "metric": "walk steps/s & spanning trees/s at 1 GPU, batched vs plain; p99 query latency",
        "value": value,
        "unit": "walk steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64 counts, f64 estimates",
        "data": "synthetic (seeded Barabasi-Albert graph; no dataset)",
        "config": {"workload": "plain LEWalk closeness + Kemeny: Barabasi-Albert n=100000 m=5, "
                               "root=max degree, omega=4096 trees, Philox seed 1",
                   "n": g.n, "nnz": g.nnz, "omega": omega, "mode": "wave"},
        "trees_per_s": omega * args.steps / dt,
        "wilson_steps_per_step": st["wilson_steps"],
        "wave_iterations_per_step": st["iterations"], "cycle_pops": st["pops"], "rescans": st["rescans"],
        "absorbed_steps_per_step": st["absorbed_steps"],
        "kernel_ms": {"wilson_wave": wave_ms, "absorbed": ms_a / max(n_a, 1),
                      "assemble": ms_s / max(n_s, 1)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "wilson_wave_kernel",
                     "bytes_per_launch": alg_bytes},
        "estimates": {"kemeny": float(out["kemeny"].item()), "kemeny_se": float(out["kemeny_se"].item()),
                      "trace_Ldagger": float(out["trace"].item())},
    }
    peaks = {}
    if not args.no_gather:
        log("random-gather peak")
        lanes = 256 * 24 * 64
        for label, nbytes in (("4MiB", 4 << 20), ("128MiB", 128 << 20), ("4GiB", 4 << 30)):
            peaks[label] = {"chase": lap.bench_gather(nbytes, lanes, 1),
                            "independent": lap.bench_gather(nbytes, lanes // 4, 0)}
        loads = LOADS_PER_WILSON_STEP * st["wilson_steps"]
        achieved_loads = loads / (wave_ms * 1e-3)
        res["gather"] = {"loads_per_wilson_step": LOADS_PER_WILSON_STEP,
                         "achieved_loads_per_s": achieved_loads,
                         "peak_loads_per_s": peaks,
                         "frac_of_chase_peak_4GiB": achieved_loads / peaks["4GiB"]["chase"],
                         "state_bytes": 8 * g.n * min(omega, 4096)}
        # line fetches: every 4 GiB chase load fetches one 128-byte line
        # (FETCH_SIZE); the kernel's fetched bytes come from its counter summary
        fetch = measured_traffic("FETCH_SIZE")
        chase_line = peaks["4GiB"]["chase"] * CHASE_BYTES_PER_LOAD
        res["gather"]["chase_line_bytes_per_s_4GiB"] = chase_line
        res["gather"]["wilson_fetch_bytes_per_s"] = fetch / (wave_ms * 1e-3) if fetch else None
        res["gather"]["frac_of_chase_line_rate"] = fetch / (wave_ms * 1e-3) / chase_line if fetch else None
    if not args.no_spantree:
        log("spantree")
        res["spantree"] = bench_spantree(lap, g, root, 1024)
    if not args.no_loop_paths:
        log("loop-included paths")
        res["loop_paths"] = bench_loop_paths(lap, g, root, omega)
    if not args.no_pairs:
        log("node-pair paths")
        res["pairs"] = bench_pairs(lap, g, root, n)
    if not args.no_landmark:
        log("landmark study")
        res["landmark"] = bench_landmark(lap, gg)
    if not args.no_kc_families:
        log("Kemeny's constant of synthetic families")
        res["kc_families"] = bench_kc_families(lap, gg, args.kc_n)
    if not args.no_batch:
        res["batched"] = bench_batch(lap, gg, args.batch_jobs)
    if not args.no_serve:
        res["serving"] = bench_serve(lap, gg, args.serve_queries)
    if not args.no_large:
        res["large"] = bench_large(lap, gg, peaks if not args.no_gather else None)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        from oracle import csr as ocsr
        og = ocsr.build_csr(n, src, dst)
        res["cpu_baseline"] = cpu_baseline(og, root, omega, seed)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
