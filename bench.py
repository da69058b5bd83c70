"""Benchmark of the hot path.  One step = Wilson loop-erased-walk sampling
(omega trees rooted at the max-degree node), omega uniform-start and omega
stationary-start absorbed walks, and the FP64 assembly of diag(L^dagger),
closeness and Kemeny's constant (Alg. 2 + Alg. 4), with inputs resident in
HBM before timing.

Headline: R-MAT scale 22 (edge factor 16, a/b/c/d = .57/.19/.19/.05),
symmetrised, self-loops and duplicates dropped, largest component kept
(n = 2.39 M, 2m = 128.3 M), omega = 512 -- the largest single-GPU workload.
`value` is walk steps per second (Wilson draws plus absorbed-walk draws).

Sub-records: the small ER(256, 0.05) workload (omega = 2^14, with its accuracy
against the dense pseudo-inverse), the mid Barabasi-Albert workload (n = 10^5,
m = 5, omega = 4096), the random-gather sweep, the 512-graph batch, serving on
a resident R-MAT 21 graph, SpanTree, loop-included paths, node pairs, the
landmark study and Kemeny's constant of synthetic families.  Each workload
with a CPU figure times the oracle on the host's cores on a bounded sample.
The small, mid, large, batched and serving workloads are defined in
graphgen/workloads.json (graph recipe, preparation, landmark, sample budget,
blocks and seeds).

Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# vector ALU issue peak: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD
# every 4 cycles (16 lanes wide), at 2.4 GHz
VALU_PEAK_WAVE_INSTR = 256 * 4 * 2.4e9 / 4
WILSON_BYTES_PER_STEP = 33.0     # offsets 16 + column 4 + draw count 8 + next 4 + tree flag 1
RETRACE_BYTES_PER_NODE = 5.0
SEED = 1

# everything the Wilson kernels and their launch configuration are built from:
# a counter summary taken on other sources is not used
KERNEL_SOURCES = ["paper_2311_10290_amd/csrc/" + f for f in
                  ("wilson.hip", "wave_sample.h", "group_sample.h", "lap_device.h", "lap_params.h",
                   "lap_launch.h", "lap_host.h", "capi.cpp")]
TRAFFIC = {
    "large": dict(file="profiles/traffic_wilson_group_rmat22.json", kernel="wilson_group_kernel<8, true>",
                  workload="R-MAT scale 22 LCC numbered by decreasing degree, omega=512, one launch"),
    "mid": dict(file="profiles/traffic_wilson_wave_ba100k.json", kernel="wilson_wave_kernel<true>",
                workload="Barabasi-Albert n=100000 m=5 numbered by decreasing degree, omega=4096, one launch"),
    "small": dict(file="profiles/traffic_wilson_wave_er256.json", kernel="wilson_wave_kernel<true>",
                  workload="ER(256, 0.05), omega=2^14, one launch"),
}
SECTIONS = ("large", "small", "mid", "gather", "spantree", "loop_paths", "pairs", "landmark", "kc_families",
            "batched", "serving")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(which):
    """The committed counter summary of one Wilson launch of the workload, if
    it was taken on the current kernel sources; otherwise None."""
    try:
        with open(os.path.join(ROOT, TRAFFIC[which]["file"])) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    return t if t.get("kernel_hash") == kernel_hash() else None


def _csv_counters(path, kernel):
    """Per-dispatch counter values {counter: [v per dispatch]} of the dispatches
    whose kernel name contains `kernel`, from rocprofv3 CSV output under path."""
    import csv
    import glob
    files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    if len(files) != 1:
        raise SystemExit(f"expected one counter_collection.csv under {path}, found {files}")
    per = {}
    with open(files[0]) as fh:
        for r in csv.DictReader(fh):
            if kernel in r["Kernel_Name"]:
                per.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
    return [per[k] for k in sorted(per)]


def write_traffic(pmc_dir, which):
    """Reduce the counter runs under pmc_dir to the traffic summary of one
    Wilson launch of the workload.  Expects four runs (rocprofv3 CSV output):
    copy_fetch/ and copy_write/ (``--copy-calibration``: a 1 GiB device copy)
    and <which>_fetch/, <which>_write/ (``--only <which> --steps 1 --warmup 0``),
    fetch runs with TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_BUBBLE_sum, write
    runs with TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum (the inputs of FETCH_SIZE
    and WRITE_SIZE), plus <which>_fetch/bench.json (the run's JSON line, for
    the draws per launch), and optionally <which>_tcc/ with TCC_HIT_sum
    TCC_MISS_sum TCC_REQ_sum TCP_TCC_READ_REQ_sum TCP_TCC_WRITE_REQ_sum (the
    L1-to-L2 requests) and <which>_valu/ with SQ_INSTS_VALU and
    SQ_INSTS_VALU_INT64 (vector instructions issued, 64-bit integer ones among
    them).  Each byte count is scaled by the copy's bytes over
    what the same counters read for the copy; several launches of the kernel
    in one run are averaged."""
    def fetch_bytes(c):
        rd, r32, bub = c["TCC_EA0_RDREQ_sum"], c["TCC_EA0_RDREQ_32B_sum"], c["TCC_BUBBLE_sum"]
        return bub * 128 + (rd - bub - r32) * 64 + r32 * 32

    def write_bytes(c):
        wr, w64 = c["TCC_EA0_WRREQ_sum"], c["TCC_EA0_WRREQ_64B_sum"]
        return (wr - w64) * 32 + w64 * 64

    spec = TRAFFIC[which]
    copy_bytes = 1 << 30
    cal_f = copy_bytes / fetch_bytes(_csv_counters(os.path.join(pmc_dir, "copy_fetch"), "copyBuffer")[0])
    cal_w = copy_bytes / write_bytes(_csv_counters(os.path.join(pmc_dir, "copy_write"), "copyBuffer")[0])
    def mean(rows):
        if not rows:
            raise SystemExit(f"no {spec['kernel']} dispatch found")
        return {k: sum(r[k] for r in rows) / len(rows) for k in rows[0]}

    f = mean(_csv_counters(os.path.join(pmc_dir, f"{which}_fetch"), spec["kernel"]))
    w = mean(_csv_counters(os.path.join(pmc_dir, f"{which}_write"), spec["kernel"]))
    with open(os.path.join(pmc_dir, f"{which}_fetch", "bench.json")) as fh:
        b = json.loads(fh.read().strip().splitlines()[-1])
    draws = b["wilson_steps_per_step"] if which == "large" else b[which]["wilson_steps_per_step"]
    res = {"kernel": spec["kernel"], "workload": spec["workload"], "kernel_hash": kernel_hash(),
           "draws_per_launch": draws,
           "fetch": {"counters": f, "raw_bytes": fetch_bytes(f), "calibration": cal_f,
                     "bytes": fetch_bytes(f) * cal_f},
           "write": {"counters": w, "raw_bytes": write_bytes(w), "calibration": cal_w,
                     "bytes": write_bytes(w) * cal_w},
           "read_requests_per_launch": f["TCC_EA0_RDREQ_sum"]}
    tcc_dir = os.path.join(pmc_dir, f"{which}_tcc")
    if os.path.isdir(tcc_dir):
        t = mean(_csv_counters(tcc_dir, spec["kernel"]))
        res["l2"] = {"counters": t, "l1_to_l2_read_requests_per_draw": t["TCP_TCC_READ_REQ_sum"] / draws,
                     "l2_hit_rate": t["TCC_HIT_sum"] / max(t["TCC_REQ_sum"], 1.0)}
    valu_dir = os.path.join(pmc_dir, f"{which}_valu")
    if os.path.isdir(valu_dir):
        v = mean(_csv_counters(valu_dir, spec["kernel"]))
        res["valu"] = {"counters": v, "instructions_per_launch": v["SQ_INSTS_VALU"],
                       "instructions_per_draw": v["SQ_INSTS_VALU"] / draws,
                       "int64_share": v["SQ_INSTS_VALU_INT64"] / max(v["SQ_INSTS_VALU"], 1.0)}
    res["bytes_per_launch"] = res["fetch"]["bytes"] + res["write"]["bytes"]
    res["bytes_per_draw"] = res["bytes_per_launch"] / draws
    res["read_requests_per_draw"] = res["read_requests_per_launch"] / draws
    with open(os.path.join(ROOT, spec["file"]), "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


def host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return model


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_baseline(og, root, omega_full, budget_s=15.0, probe=64, seed=SEED):
    """The oracle (C, OpenMP over samples) on a bounded sample of the same
    workload: the first n_s samples (Wilson + both absorbed-walk kinds), n_s
    sized from a probe run to take about budget_s; repeated when the whole
    workload is shorter than that.  Then one thread on a smaller sample."""
    from oracle import native
    threads = oracle_threads()
    probe = min(probe, omega_full)
    t = time.perf_counter()
    native.wilson(og, root, omega_full, seed, n_samples=probe, want_y1=True, threads=threads)
    dt = time.perf_counter() - t
    n_s = int(min(omega_full, max(probe, probe * budget_s / max(dt, 1e-3))))
    reps, steps, trees, t = 0, 0, 0, time.perf_counter()
    while True:
        w = native.wilson(og, root, omega_full, seed, n_samples=n_s, threads=threads)
        a1 = native.absorbed(og, root, n_s, seed, 1, omega_total=omega_full, threads=threads)
        a2 = native.absorbed(og, root, n_s, seed, 2, omega_total=omega_full, want_y2=False, threads=threads)
        steps += int(w["y1"].sum() + a1["len"].sum() + a2["len"].sum())
        trees += n_s
        reps += 1
        dt = time.perf_counter() - t
        if n_s < omega_full or dt >= 0.7 * budget_s:
            break
    n1 = max(2, min(n_s, n_s // (2 * threads)))
    t1 = time.perf_counter()
    w = native.wilson(og, root, omega_full, seed, n_samples=n1, threads=1)
    a1 = native.absorbed(og, root, n1, seed, 1, omega_total=omega_full, threads=1)
    a2 = native.absorbed(og, root, n1, seed, 2, omega_total=omega_full, want_y2=False, threads=1)
    steps1 = int(w["y1"].sum() + a1["len"].sum() + a2["len"].sum())
    dt1 = time.perf_counter() - t1
    return {"value": steps / dt, "unit": "walk steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_s} of {omega_full} samples (Wilson + both absorbed-walk kinds), "
                      f"{reps} pass(es), {dt:.1f} s",
            "trees_per_s": trees / dt,
            "single_thread": {"value": steps1 / dt1, "unit": "walk steps/s",
                              "sample": f"first {n1} samples, {dt1:.1f} s"},
            "host_cpu": host_cpu(), "host_cpus": os.cpu_count()}


def _out_tensors(n):
    import torch
    dev = torch.device("cuda:0")
    out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("diag", "diag_se", "closeness")}
    out.update({k: torch.empty(1, dtype=torch.float64, device=dev) for k in ("trace", "kemeny", "kemeny_se")})
    return out


def timed_steps(lap, g, omega, root, steps, warmup, B=64, walks=0, seed=SEED):
    """Run warmup + steps plain steps on torch's current stream; time the
    steps between two device synchronisations, with per-kernel HIP-event
    timing (on the streams the kernels run on) over the timed region."""
    import torch
    out = _out_tensors(g.n)
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        g.estimate(omega, seed, root, B=B, out=out, stream=stream, walks=walks)
    torch.cuda.synchronize()
    lap.prof_reset()
    lap.prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        g.estimate(omega, seed, root, B=B, out=out, stream=stream, walks=walks)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lap.prof_enable(False)
    st = g.last_stats()
    kern = {}
    for name in ("wilson_group", "wilson_wave", "wilson_lane", "wilson_lds", "absorbed", "loop_included",
                 "assemble"):
        ms, n = lap.prof_read(name)
        if n:
            kern[name] = {"ms_avg": ms / n, "launches": n}
    wk = next(k for k in ("wilson_group", "wilson_wave", "wilson_lane", "wilson_lds") if k in kern)
    return dt, st, kern, wk, out


def roofline(st, n, kern_ms, traffic, kernel):
    alg = WILSON_BYTES_PER_STEP * st["wilson_steps"] + RETRACE_BYTES_PER_NODE * n * st["trees"]
    achieved = alg / (kern_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic["bytes_per_launch"] if traffic else None,
            "kernel": kernel, "bytes_per_launch": alg, "kernel_ms": kern_ms}


def valu_rate(traffic, kern_ms):
    """Vector instructions issued per second (counted) against the issue peak."""
    if not traffic or "valu" not in traffic:
        return None
    rate = traffic["valu"]["instructions_per_launch"] / (kern_ms * 1e-3)
    return {"bound": "alu", "achieved": rate / 1e9, "peak": VALU_PEAK_WAVE_INSTR / 1e9,
            "unit": "G wave64 VALU instructions/s", "frac": rate / VALU_PEAK_WAVE_INSTR,
            "instructions_per_draw": traffic["valu"]["instructions_per_draw"],
            "int64_share": traffic["valu"]["int64_share"]}


def request_rate(traffic, kern_ms, gather):
    """Read requests per second that reach memory (L2 misses, counted) against
    the measured random-request peak at the 4 GiB tier."""
    if not traffic:
        return None
    rps = traffic["read_requests_per_launch"] / (kern_ms * 1e-3)
    out = {"read_requests_per_draw": traffic["read_requests_per_draw"], "read_requests_per_s": rps,
           "bytes_per_draw": traffic["bytes_per_draw"]}
    if gather:
        peak = gather["tiers"]["4GiB"]["peak"]
        out["frac_of_random_request_peak_4GiB"] = rps / peak
    # reads and writes together against the mixed sweep at the nearest write share
    wr = traffic["write"]["counters"].get("TCC_EA0_WRREQ_sum")
    if wr is not None:
        ratio = wr / max(traffic["read_requests_per_launch"], 1.0)
        out["writes_per_read"] = ratio
        out["read_write_requests_per_s"] = (traffic["read_requests_per_launch"] + wr) / (kern_ms * 1e-3)
        if gather:
            # against the highest random-request rate measured at 4 GiB (the
            # read-only one: random stores only lower the sweep's rates)
            out["read_write_frac_of_random_request_peak_4GiB"] = (out["read_write_requests_per_s"] /
                                                                   gather["tiers"]["4GiB"]["peak"])
    return out


# ----------------------------------------------------------------- workloads
def workload_graph(lap, gg, name):
    """The graph of a workload of graphgen/workloads.json, prepared as it says."""
    w = gg.workload(name)
    t = time.perf_counter()
    n, src, dst = gg.workload_edges(name)
    g = lap.Graph(n, src, dst, keep_lcc=w["keep_lcc"], degree_order=w["degree_order"])
    log(f"{name}: n={g.n} 2m={g.nnz} prepared in {time.perf_counter() - t:.1f} s")
    return g, n, src, dst


def lds_form_rate(lap, g, omega, root, draws, reps=3, B=64, seed=SEED):
    """The LDS lane form (graph and state in LDS) on the same samples, against
    the LDS random-read rate of the device (lap_bench_gather mode 4: a sweep of
    lanes and reads in flight per round).  A draw of that form makes about six
    LDS accesses: two row offsets, one column, the state word read and written
    at the node, the target's state word."""
    lds_peak = max(lap.bench_gather(1 << 20, 1 << lg, 4, d) for lg in (14, 16, 18, 20) for d in (1, 4, 16))
    g.sample_forests(omega, seed, root, B=B, mode=4)
    lap.prof_reset()
    lap.prof_enable(True)
    for _ in range(reps):
        g.sample_forests(omega, seed, root, B=B, mode=4)
    lap.prof_enable(False)
    ms, n = lap.prof_read("wilson_lds")
    ms /= max(n, 1)
    rate = 6.0 * draws / (ms * 1e-3)
    return {"wilson_lds_kernel_ms": ms, "draws_per_s": draws / (ms * 1e-3), "lds_accesses_per_draw": 6,
            "lds_accesses_per_s": rate, "lds_random_read_peak": lds_peak, "frac_of_lds_peak": rate / lds_peak}


def bench_small(lap, gg, steps, warmup, with_cpu, gather):
    """Small workload (workloads.json "small": ER(256, 0.05), graph seed 0,
    resampled until connected, root = max degree, omega = 2^14); accuracy
    against the dense FP64 pseudo-inverse at its Philox seed (CPU leg), GPU
    and CPU rates.  A step takes about 2 ms, so four are timed per headline
    step."""
    w = gg.workload("small")
    g, n, src, dst = workload_graph(lap, gg, "small")
    omega, B, seed = w["omega"], w["blocks"], w["philox_seed"]
    root = g.max_deg_node
    reps = 4 * steps
    dt, st, kern, wk, out = timed_steps(lap, g, omega, root, reps, warmup, B=B, seed=seed)
    kms = kern[wk]["ms_avg"]
    res = {"workload": gg.describe_workload("small"),
           "s_per_step": dt / reps, "walk_steps_per_s": (st["wilson_steps"] + st["absorbed_steps"]) * reps / dt,
           "trees_per_s": omega * reps / dt, "wilson_kernel": wk, "wilson_kernel_ms": kms,
           "kernel_ms": {k: v["ms_avg"] for k, v in kern.items()},
           "wilson_steps_per_step": st["wilson_steps"],
           "kemeny": float(out["kemeny"].item()), "kemeny_se": float(out["kemeny_se"].item())}
    # the walk state of 4096 slots x 256 nodes (8 MB) sits in the caches: the
    # reference is the L2-tier random-request rate of the sweep, against the
    # kernel's counted L1-to-L2 read requests
    traffic = measured_traffic("small")
    # everything sits in the caches and the generator runs once per draw: the
    # vector ALU issue rate is the roofline that applies
    res["roofline"] = valu_rate(traffic, kms)
    res["lds_form"] = lds_form_rate(lap, g, omega, root, st["wilson_steps"], B=B, seed=seed)
    if gather and traffic and "l2" in traffic:
        per = traffic["l2"]["l1_to_l2_read_requests_per_draw"]
        rate = per * st["wilson_steps"] / (kms * 1e-3)
        res["cache_tier"] = {"state_bytes": 8 * n * min(omega, 4096), "l1_to_l2_read_requests_per_draw": per,
                             "l2_hit_rate": traffic["l2"]["l2_hit_rate"], "requests_per_s": rate,
                             "peak_4MiB": gather["tiers"]["4MiB"]["peak"],
                             "frac_of_4MiB_peak": rate / gather["tiers"]["4MiB"]["peak"]}
    if with_cpu:
        from oracle import csr as ocsr, dense, native
        og = ocsr.build_csr(n, src, dst, keep_lcc=w["keep_lcc"], degree_order=w["degree_order"])
        L = dense.laplacian(og)
        t = time.perf_counter()
        Ld = dense.pinv_eigh(L)
        t_eigh = time.perf_counter() - t
        t = time.perf_counter()
        Ld2 = dense.pinv_inverse(L)
        t_inv = time.perf_counter() - t
        c_true = dense.closeness(Ld)
        k_true = dense.kemeny_spectral(og)
        c_gpu = out["closeness"].cpu().numpy()
        k_gpu = float(out["kemeny"].item())
        rel_c = np.abs(c_gpu - c_true) / c_true
        # the same samples with loop-included paths in place of fresh walks
        dtl, stl, kernl, _, outl = timed_steps(lap, g, omega, root, reps, warmup, B=B, walks=1, seed=seed)
        c_loop = outl["closeness"].cpu().numpy()
        k_loop = float(outl["kemeny"].item())
        rel_l = np.abs(c_loop - c_true) / c_true
        res["loop_included_estimator"] = {
            "s_per_step": dtl / reps, "kernel_ms": {k: v["ms_avg"] for k, v in kernl.items()},
            "kemeny_rel_err": abs(k_loop - k_true) / k_true,
            "kemeny_z": (k_loop - k_true) / float(outl["kemeny_se"].item()),
            "closeness_mean_rel_err": float(rel_l.mean()), "closeness_max_rel_err": float(rel_l.max())}
        res["accuracy_vs_dense_pinv"] = {
            "kemeny_rel_err": abs(k_gpu - k_true) / k_true, "kemeny_exact": k_true,
            "kemeny_z": (k_gpu - k_true) / float(out["kemeny_se"].item()),
            "closeness_mean_rel_err": float(rel_c.mean()), "closeness_max_rel_err": float(rel_c.max()),
            "target": "<= 1e-2 relative (kappa and mean closeness)",
            "routes_agree": float(np.abs(Ld - Ld2).max())}
        # the SpanTree estimators (Alg. 1, Alg. 3) on the same 2^14 Wilson trees
        sp = g.spantree_estimate(omega, seed, root, B=B)
        rel_cs = np.abs(sp["closeness"] - c_true) / c_true
        res["accuracy_vs_dense_pinv"]["spantree_same_trees"] = {
            "kemeny_rel_err": abs(float(sp["kemeny"][0]) - k_true) / k_true,
            "kemeny_z": (float(sp["kemeny"][0]) - k_true) / float(sp["kemeny_se"][0]),
            "closeness_mean_rel_err": float(rel_cs.mean()), "closeness_max_rel_err": float(rel_cs.max())}
        res["cpu_baseline"] = cpu_baseline(og, root, omega, budget_s=5.0, seed=seed)
        res["cpu_baseline"]["dense_pinv_s"] = {"eigh": t_eigh, "inverse": t_inv}
    g.close()
    return res


def bench_mid(lap, gg, steps, warmup, with_cpu, gather):
    """Mid workload (workloads.json "mid": Barabasi-Albert n = 100,000, m = 5,
    graph seed 0, numbered by decreasing degree, root = max degree, omega =
    4096; wave form)."""
    w = gg.workload("mid")
    g, n, src, dst = workload_graph(lap, gg, "mid")
    omega, B, seed = w["omega"], w["blocks"], w["philox_seed"]
    root = g.max_deg_node
    dt, st, kern, wk, out = timed_steps(lap, g, omega, root, steps, warmup, B=B, seed=seed)
    kms = kern[wk]["ms_avg"]
    traffic = measured_traffic("mid")
    res = {"workload": gg.describe_workload("mid"),
           "n": g.n, "nnz": g.nnz, "omega": omega, "s_per_step": dt / steps,
           "walk_steps_per_s": (st["wilson_steps"] + st["absorbed_steps"]) * steps / dt,
           "trees_per_s": omega * steps / dt, "wilson_steps_per_step": st["wilson_steps"],
           "absorbed_steps_per_step": st["absorbed_steps"],
           "kernel_ms": {k: v["ms_avg"] for k, v in kern.items()},
           "roofline": roofline(st, g.n, kms, traffic, TRAFFIC["mid"]["kernel"]),
           "requests": request_rate(traffic, kms, gather), "valu": valu_rate(traffic, kms),
           "kemeny": float(out["kemeny"].item()), "kemeny_se": float(out["kemeny_se"].item())}
    if with_cpu:
        from oracle import csr as ocsr
        res["cpu_baseline"] = cpu_baseline(ocsr.build_csr(n, src, dst, keep_lcc=w["keep_lcc"],
                                                          degree_order=w["degree_order"]),
                                           root, omega, budget_s=10.0, seed=seed)
    return res, g, root


def hot_vertex_share(g, omega, samples=64, seed=SEED):
    """What staging the hubs' data in LDS or a cache could serve, from the
    draw counts of `samples` trees: with nodes numbered by decreasing degree
    the hubs' arc records open the arc array and their state words open each
    slot.  A draw at u lands uniformly in u's row, so the share of draws whose
    arc record lies in the first B bytes is sum_u Y1[u] * frac_u(B) / sum Y1;
    arrivals at u are expected sum over neighbours w of Y1[w] / d_w, and the
    share of arrivals at the first K nodes is their sum over the total."""
    got = g.sample_forests(min(samples, omega), seed, -1, B=1, per_sample=False)
    y1 = got["Y1"][0].astype(np.float64)
    rp, col, _ = g.csr()
    deg = np.diff(rp).astype(np.float64)
    total = y1.sum()
    arcs = {}
    for label, nbytes in (("64KiB", 64 << 10), ("4MiB", 4 << 20), ("256MiB", 256 << 20)):
        first = nbytes // 16          # 16-byte arc records
        frac = np.clip((first - rp[:-1]) / np.maximum(deg, 1.0), 0.0, 1.0)
        arcs[label] = float((y1 * frac).sum() / total)
    arrivals = np.bincount(col, weights=np.repeat(y1 / np.maximum(deg, 1.0), np.diff(rp)), minlength=g.n)
    state = {str(k): float(arrivals[:k].sum() / arrivals.sum()) for k in (768, 8192, 1 << 16)}
    del col
    return {"samples": int(min(samples, omega)), "draw_share_of_first_arc_bytes": arcs,
            "arrival_share_of_first_nodes": state}


def bench_gather(lap):
    """Random 8-byte gather rates at three working sets: the pointer chase over
    lanes 2^14..2^22, independent loads over lanes {2^14, 2^16, 2^18, 2^20} x
    loads in flight {1, 2, 4, 8, 16}; the peak of each tier is the maximum,
    at 4 GiB over the four load flavours as well."""
    tiers = {}
    for label, nbytes in (("4MiB", 4 << 20), ("128MiB", 128 << 20), ("4GiB", 4 << 30)):
        chase = {str(1 << lg): lap.bench_gather(nbytes, 1 << lg, 1) for lg in range(14, 23)}
        indep = {f"{1 << lg}x{d}": lap.bench_gather(nbytes, 1 << lg, 0, d) for lg in (14, 16, 18, 20)
                 for d in (1, 2, 4, 8, 16)}
        tiers[label] = {"chase": chase, "independent": indep,
                        "chase_peak": max(chase.values()), "independent_peak": max(indep.values()),
                        "peak": max(max(chase.values()), max(indep.values()))}
        log(f"gather {label}: chase peak {tiers[label]['chase_peak'] / 1e9:.1f} G/s, "
            f"independent peak {tiers[label]['independent_peak'] / 1e9:.1f} G/s")
    # the cache policy of the loads (plain, non-temporal, relaxed atomic at
    # device and at system scope) at 4 GiB: chase with 2^19 lanes, independent
    # with 2^18 lanes x 8 loads in flight
    flavors = {name: {"chase": lap.bench_gather(4 << 30, 1 << 19, 1, 1, fl),
                      "independent": lap.bench_gather(4 << 30, 1 << 18, 0, 8, fl)}
               for fl, name in enumerate(("plain", "nontemporal", "atomic_device", "atomic_system"))}
    # the 4 GiB peak is the highest rate of any flavour: non-temporal loads
    # run a few percent above plain ones there
    t4 = tiers["4GiB"]
    t4["plain_peak"] = t4["peak"]
    t4["peak"] = max(t4["peak"], max(max(v.values()) for v in flavors.values()))
    # loads mixed with random stores (one per round of d loads) at 4 GiB, by
    # write share: 8-byte stores reach memory as 32-byte partial writes, line
    # stores as 64-byte writes.  Uniformly random stores cost more than the
    # walkers' write-backs, so these rates are context, not a ceiling.
    mixed = {}
    for mode, label in ((2, "stores_8B"), (3, "stores_64B_lines")):
        sweep = {f"{1 << lg}x{d}": lap.bench_gather(4 << 30, 1 << lg, mode, d) for lg in (16, 18, 20)
                 for d in (1, 2, 4, 8)}
        by_ratio = {str(1.0 / d): max(v for k, v in sweep.items() if k.endswith(f"x{d}")) for d in (1, 2, 4, 8)}
        mixed[label] = {"sweep": sweep, "best_by_writes_per_read": by_ratio}
        log(f"gather 4GiB with {label}: " + ", ".join(f"{float(r):.3f} writes/read {v / 1e9:.1f} G/s"
                                                      for r, v in by_ratio.items()))
    mixed["unit"] = "random loads + stores per second (one memory request each)"
    return {"unit": "random 8-byte loads/s (one memory request each at the 4 GiB tier)", "tiers": tiers,
            "flavors_4GiB": flavors, "with_stores_4GiB": mixed}


def bench_batch(lap, gg, n_jobs, with_cpu):
    """Many-graph batch (workloads.json "batched": 512 jobs, half ER with
    average degree in [8, 20], half BA with m in 2..8, n log-uniform in
    [1000, 200000], omega uniform in [256, 4096], job list seed 2), each
    estimating closeness and Kemeny's constant, in one persistent launch;
    against the same jobs run one by one through the plain path (identical
    counts, so equal accuracy)."""
    import torch
    wb = gg.workload("batched")
    n_jobs = n_jobs or wb["jobs"]
    t0 = time.perf_counter()
    specs = gg.batch_jobs(n_jobs, seed=wb["job_seed"], n_lo=wb["n_range"][0], n_hi=wb["n_range"][1],
                          omega_lo=wb["omega_range"][0], omega_hi=wb["omega_range"][1])
    jobs = []
    for sp in specs:
        s, d = gg.job_edges(sp)
        jobs.append(dict(n=sp["n"], src=s, dst=d, keep_lcc=wb["keep_lcc"], root=-1, omega=sp["omega"],
                         seed=wb["philox_seed"]))
    log(f"batch: generated {n_jobs} graphs in {time.perf_counter() - t0:.1f} s")
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
    plain_s = 0.0
    for j, job in enumerate(jobs):
        g = lap.Graph(job["n"], job["src"], job["dst"], keep_lcc=job["keep_lcc"])
        out = _out_tensors(g.n)
        g.estimate(job["omega"], job["seed"], -1, B=1, se=False, out=out)         # warm the workspace
        torch.cuda.synchronize()
        t = time.perf_counter()
        g.estimate(job["omega"], job["seed"], -1, B=1, se=False, out=out)
        torch.cuda.synchronize()
        plain_s += time.perf_counter() - t
        g.close()
        if (j + 1) % 128 == 0:
            log(f"batch: plain path {j + 1}/{len(jobs)}")
    res = {"workload": f"{n_jobs} graphs (ER/BA mix, n log-uniform 1e3..2e5, omega 256..4096), one launch",
           "jobs": n_jobs, "total_nodes": int(sum(i["n"] for i in b.info)),
           "total_trees": st["trees"], "walk_steps": steps,
           "batched_s": bt, "batched_steps_per_s": steps / bt, "batched_trees_per_s": st["trees"] / bt,
           "plain_s": plain_s, "plain_steps_per_s": steps / plain_s, "plain_trees_per_s": st["trees"] / plain_s,
           "speedup_batched_vs_plain": plain_s / bt,
           "tuning": {"pool": tuning.pool, "chunk_nodes": tuning.chunk_nodes, "use_graph": tuning.use_graph,
                      "tuned_ms": tune_ms}}
    if with_cpu:
        # the oracle on every 32nd job (16 jobs, whole sample budgets)
        from oracle import csr as ocsr, native
        threads = oracle_threads()
        steps_c, trees_c, dt = 0, 0, 0.0
        for j in range(0, n_jobs, 32):
            job = jobs[j]
            og = ocsr.build_csr(job["n"], job["src"], job["dst"], keep_lcc=job["keep_lcc"])
            root = ocsr.landmark(og)
            tt = time.perf_counter()
            w = native.wilson(og, root, job["omega"], job["seed"], threads=threads)
            a1 = native.absorbed(og, root, job["omega"], job["seed"], 1, threads=threads)
            a2 = native.absorbed(og, root, job["omega"], job["seed"], 2, want_y2=False, threads=threads)
            dt += time.perf_counter() - tt      # graph preparation untimed
            steps_c += int(w["y1"].sum() + a1["len"].sum() + a2["len"].sum())
            trees_c += job["omega"]
        res["cpu_baseline"] = {"value": steps_c / dt, "unit": "walk steps/s", "cores": threads, "kind": "oracle",
                               "sample": f"every 32nd job ({len(range(0, n_jobs, 32))} jobs, whole budgets), "
                                         f"{dt:.1f} s", "trees_per_s": trees_c / dt,
                               "est_total_s": steps / (steps_c / dt), "host_cpu": host_cpu()}
    b.close()
    return res


def _replay(lap, srv, qs, qid0):
    """Submit each query at its arrival time (seconds from start), drive the
    loop, return per-query results with latency (completion - submission)."""
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
    return out, wall


def _latency_summary(out):
    lat = np.array([r["t_done"] - r["t_submit"] for r in out])
    res = {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "errors": int(sum(r["status"] != 0 for r in out)), "by_kind": {}}
    for k, name in ((0, "closeness"), (1, "resistance"), (2, "kemeny")):
        lk = np.array([r["t_done"] - r["t_submit"] for r in out if r["kind"] == k])
        if len(lk):
            res["by_kind"][name] = {"queries": len(lk), "p50_ms": float(np.percentile(lk, 50) * 1e3),
                                    "p99_ms": float(np.percentile(lk, 99) * 1e3)}
    return res


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


def bench_serve(lap, gg, n_queries, with_cpu):
    """Serving (workloads.json "serving"): resident R-MAT scale-21 graph (edge factor 16, a/b/c/d =
    .57/.19/.19/.05, symmetrised, self-loops and duplicates dropped, largest
    component); Poisson arrivals mixing single-node closeness (64..1024 walks,
    log-uniform), pairwise resistance (1024 walk pairs) and Kemeny (256
    samples) in proportions 45/45/10.  Saturation throughput is measured with
    every query submitted at once; latency percentiles (overall and per query
    kind) at 50% and 80% of it, the 80% run repeated on the same server."""
    w = gg.workload("serving")
    n_queries = n_queries or w["queries"]
    g, n_graph, src, dst = workload_graph(lap, gg, "serving")
    if not with_cpu:
        del src, dst
    srv = lap.Server(g, seed=w["server_seed"], global_samples=w["global_samples"])
    mix = dict(mix=tuple(w["mix"]), ecc_budget=tuple(w["closeness_walks"]), res_pairs=w["resistance_pairs"],
               kemeny_samples=w["kemeny_samples"])
    qs = gg.query_stream(g.n, n_queries, qps=1.0, seed=w["saturation_stream_seed"], **mix)
    for q in qs:
        q["t"] = 0.0
    out_sat, wall = _replay(lap, srv, qs, 0)
    sat = n_queries / wall
    log(f"serve: saturation {sat:.1f} queries/s")
    n_serial = min(n_queries, 100)
    wall_serial, bad_serial = _serial(lap, srv, qs[:n_serial], 10_000_000)
    log(f"serve: one query at a time {n_serial / wall_serial:.1f} queries/s")
    res = {"workload": gg.describe_workload("serving") + ", resident; Poisson mix "
                       f"{w['mix'][0]:.0%} closeness ({w['closeness_walks'][0]}-{w['closeness_walks'][1]} walks), "
                       f"{w['mix'][1]:.0%} resistance ({w['resistance_pairs']} walk pairs), "
                       f"{w['mix'][2]:.0%} Kemeny ({w['kemeny_samples']} samples)",
           "n": g.n, "nnz": g.nnz, "queries": n_queries, "saturation_qps": sat,
           "closed_loop": _latency_summary(out_sat),
           "errors": int(sum(r["status"] != 0 for r in out_sat)) + int(bad_serial),
           "one_at_a_time_qps": n_serial / wall_serial,
           "speedup_served_vs_one_at_a_time": sat / (n_serial / wall_serial), "runs": []}
    for frac, stream_seed in zip(w["loads"], w["load_stream_seeds"]):
        k = len(res["runs"])
        qs = gg.query_stream(g.n, n_queries, qps=frac * sat, seed=stream_seed, **mix)
        out, wall = _replay(lap, srv, qs, (k + 1) * 1_000_000)
        r = {"offered_qps": frac * sat, "load": frac, "achieved_qps": n_queries / wall}
        r.update(_latency_summary(out))
        res["runs"].append(r)
        log(f"serve: {frac:.0%} load p50 {r['p50_ms']:.1f} ms p99 {r['p99_ms']:.1f} ms")
    p99s = [r["p99_ms"] for r in res["runs"] if r["load"] == 0.8]
    res["p99_80pct_spread"] = (max(p99s) - min(p99s)) / min(p99s)
    srv.close()
    if with_cpu:
        res["cpu_baseline"] = serve_cpu(gg, w, n_graph, src, dst, mix)
    g.close()
    return res


def serve_cpu(gg, w, n_graph, src, dst, mix, budget_s=12.0):
    """The oracle answering the query stream's first queries one after another
    (closeness and resistance walks on one thread, Kemeny samples on all
    cores), as a reference for the served latencies."""
    from oracle import csr as ocsr, native
    og = ocsr.build_csr(n_graph, src, dst, keep_lcc=w["keep_lcc"], degree_order=w["degree_order"])
    root = ocsr.landmark(og)
    threads = oracle_threads()
    sd = w["server_seed"]
    qs = gg.query_stream(og.n, 200, qps=1.0, seed=w["saturation_stream_seed"], **mix)
    lat = {0: [], 1: [], 2: []}
    t_all = time.perf_counter()
    for q in qs:
        t = time.perf_counter()
        if q["kind"] == 0:
            native.query_walks(og, root, sd, q["qid"], q["u"], 0, q["u"], q["u"], q["budget"])
        elif q["kind"] == 1:
            native.query_walks(og, root, sd, q["qid"], q["u"], 0, q["u"], q["w"], q["budget"])
            native.query_walks(og, root, sd, q["qid"], q["w"], 1, q["w"], q["u"], q["budget"])
        else:
            native.wilson(og, root, q["budget"], sd, qid=q["qid"], threads=threads)
            native.absorbed(og, root, q["budget"], sd, 2, qid=q["qid"], want_y2=False, threads=threads)
        lat[q["kind"]].append(time.perf_counter() - t)
        if time.perf_counter() - t_all > budget_s:
            break
    done = sum(len(v) for v in lat.values())
    wall = time.perf_counter() - t_all
    return {"kind": "oracle", "cores": threads, "queries": done, "qps": done / wall,
            "sample": f"first {done} queries of the stream, one after another, {wall:.1f} s",
            "mean_ms_by_kind": {name: float(np.mean(lat[k]) * 1e3) for k, name in
                                ((0, "closeness"), (1, "resistance"), (2, "kemeny")) if lat[k]},
            "host_cpu": host_cpu()}


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


def bench_kc_families(lap, gg, n, er_omega, loop_omega=256):
    """Kemeny's constant of synthetic families (the paper's Sec. 6 study on
    BA, ER and hyperbolic graphs): BA with m = 2..6; ER with average degree
    200..1000 (p = 2..10 x 1e-4 at 1e6 nodes); hyperbolic with gamma =
    2.2..3.0 and average degree 10 (largest component).  All 15 graphs in one
    batched launch: 256 samples each, er_omega for the ER graphs (their
    stationary-start walk lengths vary most).  Beside it, per graph, the same
    Kemeny estimate with the stationary-start lengths taken from the
    loop-included paths of the same Wilson samples (Sec. 3.4), loop_omega
    samples: the two terms are then strongly correlated and the standard
    error falls."""
    import torch
    t0 = time.perf_counter()
    jobs, labels = [], []
    for m in (2, 3, 4, 5, 6):
        s, d = gg.barabasi_albert(n, m, 100 + m)
        jobs.append(dict(n=n, src=s, dst=d, keep_lcc=True, root=-1, omega=256, seed=1))
        labels.append(f"BA m={m}")
    for k in (200, 400, 600, 800, 1000):
        s, d = gg.erdos_renyi(n, k / (n - 1), 200 + k)
        jobs.append(dict(n=n, src=s, dst=d, keep_lcc=True, root=-1, omega=er_omega, seed=1))
        labels.append(f"ER avg degree {k}")
    for gamma in (2.2, 2.4, 2.6, 2.8, 3.0):
        s, d = gg.hyperbolic(n, 10.0, gamma, 300 + int(round(gamma * 10)))
        jobs.append(dict(n=n, src=s, dst=d, keep_lcc=True, root=-1, omega=256, seed=1))
        labels.append(f"hyperbolic gamma={gamma}")
    log(f"kc families: {len(jobs)} graphs generated in {time.perf_counter() - t0:.1f} s "
        f"({sum(len(j['src']) for j in jobs) / 1e6:.0f} M edges)")
    b = lap.Batch(jobs)
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
        rows.append({"graph": lab, "n_lcc": int(b.info[j]["n"]), "omega": int(b.info[j]["omega"]),
                     "kemeny": float(r["kemeny"][0]), "kemeny_se": float(r["kemeny_se"][0]),
                     "kemeny_over_n": float(r["kemeny"][0]) / b.info[j]["n"],
                     "rel_se": float(r["kemeny_se"][0] / r["kemeny"][0])})
    st = b.stats()
    b.close()
    loop_s = 0.0
    for j, job in enumerate(jobs):
        g = lap.Graph(job["n"], job["src"], job["dst"], keep_lcc=True)
        tt = time.perf_counter()
        y1 = g.sample_forests(loop_omega, 1, -1, y1=False, per_sample=True)["y1"]
        ln = g.loop_included(loop_omega, 1, 2, -1)["len"]
        loop_s += time.perf_counter() - tt
        z = (y1 - ln).astype(np.float64)
        k, se = float(z.mean()), float(z.std(ddof=1) / math.sqrt(loop_omega))
        rows[j].update({"kemeny_loop": k, "kemeny_loop_se": se, "loop_rel_se": se / k, "loop_omega": loop_omega,
                        "corr_y1_len_loop": float(np.corrcoef(y1, ln)[0, 1])})
        g.close()
    return {"workload": f"15 synthetic graphs, n={n}, 256 samples each ({er_omega} for ER), one batched launch; "
                        f"loop-included estimate with {loop_omega} samples per graph",
            "s": dt, "prepare_s": gen_s, "walk_steps_per_s": (st["wilson_steps"] + st["absorbed_steps"]) / dt,
            "loop_estimate_s": loop_s, "graphs": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default="", help="comma-separated sections to run (default: all): " +
                                               ",".join(SECTIONS))
    ap.add_argument("--skip", default="", help="comma-separated sections to leave out")
    ap.add_argument("--batch-jobs", type=int, default=0, help="jobs of the batch (0: the workload's 512)")
    ap.add_argument("--kc-n", type=int, default=100_000)
    ap.add_argument("--kc-er-omega", type=int, default=16384)
    ap.add_argument("--serve-queries", type=int, default=0, help="queries per serving run (0: the workload's 2000)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of 1 GiB (counter calibration) and exit")
    ap.add_argument("--write-traffic", metavar="DIR",
                    help="only reduce the counter runs under DIR to a traffic summary and exit")
    ap.add_argument("--traffic-of", default="large", choices=sorted(TRAFFIC))
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args.write_traffic, args.traffic_of)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    only = set(filter(None, args.only.split(","))) or set(SECTIONS)
    only -= set(filter(None, args.skip.split(",")))
    unknown = only - set(SECTIONS)
    if unknown:
        raise SystemExit(f"unknown sections {sorted(unknown)}")
    with_cpu = not args.no_cpu_baseline

    import torch

    import graphgen as gg
    import paper_2311_10290_amd as lap

    torch.cuda.set_device(0)
    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")     # 1 GiB
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 8}), flush=True)
        return

    res = {"metric": "walk steps/s & spanning trees/s at 1 GPU, batched vs plain; p99 query latency",
           "unit": "walk steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int64 counts, f64 estimates",
           "data": "synthetic (seeded R-MAT, Erdos-Renyi, Barabasi-Albert and hyperbolic graphs; no dataset)"}
    gather = None
    if "gather" in only:
        log("random-gather sweep")
        gather = bench_gather(lap)
    if "large" in only:
        wl = gg.workload("large")
        g, n_large, src, dst = workload_graph(lap, gg, "large")
        omega, B, seed = wl["omega"], wl["blocks"], wl["philox_seed"]
        log(f"large: {args.warmup} warm-up + {args.steps} timed steps")
        dt, st, kern, wk, out = timed_steps(lap, g, omega, -1, args.steps, args.warmup, B=B, seed=seed)
        kms = kern[wk]["ms_avg"]
        traffic = measured_traffic("large")
        res.update({
            "value": (st["wilson_steps"] + st["absorbed_steps"]) * args.steps / dt,
            "ms_per_step": dt * 1e3 / args.steps,
            "config": {"workload": "plain LEWalk closeness + Kemeny: " + gg.describe_workload("large"),
                       "n": g.n, "nnz": g.nnz, "omega": omega, "wilson_kernel": TRAFFIC["large"]["kernel"]},
            "trees_per_s": omega * args.steps / dt,
            "wilson_steps_per_step": st["wilson_steps"], "absorbed_steps_per_step": st["absorbed_steps"],
            "wilson_steps_per_tree_over_n": st["wilson_steps"] / omega / g.n,
            "kernel_ms": {k: v["ms_avg"] for k, v in kern.items()},
            "roofline": roofline(st, g.n, kms, traffic, TRAFFIC["large"]["kernel"]),
            "requests": request_rate(traffic, kms, gather), "valu": valu_rate(traffic, kms),
            "estimates": {"kemeny": float(out["kemeny"].item()), "kemeny_se": float(out["kemeny_se"].item()),
                          "trace_Ldagger": float(out["trace"].item())},
        })
        log(f"large: {res['ms_per_step']:.2f} ms per step, {res['value'] / 1e9:.2f} G walk steps/s, "
            f"Wilson {kms:.2f} ms")
        root = g.max_deg_node
        # the same step with the walk counts from the loop-included paths of
        # the same Wilson samples (Sec. 3.4): after the trees, not beside them
        dtl, stl, kernl, _, outl = timed_steps(lap, g, omega, -1, 2, 1, B=B, walks=1, seed=seed)
        res["large_loop_included"] = {
            "s_per_step": dtl / 2, "kernel_ms": {k: v["ms_avg"] for k, v in kernl.items()},
            "path_steps_per_step": stl["absorbed_steps"],
            "kemeny": float(outl["kemeny"].item()), "kemeny_se": float(outl["kemeny_se"].item()),
            "trace_Ldagger": float(outl["trace"].item())}
        res["hot_vertex_share"] = hot_vertex_share(g, omega, seed=seed)
        g.close()
        if with_cpu:
            log("large: cpu baseline (oracle)")
            from oracle import csr as ocsr
            og = ocsr.build_csr(n_large, src, dst, keep_lcc=wl["keep_lcc"], degree_order=wl["degree_order"])
            res["cpu_baseline"] = cpu_baseline(og, root, omega, budget_s=15.0, probe=16, seed=seed)
            del og
        del src, dst
    if "small" in only:
        log("small workload")
        res["small"] = bench_small(lap, gg, args.steps, args.warmup, with_cpu, gather)
    mid = None
    if only & {"mid", "spantree", "loop_paths", "pairs"}:
        log("mid workload")
        r_mid, g_mid, root_mid = bench_mid(lap, gg, args.steps, args.warmup, with_cpu and "mid" in only, gather)
        if "mid" in only:
            res["mid"] = r_mid
        mid = (g_mid, root_mid)
    if "spantree" in only:
        log("spantree")
        res["spantree"] = bench_spantree(lap, mid[0], mid[1], 1024)
    if "loop_paths" in only:
        log("loop-included paths")
        res["loop_paths"] = bench_loop_paths(lap, mid[0], mid[1], 4096)
    if "pairs" in only:
        log("node-pair paths")
        res["pairs"] = bench_pairs(lap, mid[0], mid[1], mid[0].n)
    if mid:
        mid[0].close()
    if "landmark" in only:
        log("landmark study")
        res["landmark"] = bench_landmark(lap, gg)
    if "kc_families" in only:
        log("Kemeny's constant of synthetic families")
        res["kc_families"] = bench_kc_families(lap, gg, args.kc_n, args.kc_er_omega)
    if "batched" in only:
        res["batched"] = bench_batch(lap, gg, args.batch_jobs, with_cpu)
    if "serving" in only:
        res["serving"] = bench_serve(lap, gg, args.serve_queries, with_cpu)
    if gather:
        res["gather"] = gather
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
