"""Benchmark of the H0 barcode hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one whole barcode -- distances, LSD radix sort, grades, F2 column
reduction, read-off -- of the N=16384, d=64 int8 Gaussian-mixture cloud (32
clusters, std 12, seed 0), from points already resident in HBM to the
canonical barcode in HBM, through ph0_barcodes_device.  The K timed steps
run without statistics; the same number of steps with the library's HIP
events then gives the stage and kernel times (the rooflines).  First-call
latency (module load, workspace allocation), the host<->HBM copies and the
host-memory entry point are reported separately, never as the headline.

value = E_eff / step time: sorted edge columns up to the last pivot, i.e. the
columns the reduction actually processes (the remaining E - E_eff columns are
zero by the early-exit argument and cost nothing), per second of the whole
step.  One JSON line is printed; beside the headline figures it carries the
batched launch over 10,000 small clouds, the serving stream, the H1 barcode
of a 256-point cloud, and the single-threaded CPU oracle.

Other modes: --paper-scaling (the paper's unit-square run-time experiment),
--cpu-openmp (the paper's multi-core CPU scheme), --calibrate-copy (a copy
of known size for the hardware byte counters).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "mixture_n16384_d64_i8"
HBM_PEAK_GBS = 8000.0
RECOMPUTE_MIN_E = 1 << 22  # edges from which the library recomputes keys per distance range


def note(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--window", type=int, default=0, help="reduction window (0 = built-in)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-h1", action="store_true")
    ap.add_argument("--h1-only", action="store_true",
                    help="only run the H1 leg (no CPU oracle) and print its JSON")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the batched leg (10,000 clouds, with its roofline) and print "
                         "its JSON")
    ap.add_argument("--batched-launches", type=int, default=0, metavar="K",
                    help="only make K batched launches of the 10,000-cloud workload (after one "
                         "untimed), nothing else: the command profiled for the batched kernel")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--paper-scaling", action="store_true",
                    help="only run the paper's experiment: N uniform points in [0,1]^2 (on a "
                         "fixed-point grid), N = 50..700 and beyond, GPU and CPU-oracle time "
                         "per barcode with fitted run-time exponents, and the paper's OpenMP "
                         "CPU scheme at 1..all host threads, and exit")
    ap.add_argument("--cpu-openmp", action="store_true",
                    help="only run the paper's OpenMP CPU scheme on the unit-square clouds at "
                         "1..all host threads (no GPU needed), and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 5 times (a reference kernel of "
                         "known traffic for hardware byte counters) and exit")
    return ap.parse_args()


SCALING_N = (50, 100, 150, 200, 300, 400, 500, 600, 700, 1000, 2000, 4096, 8192, 16384)
OMP_N = (50, 100, 150, 200, 300, 400, 500, 600, 700, 1000, 2000)
OMP_REPS = 5


def paper_scaling(reps=10, seed=0):
    """The paper's run-time experiment on this GPU: N uniform random points in
    [0,1]^2, the mean of `reps` whole barcodes per N (points resident in HBM),
    beside the single-threaded CPU oracle for N <= 2000, and the slopes of
    log(time) against log(N) over the ranges the paper fits."""
    import numpy as np
    import torch

    import oracle
    from paper_2203_02527_amd import ph0, synth

    rows = []
    for n in SCALING_N:
        x = synth.unit_square_cloud(n, seed=seed + n)
        xd = torch.from_numpy(x).to("cuda:0")
        ws = ph0.alloc_workspace(n, 2, x.dtype, "cuda:0")
        out = torch.empty((n, 2), dtype=torch.int32, device="cuda:0")
        for _ in range(2):
            ph0.ph0_barcodes_device(xd, out=out, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ph0.ph0_barcodes_device(xd, out=out, workspace=ws)
        torch.cuda.synchronize()
        gpu_ms = 1000.0 * (time.perf_counter() - t0) / reps
        got = out.cpu().numpy().view(np.uint32)[:, 1]
        row = {"n": n, "gpu_ms": round(gpu_ms, 4)}
        if n <= 2000:
            creps = 3 if n > 700 else reps
            t0 = time.perf_counter()
            for _ in range(creps):
                ref = oracle.barcode(x)
            row["cpu_oracle_ms"] = round(1000.0 * (time.perf_counter() - t0) / creps, 3)
            row["matches_oracle"] = bool(np.array_equal(got, ref.canonical))
        rows.append(row)
        note("scaling N=%d: %s" % (n, row))

    def slope(key, lo, hi):
        pts = [(r["n"], r[key]) for r in rows if lo <= r["n"] <= hi and key in r]
        if len(pts) < 2:
            return None
        lx = np.log([p[0] for p in pts])
        ly = np.log([p[1] for p in pts])
        return round(float(np.polyfit(lx, ly, 1)[0]), 3)

    omp = omp_sweep(seed)
    omp_rows = omp["points"]
    for r in rows:
        for o in omp_rows:
            if o["n"] == r["n"]:
                r["cpu_omp_best_ms"] = min(v for k, v in o.items() if k.endswith("_ms"))

    exps = {}
    for key in ("gpu_ms", "cpu_oracle_ms"):
        for lo, hi in ((50, 150), (200, 700), (1000, 16384)):
            v = slope(key, lo, hi)
            if v is not None:
                exps["%s_N%d_%d" % (key.replace("_ms", ""), lo, hi)] = v
    return {"mode": "paper_scaling",
            "workload": "N uniform points in [0,1]^2 on the grid rint(u * %d) (int16), seed "
                        "%d + N; mean of %d barcodes per N from HBM-resident points"
                        % (synth.UNIT_SCALE, seed, reps),
            "points": rows, "exponents": exps,
            "cpu_openmp": omp}


def omp_sweep(seed=0):
    """The paper's multi-core CPU scheme (Section 3) on the same unit-square
    clouds, at the thread counts of its two CPU figures (1, 2; 3, 4, 6) and
    at all host cores; each run's barcode is checked against the oracle."""
    import numpy as np

    import oracle
    from paper_2203_02527_amd import synth

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = sorted({t for t in (1, 2, 3, 4, 6, cores) if t <= max(cores, 1)})
    omp_rows = []
    for n in OMP_N:
        x = synth.unit_square_cloud(n, seed=seed + n)
        ref = oracle.barcode(x)
        row = {"n": n}
        for t in threads:
            oracle.omp_barcode(x, t)
            t0 = time.perf_counter()
            for _ in range(OMP_REPS):
                got = oracle.omp_barcode(x, t)
            row["t%d_ms" % t] = round(1000.0 * (time.perf_counter() - t0) / OMP_REPS, 3)
            if not np.array_equal(got.canonical, ref.canonical):
                raise RuntimeError("OpenMP baseline differs from the oracle at N=%d" % n)
        if "t2_ms" in row:
            row["speedup_2_vs_1"] = round(row["t1_ms"] / row["t2_ms"], 3)
        omp_rows.append(row)
        note("openmp N=%d: %s" % (n, row))
    return {"scheme": "Section 3: OpenMP loops inside the sequential column loop (parallel "
                      "distances; each column addition with its low search is one parallel "
                      "region); stop at the (N-1)-th pivot",
            "host_cores": cores, "threads": threads, "reps": OMP_REPS, "points": omp_rows}


def calibrate_copy(mib):
    """Five device-to-device copies of mib MiB: each reads and writes exactly
    mib MiB, which scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": mib << 20, "copies": 5}), flush=True)


def host_cpu():
    """Model name and logical CPU count of this host (from /proc/cpuinfo), and
    the CPUs this process may run on."""
    model, logical = "unknown", 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model == "unknown":
                    model = line.split(":", 1)[1].strip()
                if line.startswith("processor"):
                    logical += 1
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "logical_cpus": logical or os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(points, n_sample):
    """The CPU oracle (single-threaded, the same source built with -O3
    -march=native for this host) on the first n_sample points."""
    import tempfile

    import oracle

    lib = oracle.build_native(tempfile.mkdtemp(prefix="ph0_native_"))
    sub = points[:n_sample].copy()
    t0 = time.perf_counter()
    res = oracle.barcode(sub, lib=lib)
    t = time.perf_counter() - t0
    return {
        "value": res.E_eff / t,
        "unit": "edge columns/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "%s (N=%d, E=%d, E_eff=%d), one whole oracle run (distances, std::sort, "
                  "grades, dense F2 reduction with early exit, read-off), g++ -O3 -march=native, "
                  "one thread, in %.2f s"
                  % ("the whole benchmark cloud" if n_sample >= len(points) else
                     "the first %d points of the benchmark cloud" % n_sample,
                     n_sample, res.E, res.E_eff, t),
        "seconds": res.seconds,
        "host": host_cpu(),
    }


def bench_batched(torch, ph0, synth, reps=3):
    """10,000 uneven clouds: one persistent launch vs one cloud per call."""
    import numpy as np

    pts, offsets = synth.batch_clouds(count=10000, seed=0)
    x = torch.from_numpy(pts).to("cuda:0")
    out = torch.empty((pts.shape[0], 2), dtype=torch.int32, device="cuda:0")
    nbytes = ph0.ph0_batched_workspace_bytes(offsets, 3, pts.dtype)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    ph0.ph0_barcodes_batched_device(x, offsets, out=out, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ph0.ph0_barcodes_batched_device(x, offsets, out=out, workspace=ws)
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / reps
    # plain path: the first 500 clouds, one ph0_barcodes_device call each
    k = 500
    pws = ph0.alloc_workspace(512, 3, pts.dtype, "cuda:0")
    pout = torch.empty((512, 2), dtype=torch.int32, device="cuda:0")
    for c in range(5):
        ph0.ph0_barcodes_device(x[offsets[c]:offsets[c + 1]], out=pout[: offsets[c + 1] - offsets[c]],
                                workspace=pws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(k):
        n = int(offsets[c + 1] - offsets[c])
        ph0.ph0_barcodes_device(x[offsets[c]:offsets[c + 1]], out=pout[:n], workspace=pws)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / k
    table = ph0.default_tuning()
    roof = batched_roofline(torch, ph0, x, offsets, pts, out, ws, reps)
    return {
        "workload": "10000 clouds, N uniform in [32,512], d=3 int16, circles or 2-4 blobs, seed 0",
        "roofline": roof,
        "tuning": ("autotuned table: chunk_mult %s, blocks_per_cu %d"
                   % (list(table.chunk_mult), table.blocks_per_cu)) if table else "built-in",
        "clouds_per_s": 10000 / t_batched,
        "ms_per_launch": round(1000 * t_batched, 3),
        "plain_clouds_per_s": 1.0 / t_plain,
        "plain_sample": "first %d clouds, one ph0_barcodes_device call each" % k,
        "speedup_vs_plain": (10000 / t_batched) * t_plain,
        "edges_total": int(np.sum(np.diff(offsets) * (np.diff(offsets) - 1) // 2)),
    }


def batched_roofline(torch, ph0, x, offsets, pts, out, ws, reps):
    """Roofline of the batched launch on the method's own bytes: every cloud
    sorts at least its keys up to its last pivot (E_eff of them, from the
    single-cloud path's statistics), 8 B written and P passes of 8 B read +
    8 B written each, P = ceil(b / 8) for the b distance bits of the cloud's
    coordinate ranges (as the kernel sorts).  The launch is timed with events
    on the stream it runs on."""
    import numpy as np

    alg = 0
    e_eff = 0
    pws = ph0.alloc_workspace(512, 3, pts.dtype, "cuda:0")
    pout = torch.empty((512, 2), dtype=torch.int32, device="cuda:0")
    for c in range(len(offsets) - 1):
        lo, hi = int(offsets[c]), int(offsets[c + 1])
        _, st = ph0.ph0_barcodes_device(x[lo:hi], out=pout[: hi - lo], workspace=pws,
                                        with_stats=True)
        span = pts[lo:hi].astype(np.int64)
        bound = int(((span.max(0) - span.min(0)) ** 2).sum())
        passes = (max(bound, 1).bit_length() + 7) // 8
        alg += 8 * st["E_eff"] * (1 + 2 * passes)
        e_eff += st["E_eff"]
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        ev0.record(stream)
        ph0.ph0_barcodes_batched_device(x, offsets, out=out, workspace=ws)
        ev1.record(stream)
        ev1.synchronize()
        best = min(best, ev0.elapsed_time(ev1) / 1e3)
    achieved = alg / best / 1e9
    traffic = measured_traffic("batched", "batch10000_d3_i16")
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": 8000.0, "unit": "GB/s",
            "frac": round(achieved / 8000.0, 5), "traffic": traffic,
            "basis": "8 B x E_eff x (1 + 2P) per cloud over the whole launch (best of %d, "
                     "events on its stream); sum E_eff = %d" % (reps, e_eff),
            "algorithmic_bytes": int(alg), "launch_s": round(best, 6)}
    if traffic is not None:
        roof["traffic_gbs"] = round(traffic / best / 1e9, 1)
    return roof


H1_N = 256
H1_CPU_N = 128


def bench_h1(torch, ph0, synth, with_cpu, reps=5):
    """H1 (edge-by-triangle boundary matrix) of the uniform N=256, d=3 int16
    cloud: whole calls from HBM-resident points, the oracle beside it on a
    128-point cloud of the same recipe, and the dense-column rate: each
    column addition of the dense method moves one E-bit column (the kernel
    reads only the part of it at or below the stored column's low; the stored
    columns stay in the last-level cache, so the rate is not an HBM one)."""
    x = synth.uniform_cloud(H1_N, 3, seed=0)
    xd = torch.from_numpy(x).to("cuda:0")
    ws = torch.empty(ph0.ph0_h1_workspace_bytes(H1_N, 3, x.dtype), dtype=torch.uint8,
                     device="cuda:0")
    ph0.ph0_h1_device(xd, workspace=ws)
    torch.cuda.synchronize()
    sts = []
    t0 = time.perf_counter()
    for _ in range(reps):
        _, _, st = ph0.ph0_h1_device(xd, workspace=ws, with_stats=True)
        sts.append(st)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    st = sts[-1]
    E = H1_N * (H1_N - 1) // 2
    dense_bytes = 8.0 * ((E + 63) // 64) * st["additions"]
    rec = {
        "workload": "uniform_n256_d3_i16 (integers in [-100, 100]^3, seed 0)",
        "ms_per_call": round(1000 * t, 3),
        "triangles": st["T"],
        "triangles_per_s": st["T"] / t,
        "additions_per_s": st["additions"] / t,
        "pairs": st["pivots"], "emergent": st["emergent"], "bars": st["bars"],
        "rounds": st["rounds"], "walks": st["walks"],
        # E-bit stored columns: 2.1 MB per column at N=256 x E/64 words; the
        # table of E columns (0.13 GB) lives in the 256 MB last-level cache,
        # so this is a rate through the cache hierarchy, not an HBM fraction.
        "dense_column_gbs_cached": round(dense_bytes / t / 1e9, 1),
    }
    if with_cpu:
        import oracle

        xs = synth.uniform_cloud(H1_CPU_N, 3, seed=0)
        t0 = time.perf_counter()
        ref = oracle.h1_barcode(xs)
        tc = time.perf_counter() - t0
        got, _ = ph0.ph0_h1_device(torch.from_numpy(xs).to("cuda:0"))
        torch.cuda.synchronize()
        import numpy as np

        rec["cpu_oracle"] = {
            "sample": "uniform N=%d, d=3 int16, seed 0: %d triangles" % (H1_CPU_N, ref.T),
            "seconds": round(tc, 3), "cores": 1,
            "triangles_per_s": ref.T / tc,
            "gpu_matches": bool(np.array_equal(got.cpu().numpy().view(np.uint32), ref.bars)),
        }
    return rec


SERVE_LOADS = (0.5, 0.8, 0.95)


def bench_serving(ph0, synth, count, warm=200):
    """Mixed request stream: `warm` warm-up requests, then `count` requests
    closed-loop (the saturation rate), then the same `count` requests with
    Poisson arrivals at 0.5, 0.8 and 0.95 x saturation; the same requests one
    at a time through the single-cloud path beside them."""
    from paper_2203_02527_amd import serve

    reqs = synth.serving_requests(warm + count, seed=0)
    warmup, reqs = reqs[:warm], reqs[warm:]
    serve.serve(warmup, rate=None, mem_budget=8 << 30, slots=4)
    sat = serve.serve(reqs, rate=None, mem_budget=8 << 30, slots=4)
    points = []
    for load in SERVE_LOADS:
        rate = load * sat["clouds_per_s"]
        r = serve.serve(reqs, rate=rate, mem_budget=8 << 30, slots=4, seed=1)
        points.append({"load": load, "rate": round(rate, 1),
                       "clouds_per_s": round(r["clouds_per_s"], 1),
                       "p50_ms": round(r["p50_ms"], 3), "p99_ms": round(r["p99_ms"], 3)})
        note("serving at %.2f x saturation: p50 %.2f ms p99 %.2f ms"
             % (load, r["p50_ms"], r["p99_ms"]))
    pl = serve.plain(reqs)
    pl.pop("results")
    return {
        "workload": "%d requests after %d warm-up, N log-uniform in [64,8192], d in {3,16,64}, "
                    "int8/int16 mixtures, seed 0; 4 slots, 8 GiB pool" % (count, warm),
        "saturation_clouds_per_s": round(sat["clouds_per_s"], 1),
        "poisson": points,
        "plain_clouds_per_s": round(pl["clouds_per_s"], 1),
        "plain_p50_ms": round(pl["p50_ms"], 3),
        "plain_p99_ms": round(pl["p99_ms"], 3),
    }


KERNEL_SOURCES = {"reduce_walk": "reduce.hip", "radix_pass": "radix.hip",
                  "batched": "batched.hip"}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    profiles/traffic_<kernel>_<workload>.txt (FETCH_SIZE and WRITE_SIZE per
    dispatch, each scaled by what the counter reads for a copy of known
    size), or None when there is no summary or the kernel's source has
    changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.txt" % (kernel, workload))
    src = os.path.join(ROOT, "paper_2203_02527_amd", "csrc", KERNEL_SOURCES[kernel])
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != fields.get("source_sha256"):
            return None
    try:
        return int(float(fields["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def sort_bytes(st):
    """Algorithmic bytes of one call's radix passes: a pass reads each of its
    input keys once and writes each output key once (8 bytes each).  Above
    2^22 edges the keys of a distance range are recomputed and written only
    for that range (sorted_keys of them), so every pass moves 16 bytes per
    sorted key.  Below it all E keys are stored: a distance range's first
    pass reads all E keys and keeps the range's, its later passes move the
    range's keys; a sort that ends whole moves all E keys in every pass."""
    E, P, k, c = st["E"], st["sort_passes"], st["sorted_keys"], st["sort_chunks"]
    if P == 0:
        return 0.0
    if E >= RECOMPUTE_MIN_E:
        return 16.0 * k * P
    if k < E:
        return 8.0 * E * c + 8.0 * k + 16.0 * (P - 1) * k
    return 8.0 * E * (c - 1) + 16.0 * E * P


def walk_bytes(st):
    """Algorithmic bytes of one call's reduction walks, counted for the
    2-sparse representation the kernel uses: a column addition reads one
    4-byte table entry (additions of the sequential count), each column up
    to the last pivot reads its 8-byte sorted key, and each of the n - 1
    pivots writes one 4-byte table entry."""
    return 4.0 * st["additions"] + 8.0 * st["E_eff"] + 4.0 * (st["n"] - 1)


def dense_walk_bytes(st):
    """The same reduction counted for the dense method of the survey's
    per-unit figure: one N-bit column (8 * ceil(N/64) bytes) per addition."""
    return 8.0 * ((st["n"] + 63) // 64) * st["additions"] + 8.0 * st["E_eff"]


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU; this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.cpu_openmp:
        print(json.dumps({"mode": "cpu_openmp", **omp_sweep(args.seed)}), flush=True)
        return
    if args.paper_scaling:
        print(json.dumps(paper_scaling()), flush=True)
        return
    import numpy as np
    import torch

    from paper_2203_02527_amd import ph0, synth

    if not os.path.exists(ph0.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    if args.window:
        ph0.ph0_set_window(args.window)
    if args.h1_only:
        print(json.dumps({"mode": "h1", **bench_h1(torch, ph0, synth, False,
                                                  reps=max(args.steps, 1))}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"mode": "batched", **bench_batched(torch, ph0, synth)}), flush=True)
        return
    if args.batched_launches:
        bpts, boffs = synth.batch_clouds(count=10000, seed=0)
        bx = torch.from_numpy(bpts).to("cuda:0")
        bout = torch.empty((bpts.shape[0], 2), dtype=torch.int32, device="cuda:0")
        bws = torch.empty(ph0.ph0_batched_workspace_bytes(boffs, 3, bpts.dtype),
                          dtype=torch.uint8, device="cuda:0")
        for _ in range(args.batched_launches + 1):
            ph0.ph0_barcodes_batched_device(bx, boffs, out=bout, workspace=bws)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "batched-launches", "launches": args.batched_launches + 1}),
              flush=True)
        return
    pts = synth.workload(args.workload, seed=args.seed)
    n, d = pts.shape
    dev = torch.device("cuda:0")
    torch.zeros(1, device=dev)
    torch.cuda.synchronize()
    # Host -> HBM copy of the points; first call (kernel module load, workspace
    # allocation, first launch); HBM -> host copy of the barcode.
    t0 = time.perf_counter()
    x = torch.from_numpy(pts).to(dev)
    torch.cuda.synchronize()
    h2d_ms = 1000.0 * (time.perf_counter() - t0)
    t0 = time.perf_counter()
    ws = ph0.alloc_workspace(n, d, pts.dtype, dev)
    out = torch.empty((n, 2), dtype=torch.int32, device=dev)
    ph0.ph0_barcodes_device(x, out=out, workspace=ws)
    torch.cuda.synchronize()
    first_call_ms = 1000.0 * (time.perf_counter() - t0)
    t0 = time.perf_counter()
    bars_host = out.cpu()
    d2h_ms = 1000.0 * (time.perf_counter() - t0)
    del bars_host
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        ph0.ph0_barcodes_device(x, out=out, workspace=ws, stream=stream)
    torch.cuda.synchronize()

    # The timed steps: whole barcodes from HBM-resident points, no statistics
    # (each call returns when its work is complete, so per-step wall times
    # are exact too).
    step_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t1 = time.perf_counter()
        ph0.ph0_barcodes_device(x, out=out, workspace=ws, stream=stream)
        step_ms.append(1000.0 * (time.perf_counter() - t1))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ms_step = 1000.0 * t / args.steps

    # The same number of steps again with the library's HIP events (stage
    # marks and one pair around every walk and radix launch, on the call's
    # stream): stage and kernel times come from these.
    stats = []
    for _ in range(args.steps):
        _, st = ph0.ph0_barcodes_device(x, out=out, workspace=ws, stream=stream, with_stats=True)
        stats.append(st)
    torch.cuda.synchronize()
    for st in stats:
        st["radix_bytes"] = sort_bytes(st)
        st["walk_bytes"] = walk_bytes(st)
        st["dense_walk_bytes"] = dense_walk_bytes(st)
    st0 = stats[-1]
    E, E_eff = st0["E"], st0["E_eff"]

    def mean(k):
        return float(np.mean([s[k] for s in stats]))

    # Kernel rooflines from the event timings.  Walk: the bytes of the
    # 2-sparse reduction (walk_bytes); the dense method's figure is given
    # beside it.  Radix: 16 bytes per key per pass (sort_bytes).
    walk_ms = mean("ms_walk_kernel")
    walk_launches = mean("walk_launches")
    radix_ms = mean("ms_radix_kernel")
    radix_launches = mean("radix_launches")
    kern = {
        "reduce_walk": dict(ms=walk_ms, launches=walk_launches, bytes=mean("walk_bytes")),
        "radix_pass": dict(ms=radix_ms, launches=radix_launches, bytes=mean("radix_bytes")),
    }
    for k in kern.values():
        k["per_launch_ms"] = k["ms"] / max(k["launches"], 1)
        k["achieved_gbs"] = k["bytes"] / max(k["ms"], 1e-9) / 1e6
    dom = max(kern, key=lambda k: kern[k]["ms"])
    kd = kern[dom]
    per_launch = kd["bytes"] / max(kd["launches"], 1)
    traffic = measured_traffic(dom, args.workload)
    roofline = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": round(kd["achieved_gbs"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(kd["achieved_gbs"] / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "avg_launch_ms": round(kd["per_launch_ms"], 4),
        "algorithmic_bytes_per_launch": round(per_launch),
    }
    if dom == "reduce_walk":
        roofline["basis"] = ("bytes of the 2-sparse reduction: 4 B table entry per column "
                             "addition of the sequential count + 8 B sorted key per column up "
                             "to the last pivot + 4 B per pivot written; the walk is bound by "
                             "chains of dependent table loads and by row-minimum atomics, not "
                             "by HBM bandwidth")
        roofline["dense_equivalent_gbs"] = round(mean("dense_walk_bytes") / max(walk_ms, 1e-9)
                                                 / 1e6, 1)
    else:
        roofline["basis"] = "16 B per sorted key per radix pass (read once, written once)"
    if traffic is not None:
        roofline["traffic_gbs"] = round(traffic / (kd["per_launch_ms"] * 1e6), 1)
    others = {k: {"achieved_gbs": round(v["achieved_gbs"], 1), "frac": round(
        v["achieved_gbs"] / HBM_PEAK_GBS, 4), "ms_per_step": round(v["ms"], 3),
        "launches": v["launches"]} for k, v in kern.items()}

    rec = {
        "metric": "edge columns reduced/s at N=16384",
        "value": E_eff / (ms_step / 1000.0),
        "unit": "edge columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_median": round(float(np.median(step_ms)), 4),
        "ms_per_step_min": round(float(np.min(step_ms)), 4),
        "ms_per_step_max": round(float(np.max(step_ms)), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "n": int(n), "d": int(d), "seed": args.seed,
            "E": int(E), "E_eff": int(E_eff),
            "edges_per_s_all_E": E / (ms_step / 1000.0),
            "window": st0["window"],
        },
        "first_call_ms": round(first_call_ms, 3),
        "h2d_points_ms": round(h2d_ms, 3),
        "d2h_bars_ms": round(d2h_ms, 3),
        "stages_ms": {k: round(mean(k), 4) for k in
                      ("ms_keys", "ms_sort", "ms_reduce", "ms_rank", "ms_emit", "ms_total")},
        "reduction": {k: st0[k] for k in ("additions", "additions_all", "find_steps",
                                          "words_read", "rounds", "distinct_eff",
                                          "sort_passes", "sort_chunks", "sorted_keys",
                                          "delta_bits", "keys_path")},
        "roofline": roofline,
        "kernels": others,
        "rates": {
            # E_eff over the reduce stage alone (ranks + reduction + read-off)
            "edge_columns_per_s_reduce_stage": E_eff / ((mean("ms_rank") + mean("ms_reduce")
                                                          + mean("ms_emit")) / 1000.0),
            "additions_per_s": mean("additions") / (ms_step / 1000.0),
            "all_edges_per_s": E / (ms_step / 1000.0),
        },
    }
    # The host-memory entry point (copies in, barcode, copies out, and its own
    # device allocations) for the PCIe-inclusive rate; never the headline.
    ph0.ph0_barcodes(pts)
    t0 = time.perf_counter()
    for _ in range(3):
        ph0.ph0_barcodes(pts)
    host_ms = 1000.0 * (time.perf_counter() - t0) / 3
    rec["host_entry_point"] = {"ms_per_call": round(host_ms, 3),
                               "edge_columns_per_s": E_eff / (host_ms / 1000.0)}
    note("timed %d steps: %.3f ms/step" % (args.steps, ms_step))
    if not args.no_batched:
        rec["batched"] = bench_batched(torch, ph0, synth)
        note("batched done")
    if not args.no_serving:
        rec["serving"] = bench_serving(ph0, synth, args.serve_requests)
        note("serving done")
    if not args.no_h1:
        rec["h1"] = bench_h1(torch, ph0, synth, not args.no_cpu_baseline)
        note("h1 done")
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(pts, n)
        note("cpu baseline done")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
