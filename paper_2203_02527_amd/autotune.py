"""Autotuner for the launch parameters of the batched persistent kernel.

    python -m paper_2203_02527_amd.autotune [--clouds 2000] [--reps 3] [--out PATH]

The batched kernel (ph0_barcodes_batched_device) has two free parameters
that change speed but never results:

* chunk_mult[b] -- per cloud-size bucket b (n <= 64, <= 128, <= 256, <= 512),
  the first distance chunk a workgroup writes and sorts holds about
  chunk_mult * n edges.  Too small and clouds whose last pivot lies further
  out need extra chunks (another histogram-guided pass over all edges); too
  large and edges past the last pivot are written and sorted for nothing.
* blocks_per_cu -- workgroups launched per compute unit (1 or 2; a workgroup
  holds about 60 KB of LDS, so two fit the 160 KB of a CU).
* waves_per_cloud -- the size of the workgroup that runs one cloud: 8 or 16
  waves (512 or 1024 threads; the wider one keeps 16 digit histograms in
  LDS, 68 KB, so two still fit a CU).
* digit_bits -- the digit width of the chunk's LSD radix passes (5..8 bits:
  a wider digit means fewer passes, each ranking on more ballots; the
  per-wave digit histograms in LDS bound it at 8).

The search is coordinate-wise: for each bucket, one launch per candidate
multiplier over a seeded sample of that bucket's clouds (the batch
workload's generator restricted to the bucket's sizes), best of `reps`
timed launches; then blocks_per_cu, waves_per_cloud and digit_bits, one
after the other, over the mixed sample with the values chosen so far.
Every candidate's barcodes must equal the first candidate's (bit for bit);
a mismatch aborts the search.  The winners go to a JSON
table (default: tuning/batched.json beside this file), which
ph0.ph0_barcodes_batched_device loads when no tuning is passed.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(_PKG, "tuning", "batched.json")
BUCKETS = ((32, 64), (65, 128), (129, 256), (257, 512))
MULTS = (4, 6, 8, 12, 16, 24, 32, 48, 64)
BLOCKS_PER_CU = (1, 2)
WAVES_PER_CLOUD = (8, 16)
DIGIT_BITS = (5, 6, 7, 8)


def _time_launch(torch, ph0, x, offsets, tuning, reps):
    nbytes = ph0.ph0_batched_workspace_bytes(offsets, x.shape[1], x.dtype, tuning)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    out = torch.empty((x.shape[0], 2), dtype=torch.int32, device=x.device)
    ph0.ph0_barcodes_batched_device(x, offsets, out=out, workspace=ws, tuning=tuning)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        ph0.ph0_barcodes_batched_device(x, offsets, out=out, workspace=ws, tuning=tuning)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best, out.cpu().numpy()


def tune(clouds: int = 2000, reps: int = 3, seed: int = 12345, log=print) -> dict:
    """Run the search on cuda:0 and return the table (see module doc)."""
    import torch

    from . import ph0, synth

    mults = [24, 24, 24, 24]
    measured = {}
    for b, (lo, hi) in enumerate(BUCKETS):
        pts, offs = synth.batch_clouds(count=clouds, n_lo=lo, n_hi=hi, seed=seed + b)
        x = torch.from_numpy(pts).to("cuda:0")
        ref = None
        times = {}
        for m in MULTS:
            cand = list(mults)
            cand[b] = m
            t, bars = _time_launch(torch, ph0, x, offs, ph0.make_tuning(cand, 1), reps)
            if ref is None:
                ref = bars
            elif not np.array_equal(bars, ref):
                raise RuntimeError("bucket %d: chunk_mult %d changed the barcodes" % (b, m))
            times[m] = t
            log("bucket n in [%d,%d]: chunk_mult %3d  %.3f ms" % (lo, hi, m, 1e3 * t))
        mults[b] = min(times, key=times.get)
        measured["bucket_%d_%d" % (lo, hi)] = {str(m): round(1e3 * t, 4) for m, t in times.items()}
    pts, offs = synth.batch_clouds(count=clouds, seed=seed + 9)
    x = torch.from_numpy(pts).to("cuda:0")
    ref = [None]
    chosen = {"blocks_per_cu": 2, "waves_per_cloud": 8, "digit_bits": 8}

    def search(name, values):
        times = {}
        for v in values:
            cand = dict(chosen, **{name: v})
            t, bars = _time_launch(torch, ph0, x, offs, ph0.make_tuning(mults, **cand), reps)
            if ref[0] is None:
                ref[0] = bars
            elif not np.array_equal(bars, ref[0]):
                raise RuntimeError("%s %d changed the barcodes" % (name, v))
            times[v] = t
            log("mixed sample: %s %d  %.3f ms" % (name, v, 1e3 * t))
        chosen[name] = min(times, key=times.get)
        measured["mixed_" + name] = {str(k): round(1e3 * t, 4) for k, t in times.items()}

    search("blocks_per_cu", BLOCKS_PER_CU)
    search("waves_per_cloud", WAVES_PER_CLOUD)
    search("digit_bits", DIGIT_BITS)
    props = torch.cuda.get_device_properties(0)
    return {
        "device": getattr(props, "gcnArchName", props.name),
        "compute_units": props.multi_processor_count,
        "sample": "%d clouds per bucket from the batch generator (d=3 int16 circles or "
                  "2-4 blobs), seeds %d..%d; best of %d launches" % (clouds, seed, seed + 9, reps),
        "chunk_mult": mults,
        "blocks_per_cu": chosen["blocks_per_cu"],
        "waves_per_cloud": chosen["waves_per_cloud"],
        "digit_bits": chosen["digit_bits"],
        "launch_ms": measured,
    }


def load(path: str | None = None) -> dict | None:
    """The tuning table at `path` (default: the package's), or None if absent.
    Raises ValueError on a malformed table."""
    path = path or TABLE
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    cm = t.get("chunk_mult")
    bpc = t.get("blocks_per_cu")
    if (not isinstance(cm, list) or len(cm) != 4 or not all(isinstance(v, int) and v > 0 for v in cm)
            or bpc not in BLOCKS_PER_CU
            or t.get("waves_per_cloud", 8) not in WAVES_PER_CLOUD
            or t.get("digit_bits", 8) not in DIGIT_BITS):
        raise ValueError("malformed tuning table %s" % path)
    return t


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--clouds", type=int, default=2000)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=12345)
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args(argv)
    table = tune(args.clouds, args.reps, args.seed, log=lambda m: print(m, flush=True))
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
        f.write("\n")
    print("wrote %s: chunk_mult %s, blocks_per_cu %d, waves_per_cloud %d, digit_bits %d"
          % (args.out, table["chunk_mult"], table["blocks_per_cu"], table["waves_per_cloud"],
             table["digit_bits"]), flush=True)


if __name__ == "__main__":
    sys.exit(main())
