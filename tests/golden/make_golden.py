"""Write oracle_<workload>_s<seed>.json: expected values at full workload size.

Calls only the CPU oracle (oracle/) on the seeded generators; no value here
comes from the GPU library.  Run from the repository root:

    python tests/golden/make_golden.py [--seeds A-B] [workload ...]
    python tests/golden/make_golden.py --h1 N SEED     (H1 of the uniform N-point cloud)

Seeds 0-9 of every workload are stored (the parity seeds); --seeds limits
the run to a range.
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2203_02527_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def record(name: str, seed: int) -> dict:
    pts = synth.workload(name, seed=seed)
    res = oracle.barcode(pts, early_exit=True)
    return {
        "workload": name,
        "seed": seed,
        "n": int(pts.shape[0]),
        "d": int(pts.shape[1]),
        "points_sha256": digest(pts),
        "E": res.E,
        "E_eff": res.E_eff,
        "additions": res.additions,
        "pivots": res.pivots,
        "canonical_sha256": digest(res.canonical.astype("<u4")),
        "death_by_vertex_sha256": digest(res.death_by_vertex.astype("<u4")),
        "killer_pos_sha256": digest(res.killer_pos.astype("<i8")),
        "partner_sha256": digest(res.partner.astype("<i4")),
        "max_finite_death": int(res.canonical[-2]) if res.canonical.size > 1 else None,
        "oracle_seconds": res.seconds,
    }


def record_h1(n: int, seed: int) -> dict:
    """H1 of the uniform integer cloud (the H1 benchmark recipe), literal
    mode (every column reduced, as the GPU does)."""
    pts = synth.uniform_cloud(n, 3, seed=seed)
    res = oracle.h1_barcode(pts, early_exit=False)
    return {
        "workload": "h1_uniform_n%d_d3_i16" % n,
        "seed": seed,
        "n": n,
        "points_sha256": digest(pts),
        "E": res.E,
        "T": res.T,
        "pivots": res.pivots,
        "additions": res.additions,
        "zero_length": res.zero_length,
        "bars": int(res.bars.shape[0]),
        "bars_sha256": digest(res.bars.astype("<u4")),
        "tri_of_edge_sha256": digest(res.tri_of_edge.astype("<i8")),
    }


def main(names, seeds):
    for name in names:
        for seed in seeds:
            rec = record(name, seed)
            with open(os.path.join(HERE, "oracle_%s_s%d.json" % (name, seed)), "w") as f:
                json.dump(rec, f, indent=1, sort_keys=True)
                f.write("\n")
            print(name, seed, rec["E_eff"], rec["additions"], flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--h1":  # python tests/golden/make_golden.py --h1 N SEED
        n, seed = int(args[1]), int(args[2])
        rec = record_h1(n, seed)
        with open(os.path.join(HERE, "oracle_h1_uniform_n%d_d3_i16_s%d.json" % (n, seed)), "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
            f.write("\n")
        print(rec["workload"], seed, rec["pivots"], rec["additions"], flush=True)
        sys.exit(0)
    seeds = range(10)
    if args and args[0] == "--seeds":
        lo, hi = args[1].split("-")
        seeds = range(int(lo), int(hi) + 1)
        args = args[2:]
    main(args or list(synth.WORKLOADS), seeds)
