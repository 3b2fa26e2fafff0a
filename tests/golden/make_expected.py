"""Write tests/golden/expected_counts.json from the CPU oracle.

Every value in that file comes from ``oracle`` run on inputs from
``graphgen``; nothing is taken from the device path.  Re-run after any change
to the generators or to the oracle's arithmetic:

    python tests/golden/make_expected.py [--large] [--huge]

Stored per workload: the total, the cleaned edge count m, W+ (the total
number of 2-hop probes), the largest out-degree, a checksum of the whole
per-vertex array and the exact per-vertex counts of a seeded sample of
vertices (plus the 32 vertices with the largest counts).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen.workloads as W  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "expected_counts.json")
MUL = np.uint64(0x9E3779B97F4A7C15)


def checksum(per_vertex: np.ndarray) -> int:
    """sum_x t(x) * (x * 0x9E3779B97F4A7C15 + 1) mod 2^64."""
    x = np.arange(per_vertex.shape[0], dtype=np.uint64)
    with np.errstate(over="ignore"):
        w = x * MUL + np.uint64(1)
        return int(np.sum(per_vertex.astype(np.uint64) * w, dtype=np.uint64))


def record(g, sample=512, seed=1):
    t = time.time()
    r = oracle.count(g.n, g.src, g.dst, per_vertex=True)
    rng = np.random.default_rng(seed)
    q = np.unique(np.concatenate([rng.integers(0, g.n, sample), np.argsort(r.per_vertex)[-32:]]))
    return {
        "n": g.n, "m_in": g.m_in, "total": r.total, "m": r.m, "wedges_plus": r.wedges_plus,
        "max_dplus": r.max_dplus, "per_vertex_checksum": checksum(r.per_vertex),
        "sample_ids": q.astype(int).tolist(), "sample_counts": r.per_vertex[q].astype(int).tolist(),
        "oracle_seconds": round(time.time() - t, 2),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--large", action="store_true", help="also the R-MAT scale 22 workload")
    ap.add_argument("--huge", action="store_true",
                    help="also the single large instances: R-MAT scale 26 and Erdos-Renyi n = 2^25")
    ap.add_argument("--keep", action="store_true", help="keep large-instance values already stored")
    args = ap.parse_args()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data["rmat16"] = record(W.small_rmat())
    if args.large:
        data["rmat22"] = record(W.large_rmat())
    if args.huge:
        for name, fn in (("er25", W.uniform_er), ("rmat26", W.huge_rmat)):
            if args.keep and name in data:
                continue
            data[name] = record(fn())
            json.dump(data, open(OUT, "w"), indent=1)
            print(name, data[name]["total"], data[name]["oracle_seconds"], flush=True)
    json.dump(data, open(OUT, "w"), indent=1)
    print({k: (v["total"], v["oracle_seconds"]) for k, v in data.items()})


if __name__ == "__main__":
    main()
