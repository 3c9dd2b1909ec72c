"""Writes tests/golden/full_size.json: oracle results for the full-size
workloads (R-MAT scale 24 and Erdos-Renyi n=2^24, average degree 32; p=64,
balanced cuts).  Calls only the generators and the oracle.

Stored per workload: n, m, total, the SHA-256 of the per-task vector (uint64
little-endian, Alg. 4 order) and every 97th per-task entry.

Usage: python tests/golden/make_goldens.py [workload ...]
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size.json")
P = 64
STRIDE = 97


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        t = time.time()
        g = graphgen.workload(name)
        og = oracle.OracleGraph.from_graph(g)
        del g
        cuts = og.cuts(P)
        tot, per, bn = og.tasks(P, cuts)
        data[name] = {
            "n": og.n, "m": og.m, "p": P, "total": tot,
            "per_task_sha256": hashlib.sha256(per.astype("<u8").tobytes()).hexdigest(),
            "sample_stride": STRIDE,
            "per_task_sample": [int(x) for x in per[::STRIDE]],
            "cuts_sha256": hashlib.sha256(cuts.astype("<i4").tobytes()).hexdigest(),
            "seconds": round(time.time() - t, 1),
        }
        print(name, data[name]["total"], data[name]["seconds"], flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or ["rmat24", "er24"])
