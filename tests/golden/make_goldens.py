"""Writes tests/golden/full_size.json: oracle results for the full-size
workloads (R-MAT scale 24 and Erdos-Renyi n=2^24, average degree 32; p=64,
balanced cuts).  Calls only the generators and the oracle.

Stored per workload: n, m, total, the SHA-256 of the per-task vector (uint64
little-endian, Alg. 4 order) and every 97th per-task entry; under "by_p", the
total, per-task SHA-256 and cut-vector SHA-256 for every p the autotuner may
pick from a base of 64: its candidates 16, 32, 64, 128 and, past them, the
halvings down to 1 and the doubling to 256.  Values of p already stored are
kept unless --all is given.

R-MAT scale 27 (the device-budget workload, p=128) is built by the oracle
from the raw R-MAT samples (its own canonicalisation; the samples take 17 GB
against about 40 GB for the symmetric CSR route) and stores n, m, the total,
the per-task SHA-256 and the cut-vector SHA-256 at p=128.

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
TUNER_PS = (1, 2, 4, 8, 16, 32, 64, 128, 256)


def rmat27_entry():
    t = time.time()
    src, dst = graphgen.rmat_edges(27, 16, 27)
    print("rmat27 samples", round(time.time() - t, 1), flush=True)
    og = oracle.OracleGraph(1 << 27, src=src, dst=dst)
    del src, dst
    print("rmat27 oracle graph", og.m, round(time.time() - t, 1), flush=True)
    p = 128
    cuts = og.cuts(p)
    tot, per, _ = og.tasks(p, cuts)
    return {"n": og.n, "m": og.m, "p": p, "total": tot,
            "per_task_sha256": hashlib.sha256(per.astype("<u8").tobytes()).hexdigest(),
            "sample_stride": STRIDE, "per_task_sample": [int(x) for x in per[::STRIDE]],
            "cuts_sha256": hashlib.sha256(cuts.astype("<i4").tobytes()).hexdigest(),
            "seconds": round(time.time() - t, 1)}


def main(names, redo):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        if name == "rmat27":
            data[name] = rmat27_entry()
            print(name, data[name]["total"], data[name]["seconds"], flush=True)
            with open(OUT, "w") as f:
                json.dump(data, f, indent=1)
            continue
        t = time.time()
        g = graphgen.workload(name)
        og = oracle.OracleGraph.from_graph(g)
        del g
        entry = data.get(name) if not redo else None
        if entry is None:
            cuts = og.cuts(P)
            tot, per, bn = og.tasks(P, cuts)
            entry = {
                "n": og.n, "m": og.m, "p": P, "total": tot,
                "per_task_sha256": hashlib.sha256(per.astype("<u8").tobytes()).hexdigest(),
                "sample_stride": STRIDE,
                "per_task_sample": [int(x) for x in per[::STRIDE]],
                "cuts_sha256": hashlib.sha256(cuts.astype("<i4").tobytes()).hexdigest(),
                "by_p": {},
            }
        by_p = entry.setdefault("by_p", {})
        for q in TUNER_PS:
            if str(q) in by_p:
                continue
            qc = og.cuts(q)
            qt, qper, _ = og.tasks(q, qc)
            by_p[str(q)] = {"total": qt, "per_task_sha256": hashlib.sha256(qper.astype("<u8").tobytes()).hexdigest(),
                            "cuts_sha256": hashlib.sha256(qc.astype("<i4").tobytes()).hexdigest()}
            print(name, "p", q, qt, round(time.time() - t, 1), flush=True)
            data[name] = entry
            with open(OUT, "w") as f:
                json.dump(data, f, indent=1)
        entry["by_p"] = {str(q): by_p[str(q)] for q in sorted(int(x) for x in by_p)}
        entry["seconds"] = round(time.time() - t, 1)
        data[name] = entry
        print(name, entry["total"], entry["seconds"], flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1)


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "--all"]
    main(args or ["rmat24", "er24"], "--all" in sys.argv[1:])
