"""Full-size parity for the 2^24-vertex workloads (R-MAT scale 24 and
Erdos-Renyi average degree 32) at p = 64, against oracle results stored by
tests/golden/make_goldens.py (total, SHA-256 of the whole per-task vector in
Alg. 4 order, every 97th per-task entry, SHA-256 of the cut vector); and the
autotuner's choice, whose per-task vector must equal the oracle's for the p
it picks."""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import graphgen
import paper_2009_12457_amd as bb
from helpers import in_alg4_order

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "full_size.json")))


def alg4_positions(p, tasks):
    base = np.zeros((p, p), np.int64)
    t = 0
    for i in range(p):
        for j in range(i, p):
            base[i, j] = t
            t += p - j
    return base[tasks["i"], tasks["j"]] + (tasks["k"] - tasks["j"])


@pytest.fixture(scope="module", params=["rmat24", "er24"])
def workload(request):
    g = graphgen.workload(request.param)
    n, rp, ci = bb.csr_of(g, "cuda")
    yield request.param, g, n, rp, ci
    del rp, ci
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mode", ["persistent", "hmap"])
def test_full_size_per_task_parity(workload, mode):
    name, g, n, rp, ci = workload
    gold = GOLD[name]
    p = gold["p"]
    opt = bb.bbtc_options_default(p=p, mode={"persistent": bb.BBTC_MODE_PERSISTENT,
                                             "hmap": bb.BBTC_MODE_PLAIN_HMAP}[mode])
    plan = bb.bbtc_partition(n, rp, ci, options=opt, trusted=True)
    per, tot = bb.bbtc_count(plan)
    torch.cuda.synchronize()
    st = plan.stats()
    assert st["m"] == gold["m"] and st["n"] == gold["n"]
    assert hashlib.sha256(plan.cuts().astype("<i4").tobytes()).hexdigest() == gold["cuts_sha256"]
    assert int(tot.item()) == gold["total"]
    tasks = plan.tasks()
    got = np.zeros(len(tasks), np.uint64)
    got[alg4_positions(p, tasks)] = per.cpu().numpy().view(np.uint64)[:len(tasks)]
    assert [int(x) for x in got[::gold["sample_stride"]]] == gold["per_task_sample"]
    assert hashlib.sha256(got.astype("<u8").tobytes()).hexdigest() == gold["per_task_sha256"]
    plan.destroy()


def test_autotuned_per_task(workload):
    """The autotuner's choice (p from {16, 32, 64, 128}, or past them by
    halving down to 1 or doubling, and the row-mapping knobs) gives the
    oracle's per-task vector for that p, stored by
    tests/golden/make_goldens.py for p from 1 to 256."""
    name, g, n, rp, ci = workload
    opt, ms = bb.bbtc_autotune(n, rp, ci, base=bb.bbtc_options_default(p=GOLD[name]["p"]), reps=2, trusted=True)
    assert ms > 0
    assert str(opt.p) in GOLD[name]["by_p"], f"no stored oracle result at p={opt.p}"
    gold = GOLD[name]["by_p"][str(opt.p)]
    plan = bb.bbtc_partition(n, rp, ci, options=opt, trusted=True)
    per, tot = bb.bbtc_count(plan)
    torch.cuda.synchronize()
    assert hashlib.sha256(plan.cuts().astype("<i4").tobytes()).hexdigest() == gold["cuts_sha256"]
    assert int(tot.item()) == gold["total"]
    got = in_alg4_order(opt.p, plan.tasks(), per.cpu().numpy().view(np.uint64))
    assert hashlib.sha256(got.astype("<u8").tobytes()).hexdigest() == gold["per_task_sha256"]
    plan.destroy()
