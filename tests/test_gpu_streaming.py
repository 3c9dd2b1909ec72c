"""Counting under a device budget: stripes stream from pinned host memory.
Results must be identical to the oracle's, task by task."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
import paper_2009_12457_amd as bb
from helpers import in_alg4_order

pytestmark = pytest.mark.gpu


def count(plan):
    per, tot = bb.bbtc_count(plan)
    torch.cuda.synchronize()
    return per.cpu().numpy().view(np.uint64)[:plan.ntasks].copy(), int(tot.item())


def _graph(name):
    if name == "er200k":
        return graphgen.er(200000, 16.0 / 199999, 3)
    return graphgen.workload(name)


@pytest.mark.parametrize("name,p,frac,bound", [("rmat16", 12, 4, 0), ("rmat14_ef8", 5, 3, 0), ("er200k", 8, 4, 0),
                                                ("rmat16", 24, 4, -1), ("rmat16", 24, 4, 1 << 30)])
def test_streamed_equals_oracle(name, p, frac, bound):
    """Every per-task count of a streamed plan equals the oracle's (Alg. 4
    order, given the plan's cuts), on both counts; with the cache holding
    fewer than the 2p stripes, the second count must evict and re-upload."""
    g = _graph(name)
    og = oracle.OracleGraph.from_graph(g)
    n, rp, ci = bb.csr_of(g, "cuda")
    res = bb.bbtc_partition(n, rp, ci, options=bb.bbtc_options_default(p=p, bound_min_deg=bound), trusted=True)
    foot = res.stats()["footprint"]
    streamed = None
    for f in (frac, frac * 0.75, frac * 0.5, 1.5):
        try:
            streamed = bb.bbtc_partition(n, rp, ci, options=bb.bbtc_options_default(
                p=p, device_budget_bytes=int(foot / f), bound_min_deg=bound), trusted=True)
            budget = int(foot / f)
            break
        except bb.BbtcError as e:
            assert e.status == bb.BBTC_EBUDGET
    assert streamed is not None, "no budget below the resident footprint was usable"
    st = streamed.stats()
    assert st["streamed"] == 1 and st["stripe_slots"] >= 2
    streamed.verify()
    assert st["footprint"] <= budget
    cuts = streamed.cuts()
    assert np.array_equal(cuts, og.cuts(p))
    want_tot, want_per, _ = og.tasks(p, cuts)
    tasks = streamed.tasks()
    for rep in range(2):
        per_s, tot_s = count(streamed)
        assert tot_s == want_tot
        assert np.array_equal(in_alg4_order(p, tasks, per_s), want_per), f"count {rep}: per-task counts differ"
        if st["stripe_slots"] < 2 * p:
            # fewer slots than stripes: every count walks all block pairs, so
            # it must upload more stripes than the cache holds
            assert streamed.stats()["stripe_uploads"] > st["stripe_slots"]
    orow, ocol = streamed.oriented()
    w_orow, w_ocol = og.oriented()
    assert np.array_equal(orow.astype(np.int64), w_orow) and np.array_equal(ocol, w_ocol)
    if frac == 4:
        assert st["stripe_slots"] < 2 * p, "this case is meant to evict"


def test_budget_too_small_is_ebudget():
    g = graphgen.workload("rmat14_ef8")
    n, rp, ci = bb.csr_of(g, "cuda")
    with pytest.raises(bb.BbtcError) as ei:
        bb.bbtc_partition(n, rp, ci, options=bb.bbtc_options_default(p=8, device_budget_bytes=4096), trusted=True)
    assert ei.value.status == bb.BBTC_EBUDGET


def test_streamed_plan_rejected_by_shared_launch():
    g = graphgen.workload("rmat12")
    n, rp, ci = bb.csr_of(g, "cuda")
    res = bb.bbtc_partition(n, rp, ci, options=bb.bbtc_options_default(p=6), trusted=True)
    foot = res.stats()["footprint"]
    plan = None
    for frac in (3, 2, 1.5):
        try:
            plan = bb.bbtc_partition(n, rp, ci, options=bb.bbtc_options_default(
                p=6, device_budget_bytes=int(foot / frac)), trusted=True)
            break
        except bb.BbtcError:
            pass
    if plan is None:
        pytest.skip("graph too small to stream")
    with pytest.raises(bb.BbtcError) as ei:
        bb.bbtc_count_multi([plan, res])
    assert ei.value.status == bb.BBTC_ESTATE


@pytest.mark.parametrize("where,trusted", [("host", True), ("host", False), ("device", False)])
def test_budgeted_partition_inputs(where, trusted):
    """A budget below the resident partition's needs partitions in pieces from
    host or device input, trusted or validated, and counts by streaming: the
    per-task vector equals the oracle's, and the plan's tables check out."""
    g = graphgen.workload("rmat15")
    og = oracle.OracleGraph.from_graph(g)
    p = 20
    if where == "host":
        n, rp, ci = bb.csr_of(g)
    else:
        n, rp, ci = bb.csr_of(g, "cuda")
    res = bb.bbtc_partition(n, rp, ci, options=bb.bbtc_options_default(p=p), trusted=True)
    budget = res.stats()["footprint"] // 3
    res.destroy()
    plan = bb.bbtc_partition(n, rp, ci, options=bb.bbtc_options_default(p=p, device_budget_bytes=budget),
                             trusted=trusted)
    st = plan.stats()
    assert st["streamed"] == 1 and st["footprint"] <= budget
    plan.verify()
    cuts = plan.cuts()
    assert np.array_equal(cuts, og.cuts(p))
    want_tot, want_per, _ = og.tasks(p, cuts)
    per, tot = count(plan)
    assert tot == want_tot
    assert np.array_equal(in_alg4_order(p, plan.tasks(), per), want_per)
    assert np.array_equal(plan.perm(), og.rank())


def test_budgeted_partition_rejects_bad_input():
    """Validation still applies when the partition runs in pieces."""
    n, rp, ci = 3, np.array([0, 2, 3, 4], np.int64), np.array([0, 1, 0, 0], np.int32)  # a self-loop
    with pytest.raises(bb.BbtcError) as ei:
        bb.bbtc_partition(n, rp, ci, options=bb.bbtc_options_default(p=1, device_budget_bytes=1 << 20))
    assert ei.value.status == bb.BBTC_EINVAL
    with pytest.raises(bb.BbtcError) as ei:
        bb.bbtc_partition(n, torch.tensor(rp, device="cuda"), torch.tensor(ci, device="cuda"),
                          options=bb.bbtc_options_default(p=1, device_budget_bytes=1 << 20))
    assert ei.value.status == bb.BBTC_EINVAL
