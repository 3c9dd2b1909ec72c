"""Counting under a device budget: stripes stream from pinned host memory.
Results must be identical to the resident plan (and the oracle)."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
import paper_2009_12457_amd as bb

pytestmark = pytest.mark.gpu


def count(plan):
    per, tot = bb.bbtc_count(plan)
    torch.cuda.synchronize()
    return per.cpu().numpy().view(np.uint64)[:plan.ntasks].copy(), int(tot.item())


def _graph(name):
    if name == "er200k":
        return graphgen.er(200000, 16.0 / 199999, 3)
    return graphgen.workload(name)


@pytest.mark.parametrize("name,p", [("rmat16", 12), ("rmat14_ef8", 5), ("er200k", 8)])
def test_streamed_equals_resident(name, p):
    g = _graph(name)
    n, rp, ci = bb.csr_of(g, "cuda")
    res = bb.bbtc_partition(n, rp, ci, options=bb.bbtc_options_default(p=p), trusted=True)
    per_r, tot_r = count(res)
    foot = res.stats()["footprint"]
    streamed = None
    for frac in (4, 3, 2, 1.5):
        try:
            streamed = bb.bbtc_partition(n, rp, ci, options=bb.bbtc_options_default(
                p=p, device_budget_bytes=int(foot / frac)), trusted=True)
            break
        except bb.BbtcError as e:
            assert e.status == bb.BBTC_EBUDGET
    assert streamed is not None, "no budget below the resident footprint was usable"
    st = streamed.stats()
    assert st["streamed"] == 1 and st["stripe_slots"] >= 3
    assert st["footprint"] <= int(foot / frac)
    for rep in range(2):
        per_s, tot_s = count(streamed)
        assert tot_s == tot_r
        assert np.array_equal(per_s, per_r)
        if rep == 0:
            assert streamed.stats()["stripe_uploads"] > 0
    og = oracle.OracleGraph.from_graph(g)
    assert tot_r == og.total()
    # tasks and cuts are those of the resident plan
    assert np.array_equal(streamed.cuts(), res.cuts())
    orow, ocol = streamed.oriented()
    w_orow, w_ocol = og.oriented()
    assert np.array_equal(orow.astype(np.int64), w_orow) and np.array_equal(ocol, w_ocol)


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
