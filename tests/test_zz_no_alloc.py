"""bbtc_count_multi_static (launch state in the library's fixed device array,
no allocation inside the call) against bbtc_count_multi, through the C ABI:
two calls in a row, the second with a smaller input, each compared task by
task with the allocating entry point's results (exact integer counts)."""
import numpy as np
import pytest
import torch

import graphgen
import paper_2009_12457_amd as bb

pytestmark = pytest.mark.gpu


def _plans(specs):
    out = []
    for name, p, mode in specs:
        g = graphgen.workload(name)
        n, rp, ci = bb.csr_of(g, "cuda")
        out.append(bb.bbtc_partition(n, rp, ci, options=bb.bbtc_options_default(p=p, mode=mode), trusted=True))
    return out


def _counts(plans, static):
    pers = [torch.full((max(pl.ntasks, 1),), -1, dtype=torch.int64, device="cuda") for pl in plans]
    tots = torch.full((len(plans),), -1, dtype=torch.int64, device="cuda")
    bb.bbtc_count_multi(plans, pers, tots, static=static)
    torch.cuda.synchronize()
    return [p.cpu().numpy()[:pl.ntasks].copy() for p, pl in zip(pers, plans)], tots.cpu().numpy().copy()


def test_static_multi_matches_allocating_entry_point():
    big = _plans([("rmat14_ef8", 16, bb.BBTC_MODE_PERSISTENT), ("er2000", 4, bb.BBTC_MODE_PLAIN_HMAP),
                  ("rmat12", 7, bb.BBTC_MODE_PERSISTENT), ("rmat10", 1, bb.BBTC_MODE_PLAIN_INTERSECT),
                  ("rmat13", 9, bb.BBTC_MODE_PERSISTENT)])
    small = _plans([("rmat10", 3, bb.BBTC_MODE_PERSISTENT), ("er2000", 2, bb.BBTC_MODE_PERSISTENT)])
    for plans in (big, small):  # the second call is smaller: fewer plans, fewer items
        want_per, want_tot = _counts(plans, static=False)
        got_per, got_tot = _counts(plans, static=True)
        assert np.array_equal(got_tot, want_tot)
        for q in range(len(plans)):
            assert np.array_equal(got_per[q], want_per[q]), q
    # repeated calls on the same stream reuse the array in order
    for _ in range(3):
        got_per, got_tot = _counts(big, static=True)
        assert np.array_equal(got_tot, _counts(big, static=False)[1])


def test_static_multi_limits():
    plans = _plans([("rmat10", 2, bb.BBTC_MODE_PERSISTENT)])
    with pytest.raises(bb.BbtcError) as ei:
        bb.bbtc_count_multi(plans * (bb.BBTC_STATIC_MAX_PLANS + 1), static=True)
    assert ei.value.status == bb.BBTC_EINVAL
    # exactly the maximum is accepted (one plan counted 64 times into 64 outputs)
    pers, tots = bb.bbtc_count_multi(plans * bb.BBTC_STATIC_MAX_PLANS, static=True)
    torch.cuda.synchronize()
    want = _counts(plans, static=False)[1][0]
    assert np.all(tots.cpu().numpy() == want)
