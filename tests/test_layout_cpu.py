"""The block-table checker (bbtc_check_tables, pure host code) on the CPU:
tables built here from the oracle's oriented graph by the definitions the
header states are accepted, and a single wrong entry of any table -- of the
kinds the counting kernels would turn into out-of-row reads (a boundary
outside its row, a wrong stride, an active column without an in-neighbour,
an in-row not grouped by part) -- is rejected.  The same checker runs on the
GPU plans in tests/test_gpu_parity.py (bbtc_plan_verify)."""
import numpy as np
import pytest

import graphgen
import oracle
import paper_2009_12457_amd as bb


def reference_tables(g, p, T):
    og = oracle.OracleGraph.from_graph(g)
    n, m = og.n, og.m
    orow, ocol = og.oriented()
    cuts = og.cuts(p).astype(np.int64)
    part = np.searchsorted(cuts, np.arange(n), side="right") - 1
    src = np.repeat(np.arange(n), np.diff(orow))
    order = np.lexsort((src, ocol))  # in-rows: by head, then tail ascending
    icol = src[order].astype(np.int32)
    irow = np.zeros(n + 1, np.int64)
    np.add.at(irow, ocol + 1, 1)
    irow = np.cumsum(irow)
    deg = np.diff(orow) + np.diff(irow)
    rT = int((deg <= T).sum()) if T >= 0 else 0
    botp, bot = [0], []
    for a in range(p):  # column-major per part: column b-a lists entry b-a of every stored row
        sa = max(cuts[a], rT)
        rows = [[orow[u] + int(np.searchsorted(ocol[orow[u]:orow[u + 1]], cuts[b])) for b in range(a, p)]
                + [orow[u + 1]] for u in range(sa, cuts[a + 1])]
        for col in range(p - a + 1):
            bot += [r[col] for r in rows]
        botp.append(botp[-1] + max(0, cuts[a + 1] - sa) * (p - a + 1))
    slices = {}
    for v in range(n):
        ins = icol[irow[v]:irow[v + 1]]
        for a in sorted(set(part[ins].tolist())):
            slices.setdefault((a, part[v]), []).append((v, ins[part[ins] == a][::-1]))  # any order inside
    acp, acol, aoff, icolb = [0], [], [], []
    for b in range(p):
        for a in range(b + 1):
            for v, sl in slices.get((a, b), []):
                acol.append(v)
                aoff.append(len(icolb))
                icolb += sl.tolist()
            acp.append(len(acol))
    aoff.append(len(icolb))
    return dict(n=n, m=m, p=p, rT=rT, cuts=cuts, orow=orow, ocol=ocol, botp=botp, bot=bot, acp=acp, acol=acol,
                aoff=aoff, icolb=icolb)


def tables_np(t):
    out = dict(t)
    for k, dt in (("cuts", np.int32), ("orow", np.uint32), ("ocol", np.int32), ("botp", np.uint64),
                  ("bot", np.uint32), ("acp", np.uint64), ("acol", np.int32), ("aoff", np.uint32),
                  ("icolb", np.int32)):
        out[k] = np.array(t[k], dtype=dt)
    return out


@pytest.mark.parametrize("name,p,T", [("er2000", 4, 32), ("rmat10", 7, 8), ("rmat10", 16, -1), ("rmat11", 3, 0),
                                      ("rmat10", 31, 1 << 30)])
def test_reference_tables_accepted(name, p, T):
    t = tables_np(reference_tables(graphgen.workload(name), p, T))
    bb.bbtc_check_tables(**t)


def _expect_reject(t, what):
    with pytest.raises(bb.BbtcError) as ei:
        bb.bbtc_check_tables(**t)
    assert ei.value.status == bb.BBTC_EINVAL
    assert what in str(ei.value), str(ei.value)


def test_single_wrong_entries_rejected():
    base = tables_np(reference_tables(graphgen.workload("rmat10"), 7, 8))
    assert len(base["bot"]) > 0 and len(base["acol"]) > 3

    def mutated(key, fn):
        t = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in base.items()}
        fn(t[key])
        return t

    # a boundary moved by one inside and one outside its row
    _expect_reject(mutated("bot", lambda a: a.__setitem__(3, a[3] + 1)), "out-side boundary")
    _expect_reject(mutated("bot", lambda a: a.__setitem__(len(a) - 1, a[-1] + 100)), "out-side boundary")
    # the part table with a wrong stride; rT moved so that the stored rows no
    # longer match the table
    _expect_reject(mutated("botp", lambda a: a.__setitem__(len(a) - 1, a[-1] + 1)), "botp")
    t = dict(base)
    t["rT"] = base["rT"] - 1
    _expect_reject(t, "botp")
    # active columns: a wrong column, a wrong count
    _expect_reject(mutated("acol", lambda a: a.__setitem__(2, a[2] + 1)), "active column")
    _expect_reject(mutated("acp", lambda a: a.__setitem__(len(a) - 1, a[-1] - 1)), "active-column count")
    # in slices: an offset moved, an entry replaced by a vertex of another part
    x = int(np.argmax(np.diff(base["aoff"].astype(np.int64)) >= 2))
    _expect_reject(mutated("aoff", lambda a: a.__setitem__(x + 1, a[x + 1] - 1)), "in-slice")

    def foreign_entry(a):
        a[int(base["aoff"][x])] = base["n"] - 1  # the highest rank is never an in-neighbour
    _expect_reject(mutated("icolb", foreign_entry), "in-slice entries")
    # oriented rows: an entry out of order
    def swap_out(a):
        r = int(np.argmax(np.diff(base["orow"].astype(np.int64)) >= 2))
        s0 = int(base["orow"][r])
        a[s0], a[s0 + 1] = a[s0 + 1], a[s0]
    _expect_reject(mutated("ocol", swap_out), "out-row")
    # cut vector not strictly increasing
    _expect_reject(mutated("cuts", lambda a: a.__setitem__(2, a[1])), "cut vector")
