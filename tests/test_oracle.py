"""Pins for the CPU oracle against facts the paper and mathematics fix.

None of these tests re-types the oracle's own formula: totals are checked
against brute-force enumeration of vertex triples, closed forms, trace(A^3)/6
and networkx; per-task counts against brute-force classification of every
triangle and against the p = n closed form; the task list against the
paper's printed example and Table 4.
"""
import itertools
import json
import math
import os

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp

import graphgen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "task_examples.json")


# ---------------------------------------------------------------- helpers
def og_from_edges(n, edges):
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return oracle.OracleGraph(n, src=edges[:, 0], dst=edges[:, 1])


def simple_adj(n, edges):
    A = np.zeros((n, n), dtype=bool)
    for x, y in edges:
        if x != y:
            A[x, y] = A[y, x] = True
    return A


def brute_triangles(A):
    """All vertex triples {x<y<z} with all three edges present."""
    n = A.shape[0]
    return [(x, y, z) for x, y, z in itertools.combinations(range(n), 3) if A[x, y] and A[y, z] and A[x, z]]


def random_edges(rng, n, ne):
    return rng.integers(0, n, size=(ne, 2))


def alg4_index(p):
    """Position of each (i,j,k) when enumerated i<=j<=k in nested loop order."""
    idx, t = {}, 0
    for i in range(p):
        for j in range(i, p):
            for k in range(j, p):
                idx[(i, j, k)] = t
                t += 1
    return idx


def degree_rank(A):
    """rank[x] from sorting ids by (degree, id)."""
    deg = A.sum(axis=1)
    order = sorted(range(A.shape[0]), key=lambda x: (deg[x], x))
    rank = np.empty(A.shape[0], np.int64)
    rank[order] = np.arange(A.shape[0])
    return rank


# ------------------------------------------------------- totals: brute force
@pytest.mark.parametrize("seed", range(60))
def test_total_matches_brute_force_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    ne = int(rng.integers(0, 4 * n + 1))
    e = random_edges(rng, n, ne)
    A = simple_adj(n, e)
    og = og_from_edges(n, e)
    want = len(brute_triangles(A))
    assert og.m == int(A.sum()) // 2
    assert og.total(threads=2) == want
    assert og.total_hmap(threads=2) == want


@pytest.mark.parametrize("scale,seed", [(3, 1), (4, 2), (5, 3), (6, 4), (6, 5)])
def test_total_matches_brute_force_rmat(scale, seed):
    src, dst = graphgen.rmat_edges(scale, 8, seed)
    n = 1 << scale
    A = simple_adj(n, zip(src.tolist(), dst.tolist()))
    og = oracle.OracleGraph(n, src=src, dst=dst)
    want = len(brute_triangles(A))
    assert og.total(threads=3) == want
    assert og.total_hmap(threads=3) == want


# ------------------------------------------------------- totals: closed forms
def complete(n):
    return [(x, y) for x in range(n) for y in range(x + 1, n)]


def cycle(n):
    return [(x, (x + 1) % n) for x in range(n)]


CLOSED_FORMS = []
for n in (3, 4, 5, 7, 10, 23, 40):
    CLOSED_FORMS.append((f"K{n}", n, complete(n), math.comb(n, 3)))
for k in (2, 3, 5, 9):  # K_{2k} minus a perfect matching
    n = 2 * k
    CLOSED_FORMS.append((f"K{n}-M", n, [(x, y) for x, y in complete(n) if not (y == x + 1 and x % 2 == 0)],
                         math.comb(n, 3) - k * (n - 2)))
CLOSED_FORMS.append(("C3", 3, cycle(3), 1))
for n in (4, 6, 10, 31):
    CLOSED_FORMS.append((f"C{n}", n, cycle(n), 0))
for n in (4, 5, 8, 20):  # wheel: hub n, rim 0..n-1
    CLOSED_FORMS.append((f"W{n}", n + 1, cycle(n) + [(n, x) for x in range(n)], n))
for k in (1, 2, 5, 12):  # friendship graph F_k: k triangles sharing vertex 0
    CLOSED_FORMS.append((f"F{k}", 2 * k + 1, [e for t in range(k) for e in ((0, 2 * t + 1), (0, 2 * t + 2), (2 * t + 1, 2 * t + 2))], k))
for a, b in ((1, 1), (2, 3), (5, 7)):  # complete bipartite
    CLOSED_FORMS.append((f"K{a},{b}", a + b, [(x, a + y) for x in range(a) for y in range(b)], 0))
for a, b, c in ((1, 1, 1), (2, 3, 4), (3, 3, 5)):  # complete tripartite
    parts = [range(0, a), range(a, a + b), range(a + b, a + b + c)]
    es = [(x, y) for P, Q in itertools.combinations(parts, 2) for x in P for y in Q]
    CLOSED_FORMS.append((f"K{a},{b},{c}", a + b + c, es, a * b * c))
for r, c in ((2, 2), (3, 5), (7, 4)):  # grid graph
    idx = lambda x, y: x * c + y
    es = [(idx(x, y), idx(x + 1, y)) for x in range(r - 1) for y in range(c)]
    es += [(idx(x, y), idx(x, y + 1)) for x in range(r) for y in range(c - 1)]
    CLOSED_FORMS.append((f"grid{r}x{c}", r * c, es, 0))
CLOSED_FORMS.append(("star50", 51, [(0, x) for x in range(1, 51)], 0))
CLOSED_FORMS.append(("path30", 30, [(x, x + 1) for x in range(29)], 0))
CLOSED_FORMS.append(("empty", 10, [], 0))
CLOSED_FORMS.append(("single", 1, [], 0))
# disjoint union K5 + W6 + F3 -> 10 + 6 + 3
_u = complete(5) + [(5 + x, 5 + y) for x, y in cycle(6) + [(6, t) for t in range(6)]]
_u += [(12 + x, 12 + y) for t in range(3) for x, y in ((0, 2 * t + 1), (0, 2 * t + 2), (2 * t + 1, 2 * t + 2))]
CLOSED_FORMS.append(("union", 19, _u, 10 + 6 + 3))


@pytest.mark.parametrize("name,n,edges,want", CLOSED_FORMS, ids=[c[0] for c in CLOSED_FORMS])
def test_total_closed_forms(name, n, edges, want):
    og = og_from_edges(n, edges if edges else np.zeros((0, 2), np.int64))
    assert og.total(threads=2) == want
    assert og.total_hmap(threads=2) == want
    for p in sorted({1, 2, min(3, n), n}):
        if 1 <= p <= n:
            tot, per, _ = og.tasks(p, threads=2)
            assert tot == want and int(per.sum()) == want


def test_random_tree_and_forest_have_no_triangles():
    rng = np.random.default_rng(7)
    n = 500
    parent = [int(rng.integers(0, x)) for x in range(1, n)]
    tree = [(x + 1, parent[x]) for x in range(n - 1)]
    assert og_from_edges(n, tree).total() == 0
    forest = [e for e in tree if rng.random() < 0.7]
    assert og_from_edges(n, forest).total() == 0


def test_random_bipartite_has_no_triangles():
    rng = np.random.default_rng(8)
    a, b = 300, 400
    es = [(x, a + y) for x in range(a) for y in range(b) if rng.random() < 0.05]
    assert og_from_edges(a + b, es).total() == 0


# ------------------------------------------------------- totals: linear algebra
def test_trace_a_cubed_er2000():
    g = graphgen.workload("er2000")
    A = np.zeros((g.n, g.n))
    u, v = g.edges()
    A[u, v] = A[v, u] = 1.0
    want = int(round(np.trace(A @ A @ A) / 6.0))  # exact: entries < 2^53
    og = oracle.OracleGraph.from_graph(g)
    assert og.total() == want
    assert og.total_hmap() == want


@pytest.mark.parametrize("name", ["rmat12", "rmat14_ef8"])
def test_sparse_trace_and_networkx(name):
    g = graphgen.workload(name)
    A = sp.csr_matrix((np.ones(len(g.colidx), np.int64), g.colidx, g.rowptr), shape=(g.n, g.n))
    want = int((A @ A).multiply(A).sum()) // 6
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from(zip(*[a.tolist() for a in g.edges()]))
    assert sum(nx.triangles(G).values()) // 3 == want
    og = oracle.OracleGraph.from_graph(g)
    assert og.total() == want


# ------------------------------------------------------- invariants
@pytest.mark.parametrize("name", ["er2000", "rmat10", "rmat12_ef32"])
def test_relabel_and_p_invariance(name):
    g = graphgen.workload(name)
    base = oracle.OracleGraph.from_graph(g).total()
    for s in (1, 2):
        assert oracle.OracleGraph.from_graph(graphgen.relabel(g, s)).total() == base
    og = oracle.OracleGraph.from_graph(g)
    for p in (1, 2, 3, 4, 7, 16, 33):
        for mode in (oracle.CUT_BALANCED, oracle.CUT_UNIFORM):
            tot, per, bn = og.tasks(p, og.cuts(p, mode))
            assert tot == base and int(per.sum()) == base
            assert int(bn.sum()) == og.m


def test_canonicalisation_of_raw_rmat_samples():
    """Raw samples (with repeats and loops) and the generator's CSR agree."""
    src, dst = graphgen.rmat_edges(12, 16, 12)
    g = graphgen.rmat(12, 16, 12)
    a = oracle.OracleGraph(g.n, src=src, dst=dst)
    b = oracle.OracleGraph.from_graph(g)
    G = nx.Graph()
    G.add_edges_from((x, y) for x, y in zip(src.tolist(), dst.tolist()) if x != y)
    assert a.m == b.m == G.number_of_edges() == g.m
    assert a.total() == b.total() == sum(nx.triangles(G).values()) // 3


# ------------------------------------------------------- ordering and cuts
@pytest.mark.parametrize("seed", range(10))
def test_degree_order_is_nondecreasing_with_id_ties(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 60))
    e = random_edges(rng, n, int(rng.integers(0, 5 * n)))
    A = simple_adj(n, e)
    og = og_from_edges(n, e)
    assert np.array_equal(og.rank(), degree_rank(A))
    # every oriented entry points from lower to higher rank, lists sorted
    orow, ocol = og.oriented()
    for r in range(n):
        row = ocol[orow[r]:orow[r + 1]]
        assert np.all(row > r) and np.all(np.diff(row) > 0)


@pytest.mark.parametrize("name,p", [("er2000", 4), ("rmat12", 16), ("rmat12", 64), ("rmat10", 3)])
def test_balanced_cut_properties(name, p):
    g = graphgen.workload(name)
    og = oracle.OracleGraph.from_graph(g)
    orow, _ = og.oriented()
    c = og.cuts(p)
    m, n = og.m, og.n
    assert c[0] == 0 and c[-1] == n and np.all(np.diff(c) > 0)
    for i in range(1, p):
        target = -(-i * m // p)
        clamped = c[i] == n - (p - i)
        forced = c[i] == c[i - 1] + 1
        if not clamped:
            assert orow[c[i]] >= target  # reaches its share ...
        if not forced and not clamped:
            assert orow[c[i] - 1] < target  # ... and is the first to do so


def uniform_part_of(x, n, p):
    """Part of vertex x under an even split, vertex by vertex: the unit cell
    (x, x+1] of the interval (0, n] belongs to the part a whose share
    (a*n/p, (a+1)*n/p] holds its right end, i.e. a*n < (x+1)*p <= (a+1)*n."""
    return -(-(x + 1) * p // n) - 1


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 10, 16, 31, 40, 97])
def test_uniform_cut_rule(n):
    """The uniform cut (Sec. 4.1 partitions V into p contiguous parts; the
    uniform reading splits the rank range evenly).  Pinned without the cut
    formula: (1) every part has floor(n/p) or ceil(n/p) vertices, exactly
    n mod p of them the larger size, in the order that integer rounding of
    a*n/p gives; (2) the part of each vertex, computed vertex by vertex from
    (x+1)*p/n, agrees with the cut vector; (3) the clamps into
    [c_{i-1}+1, n-(p-i)] never bind for p <= n (floor(i*n/p) rises by at
    least floor(n/p) >= 1 per step and i*n/p <= n-(p-i) iff p <= n), so the
    rule is the plain even split for every valid p."""
    g = graphgen.from_edges(n, np.zeros(0, np.int32), np.zeros(0, np.int32))
    og = oracle.OracleGraph.from_graph(g)
    for p in range(1, n + 1):
        c = og.cuts(p, oracle.CUT_UNIFORM).astype(np.int64)
        sizes = np.diff(c)
        q = n // p
        assert c[0] == 0 and c[-1] == n
        assert set(sizes.tolist()) <= {q, q + 1}
        assert int((sizes == q + 1).sum()) == n % p
        part = np.array([uniform_part_of(x, n, p) for x in range(n)])
        assert np.array_equal(np.searchsorted(c, np.arange(n), side="right") - 1, part)
    with pytest.raises(ValueError):
        og.cuts(n + 1, oracle.CUT_UNIFORM)


def test_uniform_cut_on_edge_graph_ignores_edges():
    """The uniform rule depends on n and p only: adding edges moves no cut."""
    g = graphgen.workload("rmat10")
    og = oracle.OracleGraph.from_graph(g)
    empty = oracle.OracleGraph.from_graph(graphgen.from_edges(g.n, np.zeros(0, np.int32), np.zeros(0, np.int32)))
    for p in (1, 3, 16, 100, g.n):
        assert np.array_equal(og.cuts(p, oracle.CUT_UNIFORM), empty.cuts(p, oracle.CUT_UNIFORM))


# ------------------------------------------------------- per-task counts
def brute_per_task(A, rank, cuts, p):
    part = np.searchsorted(cuts, np.arange(A.shape[0]), side="right") - 1
    idx = alg4_index(p)
    per = np.zeros(len(idx), np.uint64)
    for x, y, z in brute_triangles(A):
        a, b, c = sorted((rank[x], rank[y], rank[z]))
        per[idx[(part[a], part[b], part[c])]] += 1
    return per


@pytest.mark.parametrize("seed", range(25))
def test_per_task_matches_brute_classification(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(3, 36))
    e = random_edges(rng, n, int(rng.integers(n, 6 * n)))
    A = simple_adj(n, e)
    og = og_from_edges(n, e)
    rank = degree_rank(A)
    for p in sorted({1, 2, 3, min(5, n), n}):
        for mode in (oracle.CUT_BALANCED, oracle.CUT_UNIFORM):
            cuts = og.cuts(p, mode)
            tot, per, _ = og.tasks(p, cuts, threads=2)
            assert np.array_equal(per, brute_per_task(A, rank, cuts, p))
            assert tot == len(brute_triangles(A))


@pytest.mark.parametrize("seed", range(8))
def test_per_task_p_equals_n_closed_form(seed):
    """Singleton parts: task (i,j,k) counts A_ij A_jk A_ik in rank space for
    i<j<k; any repeated index has no internal edge, so it counts 0."""
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(3, 24))
    e = random_edges(rng, n, int(rng.integers(n, 5 * n)))
    A = simple_adj(n, e)
    og = og_from_edges(n, e)
    rank = og.rank()
    R = np.zeros_like(A)
    R[np.ix_(rank, rank)] = A  # R[rank x, rank y] = A[x, y]
    _, per, _ = og.tasks(n, np.arange(n + 1, dtype=np.int32))
    tl = oracle.task_list(n)
    for t, (i, j, k) in enumerate(tl):
        want = int(R[i, j] and R[j, k] and R[i, k]) if i < j < k else 0
        assert per[t] == want


def test_per_task_hand_example():
    """A 6-vertex graph worked by hand (triangles listed explicitly)."""
    # triangles: {0,1,2}, {2,3,4}, {0,2,4}; extra edge 4-5
    es = [(0, 1), (1, 2), (0, 2), (2, 3), (3, 4), (2, 4), (0, 4), (4, 5)]
    og = og_from_edges(6, es)
    # degrees: 0:3 1:2 2:4 3:2 4:4 5:1 -> order 5,1,3,0,2,4 -> ranks
    assert list(og.rank()) == [3, 1, 4, 2, 5, 0]
    cuts = np.array([0, 2, 4, 6], np.int32)  # parts {5,1} {3,0} {2,4}
    _, per, bn = og.tasks(3, cuts)
    idx = alg4_index(3)
    want = np.zeros(10, np.uint64)
    # {0,1,2} -> ranks {3,1,4} -> parts (0,1,2); {2,3,4} -> {4,2,5} -> (1,2,2);
    # {0,2,4} -> {3,4,5} -> (1,2,2)
    want[idx[(0, 1, 2)]] += 1
    want[idx[(1, 2, 2)]] += 2
    assert np.array_equal(per, want)
    # block nnz (a<=b row-major): edges in rank space
    # 0-1:(3,1) 1-2:(1,4) 0-2:(3,4) 2-3:(4,2) 3-4:(2,5) 2-4:(4,5) 0-4:(3,5) 4-5:(5,0)
    # parts: r0,r1 ->0 ; r2,r3 ->1 ; r4,r5 ->2
    # (1,3)->(0,1) (1,4)->(0,2) (3,4)->(1,2) (2,4)->(1,2) (2,5)->(1,2) (4,5)->(2,2) (3,5)->(1,2) (0,5)->(0,2)
    assert list(bn) == [0, 1, 2, 0, 4, 1]


# ------------------------------------------------------- task list
def test_task_list_matches_paper_example_and_table4():
    gold = json.load(open(GOLD))
    assert oracle.task_list(3).tolist() == gold["p3_tasks_in_order"]
    assert list(gold["p3_triangle_example"]["task"]) in oracle.task_list(3).tolist()
    for tiles, tasks in gold["table4_tiles_tasks"]:
        p = math.isqrt(tiles)
        assert p * p == tiles
        assert len(oracle.task_list(p)) == tasks == p * (p + 1) * (p + 2) // 6


@pytest.mark.parametrize("name,p", [("er2000", 4), ("rmat12", 16), ("rmat10", 5)])
def test_role_counted_block_nnz(name, p):
    """Each block (a,b) is G_ij in p-b tasks, G_jk in a+1, G_ik in b-a+1:
    p+2 role appearances, so the sum over tasks of the three block sizes is
    exactly (p+2)*m."""
    og = oracle.OracleGraph.from_graph(graphgen.workload(name))
    _, _, bn = og.tasks(p)
    bid, t = {}, 0
    for a in range(p):
        for b in range(a, p):
            bid[(a, b)] = t
            t += 1
    s = 0
    for i, j, k in oracle.task_list(p):
        s += int(bn[bid[(i, j)]] + bn[bid[(j, k)]] + bn[bid[(i, k)]])
    assert s == (p + 2) * og.m


def test_er_statistics_smoke():
    """Not parity: G(2000, 0.005) should land near C(n,3) p^3 ~ 166 triangles."""
    og = oracle.OracleGraph.from_graph(graphgen.workload("er2000"))
    assert 60 < og.total() < 320


@pytest.mark.parametrize("name", ["er2000", "rmat12"])
def test_total_rows_tiles_the_total(name):
    """Row-list counts (used for bounded CPU timing samples) over lists that
    partition the ranks add up to the total, and each equals the
    brute-force count of triangles whose lowest-ranked vertex is listed
    (checked on the 2000-vertex graph by dense enumeration over ranks)."""
    g = graphgen.workload(name)
    og = oracle.OracleGraph.from_graph(g)
    tot = og.total()
    rng = np.random.default_rng(3)
    lab = rng.integers(0, 4, size=og.n)
    lists = [np.nonzero(lab == c)[0] for c in range(4)]
    parts = [og.total_rows(r) for r in lists]
    assert sum(parts) == tot
    assert og.total_rows(np.zeros(0, np.int64)) == 0
    with pytest.raises(ValueError):
        og.total_rows([og.n])
    if name == "er2000":
        rank = og.rank()
        A = np.zeros((og.n, og.n), bool)
        u, v = g.edges()
        A[rank[u], rank[v]] = A[rank[v], rank[u]] = True
        low = np.zeros(og.n, np.int64)
        for a in range(og.n):
            nb = np.nonzero(A[a, a + 1:])[0] + a + 1
            for x in range(len(nb)):
                low[a] += int(A[nb[x], nb[x + 1:]].sum())
        for r, got in zip(lists, parts):
            assert got == int(low[r].sum())
