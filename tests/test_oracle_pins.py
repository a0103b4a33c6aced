"""Pins for the CPU oracle against facts that do not come from the oracle itself.

* brute force on every labelled simple graph with n <= 5 and random small
  multigraphs (distances by repeated relaxation over the raw edge list, the
  valid-parent sets enumerated);
* an independent library routine (scipy's unweighted shortest paths);
* closed forms (grids, paths, stars, complete graphs, isolated sources);
* the worked 6x6 block of Fig. 2 (tests/golden/fig2_block.json);
* BFS-tree invariants rejecting corrupted outputs;
* an emulated p_r x p_c grid whose merged block results must equal a
  whole-graph level;
* planted mistakes in copies of the oracle source that these pins must catch.
"""
import itertools
import json
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import graphgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- brute force
def brute_dist(n, edges, s):
    """Hop distances by n rounds of relaxation over an undirected edge list."""
    INF = 10 ** 9
    d = [INF] * n
    d[s] = 0
    for _ in range(n):
        for (u, v) in edges:
            if d[u] + 1 < d[v]:
                d[v] = d[u] + 1
            if d[v] + 1 < d[u]:
                d[u] = d[v] + 1
    return [x if x < INF else -1 for x in d]


def brute_parent_sets(n, edges, dist):
    ps = [set() for _ in range(n)]
    for (u, v) in edges:
        if u == v:
            continue
        if dist[u] >= 0 and dist[v] == dist[u] + 1:
            ps[v].add(u)
        if dist[v] >= 0 and dist[u] == dist[v] + 1:
            ps[u].add(v)
    return ps


def check_against_brute(orc, n, edges, s):
    src = np.array([e[0] for e in edges], np.int64)
    dst = np.array([e[1] for e in edges], np.int64)
    off, cols = graphgen.csr_from_edges(n, src, dst)
    dist = brute_dist(n, edges, s)
    ps = brute_parent_sets(n, edges, dist)
    parent, depth = orc.bfs(off, cols, s)
    assert depth.tolist() == dist
    pmin = orc.min_parent(off, cols, depth)
    pbu, dbu = orc.bfs_bottom_up(off, cols, s)
    assert dbu.tolist() == dist
    for v in range(n):
        if v == s:
            assert parent[v] == s and pmin[v] == s and pbu[v] == s
        elif dist[v] < 0:
            assert parent[v] == -1 and pmin[v] == -1 and pbu[v] == -1
        else:
            assert parent[v] in ps[v]
            assert pmin[v] == min(ps[v])
            assert pbu[v] == min(ps[v])  # first hit over a sorted row is the minimum
    assert orc.validate(off, cols, s, parent, depth)[0] == "ok"
    assert orc.validate(off, cols, s, pmin, depth)[0] == "ok"


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exhaustive_small_graphs(orc, n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        for s in range(n):
            check_against_brute(orc, n, edges, s)


def test_random_multigraphs_with_loops_and_duplicates(orc):
    rng = np.random.default_rng(11)
    for trial in range(120):
        n = int(rng.integers(1, 65))
        m = int(rng.integers(0, 3 * n + 1))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
        edges += edges[: m // 4]            # duplicates
        edges += [(0, 0)] if n else []      # a self-loop
        s = int(rng.integers(0, n))
        check_against_brute(orc, n, edges, s)


# ----------------------------------------------------------------- library routine
def test_against_scipy_shortest_paths(orc):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    for (off, cols) in [graphgen.kronecker(11, seed=5), graphgen.erdos_renyi(3000, 3.0, seed=4)]:
        n = off.size - 1
        A = csr_matrix((np.ones(cols.size), cols, off), shape=(n, n))
        srcs = graphgen.random_sources(off, 6, seed=9)
        D = shortest_path(A, unweighted=True, directed=True, indices=srcs)
        for i, s in enumerate(srcs):
            parent, depth = orc.bfs(off, cols, int(s))
            ref = np.where(np.isinf(D[i]), -1, D[i]).astype(np.int64)
            assert np.array_equal(depth.astype(np.int64), ref)
            assert orc.validate(off, cols, int(s), parent, depth)[0] == "ok"


# ----------------------------------------------------------------- closed forms
def grid_min_parent(H, W, r0, c0, v):
    r, c = divmod(v, W)
    if (r, c) == (r0, c0):
        return v
    if r > r0:
        return v - W
    if c > c0:
        return v - 1
    if c < c0:
        return v + 1
    return v + W


@pytest.mark.parametrize("H,W", [(1, 1), (1, 7), (6, 1), (4, 5), (7, 7)])
def test_grid_closed_form(orc, H, W):
    off, cols = graphgen.grid2d(H, W)
    for s in range(H * W):
        r0, c0 = divmod(s, W)
        pmin, depth = orc.bfs_min(off, cols, s)
        for v in range(H * W):
            r, c = divmod(v, W)
            assert depth[v] == abs(r - r0) + abs(c - c0)
            assert pmin[v] == grid_min_parent(H, W, r0, c0, v)


def test_path_star_complete_isolated(orc):
    n = 9
    # path 0-1-...-8
    off, cols = graphgen.csr_from_edges(n, np.arange(n - 1), np.arange(1, n))
    for s in range(n):
        pmin, depth = orc.bfs_min(off, cols, s)
        assert depth.tolist() == [abs(v - s) for v in range(n)]
        assert pmin.tolist() == [s if v == s else (v - 1 if v > s else v + 1) for v in range(n)]
    # star centred at 4
    leaves = [v for v in range(n) if v != 4]
    off, cols = graphgen.csr_from_edges(n, np.full(n - 1, 4), np.array(leaves))
    pmin, depth = orc.bfs_min(off, cols, 4)
    assert depth.tolist() == [0 if v == 4 else 1 for v in range(n)]
    assert pmin.tolist() == [4] * n
    pmin, depth = orc.bfs_min(off, cols, 0)
    assert depth.tolist() == [0 if v == 0 else (1 if v == 4 else 2) for v in range(n)]
    assert pmin.tolist() == [0 if v in (0, 4) else 4 for v in range(n)]
    # complete graph: everything at depth 1 with parent s
    src, dst = zip(*itertools.combinations(range(n), 2))
    off, cols = graphgen.csr_from_edges(n, np.array(src), np.array(dst))
    for s in range(n):
        parent, depth = orc.bfs(off, cols, s)
        assert depth.tolist() == [0 if v == s else 1 for v in range(n)]
        assert parent.tolist() == [s] * n
    # isolated source among other edges
    off, cols = graphgen.csr_from_edges(n, np.array([1, 2]), np.array([2, 3]))
    parent, depth = orc.bfs(off, cols, 7)
    assert depth.tolist() == [0 if v == 7 else -1 for v in range(n)]
    assert parent.tolist() == [7 if v == 7 else -1 for v in range(n)]


def test_bottom_up_scan_lengths_closed_form(orc):
    n = 8
    src, dst = zip(*itertools.combinations(range(n), 2))
    off, cols = graphgen.csr_from_edges(n, np.array(src), np.array(dst))
    for s in range(n):
        _, depth = orc.bfs(off, cols, s)
        scanned, unvisited = orc.bu_scan_lengths(off, cols, depth, 0)
        # row of v is [0..n-1] without v; s sits at index s if s < v else s-1
        assert unvisited == n - 1
        assert scanned == sum((s + 1) if s < v else s for v in range(n) if v != s)
        # level 1: nobody is left
        assert orc.bu_scan_lengths(off, cols, depth, 1) == (0, 0)
    # star from the centre: every leaf stops at its single entry
    off, cols = graphgen.csr_from_edges(n, np.zeros(n - 1, np.int64), np.arange(1, n))
    _, depth = orc.bfs(off, cols, 0)
    assert orc.bu_scan_lengths(off, cols, depth, 0) == (n - 1, n - 1)


# ----------------------------------------------------------------- heuristic
def test_level_stats_and_direction_schedule(orc):
    # path of 5 plus isolated vertex 5: levels {0},{1},{2},{3},{4} from s=0
    off, cols = graphgen.csr_from_edges(6, np.arange(4), np.arange(1, 5))
    _, depth = orc.bfs(off, cols, 0)
    n_f, m_f, m_u = orc.level_stats(off, depth)
    assert n_f.tolist() == [1, 1, 1, 1, 1]
    assert m_f.tolist() == [1, 2, 2, 2, 1]
    assert m_u.tolist() == [7, 5, 3, 1, 0]
    # special cases of the rule: a frontier with all remaining edges forces
    # bottom-up, a frontier of one vertex in a big graph forces top-down
    assert orc.direction_schedule(1000, [1, 500], [10, 100], [100000, 50], 15, 18).tolist() == [0, 1]
    assert orc.direction_schedule(1000, [1, 500, 1], [10, 100, 1], [100000, 50, 0], 15, 18).tolist() == [0, 1, 0]
    assert orc.direction_schedule(1000, [1, 500, 1], [10, 100, 1], [100000, 50, 0], 15, 18, mode=1).tolist() == [0, 0, 0]
    assert orc.direction_schedule(1000, [1, 500, 1], [10, 100, 1], [100000, 50, 0], 15, 18, mode=2).tolist() == [1, 1, 1]
    # the comparison is strict: m_f*alpha == m_u stays top-down
    assert orc.direction_schedule(1000, [1], [10], [150], 15, 18).tolist() == [0]
    assert orc.direction_schedule(18, [1, 1], [1000, 1], [1, 0], 15, 18).tolist() == [1, 1]


# ----------------------------------------------------------------- validator
def test_validator_rejects_corruptions(orc):
    off, cols = graphgen.grid2d(5, 6)
    s = 7
    parent, depth = orc.bfs(off, cols, s)
    assert orc.validate(off, cols, s, parent, depth)[0] == "ok"

    def bad(mut):
        p, d = parent.copy(), depth.copy()
        mut(p, d)
        return orc.validate(off, cols, s, p, d)[0]

    assert bad(lambda p, d: d.__setitem__(s, 1)) == "source"
    assert bad(lambda p, d: p.__setitem__(s, 0)) == "source"
    assert bad(lambda p, d: p.__setitem__(20, -1)) == "pairing"
    assert bad(lambda p, d: p.__setitem__(20, 999)) == "range"
    # depth one too large on a leaf-ish vertex: parent level check fires
    far = int(np.argmax(depth))
    assert bad(lambda p, d: d.__setitem__(far, d[far] + 1)) in ("parent_level", "skip")
    # parent that is not adjacent but at the right level
    v = int(np.flatnonzero(depth == 3)[0])
    cand = [u for u in np.flatnonzero(depth == 2) if u not in cols[off[v]:off[v + 1]]]
    assert bad(lambda p, d: p.__setitem__(v, cand[0])) == "not_edge"
    # two vertices that name each other (a cycle) cannot both be one level apart
    a = int(np.flatnonzero(depth == 2)[0])
    b = int(parent[a])
    assert bad(lambda p, d: p.__setitem__(b, a)) in ("parent_level", "not_edge")
    # dropping a reachable vertex from the tree
    leaf = int(np.flatnonzero(depth == depth.max())[0])
    assert bad(lambda p, d: (p.__setitem__(leaf, -1), d.__setitem__(leaf, -1))) == "leak"
    # an extra root
    assert bad(lambda p, d: (p.__setitem__(leaf, leaf), d.__setitem__(leaf, 0))) == "root"
    # a consistent parent chain that is not shortest: 4-cycle 0-1-2-3-0, vertex 3
    # hung below 2 at depth 3 although it is adjacent to the source
    off4, cols4 = graphgen.csr_from_edges(4, np.array([0, 1, 2, 3]), np.array([1, 2, 3, 0]))
    p4, d4 = orc.bfs(off4, cols4, 0)
    assert orc.validate(off4, cols4, 0, p4, d4)[0] == "ok"
    p4[3], d4[3] = 2, 3
    assert orc.validate(off4, cols4, 0, p4, d4)[0] == "skip"


# ----------------------------------------------------------------- Fig. 2 block
def _fig2():
    with open(os.path.join(GOLDEN, "fig2_block.json")) as f:
        return json.load(f)


def test_fig2_block_builder():
    g = _fig2()
    ent = np.array(g["entries_row_col"], np.int64)
    blk = graphgen.coo_block(6, 6, ent[:, 0], ent[:, 1])
    for k in ("jc", "cp", "ir"):
        assert blk[k].tolist() == g["dcsc_full"][k]
    top = ent[ent[:, 0] < 3]
    blk = graphgen.coo_block(3, 6, top[:, 0], top[:, 1])
    for k in ("jc", "cp", "ir"):
        assert blk[k].tolist() == g["dcsc_rows_0_2"][k]
    bot = ent[ent[:, 0] >= 3]
    blk = graphgen.coo_block(3, 6, bot[:, 0] - 3, bot[:, 1])
    exp = g["dcsc_rows_3_5_global_rows"]
    assert blk["jc"].tolist() == exp["jc"] and blk["cp"].tolist() == exp["cp"]
    assert (blk["ir"] + 3).tolist() == exp["ir"]
    # the row-major copy lists each row's columns in ascending order
    assert blk["jr"].tolist() == [0, 1, 2] and blk["rp"].tolist() == [0, 3, 4, 5]
    assert blk["ic"].tolist() == [0, 2, 3, 1, 2]


def test_fig2_block_td_bu(orc):
    g = _fig2()
    ent = np.array(g["entries_row_col"], np.int32)
    rows, par = orc.block_td(6, 6, ent[:, 0], ent[:, 1], 0, np.array(g["td_frontier"], np.int32))
    assert list(zip(rows.tolist(), par.tolist())) == [tuple(x) for x in g["td_expected_row_parent"]]
    fb = graphgen.bits_to_words([i in g["bu_frontier"] for i in range(6)])
    comp = np.zeros(1, np.uint64)
    rows, par, comp2 = orc.block_bu(6, 6, ent[:, 0], ent[:, 1], 0, fb, comp, 0, 6)
    assert list(zip(rows.tolist(), par.tolist())) == [tuple(x) for x in g["bu_expected_row_parent"]]
    assert np.flatnonzero(graphgen.words_to_bits(comp2, 6)).tolist() == g["bu_expected_completed_rows"]
    # completed rows are skipped, column base shifts parents, row window limits the sweep
    comp = graphgen.bits_to_words([i in (1, 4) for i in range(6)])
    rows, par, _ = orc.block_bu(6, 6, ent[:, 0], ent[:, 1], 100, fb, comp, 0, 5)
    assert list(zip(rows.tolist(), par.tolist())) == [(3, 102)]


# ----------------------------------------------------------------- emulated 2D grid
@pytest.mark.parametrize("pr,pc", [(1, 1), (2, 2), (4, 4), (2, 8), (8, 2)])
def test_emulated_2d_grid_matches_whole_graph_level(orc, pr, pc):
    off, cols = graphgen.kronecker(9, seed=3)
    n = off.size - 1
    s = int(graphgen.random_sources(off, 1, seed=4)[0])
    _, depth = orc.bfs(off, cols, s)
    pmin = orc.min_parent(off, cols, depth)
    R, C = n // pr, n // pc
    rowsz = np.repeat(np.arange(n), np.diff(off))
    for d in range(int(depth.max())):
        frontier = np.flatnonzero(depth == d)
        visited = depth.copy()
        visited_mask = (visited >= 0) & (visited <= d)
        # top-down: every block discovers, rows min-merge, then the local update keeps unvisited rows
        best = np.full(n, np.iinfo(np.int64).max)
        for i in range(pr):
            for j in range(pc):
                sel = (rowsz >= i * R) & (rowsz < (i + 1) * R) & (cols >= j * C) & (cols < (j + 1) * C)
                fl = frontier[(frontier >= j * C) & (frontier < (j + 1) * C)] - j * C
                r, p = orc.block_td(R, C, rowsz[sel] - i * R, cols[sel] - j * C, j * C, fl.astype(np.int32))
                np.minimum.at(best, r + i * R, p.astype(np.int64))
        new = (best != np.iinfo(np.int64).max) & ~visited_mask
        assert np.array_equal(np.flatnonzero(new), np.flatnonzero(depth == d + 1))
        assert np.array_equal(best[new], pmin[new])
        # bottom-up: sub-steps sweep column blocks in order 0..pc-1 with a shared completed bitmap
        par = np.full(n, -1, np.int64)
        for i in range(pr):
            comp = graphgen.bits_to_words(visited_mask[i * R:(i + 1) * R])
            for j in range(pc):
                sel = (rowsz >= i * R) & (rowsz < (i + 1) * R) & (cols >= j * C) & (cols < (j + 1) * C)
                fb = graphgen.bits_to_words((depth == d)[j * C:(j + 1) * C])
                r, p, comp = orc.block_bu(R, C, rowsz[sel] - i * R, cols[sel] - j * C, j * C, fb, comp, 0, R)
                par[r + i * R] = p
        found = par >= 0
        assert np.array_equal(np.flatnonzero(found), np.flatnonzero(depth == d + 1))
        assert np.array_equal(par[found], pmin[found])


# ----------------------------------------------------------------- planted mistakes
MUTANTS = [
    ("depth[v] = depth[u] + 1;", "depth[v] = depth[u] + 1 + (v == 3);", "exhaustive"),
    ("parent_min[v] > (int32_t)u", "parent_min[v] < (int32_t)u", "exhaustive"),
    ("                    break;\n                }\n            }\n        }\n        unsigned char* t",
     "                }\n            }\n        }\n        unsigned char* t", "exhaustive"),
    ("if (inf[ecol[e]] && col_base + ecol[e] < best[erow[e]])", "if (inf[ecol[e]] && col_base + ecol[e] > best[erow[e]] - 1)", "fig2"),
    ("if ((completed[r >> 6] >> (r & 63)) & 1ULL) continue;", "", "fig2"),
    ("if (parent[v] == (int32_t)u) edge_ok[v] = 1;", "edge_ok[v] = 1;", "validator"),
    ("if (depth[v] > depth[u] + 1) { *bad_vertex = v; code = V_SKIP; break; }", "", "validator"),
]


@pytest.mark.parametrize("old,new,pin", MUTANTS)
def test_pins_catch_planted_mistakes(orc, old, new, pin):
    import oracle
    src = open(oracle._SRC).read()
    assert old in src, old
    tmpd = tempfile.mkdtemp()
    try:
        path = os.path.join(tmpd, "bfs_oracle.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new, 1))
        so = os.path.join(tmpd, "libmut.so")
        subprocess.run(["gcc", "-O2", "-shared", "-fPIC", "-o", so, path], check=True)
        mut = oracle.load(so)
        caught = False
        try:
            if pin == "exhaustive":
                for n in (4, 5):
                    pairs = list(itertools.combinations(range(n), 2))
                    for mask in range(0, 1 << len(pairs), 3):
                        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
                        for s in range(n):
                            check_against_brute(mut, n, edges, s)
            elif pin == "fig2":
                test_fig2_block_td_bu(mut)
            elif pin == "validator":
                test_validator_rejects_corruptions(mut)
        except AssertionError:
            caught = True
        assert caught, f"planted mistake not caught: {old!r} -> {new!r}"
    finally:
        shutil.rmtree(tmpd)
