"""GPU parity: bfs_run (through the C ABI) against the CPU oracle.

Depths must be bit-exact, minimum-id parents bit-exact, and ANY-mode parents
must pass the BFS-tree invariants.  Cases cover several tiles and ragged
tails, every direction policy, forced switch schedules, int32 and int64
offsets, degenerate graphs, and error paths.
"""
import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1705_04590_amd as bfs  # noqa: E402

DEV = torch.device("cuda:0")
SYM = bfs.BFS_GRAPH_SYMMETRIC | bfs.BFS_GRAPH_SORTED | bfs.BFS_GRAPH_VALIDATE


class DevGraph:
    def __init__(self, off, cols, off_dtype=np.int64, flags=SYM):
        self.off, self.cols = off, cols
        self.n = off.size - 1
        self.d_off = torch.from_numpy(np.ascontiguousarray(off.astype(off_dtype))).to(DEV)
        self.d_cols = torch.from_numpy(np.ascontiguousarray(cols)).to(DEV)
        self.g = bfs.bfs_create_graph_csr(self.d_off, self.d_cols, flags)
        self.ws = bfs.workspace(self.g, 1, DEV)
        self.parent = torch.empty(max(self.n, 1), dtype=torch.int32, device=DEV)
        self.depth = torch.empty(max(self.n, 1), dtype=torch.int32, device=DEV)

    def run(self, s, **kw):
        # the level-by-level kernels unless a test asks for the fused search
        # (which small graphs take by default; its own tests below)
        kw.setdefault("fused_max_n", -1)
        # poison the outputs: every entry must be written by the call itself
        self.parent.fill_(-7)
        self.depth.fill_(-7)
        st = bfs.bfs_run(self.g, int(s), self.parent, self.depth, self.ws, bfs.bfs_opts_default(**kw))
        torch.cuda.synchronize()
        return self.parent[: self.n].cpu().numpy(), self.depth[: self.n].cpu().numpy(), st


def check(orc, dg, s, p, d, min_mode, ref=None):
    ref_p, ref_d = ref if ref is not None else orc.bfs_min(dg.off, dg.cols, int(s))
    assert np.array_equal(d, ref_d), f"depth mismatch at {np.flatnonzero(d != ref_d)[:8]}"
    if min_mode:
        bad = np.flatnonzero(p != ref_p)
        assert bad.size == 0, f"min parent mismatch at {bad[:8]}: {p[bad[:8]]} vs {ref_p[bad[:8]]}"
    else:
        res = orc.validate(dg.off, dg.cols, int(s), p, d)
        assert res[0] == "ok", res


def path_graph(n):
    return graphgen.csr_from_edges(n, np.arange(n - 1), np.arange(1, n))


def star_graph(n):
    return graphgen.csr_from_edges(n, np.zeros(n - 1, np.int64), np.arange(1, n))


def complete_graph(n):
    import itertools
    a, b = zip(*itertools.combinations(range(n), 2))
    return graphgen.csr_from_edges(n, np.array(a), np.array(b))


def two_pieces():
    # a Kronecker piece plus a separate path; some isolated vertices
    off, cols = graphgen.kronecker(9, seed=8)
    n1 = off.size - 1
    src = np.repeat(np.arange(n1), np.diff(off))
    keep = src < cols
    a = np.concatenate([src[keep], n1 + np.arange(99)])
    b = np.concatenate([cols[keep], n1 + np.arange(1, 100)])
    return graphgen.csr_from_edges(n1 + 120, a, b)


CASES = {
    "kron8": lambda: graphgen.kronecker(8, seed=3),
    "kron12": lambda: graphgen.kronecker(12, seed=1),
    "kron14": lambda: graphgen.kronecker(14, seed=2),
    "er": lambda: graphgen.erdos_renyi(6000, 2.5, seed=4),
    "grid": lambda: graphgen.grid2d(37, 53),
    "path": lambda: path_graph(3000),
    "star": lambda: star_graph(5000),
    "complete": lambda: complete_graph(80),
    "pieces": two_pieces,
}


@pytest.fixture(scope="module")
def graphs():
    return {}


def get(graphs, name, off_dtype=np.int64):
    key = (name, off_dtype)
    if key not in graphs:
        off, cols = CASES[name]()
        graphs[key] = DevGraph(off, cols, off_dtype)
    return graphs[key]


def sources_for(off, k=3, seed=5):
    srcs = list(graphgen.random_sources(off, k, seed=seed))
    deg = np.diff(off)
    iso = np.flatnonzero(deg == 0)
    if iso.size:
        srcs.append(int(iso[0]))
    return srcs


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("direction", ["DO", "TD", "BU"])
def test_parity_all_modes(orc, graphs, name, direction):
    dirv = {"DO": bfs.BFS_DIR_DO, "TD": bfs.BFS_DIR_TD, "BU": bfs.BFS_DIR_BU}[direction]
    for off_dtype in (np.int32, np.int64):
        dg = get(graphs, name, off_dtype)
        for s in sources_for(dg.off):
            ref = orc.bfs_min(dg.off, dg.cols, int(s))
            for pm, claim, head, pre in ((bfs.BFS_PARENT_ANY, 0, 0, 0), (bfs.BFS_PARENT_ANY, 1, 0, 0),
                                         (bfs.BFS_PARENT_ANY, 0, 1, 0), (bfs.BFS_PARENT_ANY, 0, 2, 0),
                                         (bfs.BFS_PARENT_ANY, 0, 3, 0), (bfs.BFS_PARENT_MIN, 0, 0, 0),
                                         (bfs.BFS_PARENT_MIN, 0, 3, 0), (bfs.BFS_PARENT_ANY, 0, 0, 1),
                                         (bfs.BFS_PARENT_ANY, 0, 2, 1), (bfs.BFS_PARENT_MIN, 0, 0, 1)):
                # pre = 1: every top-down level with an edge runs the hub
                # pre-pass (engine off, so the small levels do too)
                p, d, st = dg.run(s, dir=dirv, parent_mode=pm, td_claim=claim, bu_head=head, td_prepass=pre,
                                  small_edges=-1 if pre else 0)
                check(orc, dg, s, p, d, pm == bfs.BFS_PARENT_MIN, ref)
                assert st.reached == int((d >= 0).sum())
                assert st.isolated == int((np.diff(dg.off) == 0).sum())
                # per-level counts depend on the depths only, in every mode
                n_f, m_f, m_u = orc.level_stats(dg.off, ref[1])
                L = min(len(n_f), bfs.STATS_MAX_LEVELS)
                assert st.levels == len(n_f)
                assert list(st.level_nf[:L]) == n_f[:L].tolist()
                assert list(st.level_mf[:L]) == m_f[:L].tolist()
                assert list(st.level_mu[:L]) == m_u[:L].tolist()


@pytest.mark.parametrize("name", ["kron12", "kron14", "grid", "pieces"])
def test_direction_schedule_and_counters_match_oracle(orc, graphs, name):
    dg = get(graphs, name)
    for s in sources_for(dg.off, k=3, seed=11)[:3]:
        for alpha, beta in ((15.0, 18.0), (1e9, 18.0), (15.0, 1e-9), (1e9, 1e9), (2.0, 50.0)):
            p, d, st = dg.run(s, alpha=alpha, beta=beta, parent_mode=bfs.BFS_PARENT_MIN)
            check(orc, dg, s, p, d, True)
            n_f, m_f, m_u = orc.level_stats(dg.off, d)
            sched = orc.direction_schedule(dg.n, n_f, m_f, m_u, alpha, beta)
            L = min(len(n_f), bfs.STATS_MAX_LEVELS)
            # the search expands every level once, the last one finding nothing
            assert st.levels == len(n_f)
            assert list(st.level_dir[:L]) == sched[:L].tolist()
            assert list(st.level_nf[:L]) == n_f[:L].tolist()
            assert list(st.level_mf[:L]) == m_f[:L].tolist()
            assert list(st.level_mu[:L]) == m_u[:L].tolist()
            for lv in range(L):
                if st.level_dir[lv] == 1:
                    scanned, unvisited = orc.bu_scan_lengths(dg.off, dg.cols, d, lv)
                    assert st.level_examined[lv] == scanned
                    assert st.level_unvisited[lv] == unvisited
                else:
                    assert st.level_examined[lv] == m_f[lv]


def test_config1_scale16_int32_offsets(orc, graphs):
    """Kronecker scale 16, int32 CSR, 16 sources, top-down and direction-optimizing, CAS and MIN."""
    off, cols = graphgen.kronecker(16, seed=1)
    dg = DevGraph(off, cols, np.int32)
    for s in graphgen.random_sources(off, 16, seed=2):
        ref = orc.bfs_min(off, cols, int(s))
        for dirv in (bfs.BFS_DIR_TD, bfs.BFS_DIR_DO):
            for pm in (bfs.BFS_PARENT_ANY, bfs.BFS_PARENT_MIN):
                p, d, _ = dg.run(s, dir=dirv, parent_mode=pm)
                check(orc, dg, s, p, d, pm == bfs.BFS_PARENT_MIN, ref)
        # hub-rank heads: some neighbours are hubs (LDS bits), others are not
        for head in (2, 3):
            p, d, _ = dg.run(s, parent_mode=bfs.BFS_PARENT_ANY, bu_head=head)
            check(orc, dg, s, p, d, False, ref)
        p, d, _ = dg.run(s, parent_mode=bfs.BFS_PARENT_ANY, td_prepass=1, small_edges=-1)
        check(orc, dg, s, p, d, False, ref)


@pytest.mark.parametrize("name", ["kron12", "kron14", "er", "grid", "pieces", "path", "star"])
@pytest.mark.parametrize("segments", [1, 2, 4, 8])
def test_column_blocked_bottom_up(orc, graphs, name, segments):
    """bu_segments = S: the bottom-up sweep probes the row heads, then S
    sub-steps scan the remaining rows one column segment at a time in
    ascending order (Alg. 4's sub-steps inside one device).  Minimum parents
    stay exact and the entries examined equal the oracle's row-order
    first-hit scan; any-parent searches (hub heads, lazy -1 fill) pass the
    tree check."""
    for off_dtype in (np.int32, np.int64):
        dg = get(graphs, name, off_dtype)
        for s in sources_for(dg.off, k=2, seed=41):
            ref = orc.bfs_min(dg.off, dg.cols, int(s))
            for dirv in (bfs.BFS_DIR_BU, bfs.BFS_DIR_DO):
                p, d, st = dg.run(s, dir=dirv, parent_mode=bfs.BFS_PARENT_MIN, bu_segments=segments)
                check(orc, dg, s, p, d, True, ref)
                for lv in range(min(st.levels, bfs.STATS_MAX_LEVELS)):
                    if st.level_dir[lv] == 1:
                        assert st.level_examined[lv] == orc.bu_scan_lengths(dg.off, dg.cols, d, lv)[0]
                for head in (0, 1, 2, 3):
                    p, d, st = dg.run(s, dir=dirv, bu_head=head, bu_serial=4, bu_segments=segments)
                    check(orc, dg, s, p, d, False, ref)
        # a 64-entry serial limit and 1-entry one (the wave scans the rest)
        s = sources_for(dg.off, k=1, seed=43)[0]
        ref = orc.bfs_min(dg.off, dg.cols, int(s))
        for serial in (1, 64):
            p, d, _ = dg.run(s, dir=bfs.BFS_DIR_BU, parent_mode=bfs.BFS_PARENT_MIN, bu_serial=serial,
                             bu_segments=segments)
            check(orc, dg, s, p, d, True, ref)


@pytest.mark.parametrize("name", ["kron12", "kron14", "er", "grid", "pieces", "complete"])
@pytest.mark.parametrize("segments", [1, 2, 4, 8])
def test_column_blocked_top_down(orc, graphs, name, segments):
    """td_segments = S: a top-down level is expanded in S passes, one per
    column segment in ascending order, each over the frontier's entries in
    its id range (found by binary search in the sorted rows).  Every claim
    mode gives the oracle's depths, minimum parents exactly, and the same
    per-level schedule and counts."""
    for off_dtype in (np.int32, np.int64):
        dg = get(graphs, name, off_dtype)
        for s in sources_for(dg.off, k=2, seed=51):
            ref = orc.bfs_min(dg.off, dg.cols, int(s))
            n_f, m_f, _ = orc.level_stats(dg.off, ref[1])
            for dirv in (bfs.BFS_DIR_TD, bfs.BFS_DIR_DO):
                for pm, claim in ((bfs.BFS_PARENT_MIN, 0), (bfs.BFS_PARENT_ANY, 0), (bfs.BFS_PARENT_ANY, 1),
                                  (bfs.BFS_PARENT_ANY, 2)):
                    p, d, st = dg.run(s, dir=dirv, parent_mode=pm, td_claim=claim, td_segments=segments,
                                      td_seg_edges=1, small_edges=-1)
                    check(orc, dg, s, p, d, pm == bfs.BFS_PARENT_MIN, ref)
                    L = min(st.levels, bfs.STATS_MAX_LEVELS)
                    assert list(st.level_nf[:L]) == n_f[:L].tolist()
                    assert list(st.level_mf[:L]) == m_f[:L].tolist()


def test_column_blocked_bad_segment_count():
    off, cols = path_graph(100)
    dg = DevGraph(off, cols)
    with pytest.raises(bfs.BfsError) as e:
        dg.run(0, bu_segments=9)
    assert e.value.status == 1
    with pytest.raises(bfs.BfsError) as e:
        dg.run(0, td_segments=9)
    assert e.value.status == 1
    # segments are sub-ranges of sorted rows
    uns = DevGraph(off, cols, flags=bfs.BFS_GRAPH_SYMMETRIC)
    for kw in (dict(bu_segments=2), dict(td_segments=2)):
        with pytest.raises(bfs.BfsError) as e:
            uns.run(0, **kw)
        assert e.value.status == 8


@pytest.mark.parametrize("name", ["kron12", "kron14", "er", "grid", "pieces", "star", "complete"])
def test_benign_race_top_down(orc, graphs, name):
    """td_claim = 2: children are taken with no atomic test (the benign race
    of Section 5.2), so several threads may take the same child.  Depths stay
    exact and parents valid; the next frontier comes from the level's merge,
    so the per-level frontier sizes and edge counts, and the direction
    schedule, equal the oracle's; the repeated takes are counted and never
    exceed the takes."""
    for off_dtype in (np.int32, np.int64):
        dg = get(graphs, name, off_dtype)
        for s in sources_for(dg.off):
            ref = orc.bfs_min(dg.off, dg.cols, int(s))
            n_f, m_f, _ = orc.level_stats(dg.off, ref[1])
            for kw in (dict(dir=bfs.BFS_DIR_TD), dict(dir=bfs.BFS_DIR_TD, small_edges=-1),
                       dict(dir=bfs.BFS_DIR_DO), dict(dir=bfs.BFS_DIR_DO, small_edges=-1, td_prepass=1),
                       dict(dir=bfs.BFS_DIR_DO, alpha=1e9, beta=1e9, small_edges=-1)):
                p, d, st = dg.run(s, td_claim=2, **kw)
                check(orc, dg, s, p, d, False, ref)
                L = min(st.levels, bfs.STATS_MAX_LEVELS)
                assert st.levels == len(n_f)
                assert list(st.level_nf[:L]) == n_f[:L].tolist()
                assert list(st.level_mf[:L]) == m_f[:L].tolist()
                assert 0 <= st.td_duplicates <= st.td_claims
                if kw.get("small_edges") == -1 and kw["dir"] == bfs.BFS_DIR_TD:
                    # every level after the source's goes through the expansion
                    assert st.td_claims - st.td_duplicates == int((d > 0).sum())


def test_tuning_knobs_do_not_change_results(orc, graphs):
    dg = get(graphs, "kron14")
    s = int(graphgen.random_sources(dg.off, 1, seed=3)[0])
    ref = orc.bfs_min(dg.off, dg.cols, s)
    for serial in (1, 4, 16, 64, 1 << 20):
        for grid in (1, 7, 64, 4096):
            p, d, _ = dg.run(s, parent_mode=bfs.BFS_PARENT_MIN, bu_serial=serial, grid_blocks=grid)
            check(orc, dg, s, p, d, True, ref)


@pytest.mark.parametrize("name", ["kron14", "er", "pieces", "grid"])
def test_shape_knobs_do_not_change_results(orc, graphs, name):
    """Workgroup and tile shapes (td_block, bu_block, bu_group) are tuning
    only: minimum parents and depths stay the oracle's, any-parent trees stay
    valid, and the per-level counts stay the oracle's."""
    dg = get(graphs, name)
    s = int(graphgen.random_sources(dg.off, 1, seed=13)[0])
    ref = orc.bfs_min(dg.off, dg.cols, s)
    n_f, m_f, _ = orc.level_stats(dg.off, ref[1])
    runs = [dict(dir=bfs.BFS_DIR_TD, td_block=b, parent_mode=pm, td_claim=c)
            for b in (128, 256, 512) for pm, c in ((bfs.BFS_PARENT_MIN, 0), (bfs.BFS_PARENT_ANY, 0),
                                                   (bfs.BFS_PARENT_ANY, 2))]
    runs += [dict(dir=dv, bu_block=b, bu_group=gw, parent_mode=pm)
             for dv in (bfs.BFS_DIR_BU, bfs.BFS_DIR_DO) for b in (128, 256, 512) for gw in (0, 1, 8, 64)
             for pm in (bfs.BFS_PARENT_MIN, bfs.BFS_PARENT_ANY)]
    runs += [dict(td_block=b, bu_block=bb, grid_blocks=gb) for b in (128, 512) for bb in (128, 512)
             for gb in (7, 1024)]
    for kw in runs:
        p, d, st = dg.run(s, **kw)
        check(orc, dg, s, p, d, kw.get("parent_mode") == bfs.BFS_PARENT_MIN, ref)
        L = min(st.levels, bfs.STATS_MAX_LEVELS)
        assert list(st.level_nf[:L]) == n_f[:L].tolist(), kw
        assert list(st.level_mf[:L]) == m_f[:L].tolist(), kw


def test_shape_knob_errors():
    off, cols = path_graph(100)
    dg = DevGraph(off, cols)
    for kw in (dict(td_block=64), dict(td_block=1024), dict(bu_block=192), dict(bu_group=3), dict(bu_group=128),
               dict(bu_group=-1)):
        with pytest.raises(bfs.BfsError) as e:
            dg.run(0, **kw)
        assert e.value.status == 1, kw


FUSED = bfs.KERNEL_KINDS.index("fused")


@pytest.mark.parametrize("name", list(CASES))
def test_fused_search_parity(orc, graphs, name):
    """The whole search in one persistent launch (fused_max_n): oracle depths,
    minimum parents exactly, valid any-parent trees, and the oracle's level
    schedule and counts (frontier size and edges, unvisited vertices and
    edges, bottom-up entries examined in row order), in every direction
    policy, from isolated sources too, with 1 to 64 workgroups."""
    for off_dtype in (np.int32, np.int64):
        dg = get(graphs, name, off_dtype)
        for s in sources_for(dg.off, k=2, seed=71):
            ref = orc.bfs_min(dg.off, dg.cols, int(s))
            n_f, m_f, m_u = orc.level_stats(dg.off, ref[1])
            for dirv, alpha, beta in ((bfs.BFS_DIR_DO, 15.0, 18.0), (bfs.BFS_DIR_TD, 15.0, 18.0),
                                      (bfs.BFS_DIR_BU, 15.0, 18.0), (bfs.BFS_DIR_DO, 2.0, 50.0),
                                      (bfs.BFS_DIR_DO, 1e9, 1e9)):
                for pm in (bfs.BFS_PARENT_MIN, bfs.BFS_PARENT_ANY):
                    for groups in (0, 1, 3):
                        p, d, st = dg.run(s, dir=dirv, alpha=alpha, beta=beta, parent_mode=pm,
                                          fused_max_n=1 << 30, persist_groups=groups)
                        assert st.launches[FUSED] == 1 and st.launches[bfs.KERNEL_KINDS.index("bu_sweep")] == 0
                        check(orc, dg, s, p, d, pm == bfs.BFS_PARENT_MIN, ref)
                        assert st.levels == len(n_f) and st.fill_level == -1
                        assert st.reached == int((d >= 0).sum())
                        L = min(st.levels, bfs.STATS_MAX_LEVELS)
                        if dirv == bfs.BFS_DIR_DO:
                            sched = orc.direction_schedule(dg.n, n_f, m_f, m_u, alpha, beta)
                        else:
                            sched = np.full(len(n_f), 1 if dirv == bfs.BFS_DIR_BU else 0)
                        assert list(st.level_dir[:L]) == sched[:L].tolist()
                        assert list(st.level_nf[:L]) == n_f[:L].tolist()
                        assert list(st.level_mf[:L]) == m_f[:L].tolist()
                        assert list(st.level_mu[:L]) == m_u[:L].tolist()
                        assert st.td_levels + st.bu_levels == L
                        for lv in range(L):
                            if st.level_dir[lv] == 1:
                                scanned, unvisited = orc.bu_scan_lengths(dg.off, dg.cols, d, lv)
                                assert st.level_examined[lv] == scanned
                                assert st.level_unvisited[lv] == unvisited
                            else:
                                assert st.level_examined[lv] == m_f[lv]


def test_fused_search_selection(orc, graphs):
    """The fused search is the default up to 2^18 vertices (not for top-down
    only, unless a size limit is given) and is not used when switched off,
    above the size limit, or with knobs it does not take (CAS or benign
    claims, explicit heads, pre-pass, column segments)."""
    dg = get(graphs, "kron12")
    s = int(graphgen.random_sources(dg.off, 1, seed=5)[0])
    ref = orc.bfs_min(dg.off, dg.cols, s)
    for kw in (dict(fused_max_n=0), dict(fused_max_n=0, dir=bfs.BFS_DIR_BU), dict(fused_max_n=dg.n, dir=bfs.BFS_DIR_TD)):
        _, _, st = dg.run(s, **kw)
        assert st.launches[FUSED] == 1, kw
    for kw in (dict(fused_max_n=-1), dict(fused_max_n=dg.n - 1), dict(td_claim=1), dict(td_claim=2),
               dict(bu_head=2), dict(td_prepass=1), dict(bu_segments=2), dict(td_segments=2),
               dict(dir=bfs.BFS_DIR_TD)):
        p, d, st = dg.run(s, **dict(dict(fused_max_n=0), **kw))
        assert st.launches[FUSED] == 0, kw
        check(orc, dg, s, p, d, False, ref)
    _, _, st = dg.run(s, fused_max_n=dg.n)
    assert st.launches[FUSED] == 1


@pytest.mark.parametrize("name", ["kron12", "kron14", "er"])
def test_deferred_depths_reach_the_hub_prepass(orc, graphs, name):
    """Any-parent fetch-or searches leave a top-down level's depths to the next
    level until the outputs are filled. Here the next level is a top-down level
    heavy enough for the hub pre-pass, whose fill must write them: top-down
    only (alpha ~ 0), engine off, and a pre-pass threshold that the first
    level with more frontier edges than the level before reaches."""
    for off_dtype in (np.int32, np.int64):
        dg = get(graphs, name, off_dtype)
        for s in sources_for(dg.off, k=2, seed=51)[:2]:
            ref = orc.bfs_min(dg.off, dg.cols, int(s))
            n_f, m_f, _ = orc.level_stats(dg.off, ref[1])
            # the heaviest level, when some top-down level with edges runs
            # before it: the levels before leave their depths to the next one
            # (through the queue), and its pre-pass is the first to fill
            grow = [lv for lv in range(1, len(m_f)) if m_f[lv - 1] > 0 and m_f[lv] > m_f[:lv].max()]
            if not grow:
                continue
            lv = grow[-1]
            p, d, st = dg.run(s, alpha=1e-9, small_edges=-1, td_prepass=int(m_f[lv]))
            check(orc, dg, s, p, d, False, ref)
            assert st.bu_levels == 0 and st.fill_level == lv
            # and with no pre-pass at all: every level's depths come from the
            # next level's queue, and a pass after the last level fills the -1
            p, d, st = dg.run(s, alpha=1e-9, small_edges=-1, td_prepass=-1)
            check(orc, dg, s, p, d, False, ref)
            assert st.bu_levels == 0 and st.fill_level == -2


@pytest.mark.parametrize("name", ["kron12", "pieces", "grid", "path"])
def test_outputs_fully_written(orc, graphs, name):
    """Every parent/depth entry is written by the call, whatever the level
    schedule: searches with and without bottom-up levels, isolated sources,
    the default any-parent mode (whose -1 fill happens inside the first
    bottom-up sweep or in a final pass) and the modes that initialise first."""
    for off_dtype in (np.int32, np.int64):
        dg = get(graphs, name, off_dtype)
        for s in sources_for(dg.off, k=2, seed=31):
            ref = orc.bfs_min(dg.off, dg.cols, int(s))
            for kw in (dict(), dict(dir=bfs.BFS_DIR_BU), dict(dir=bfs.BFS_DIR_TD), dict(alpha=1e-9),
                       dict(alpha=1e9, beta=1e9), dict(small_edges=-1), dict(td_claim=1), dict(td_claim=2),
                       dict(parent_mode=bfs.BFS_PARENT_MIN), dict(td_prepass=1, small_edges=-1),
                       dict(td_prepass=1, small_edges=-1, alpha=1e9, beta=1e9)):
                p, d, st = dg.run(s, **kw)
                check(orc, dg, s, p, d, kw.get("parent_mode") == bfs.BFS_PARENT_MIN, ref)
                assert (p >= -1).all() and (d >= -1).all()
                # who wrote the -1 fill: initialisation (-1) in the modes that
                # compare against it, else the first bottom-up sweep or top-down
                # pre-pass, else a pass after the last level (-2)
                L = min(st.levels, bfs.STATS_MAX_LEVELS)
                eager = kw.get("parent_mode") == bfs.BFS_PARENT_MIN or kw.get("td_claim") == 1 or \
                    kw.get("dir") == bfs.BFS_DIR_TD
                if eager:
                    assert st.fill_level == -1
                elif st.fill_level >= bfs.STATS_MAX_LEVELS:
                    assert st.fill_level < st.levels   # past the recorded levels
                elif st.fill_level >= 0:
                    first_bu = [x for x in range(L) if st.level_dir[x] == 1]
                    assert st.level_dir[st.fill_level] == 1 or kw.get("td_prepass")
                    if not kw.get("td_prepass"):
                        assert st.fill_level == first_bu[0]
                else:
                    assert st.fill_level == -2 and st.bu_levels == 0


def test_uniform_degree_graph_has_no_hubs(orc):
    """A 300 x 300 grid: over 65 535 vertices share the top degree, so no hub
    threshold exists and the hub-ranked modes fall back to the plain heads."""
    off, cols = graphgen.grid2d(300, 300)
    dg = DevGraph(off, cols, np.int32)
    for s in (0, 45150, 89999):
        ref = orc.bfs_min(off, cols, s)
        for kw in (dict(bu_head=3), dict(bu_head=0), dict(td_prepass=1, small_edges=-1),
                   dict(parent_mode=bfs.BFS_PARENT_MIN)):
            p, d, _ = dg.run(s, **kw)
            check(orc, dg, s, p, d, kw.get("parent_mode") == bfs.BFS_PARENT_MIN, ref)


def test_repeat_runs_identical(graphs):
    dg = get(graphs, "kron14")
    s = int(graphgen.random_sources(dg.off, 1, seed=9)[0])
    p0, d0, _ = dg.run(s, parent_mode=bfs.BFS_PARENT_MIN)
    for _ in range(5):
        p, d, _ = dg.run(s, parent_mode=bfs.BFS_PARENT_MIN)
        assert np.array_equal(p, p0) and np.array_equal(d, d0)


def test_degenerate_graphs(orc):
    # single vertex, no edges
    dg = DevGraph(np.zeros(2, np.int64), np.zeros(0, np.int32))
    for dirv in (bfs.BFS_DIR_DO, bfs.BFS_DIR_TD, bfs.BFS_DIR_BU):
        p, d, st = dg.run(0, dir=dirv)
        assert p.tolist() == [0] and d.tolist() == [0] and st.reached == 1
    # 200 vertices, no edges at all
    dg = DevGraph(np.zeros(201, np.int64), np.zeros(0, np.int32))
    p, d, _ = dg.run(150)
    assert d[150] == 0 and p[150] == 150 and (d >= 0).sum() == 1 and (p >= 0).sum() == 1
    # n = 64 exactly and n = 65 (bitmap word boundaries)
    for n in (63, 64, 65, 129):
        off, cols = path_graph(n)
        dg = DevGraph(off, cols)
        for s in (0, n - 1, n // 2):
            for dirv in (bfs.BFS_DIR_DO, bfs.BFS_DIR_BU, bfs.BFS_DIR_TD):
                p, d, _ = dg.run(s, dir=dirv, parent_mode=bfs.BFS_PARENT_MIN)
                check(orc, dg, s, p, d, True)


def test_directed_graph_top_down(orc):
    rng = np.random.default_rng(3)
    n = 3000
    a = rng.integers(0, n, 12000)
    b = rng.integers(0, n, 12000)
    off, cols = graphgen.csr_from_edges(n, a, b, symmetrize=False)
    dg = DevGraph(off, cols, flags=bfs.BFS_GRAPH_SORTED | bfs.BFS_GRAPH_VALIDATE)
    deg = np.diff(off)
    for s in list(np.flatnonzero(deg > 0)[:5]) + [int(np.flatnonzero(deg == 0)[0])]:
        ref = orc.bfs_min(off, cols, int(s))
        for pm in (bfs.BFS_PARENT_ANY, bfs.BFS_PARENT_MIN):
            p, d, _ = dg.run(s, dir=bfs.BFS_DIR_TD, parent_mode=pm)
            check(orc, dg, s, p, d, pm == bfs.BFS_PARENT_MIN, ref)
    with pytest.raises(bfs.BfsError) as e:
        dg.run(0, dir=bfs.BFS_DIR_DO)
    assert e.value.status == 8


def test_error_paths():
    off, cols = path_graph(100)
    dg = DevGraph(off, cols)
    with pytest.raises(bfs.BfsError) as e:
        dg.run(100)
    assert e.value.status == 2
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_run(dg.g, 0, dg.parent, dg.depth, dg.ws[:100])
    assert e.value.status == 7
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_run(dg.g, 0, dg.parent, dg.depth, dg.ws, bfs.bfs_opts_default(dir=7))
    assert e.value.status == 1
    # validation on device: out-of-range id, unsorted row, missing mirror entry
    bad = cols.copy()
    bad[5] = 100
    with pytest.raises(bfs.BfsError) as e:
        DevGraph(off, bad)
    assert e.value.status == 2
    uns = cols.copy()
    uns[1], uns[2] = uns[2], uns[1]
    with pytest.raises(bfs.BfsError) as e:
        DevGraph(off, uns)
    assert e.value.status in (3, 4)
    asym_off, asym_cols = graphgen.csr_from_edges(10, np.array([0, 1]), np.array([1, 2]), symmetrize=False)
    with pytest.raises(bfs.BfsError) as e:
        DevGraph(asym_off, asym_cols)
    assert e.value.status == 4
    moff = off.copy()
    moff[-1] += 1
    with pytest.raises(bfs.BfsError) as e:
        DevGraph(moff, cols)
    assert e.value.status == 1


def test_config2_scale22_sampled_sources(orc):
    """Kronecker scale 22, int64 offsets, default launch configuration: 3 sources fully checked."""
    off, cols = graphgen.kronecker(22, seed=1)
    dg = DevGraph(off, cols, np.int64, flags=bfs.BFS_GRAPH_SYMMETRIC | bfs.BFS_GRAPH_SORTED)
    srcs = graphgen.random_sources(off, 64, seed=2)
    for s in srcs[:3]:
        ref = orc.bfs_min(off, cols, int(s))
        for pm, head in ((bfs.BFS_PARENT_ANY, 0), (bfs.BFS_PARENT_ANY, 2), (bfs.BFS_PARENT_ANY, 3),
                         (bfs.BFS_PARENT_MIN, 0)):
            p, d, _ = dg.run(s, parent_mode=pm, bu_head=head)
            check(orc, dg, s, p, d, pm == bfs.BFS_PARENT_MIN, ref)
        # the large-graph defaults at this scale: ranked hub heads on the first
        # bottom-up level and the hub pre-pass on top-down levels of 2^16+ edges
        p, d, _ = dg.run(s, bu_head=3, td_prepass=1 << 16)
        check(orc, dg, s, p, d, False, ref)


def _progress(msg):
    import sys
    import time
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", file=sys.__stderr__, flush=True)


def test_config3_scale26_full_size(orc):
    """Kronecker scale 26 (the benchmark workload, default launch configuration).

    One source compared exactly (depths and minimum-id parents, the oracle run
    on the CPU); a second source checked through the BFS-tree invariants,
    which pin the depths exactly at any size.
    """
    _progress("scale 26: generating")
    off, cols = graphgen.kronecker(26, seed=1)
    _progress("scale 26: to device")
    dg = DevGraph(off, cols, np.int64, flags=bfs.BFS_GRAPH_SYMMETRIC | bfs.BFS_GRAPH_SORTED)
    srcs = graphgen.random_sources(off, 64, seed=2)
    s = int(srcs[0])
    _progress("scale 26: oracle")
    ref = orc.bfs_min(off, cols, s)
    _progress("scale 26: GPU min parents")
    p, d, st = dg.run(s, parent_mode=bfs.BFS_PARENT_MIN)
    check(orc, dg, s, p, d, True, ref)
    assert st.bu_levels > 0 and st.td_levels > 0
    del ref
    s = int(srcs[1])
    _progress("scale 26: GPU any parents + validator")
    p, d, _ = dg.run(s, parent_mode=bfs.BFS_PARENT_ANY)
    res = orc.validate(off, cols, s, p, d)
    assert res[0] == "ok", res
    _progress("scale 26: done")


# (small_edges, persist_edges, persist_groups): engine off, one workgroup at
# various caps, many workgroups (including counts that do not divide the
# frontier evenly) from the first level on, and the defaults
ENGINE_CFGS = ((-1, 0, 0), (1, 1, 0), (7, 7, 0), (100, 100, 0), (4096, 4096, 0), (0, 0, 0),
               (1 << 30, 1 << 30, 0), (1, 1 << 30, 2), (1, 1 << 30, 7), (1, 1 << 30, 64), (8, 200, 33))


@pytest.mark.parametrize("name", ["grid", "path", "kron12", "er", "pieces"])
def test_persistent_engine_invariance(orc, graphs, name):
    """The persistent top-down engine (one workgroup, several workgroups with
    grid barriers, any edge caps, or switched off) changes neither results
    nor the per-level schedule and counters."""
    for off_dtype in (np.int32, np.int64):
        dg = get(graphs, name, off_dtype)
        for s in sources_for(dg.off, k=2, seed=21):
            ref = orc.bfs_min(dg.off, dg.cols, int(s))
            for dirv in (bfs.BFS_DIR_DO, bfs.BFS_DIR_TD):
                # bottom-up probe orders differ between parent modes, so the
                # examined counts are compared within one mode
                base = {}
                for cap, pcap, pg in ENGINE_CFGS:
                    for pm, claim in ((bfs.BFS_PARENT_MIN, 0), (bfs.BFS_PARENT_ANY, 0), (bfs.BFS_PARENT_ANY, 1)):
                        p, d, st = dg.run(s, dir=dirv, parent_mode=pm, td_claim=claim, small_edges=cap,
                                          persist_edges=pcap, persist_groups=pg)
                        check(orc, dg, s, p, d, pm == bfs.BFS_PARENT_MIN, ref)
                        L = min(st.levels, bfs.STATS_MAX_LEVELS)
                        sig = (st.levels, st.reached, st.edges_examined, st.td_levels, st.bu_levels,
                               list(st.level_dir[:L]), list(st.level_nf[:L]), list(st.level_mf[:L]),
                               list(st.level_mu[:L]), list(st.level_unvisited[:L]), list(st.level_examined[:L]))
                        ref_sig = base.setdefault((pm, claim), sig)
                        assert sig == ref_sig, (cap, pcap, pg, pm, claim)


def test_grid_many_levels_closed_form(orc):
    """A 300x700 grid from a corner (998 levels) and from an interior point:
    depths follow the Manhattan distance and minimum-id parents the closed form
    (up if below the source row, else left / right toward the source column,
    else down)."""
    H, W = 300, 700
    off, cols = graphgen.grid2d(H, W)
    dg = DevGraph(off, cols, np.int32)
    r, c = np.divmod(np.arange(H * W), W)
    for (r0, c0) in ((0, 0), (123, 456), (H - 1, W - 1)):
        s = r0 * W + c0
        dist = np.abs(r - r0) + np.abs(c - c0)
        par = np.where(r > r0, s * 0 + (r - 1) * W + c,
                       np.where(c > c0, r * W + c - 1, np.where(c < c0, r * W + c + 1, (r + 1) * W + c)))
        par[s] = s
        for dirv in (bfs.BFS_DIR_DO, bfs.BFS_DIR_TD, bfs.BFS_DIR_BU):
            p, d, st = dg.run(s, dir=dirv, parent_mode=bfs.BFS_PARENT_MIN)
            assert np.array_equal(d, dist)
            assert np.array_equal(p, par)
            assert st.levels == int(dist.max()) + 1
