"""GPU parity of bfs_run_multi (up to 64 sources, uint64 masks) against the oracle and bfs_run."""
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


class MG:
    def __init__(self, off, cols, off_dtype=np.int64):
        self.off, self.cols, self.n = off, cols, off.size - 1
        self.d_off = torch.from_numpy(off.astype(off_dtype)).to(DEV)
        self.d_cols = torch.from_numpy(cols).to(DEV)
        self.g = bfs.bfs_create_graph_csr(self.d_off, self.d_cols, SYM)
        self.ws_multi = None

    def multi(self, sources, with_parent=True, **kw):
        k = len(sources)
        if self.ws_multi is None:
            self.ws_multi = bfs.workspace(self.g, 64, DEV)
        par = torch.empty(k * self.n, dtype=torch.int32, device=DEV) if with_parent else None
        dep = torch.empty(k * self.n, dtype=torch.int32, device=DEV)
        st = bfs.bfs_run_multi(self.g, sources, par, dep, self.ws_multi, bfs.bfs_opts_default(**kw))
        torch.cuda.synchronize()
        p = par.cpu().numpy().reshape(k, self.n) if with_parent else None
        return p, dep.cpu().numpy().reshape(k, self.n), st


def check_all(orc, mg, sources, p, d):
    for j, s in enumerate(sources):
        rp, rd = orc.bfs_min(mg.off, mg.cols, int(s))
        assert np.array_equal(d[j], rd), f"source {j} ({s}): depth mismatch at {np.flatnonzero(d[j] != rd)[:5]}"
        if p is not None:
            bad = np.flatnonzero(p[j] != rp)
            assert bad.size == 0, f"source {j} ({s}): parent mismatch at {bad[:5]}: {p[j][bad[:5]]} vs {rp[bad[:5]]}"


GRAPHS = {
    "kron12": lambda: graphgen.kronecker(12, seed=1),
    "kron14": lambda: graphgen.kronecker(14, seed=2),
    "er": lambda: graphgen.erdos_renyi(5000, 2.5, seed=4),
    "grid": lambda: graphgen.grid2d(40, 37),
}


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("direction", [0, 1, 2])
def test_multi_matches_oracle(orc, name, direction):
    off, cols = GRAPHS[name]()
    for off_dtype in (np.int32, np.int64):
        mg = MG(off, cols, off_dtype)
        srcs = list(graphgen.random_sources(off, 40, seed=7))
        deg = np.diff(off)
        iso = np.flatnonzero(deg == 0)
        if iso.size:
            srcs.append(int(iso[0]))   # an isolated source
        srcs += [srcs[0], srcs[3]]     # duplicates
        p, d, st = mg.multi(srcs, dir=direction)
        check_all(orc, mg, srcs, p, d)


def test_full_batch_of_64_and_single(orc):
    off, cols = graphgen.kronecker(13, seed=5)
    mg = MG(off, cols)
    srcs = graphgen.random_sources(off, 64, seed=2)
    p, d, st = mg.multi(srcs)
    check_all(orc, mg, srcs, p, d)
    assert st.levels > 2
    # a batch of one equals bfs_run with minimum parents
    ws = bfs.workspace(mg.g, 1, DEV)
    par = torch.empty(mg.n, dtype=torch.int32, device=DEV)
    dep = torch.empty(mg.n, dtype=torch.int32, device=DEV)
    for s in srcs[:4]:
        p1, d1, _ = mg.multi([int(s)])
        bfs.bfs_run(mg.g, int(s), par, dep, ws, bfs.bfs_opts_default(parent_mode=bfs.BFS_PARENT_MIN))
        torch.cuda.synchronize()
        assert np.array_equal(p1[0], par.cpu().numpy()) and np.array_equal(d1[0], dep.cpu().numpy())


def test_multi_without_parents_and_forced_schedules(orc):
    off, cols = graphgen.kronecker(12, seed=9)
    mg = MG(off, cols)
    srcs = graphgen.random_sources(off, 17, seed=3)
    ref_p, ref_d, _ = mg.multi(srcs)
    check_all(orc, mg, srcs, ref_p, ref_d)
    _, d, _ = mg.multi(srcs, with_parent=False)
    assert np.array_equal(d, ref_d)
    for alpha, beta in ((1e9, 1e9), (1e-9, 1e-9), (2.0, 50.0), (1e9, 1e-9)):
        for serial in (1, 16, 1 << 20):
            p, d, _ = mg.multi(srcs, alpha=alpha, beta=beta, bu_serial=serial)
            assert np.array_equal(p, ref_p) and np.array_equal(d, ref_d)


def test_multi_sources_in_different_components(orc):
    # Kronecker piece + a separate path + isolated vertices
    off1, cols1 = graphgen.kronecker(10, seed=8)
    n1 = off1.size - 1
    src = np.repeat(np.arange(n1), np.diff(off1))
    keep = src < cols1
    a = np.concatenate([src[keep], n1 + np.arange(299)])
    b = np.concatenate([cols1[keep], n1 + np.arange(1, 300)])
    off, cols = graphgen.csr_from_edges(n1 + 310, a, b)
    mg = MG(off, cols)
    srcs = [n1, n1 + 150, n1 + 305] + list(graphgen.random_sources(off1, 10, seed=1))
    for direction in (0, 1, 2):
        p, d, _ = mg.multi(srcs, dir=direction)
        check_all(orc, mg, srcs, p, d)


def test_multi_errors():
    off, cols = graphgen.kronecker(8, seed=1)
    mg = MG(off, cols)
    ws = bfs.workspace(mg.g, 64, DEV)
    dep = torch.empty(65 * mg.n, dtype=torch.int32, device=DEV)
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_run_multi(mg.g, list(range(65)), None, dep, ws)
    assert e.value.status == 1
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_run_multi(mg.g, [0, mg.n], None, dep, ws)
    assert e.value.status == 2
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_run_multi(mg.g, [0], None, dep, ws[:1000])
    assert e.value.status == 7


def test_multi_long_rows_get_minimum_parents(orc):
    """Vertices whose rows exceed the resolve pass's scan limit take their
    parents from the frontier side: hubs of several stars joined in a ring,
    sources on leaves and on hubs, top-down only and direction-optimizing."""
    hubs, leaves = 6, 900
    n = hubs * (leaves + 1)
    a, b = [], []
    for h in range(hubs):
        c = h * (leaves + 1)
        a += [c] * leaves
        b += list(range(c + 1, c + 1 + leaves))
        a.append(c)
        b.append(((h + 1) % hubs) * (leaves + 1))
    # leaves of neighbouring stars share some extra edges, so a hub has
    # several frontier neighbours and the minimum matters
    rng = np.random.default_rng(3)
    for _ in range(2000):
        h = int(rng.integers(0, hubs))
        a.append(h * (leaves + 1) + 1 + int(rng.integers(0, leaves)))
        b.append(((h + 1) % hubs) * (leaves + 1) + 1 + int(rng.integers(0, leaves)))
    off, cols = graphgen.csr_from_edges(n, np.array(a), np.array(b))
    assert np.diff(off).max() > 512
    mg = MG(off, cols)
    srcs = [int(x) for x in rng.choice(np.flatnonzero(np.diff(off) > 0), 60, replace=False)] + [0, leaves + 1]
    for direction in (0, 1):
        # persistent engine on (the default) and off: both mark the long rows
        for engine in (0, -1):
            p, d, _ = mg.multi(srcs, dir=direction, small_edges=engine)
            check_all(orc, mg, srcs, p, d)


# (small_edges, persist_edges, persist_groups): engine off, default, on (a
# positive small_edges; graphs whose rows all have at most 32 entries leave it
# off by default) with tiny and huge edge caps, one workgroup, counts that do
# not divide the queue evenly
MS_ENGINE = ((-1, 0, 0), (0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 100, 3), (1, 1 << 30, 1), (1, 1 << 30, 64),
             (1, 5000, 7))


@pytest.mark.parametrize("name", ["kron12", "grid", "er"])
def test_multi_engine_invariance(orc, name):
    """The persistent multi-source engine runs small top-down levels in one
    launch.  Switched off, on with any edge cap or workgroup count, it gives
    the same parents and depths (the oracle's) and the same per-level
    schedule and counts."""
    off, cols = GRAPHS[name]()
    mg = MG(off, cols)
    srcs = list(graphgen.random_sources(off, 33, seed=12))
    ref = None
    for direction in (0, 1):
        base = None
        for eng, cap, grp in MS_ENGINE:
            p, d, st = mg.multi(srcs, dir=direction, small_edges=eng, persist_edges=cap, persist_groups=grp)
            if ref is None:
                check_all(orc, mg, srcs, p, d)
                ref = (p, d)
            assert np.array_equal(p, ref[0]) and np.array_equal(d, ref[1]), (direction, eng, cap, grp)
            L = min(st.levels, bfs.STATS_MAX_LEVELS)
            sig = (st.levels, st.edges_examined, list(st.level_dir[:L]), list(st.level_nf[:L]),
                   list(st.level_mf[:L]), list(st.level_mu[:L]), list(st.level_examined[:L]))
            base = base or sig
            assert sig == base, (direction, eng, cap, grp)


def test_multi_engine_on_a_long_grid():
    """A 3 x 2000 grid from its corners and middle: about 2000 levels, all
    inside the engine, checked against the closed form."""
    H, W = 3, 2000
    off, cols = graphgen.grid2d(H, W)
    mg = MG(off, cols)
    srcs = [0, W - 1, (H - 1) * W, H * W - 1, W // 2, W + 700]
    r, c = np.divmod(np.arange(H * W), W)
    for eng in (1, 0, -1):
        p, d, st = mg.multi(srcs, small_edges=eng)
        for j, s in enumerate(srcs):
            r0, c0 = divmod(s, W)
            dist = np.abs(r - r0) + np.abs(c - c0)
            par = np.where(r > r0, (r - 1) * W + c, np.where(c > c0, r * W + c - 1,
                                                            np.where(c < c0, r * W + c + 1, (r + 1) * W + c)))
            par[s] = s
            assert np.array_equal(d[j], dist) and np.array_equal(p[j], par), (eng, j)


def test_multi_level_cap_is_an_error():
    """Levels are 16-bit in the batched search: a path of 70 000 vertices
    searched from one end needs 70 000 levels, more than 65 535, and the call
    fails with BFS_E_UNSUPPORTED; from the middle it needs 35 000 and passes."""
    n = 70000
    off, cols = graphgen.csr_from_edges(n, np.arange(n - 1), np.arange(1, n))
    mg = MG(off, cols)
    with pytest.raises(bfs.BfsError) as e:
        mg.multi([0, 5], with_parent=False)
    assert e.value.status == 8
    p, d, st = mg.multi([n // 2], with_parent=True)
    assert np.array_equal(d[0], np.abs(np.arange(n) - n // 2))
    assert st.levels == n // 2 + 1
