"""GPU parity of the DCSC block calls (Alg. 3 / Alg. 4 local discovery) against the oracle."""
import json
import os

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1705_04590_amd as bfs  # noqa: E402

DEV = torch.device("cuda:0")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)


def t64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).to(DEV)


class DevBlock:
    def __init__(self, blk, nrows, ncols, row_base=0, col_base=0, row_major=True,
                 flags=bfs.BFS_GRAPH_SORTED | bfs.BFS_GRAPH_VALIDATE):
        self.blk, self.nrows, self.ncols, self.col_base = blk, nrows, ncols, col_base
        self.arrs = [t32(blk["jc"]), t64(blk["cp"]), t32(blk["ir"])]
        if row_major:
            self.arrs += [t32(blk["jr"]), t64(blk["rp"]), t32(blk["ic"])]
        else:
            self.arrs += [None, None, None]
        self.g = bfs.bfs_create_graph_dcsc(nrows, ncols, row_base, col_base, *self.arrs, flags=flags)
        self.ws = bfs.workspace(self.g, 1, DEV)
        self.out_r = torch.empty(max(nrows, 1), dtype=torch.int32, device=DEV)
        self.out_p = torch.empty(max(nrows, 1), dtype=torch.int32, device=DEV)
        self.nout = torch.zeros(1, dtype=torch.int64, device=DEV)
        # plain entry list for the oracle
        self.erow = blk["ir"]
        self.ecol = np.repeat(blk["jc"], np.diff(blk["cp"])).astype(np.int32)

    def td(self, fcols):
        bfs.bfs_block_td(self.g, t32(fcols), self.out_r, self.out_p, self.nout, self.ws)
        torch.cuda.synchronize()
        k = int(self.nout.item())
        return self.out_r[:k].cpu().numpy(), self.out_p[:k].cpu().numpy()

    def bu(self, fbits, completed, row_lo, row_hi):
        fb = torch.from_numpy(np.ascontiguousarray(fbits).view(np.int64)).to(DEV)
        comp = torch.from_numpy(np.ascontiguousarray(completed).view(np.int64).copy()).to(DEV)
        bfs.bfs_block_bu(self.g, fb, comp, row_lo, row_hi, self.out_r, self.out_p, self.nout, self.ws)
        torch.cuda.synchronize()
        k = int(self.nout.item())
        return self.out_r[:k].cpu().numpy(), self.out_p[:k].cpu().numpy(), comp.cpu().numpy().view(np.uint64)


def test_fig2_block_on_gpu():
    g = json.load(open(os.path.join(GOLDEN, "fig2_block.json")))
    ent = np.array(g["entries_row_col"])
    blk = graphgen.coo_block(6, 6, ent[:, 0], ent[:, 1])
    db = DevBlock(blk, 6, 6)
    r, p = db.td(np.array(g["td_frontier"]))
    assert list(zip(r.tolist(), p.tolist())) == [tuple(x) for x in g["td_expected_row_parent"]]
    fb = graphgen.bits_to_words([i in g["bu_frontier"] for i in range(6)])
    r, p, comp = db.bu(fb, np.zeros(1, np.uint64), 0, 6)
    assert list(zip(r.tolist(), p.tolist())) == [tuple(x) for x in g["bu_expected_row_parent"]]
    assert np.flatnonzero(graphgen.words_to_bits(comp, 6)).tolist() == g["bu_expected_completed_rows"]
    # an empty frontier and an empty row range
    r, p = db.td(np.zeros(0, np.int32))
    assert r.size == 0
    r, p, _ = db.bu(fb, np.zeros(1, np.uint64), 3, 3)
    assert r.size == 0


@pytest.mark.parametrize("pr,pc", [(1, 1), (2, 2), (4, 4), (2, 8), (8, 2), (8, 8)])
def test_blocks_match_oracle_on_bfs_levels(orc, pr, pc):
    off, cols = graphgen.kronecker(12, seed=3)
    n = off.size - 1
    s = int(graphgen.random_sources(off, 1, seed=4)[0])
    _, depth = orc.bfs(off, cols, s)
    R, C = n // pr, n // pc
    for (i, j) in [(0, 0), (pr - 1, pc - 1), (pr // 2, (pc + 1) // 3)]:
        blk = graphgen.csr_block(off, cols, i * R, R, j * C, C)
        db = DevBlock(blk, R, C, i * R, j * C)
        for d in range(int(depth.max())):
            fr = np.flatnonzero(depth[j * C:(j + 1) * C] == d).astype(np.int32)
            r, p = db.td(fr)
            er, ep = orc.block_td(R, C, db.erow, db.ecol, j * C, fr)
            assert np.array_equal(r, er) and np.array_equal(p, ep)
            fb = graphgen.bits_to_words(depth[j * C:(j + 1) * C] == d)
            comp0 = graphgen.bits_to_words((depth[i * R:(i + 1) * R] >= 0) & (depth[i * R:(i + 1) * R] <= d))
            for (lo, hi) in [(0, R), (R // 3, R // 2)]:
                r, p, comp = db.bu(fb, comp0, lo, hi)
                er, ep, ecomp = orc.block_bu(R, C, db.erow, db.ecol, j * C, fb, comp0, lo, hi)
                assert np.array_equal(r, er) and np.array_equal(p, ep)
                assert np.array_equal(comp, ecomp)


@pytest.mark.parametrize("density", [1e-5, 1e-3, 1e-2, 1e-1, 0.5])
def test_block_sparse_frontiers(orc, density):
    """One block of an 8x8 decomposition of a scale-18 Kronecker graph, seeded frontiers."""
    scale = 18
    n = 1 << scale
    R = C = n // 8
    blk = graphgen.kronecker_block(scale, 0, R, C, C, seed=1)
    db = DevBlock(blk, R, C, 0, C)
    k = max(1, int(round(density * C)))
    fr = graphgen.random_sorted_subset(C, k, seed=4)
    r, p = db.td(fr)
    er, ep = orc.block_td(R, C, db.erow, db.ecol, C, fr)
    assert np.array_equal(r, er) and np.array_equal(p, ep)
    fb = graphgen.random_bitmap(C, density, seed=4)
    comp = graphgen.random_bitmap(R, min(density, 0.5), seed=5)
    for (lo, hi) in [(0, R), (R // 8, 3 * R // 8)]:
        r, p, c2 = db.bu(fb, comp, lo, hi)
        er, ep, ec = orc.block_bu(R, C, db.erow, db.ecol, C, fb, comp, lo, hi)
        assert np.array_equal(r, er) and np.array_equal(p, ep) and np.array_equal(c2, ec)


@pytest.mark.parametrize("density", [0.04, 0.3, 1.0])
def test_dense_block_frontier_all_layouts(orc, density):
    """Dense frontiers take the row scan (row copy, sorted), the JC scan (no row copy) or
    the JC scan over unsorted-flagged rows; all give the oracle's minimum parents."""
    scale = 16
    n = 1 << scale
    R = C = n // 4
    blk = graphgen.kronecker_block(scale, R, R, 2 * C, C, seed=7)
    k = max(1, int(round(density * C)))
    fr = graphgen.random_sorted_subset(C, k, seed=8)
    layouts = [dict(row_major=True), dict(row_major=False),
               dict(row_major=True, flags=bfs.BFS_GRAPH_VALIDATE)]
    er = ep = None
    for kw in layouts:
        db = DevBlock(blk, R, C, R, 2 * C, **kw)
        if er is None:
            er, ep = orc.block_td(R, C, db.erow, db.ecol, 2 * C, fr)
        r, p = db.td(fr)
        assert np.array_equal(r, er) and np.array_equal(p, ep), kw
        # the frontier marks are cleared: a sparse call afterwards is unaffected
        r, p = db.td(fr[:3])
        er3, ep3 = orc.block_td(R, C, db.erow, db.ecol, 2 * C, fr[:3])
        assert np.array_equal(r, er3) and np.array_equal(p, ep3), kw


def test_accumulator_is_reset_between_calls(orc):
    off, cols = graphgen.kronecker(13, seed=6)
    n = off.size - 1
    blk = graphgen.csr_block(off, cols, 0, n // 2, n // 2, n // 2)
    db = DevBlock(blk, n // 2, n // 2, 0, n // 2)
    for seed in range(6):
        # accumulator and sorted union alternate on the same workspace
        bfs.bfs_block_set_union(db.g, -1 if seed % 2 == 0 else 1)
        fr = graphgen.random_sorted_subset(n // 2, 50 * (seed + 1), seed=seed)
        r, p = db.td(fr)
        er, ep = orc.block_td(n // 2, n // 2, db.erow, db.ecol, n // 2, fr)
        assert np.array_equal(r, er) and np.array_equal(p, ep)


@pytest.mark.parametrize("mode", [-1, 0, 1])
def test_union_modes_match_oracle(orc, mode):
    """bfs_block_set_union: the accumulator (-1 and the default 0) and the
    sorted union whenever it fits (1) give the oracle's pairs on
    frontiers from one column to an eighth of the block; columns holding
    more than the sorted union's 8192 entries fall back to the accumulator,
    and the call after such a fallback is unaffected."""
    scale = 18
    n = 1 << scale
    R = C = n // 8
    blk = graphgen.kronecker_block(scale, 0, R, C, C, seed=1)
    db = DevBlock(blk, R, C, 0, C)
    bfs.bfs_block_set_union(db.g, mode)
    lens = np.diff(blk["cp"])
    heavy = np.sort(blk["jc"][np.argsort(lens)[::-1][:64]]).astype(np.int32)
    assert lens[np.isin(blk["jc"], heavy)].sum() > 8192
    frontiers = [graphgen.random_sorted_subset(C, k, seed=10 + k) for k in (1, 7, 60, 500, 3000, C // 8)]
    frontiers += [heavy, heavy[:1], np.zeros(0, np.int32), graphgen.random_sorted_subset(C, 40, seed=3)]
    for fr in frontiers:
        r, p = db.td(fr)
        er, ep = orc.block_td(R, C, db.erow, db.ecol, C, fr)
        assert np.array_equal(r, er) and np.array_equal(p, ep), fr.size


def test_union_mode_errors():
    g = json.load(open(os.path.join(GOLDEN, "fig2_block.json")))
    ent = np.array(g["entries_row_col"])
    db = DevBlock(graphgen.coo_block(6, 6, ent[:, 0], ent[:, 1]), 6, 6)
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_block_set_union(db.g, 2)
    assert e.value.status == 1
    off, cols = graphgen.kronecker(8, seed=1)
    g2 = bfs.bfs_create_graph_csr(t64(off), t32(cols), bfs.BFS_GRAPH_SYMMETRIC)
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_block_set_union(g2, 0)
    assert e.value.status == 1


def test_block_errors():
    g = json.load(open(os.path.join(GOLDEN, "fig2_block.json")))
    ent = np.array(g["entries_row_col"])
    blk = graphgen.coo_block(6, 6, ent[:, 0], ent[:, 1])
    db = DevBlock(blk, 6, 6, row_major=False)
    fb = torch.zeros(1, dtype=torch.int64, device=DEV)
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_block_bu(db.g, fb, fb.clone(), 0, 6, db.out_r, db.out_p, db.nout, db.ws)
    assert e.value.status == 8
    db = DevBlock(blk, 6, 6)
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_block_bu(db.g, fb, fb.clone(), 4, 2, db.out_r, db.out_p, db.nout, db.ws)
    assert e.value.status == 1
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_block_td(db.g, t32(np.arange(7)), db.out_r, db.out_p, db.nout, db.ws)
    assert e.value.status == 1
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_block_td(db.g, t32([1]), db.out_r, db.out_p, db.nout, db.ws[:64])
    assert e.value.status == 7
    # validation: a row id out of range, an unsorted column
    bad = dict(blk)
    bad["ir"] = blk["ir"].copy()
    bad["ir"][0] = 9
    with pytest.raises(bfs.BfsError) as e:
        DevBlock(bad, 6, 6)
    assert e.value.status == 2
    uns = dict(blk)
    uns["ir"] = blk["ir"].copy()
    uns["ir"][0], uns["ir"][1] = uns["ir"][1], uns["ir"][0]
    with pytest.raises(bfs.BfsError) as e:
        DevBlock(uns, 6, 6)
    assert e.value.status == 3
