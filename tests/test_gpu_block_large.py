"""The GPU block generator pinned to the host generator, and the DCSC block
calls on one block of an 8x8 decomposition of a scale-30 Kronecker graph (the
full-size configuration, 2^27 x 2^27), checked on sampled rows against the
oracle and on every output row through properties that hold at any size."""
import sys
import time

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1705_04590_amd as bfs  # noqa: E402

DEV = torch.device("cuda:0")


def _progress(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", file=sys.__stderr__, flush=True)


@pytest.mark.parametrize("scale,pr,pc,i,j,permute", [(12, 1, 1, 0, 0, True), (16, 8, 8, 0, 1, True),
                                                     (16, 4, 2, 3, 0, True), (17, 8, 8, 5, 2, False),
                                                     (18, 8, 8, 7, 7, True)])
def test_gpu_generator_matches_host(scale, pr, pc, i, j, permute):
    n = 1 << scale
    R, C = n // pr, n // pc
    cpu = graphgen.kronecker_block(scale, i * R, R, j * C, C, seed=1, permute=permute)
    gpu = graphgen.kronecker_block_gpu(scale, i * R, R, j * C, C, seed=1, permute=permute)
    for k in ("nnz", "nzc", "nzr"):
        assert cpu[k] == gpu[k], k
    for k in ("jc", "cp", "ir", "jr", "rp", "ic"):
        assert np.array_equal(cpu[k], gpu[k].cpu().numpy()), k


def rows_entries(blk, rows):
    """(row, col) entries of the given block-local rows, read from the DCSR form on the device."""
    jr, rp, ic = blk["jr"], blk["rp"], blk["ic"]
    rt = torch.from_numpy(rows.astype(np.int32)).to(DEV)
    idx = torch.searchsorted(jr, rt).clamp(max=jr.numel() - 1)
    present = jr[idx] == rt
    beg = rp[idx]
    lens = torch.where(present, rp[idx + 1] - beg, torch.zeros_like(beg))
    total = int(lens.sum().item())
    starts = torch.cumsum(lens, 0) - lens
    pos = (torch.arange(total, device=DEV) - torch.repeat_interleave(starts, lens) +
           torch.repeat_interleave(beg, lens))
    erow = torch.repeat_interleave(rt.long(), lens).to(torch.int32)
    return erow.cpu().numpy(), ic[pos].cpu().numpy()


@pytest.fixture(scope="module")
def s30_block():
    scale = 30
    n = 1 << scale
    R = C = n // 8
    _progress("scale-30 8x8 block (0, 1): generating on the GPU")
    blk = graphgen.kronecker_block_gpu(scale, 0, R, C, C, seed=1)
    _progress(f"block: nnz {blk['nnz']} nzc {blk['nzc']} nzr {blk['nzr']}")
    g = bfs.bfs_create_graph_dcsc(R, C, 0, C, blk["jc"], blk["cp"], blk["ir"], blk["jr"], blk["rp"], blk["ic"],
                                  flags=bfs.BFS_GRAPH_SORTED | bfs.BFS_GRAPH_VALIDATE)
    ws = bfs.workspace(g, 1, DEV)
    yield dict(blk=blk, g=g, ws=ws, R=R, C=C)
    bfs.bfs_destroy_graph(g)


def sample_rows(out_rows, R, seed, k=1500):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, R, k)
    b = out_rows[rng.integers(0, out_rows.size, k)] if out_rows.size else np.zeros(0, np.int64)
    return np.unique(np.concatenate([a, b]).astype(np.int64))


@pytest.mark.parametrize("density", [1e-5, 1e-3, 1e-1])
def test_s30_block_td_sampled(orc, s30_block, density):
    R, C, blk = s30_block["R"], s30_block["C"], s30_block["blk"]
    k = int(round(density * C))
    fr = graphgen.random_sorted_subset(C, k, seed=4)
    out_r = torch.empty(R, dtype=torch.int32, device=DEV)
    out_p = torch.empty(R, dtype=torch.int32, device=DEV)
    nout = torch.zeros(1, dtype=torch.int64, device=DEV)
    _progress(f"block TD, density {density}: {k} frontier columns")
    bfs.bfs_block_td(s30_block["g"], torch.from_numpy(fr).to(DEV), out_r, out_p, nout, s30_block["ws"])
    torch.cuda.synchronize()
    m = int(nout.item())
    r, p = out_r[:m], out_p[:m]
    # every output row: strictly ascending, parent a frontier column of the block
    if m > 1:
        assert bool((r[1:] > r[:-1]).all())
    ft = torch.from_numpy(fr).to(DEV)
    assert bool(torch.isin(p - C, ft).all())
    # sampled rows (random rows and output rows): exactly the oracle's answer
    rows = sample_rows(r.cpu().numpy(), R, seed=int(1 / density))
    erow, ecol = rows_entries(blk, rows)
    er, ep = orc.block_td(R, C, erow, ecol, C, fr)
    sel = torch.isin(r, torch.from_numpy(rows.astype(np.int32)).to(DEV))
    assert np.array_equal(r[sel].cpu().numpy(), er) and np.array_equal(p[sel].cpu().numpy(), ep)
    _progress(f"block TD, density {density}: {m} rows out, {rows.size} sampled rows match")


@pytest.mark.parametrize("density,cdens", [(1e-3, 1e-3), (1e-1, 1e-1), (1e-1, 0.5)])
def test_s30_block_bu_sampled(orc, s30_block, density, cdens):
    R, C, blk = s30_block["R"], s30_block["C"], s30_block["blk"]
    fb = graphgen.random_bitmap(C, density, seed=4)
    comp0 = graphgen.random_bitmap(R, cdens, seed=5)
    out_r = torch.empty(R, dtype=torch.int32, device=DEV)
    out_p = torch.empty(R, dtype=torch.int32, device=DEV)
    nout = torch.zeros(1, dtype=torch.int64, device=DEV)
    comp = torch.from_numpy(comp0.view(np.int64).copy()).to(DEV)
    _progress(f"block BU, frontier density {density}, completed density {cdens}")
    bfs.bfs_block_bu(s30_block["g"], torch.from_numpy(fb.view(np.int64)).to(DEV), comp, 0, R, out_r, out_p, nout,
                     s30_block["ws"])
    torch.cuda.synchronize()
    m = int(nout.item())
    r = out_r[:m].cpu().numpy()
    p = out_p[:m].cpu().numpy()
    c1 = comp.cpu().numpy().view(np.uint64)
    before = graphgen.words_to_bits(comp0, R)
    after = graphgen.words_to_bits(c1, R)
    # properties of every output row
    assert np.all(np.diff(r) > 0)
    assert not before[r].any() and after[r].all()
    assert int(after.sum()) - int(before.sum()) == m
    fbits = graphgen.words_to_bits(fb, C)
    assert fbits[p - C].all()
    # sampled rows: the oracle's rows, parents and completed bits
    rows = sample_rows(r, R, seed=7)
    erow, ecol = rows_entries(blk, rows)
    er, ep, ec = orc.block_bu(R, C, erow, ecol, C, fb, comp0, 0, R)
    sel = np.isin(r, rows)
    assert np.array_equal(r[sel], er) and np.array_equal(p[sel], ep)
    eb = graphgen.words_to_bits(ec, R)
    assert np.array_equal(after[rows], eb[rows])
    _progress(f"block BU: {m} rows out, {rows.size} sampled rows match")
