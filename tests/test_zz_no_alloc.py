"""bfs_block_td_noalloc (the allocation-free block top-down call) against bfs_block_td.

Both calls go through the C ABI on the same blocks and frontiers; the outputs
must be identical (rows and parents are integers: bit-exact).  Calls run back
to back on one device: a larger block, then a smaller one (another workspace
layout inside the shared static array), then the larger one again, each with
sparse, medium and dense frontiers (the three top-down forms).  A block whose
workspace exceeds the static array is rejected before any launch.
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


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)


def t64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).to(DEV)


class Block:
    def __init__(self, scale, pr, i, j, seed):
        off, cols = graphgen.kronecker(scale, seed=seed)
        n = off.size - 1
        self.R = self.C = n // pr
        blk = graphgen.csr_block(off, cols, i * self.R, self.R, j * self.C, self.C)
        self.arrs = [t32(blk["jc"]), t64(blk["cp"]), t32(blk["ir"]), t32(blk["jr"]), t64(blk["rp"]),
                     t32(blk["ic"])]
        self.g = bfs.bfs_create_graph_dcsc(self.R, self.C, i * self.R, j * self.C, *self.arrs,
                                           flags=bfs.BFS_GRAPH_SORTED | bfs.BFS_GRAPH_VALIDATE)
        self.ws = bfs.workspace(self.g, 1, DEV)
        self.nzc = blk["nzc"]

    def outputs(self):
        return (torch.full((self.R,), -7, dtype=torch.int32, device=DEV),
                torch.full((self.R,), -7, dtype=torch.int32, device=DEV),
                torch.full((1,), -7, dtype=torch.int64, device=DEV))

    def both(self, fcols):
        f = t32(fcols)
        r0, p0, n0 = self.outputs()
        bfs.bfs_block_td(self.g, f, r0, p0, n0, self.ws)
        r1, p1, n1 = self.outputs()
        bfs.bfs_block_td_noalloc(self.g, f, r1, p1, n1)
        torch.cuda.synchronize()
        k0, k1 = int(n0.item()), int(n1.item())
        return (r0[:k0].cpu().numpy(), p0[:k0].cpu().numpy()), (r1[:k1].cpu().numpy(), p1[:k1].cpu().numpy())


def frontiers(C, seed):
    # sparse (binary search in JC), |F| log2 nzc > nzc (one JC pass), and
    # more than 1/32 of the columns (the row-side pull form)
    return [graphgen.random_sorted_subset(C, k, seed=seed + i)
            for i, k in enumerate((1, max(2, C // 400), C // 8, C // 2))] + [np.zeros(0, np.int32)]


def check_block(b, seed):
    rows = 0
    for f in frontiers(b.C, seed):
        (r0, p0), (r1, p1) = b.both(f)
        assert np.array_equal(r0, r1) and np.array_equal(p0, p1), f"{f.size} frontier columns"
        rows += r0.size
    assert rows > 0   # the frontiers reach some rows of the block


def test_noalloc_matches_block_td_across_calls():
    big = Block(16, 2, 0, 1, seed=1)      # 32768 x 32768 block
    small = Block(12, 4, 1, 2, seed=3)    # 1024 x 1024 block: a smaller input, another layout
    check_block(big, 10)
    check_block(small, 20)
    check_block(big, 30)
    # same block twice in a row (the scratch is not cleared again)
    check_block(small, 40)
    check_block(small, 50)


def test_noalloc_rejects_blocks_beyond_its_scratch():
    # 2^25 rows: the row accumulator alone is 128 MiB, over the 64 MiB array
    R = C = 1 << 25
    jc, cp, ir = t32([5]), t64([0, 1]), t32([7])
    g = bfs.bfs_create_graph_dcsc(R, C, 0, 0, jc, cp, ir, None, None, None, flags=bfs.BFS_GRAPH_SORTED)
    assert bfs.bfs_workspace_bytes(g, 1) > 64 << 20
    rows = torch.full((R,), -7, dtype=torch.int32, device=DEV)
    pars = torch.full((R,), -7, dtype=torch.int32, device=DEV)
    nout = torch.full((1,), -7, dtype=torch.int64, device=DEV)
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_block_td_noalloc(g, t32([5]), rows, pars, nout)
    assert e.value.status == 7
    torch.cuda.synchronize()
    assert int(nout.item()) == -7      # nothing was launched
