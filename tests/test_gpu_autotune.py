"""The autotuner returns settings that leave results unchanged."""
import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1705_04590_amd as bfs  # noqa: E402
from paper_1705_04590_amd import autotune  # noqa: E402

DEV = torch.device("cuda:0")


def test_autotune_single_and_multi_are_result_invariant(orc, tmp_path):
    off, cols = graphgen.kronecker(13, seed=4)
    n = off.size - 1
    g = bfs.bfs_create_graph_csr(torch.from_numpy(off).to(DEV), torch.from_numpy(cols).to(DEV),
                                 bfs.BFS_GRAPH_SYMMETRIC | bfs.BFS_GRAPH_SORTED)
    tune_src = graphgen.random_sources(off, 8, seed=99)
    cache = str(tmp_path / "tune.json")
    r1 = autotune.tune(g, tune_src, k=1, cache_path=cache)
    assert r1["trials"] > 10 and r1["tuned_ms"] <= r1["default_ms"] * 1.0001
    again = autotune.tune(g, tune_src, k=1, cache_path=cache)   # served from the cache
    assert again.pop("cached") is True and again == r1
    ws = bfs.workspace(g, 1, DEV)
    par = torch.empty(n, dtype=torch.int32, device=DEV)
    dep = torch.empty(n, dtype=torch.int32, device=DEV)
    for s in graphgen.random_sources(off, 4, seed=2):
        bfs.bfs_run(g, int(s), par, dep, ws, autotune.opts_from(r1, parent_mode=bfs.BFS_PARENT_MIN))
        torch.cuda.synchronize()
        rp, rd = orc.bfs_min(off, cols, int(s))
        assert np.array_equal(dep.cpu().numpy(), rd) and np.array_equal(par.cpu().numpy(), rp)
    rk = autotune.tune(g, graphgen.random_sources(off, 16, seed=99), k=16)
    srcs = graphgen.random_sources(off, 16, seed=2)
    wsm = bfs.workspace(g, 16, DEV)
    mp = torch.empty(16 * n, dtype=torch.int32, device=DEV)
    md = torch.empty(16 * n, dtype=torch.int32, device=DEV)
    bfs.bfs_run_multi(g, srcs, mp, md, wsm, autotune.opts_from(rk))
    torch.cuda.synchronize()
    mp, md = mp.cpu().numpy().reshape(16, n), md.cpu().numpy().reshape(16, n)
    for j, s in enumerate(srcs):
        rp, rd = orc.bfs_min(off, cols, int(s))
        assert np.array_equal(md[j], rd) and np.array_equal(mp[j], rp)
