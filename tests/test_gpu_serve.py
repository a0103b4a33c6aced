"""The query server: each result equals the stand-alone search, admission under a tight budget,
overlap of batches on several slots, and the replay path."""
import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1705_04590_amd as bfs  # noqa: E402
from paper_1705_04590_amd import serve  # noqa: E402

DEV = torch.device("cuda:0")
FLAGS = bfs.BFS_GRAPH_SYMMETRIC | bfs.BFS_GRAPH_SORTED


def graphs():
    out = []
    for (off, cols) in (graphgen.kronecker(11, seed=1), graphgen.kronecker(13, seed=2), graphgen.grid2d(30, 41),
                        graphgen.erdos_renyi(4000, 3.0, seed=5)):
        d_off, d_cols = torch.from_numpy(off).to(DEV), torch.from_numpy(cols).to(DEV)
        out.append((off, cols, d_off, d_cols, bfs.bfs_create_graph_csr(d_off, d_cols, FLAGS)))
    return out


def alone(entry, s):
    off, cols, _, _, g = entry
    n = off.size - 1
    ws = bfs.workspace(g, 1, DEV)
    p = torch.empty(n, dtype=torch.int32, device=DEV)
    d = torch.empty(n, dtype=torch.int32, device=DEV)
    bfs.bfs_run(g, int(s), p, d, ws, bfs.bfs_opts_default(parent_mode=bfs.BFS_PARENT_MIN))
    torch.cuda.synchronize()
    return p.cpu().numpy(), d.cpu().numpy()


def run_mix(gs, reqs, **opts):
    srv = serve.Server(serve.bfs_server_opts_default(**opts))
    gids = [srv.bfs_server_add_graph(e[4]) for e in gs]
    outs = []
    for rid, (gi, s) in enumerate(reqs):
        n = gs[gi][0].size - 1
        d = np.full(n, -7, np.int32)
        p = np.full(n, -7, np.int32)
        srv.bfs_server_submit(gids[gi], int(s), rid, d, p)
        outs.append((gi, s, p, d))
    srv.bfs_server_drain()
    st = srv.bfs_server_stats_get()
    ids, lat, bsz, seq = srv.bfs_server_records()
    srv.bfs_server_destroy()
    return outs, st, (ids, lat, bsz, seq)


def test_each_result_same_alone_and_in_the_mix(orc):
    gs = graphs()
    rng = np.random.default_rng(0)
    reqs = []
    for _ in range(150):
        gi = int(rng.integers(0, len(gs)))
        s = int(graphgen.random_sources(gs[gi][0], 1, seed=int(rng.integers(0, 1 << 30)))[0])
        reqs.append((gi, s))
    outs, st, (ids, lat, bsz, seq) = run_mix(gs, reqs, slots=3, max_batch=64, want_parent=1,
                                             hbm_budget=2 << 30)
    assert st["completed"] == len(reqs) and sorted(ids.tolist()) == list(range(len(reqs)))
    assert st["batches"] < len(reqs)          # same-graph queries were packed together
    assert (lat > 0).all() and st["p99_us"] >= st["p50_us"] > 0
    cache = {}
    for gi, s, p, d in outs:
        if (gi, s) not in cache:
            cache[(gi, s)] = alone(gs[gi], s)
        ap, ad = cache[(gi, s)]
        assert np.array_equal(d, ad) and np.array_equal(p, ap)
    # and against the oracle for a few
    for gi, s, p, d in outs[:8]:
        rp, rd = orc.bfs_min(gs[gi][0], gs[gi][1], int(s))
        assert np.array_equal(d, rd) and np.array_equal(p, rp)


def test_tight_budget_queues_and_loses_nothing():
    gs = graphs()
    big = [gs[1]]
    n = big[0][0].size - 1
    # room for one single-query batch only (single-source workspace plus depth
    # and parent): every batch shrinks to one query and they run one at a time
    one = bfs.bfs_workspace_bytes(big[0][4], 1) + 2 * 4 * n + 4096
    reqs = [(0, int(s)) for s in graphgen.random_sources(big[0][0], 40, seed=1)]
    outs, st, (ids, lat, bsz, seq) = run_mix(big, reqs, slots=4, max_batch=64, want_parent=1, hbm_budget=one)
    assert st["completed"] == 40 and st["max_inflight"] == 1 and st["batches"] == 40
    # one batch at a time: their spans on the device do not overlap either
    assert st["device_max_overlap"] == 1
    for gi, s, p, d in outs:
        ap, ad = alone(big[gi], s)
        assert np.array_equal(d, ad) and np.array_equal(p, ap)
    with pytest.raises(bfs.BfsError) as e:
        srv = serve.Server(serve.bfs_server_opts_default(hbm_budget=1 << 16))
        gid = srv.bfs_server_add_graph(gs[1][4])
        srv.bfs_server_submit(gid, 0, 0)
    assert e.value.status == 7


def test_batches_overlap_on_several_slots():
    gs = graphs()
    srv = serve.Server(serve.bfs_server_opts_default(slots=4, max_batch=8, hbm_budget=4 << 30))
    gids = [srv.bfs_server_add_graph(e[4]) for e in gs]
    rid = 0
    for rep in range(6):
        for gi in range(len(gs)):
            for s in graphgen.random_sources(gs[gi][0], 8, seed=rep):
                srv.bfs_server_submit(gids[gi], int(s), rid)
                rid += 1
    srv.bfs_server_drain()
    st = srv.bfs_server_stats_get()
    srv.bfs_server_destroy()
    assert st["completed"] == rid and st["max_inflight"] > 1
    # overlap seen on the device: HIP events around each batch on its slot's
    # stream give spans of which several are open at once
    assert st["device_max_overlap"] > 1


def test_replay_poisson_stream():
    gs = graphs()
    rng = np.random.default_rng(3)
    m = 300
    t = np.cumsum(rng.exponential(200.0, m))     # mean gap 200 us
    gi = rng.integers(0, len(gs), m).astype(np.int32)
    src = np.array([int(graphgen.random_sources(gs[g][0], 1, seed=i)[0]) for i, g in enumerate(gi)])
    srv = serve.Server(serve.bfs_server_opts_default(slots=2, hbm_budget=2 << 30))
    for e in gs:
        srv.bfs_server_add_graph(e[4])
    srv.bfs_server_replay(t, gi, src, np.arange(m))
    srv.bfs_server_drain()
    st = srv.bfs_server_stats_get()
    srv.bfs_server_destroy()
    assert st["completed"] == m and st["queries_per_s"] > 0
