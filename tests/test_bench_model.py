"""Host logic of the benchmark: the algorithmic-bytes model behind the roofline
entry, the gate on the committed traffic record, and the one-GPU refusal."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _stats(dirs, nf, mf, mu, fill_level=-1):
    return {"levels": len(dirs), "level_dir": dirs, "level_nf": nf, "level_mf": mf, "level_mu": mu,
            "fill_level": fill_level}


def _row(levels):
    return {"source": 7, "levels": levels}


# a made-up search: [n_f, m_f, m_u, u (unvisited with edges), x (first-hit scan entries)] per level
ROW = _row([[1, 16, 9000, 900, 9500], [40, 5000, 4000, 899, 9000], [7, 30, 3970, 859, 900],
            [0, 0, 3970, 852, 852]])


def test_level_bytes_model_by_hand():
    # four levels: top-down, bottom-up, top-down, and the last that finds nothing
    n, wo, iso = 1 << 20, 8, 1000
    st = _stats([0, 1, 0, 0], [1, 40, 7, 0], [16, 5000, 30, 0], [9000, 4000, 3970, 3970])
    out = bench.level_bytes(st, ROW, n, wo, iso)
    assert [k for k, _ in out] == ["td_expand", "bu_sweep", "td_expand", "td_expand"]
    # top-down: |F|(4 + 2 W_o) + 8 D_F + 12 |N|
    assert out[0][1] == 1 * (4 + 16) + 16 * 8 + 40 * 12
    # bottom-up: 3 n/8 bitmap words + 2 W_o |U| + 4 X + 8 |N|, with U and X from the table
    assert out[1][1] == 3 * (n / 8) + 2 * wo * 899 + 4 * 9000 + 8 * 7
    assert out[2][1] == 7 * (4 + 16) + 30 * 8 + 0
    assert out[3][1] == 0


def test_fill_is_counted_on_the_sweep_that_writes_it():
    n, wo, iso = 1 << 20, 8, 1000
    plain = bench.level_bytes(_stats([0, 1, 0, 0], [1, 40, 7, 0], [16, 5000, 30, 0], [9000, 4000, 3970, 3970]),
                              ROW, n, wo, iso)
    filled = bench.level_bytes(_stats([0, 1, 0, 0], [1, 40, 7, 0], [16, 5000, 30, 0], [9000, 4000, 3970, 3970],
                                      fill_level=1), ROW, n, wo, iso)
    # -1 for the isolated vertices and the unvisited ones this level did not reach
    assert filled[1][1] - plain[1][1] == 8 * (iso + 899 - 7)
    assert [b for _, b in filled[:1] + filled[2:]] == [b for _, b in plain[:1] + plain[2:]]


def test_library_counts_must_equal_the_table():
    n, wo, iso = 1 << 20, 8, 1000
    with pytest.raises(ValueError):
        bench.level_bytes(_stats([0, 1, 0, 0], [1, 41, 7, 0], [16, 5000, 30, 0], [9000, 4000, 3970, 3970]),
                          ROW, n, wo, iso)
    with pytest.raises(ValueError):
        bench.level_bytes(_stats([0, 1, 0], [1, 40, 7], [16, 5000, 30], [9000, 4000, 3970]), ROW, n, wo, iso)


def test_work_table_matches_only_its_graph(tmp_path, monkeypatch):
    import json
    doc = {"graph": {"kind": "kronecker", "scale": 9, "edgefactor": 16, "seed": 1, "n": 512, "nnz": 1000,
                     "isolated": 3}, "source_seed": 2, "level_fields": ["n_f", "m_f", "m_u", "u", "x"],
           "sources": [{"source": 7, "levels": ROW["levels"], "dir": [0, 1, 0, 0]}]}
    (tmp_path / "kron9_work_model.json").write_text(json.dumps(doc))
    monkeypatch.setattr(bench, "WORK_TABLE", str(tmp_path / "kron{scale}_work_model.json"))
    t, _ = bench.load_work_table(9, 16, 1, 2, 512, 1000)
    assert t["isolated"] == 3 and t["rows"][7]["levels"] == ROW["levels"]
    assert bench.load_work_table(9, 16, 1, 3, 512, 1000)[0] is None     # other source seed
    assert bench.load_work_table(9, 16, 1, 2, 512, 1002)[0] is None     # other graph
    assert bench.load_work_table(10, 16, 1, 2, 512, 1000)[0] is None    # no table


def test_work_counts_recount_by_hand(orc):
    """The table's u and x columns come from the oracle's bottom-up scan
    counter; on a small graph, every level's pair equals a plain recount from
    the oracle's depths (the rows scanned in order up to their first vertex of
    level d)."""
    import numpy as np

    import graphgen
    off, cols = graphgen.kronecker(10, seed=1)
    s = int(graphgen.random_sources(off, 1, seed=2)[0])
    _, depth = orc.bfs(off, cols, s)
    deg = np.diff(off)
    L = depth.max() + 1
    for d in range(L):
        x, un = orc.bu_scan_lengths(off, cols, depth, d)
        # unvisited before level d: depth -1 or deeper than d
        unv = (depth < 0) | (depth > d)
        assert un == int(unv.sum())
        # scan lengths: each unvisited row up to its first member of L_d, else whole
        xs = 0
        for v in np.flatnonzero(unv & (deg > 0)):
            row = cols[off[v]:off[v + 1]]
            hit = np.flatnonzero(depth[row] == d)
            xs += int(hit[0]) + 1 if hit.size else row.size
        assert x == xs


def test_traffic_record_is_used_only_for_the_profiled_kernels(monkeypatch):
    real = bench.kernel_source_hash()
    rec = bench.read_traffic("bu_sweep")
    if rec is None:
        pytest.skip("the committed profile does not match these kernel sources")
    assert rec > 0
    # another kernel name, or changed sources, give no traffic figure
    assert bench.read_traffic("td_expand") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: real[::-1])
    assert bench.read_traffic("bu_sweep") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
