"""Host logic of the benchmark: the algorithmic-bytes model behind the roofline
entry, the gate on the committed traffic record, and the one-GPU refusal."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _stats(dirs, nf, mf, unvisited, examined, isolated):
    return {"level_dir": dirs, "level_nf": nf, "level_mf": mf, "level_unvisited": unvisited,
            "level_examined": examined, "isolated": isolated}


def test_level_bytes_model_by_hand():
    # three levels: top-down, bottom-up, top-down (the last finds nothing)
    n, wo = 1 << 20, 8
    st = _stats([0, 1, 0], [1, 40, 7], [16, 5000, 30], [n - 1, n - 41, n - 48], [16, 9000, 30], 1000)
    out = bench.level_bytes(st, n, wo)
    assert [k for k, _ in out] == ["td_expand", "bu_sweep", "td_expand"]
    # top-down: |F|(4 + 2 W_o) + 8 D_F + 12 |N|
    assert out[0][1] == 1 * (4 + 16) + 16 * 8 + 40 * 12
    # bottom-up: 3 n/8 bitmap words + 2 W_o |U| + 4 X + 8 |N|, U without the isolated vertices
    u = (n - 41) - 1000
    assert out[1][1] == 3 * (n / 8) + 2 * wo * u + 4 * 9000 + 8 * 7
    # the last level has no next frontier
    assert out[2][1] == 7 * (4 + 16) + 30 * 8 + 0


def test_top_down_level_without_edges_costs_nothing():
    st = _stats([0], [3], [0], [10], [0], 0)
    assert bench.level_bytes(st, 64, 4) == [("td_expand", 0)]


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
