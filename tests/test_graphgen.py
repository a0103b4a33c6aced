"""Input generators: cleanup invariants, determinism, block extraction."""
import os
import subprocess
import sys

import numpy as np
import pytest

import graphgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def check_clean_symmetric(off, cols):
    n = off.size - 1
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == cols.size
    assert cols.size % 2 == 0
    rows = np.repeat(np.arange(n), np.diff(off))
    assert not np.any(rows == cols), "self-loop"
    # strictly increasing inside each row: sorted and no duplicates
    same_row = rows[1:] == rows[:-1]
    assert np.all(np.diff(cols.astype(np.int64))[same_row] > 0)
    # symmetric: the multiset of (u,v) equals that of (v,u)
    a = np.sort(rows.astype(np.int64) * n + cols)
    b = np.sort(cols.astype(np.int64) * n + rows)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("maker", [
    lambda: graphgen.kronecker(12, seed=1),
    lambda: graphgen.kronecker(10, seed=7, permute=False),
    lambda: graphgen.erdos_renyi(5000, 8, seed=3),
    lambda: graphgen.grid2d(17, 23),
])
def test_clean_symmetric(maker):
    off, cols = maker()
    check_clean_symmetric(off, cols)


def test_kronecker_matches_raw_draws():
    scale = 9
    off, cols = graphgen.kronecker(scale, seed=4)
    src, dst = graphgen.kronecker_edges(scale, seed=4)
    n = 1 << scale
    keep = src != dst
    e = set(zip(src[keep].tolist(), dst[keep].tolist())) | set(zip(dst[keep].tolist(), src[keep].tolist()))
    rows = np.repeat(np.arange(n), np.diff(off))
    assert set(zip(rows.tolist(), cols.tolist())) == e


def test_kronecker_skew_and_size():
    off, cols = graphgen.kronecker(14, seed=1)
    deg = np.diff(off)
    n = deg.size
    assert cols.size <= 2 * 16 * n and cols.size > 1.5 * 16 * n * 0.8
    # skewed degrees: the maximum is far above the mean
    assert deg.max() > 50 * deg.mean()
    # ER is not skewed
    off2, _ = graphgen.erdos_renyi(1 << 14, 8, seed=1)
    d2 = np.diff(off2)
    assert d2.max() < 6 * d2.mean()


def test_deterministic_and_thread_count_independent():
    code = ("import graphgen,hashlib;o,c=graphgen.kronecker(12,seed=9);"
            "print(hashlib.sha1(o.tobytes()+c.tobytes()).hexdigest())")
    outs = set()
    for t in ("1", "3", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=t, PYTHONPATH=ROOT)
        outs.add(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                                check=True).stdout.strip())
    assert len(outs) == 1


def test_relabel_is_a_bijection():
    for scale in (1, 2, 5, 11):
        img = {graphgen._load().gg_kron_relabel(scale, 3, x) for x in range(1 << scale)}
        assert img == set(range(1 << scale))


def test_grid_degree_and_ids():
    off, cols = graphgen.grid2d(4, 5)
    deg = np.diff(off).reshape(4, 5)
    assert deg[0, 0] == 2 and deg[0, 2] == 3 and deg[1, 1] == 4
    assert cols[off[6]:off[7]].tolist() == [1, 5, 7, 11]


def test_block_from_draws_equals_block_from_csr():
    scale = 10
    off, cols = graphgen.kronecker(scale, seed=2)
    n = 1 << scale
    R = C = n // 4
    for (i, j) in [(0, 1), (2, 2), (3, 0)]:
        a = graphgen.csr_block(off, cols, i * R, R, j * C, C)
        b = graphgen.kronecker_block(scale, i * R, R, j * C, C, seed=2)
        for k in ("jc", "cp", "ir", "jr", "rp", "ic"):
            assert np.array_equal(a[k], b[k]), k
        # DCSC and DCSR describe the same entry set
        rows_c = a["ir"]
        cols_c = np.repeat(a["jc"], np.diff(a["cp"]))
        rows_r = np.repeat(a["jr"], np.diff(a["rp"]))
        cols_r = a["ic"]
        assert set(zip(rows_c.tolist(), cols_c.tolist())) == set(zip(rows_r.tolist(), cols_r.tolist()))


def test_bitmap_helpers_roundtrip():
    rng = np.random.default_rng(0)
    for nb in (1, 63, 64, 65, 1000):
        bits = rng.random(nb) < 0.3
        w = graphgen.bits_to_words(bits)
        assert w.size == (nb + 63) // 64
        assert np.array_equal(graphgen.words_to_bits(w, nb), bits)
        for i in np.flatnonzero(bits):
            assert (int(w[i // 64]) >> int(i % 64)) & 1


def test_sources_and_subsets():
    off, _ = graphgen.kronecker(10, seed=1)
    s = graphgen.random_sources(off, 64, seed=2)
    assert len(set(s.tolist())) == 64 and np.all(np.diff(off)[s] > 0)
    assert np.array_equal(s, graphgen.random_sources(off, 64, seed=2))
    f = graphgen.random_sorted_subset(1000, 37, seed=5)
    assert f.size == 37 and np.all(np.diff(f) > 0) and f.max() < 1000
