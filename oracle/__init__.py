"""CPU oracle for the breadth-first search -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.  The arithmetic lives in ``bfs_oracle.c`` (plain serial
C, built with gcc into ``liboracle.so``); this module only marshals numpy
arrays.  See the header of ``bfs_oracle.c`` for what each function follows in
the paper (Alg. 1, Alg. 2, Section 4.2 semiring, Section 4.4 heuristic, Eq. 1
blocks with Alg. 3 / Alg. 4 local discovery).

Parity status: every function here is pinned by tests/test_oracle_pins.py
(brute force on tiny graphs, closed forms, the Fig. 2 worked block, BFS-tree
invariants, planted-mistake checks); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)

VALIDATE_CODES = {
    0: "ok", 1: "source", 2: "pairing", 3: "range", 4: "root", 5: "not_edge",
    6: "parent_level", 7: "leak", 8: "skip",
}


def build(defines=(), out_path: str | None = None, opt=("-O2",)) -> str:
    """Compile the oracle with gcc -O2 (``defines`` is for planted-mistake tests)."""
    out = out_path or _LIB_PATH
    tmp = out + ".tmp"
    cmd = ["gcc", *opt, "-shared", "-fPIC", "-o", tmp, _SRC] + [f"-D{d}" for d in defines]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_TIMING_PATH = os.path.join(_HERE, "liboracle_native.so")


def load_timing():
    """The same oracle source built for timing on this machine (gcc -O3 -march=native), loaded.

    Only the benchmark's CPU-baseline leg uses it; it is rebuilt on every call
    so that it is native to the host that runs it."""
    build(out_path=_TIMING_PATH, opt=("-O3", "-march=native"))
    return Oracle(_bind(ctypes.CDLL(_TIMING_PATH)))


def _bind(lib):
    lib.oracle_bfs.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int64, _i32p, _i32p]
    lib.oracle_bfs_bottom_up.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int64, _i32p, _i32p]
    lib.oracle_min_parent.argtypes = [ctypes.c_int64, _i64p, _i32p, _i32p, _i32p]
    lib.oracle_validate.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int64, _i32p, _i32p, _i64p]
    lib.oracle_level_stats.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int64, _i64p, _i64p,
                                       _i64p, _i64p]
    lib.oracle_direction_schedule.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i64p, _i64p,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_int, _i32p]
    lib.oracle_bu_scan_lengths.argtypes = [ctypes.c_int64, _i64p, _i32p, _i32p, ctypes.c_int32, _i64p,
                                           _i64p]
    lib.oracle_block_td.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _i32p, _i32p,
                                    ctypes.c_int64, ctypes.c_int64, _i32p, _i32p, _i32p, _i64p]
    lib.oracle_block_bu.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _i32p, _i32p,
                                    ctypes.c_int64, _u64p, _u64p, ctypes.c_int64, ctypes.c_int64, _i32p,
                                    _i32p, _i64p]
    return lib


def load(path: str | None = None):
    """Load (building on first use) the oracle library; ``path`` loads a variant build."""
    global _lib
    if path is not None:
        return Oracle(_bind(ctypes.CDLL(path)))
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return Oracle(_lib)


def _csr(offsets, cols):
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    c = np.ascontiguousarray(cols, dtype=np.int32)
    if c.size == 0:
        c = np.zeros(1, np.int32)
    return off, c


def _p(a, t):
    return a.ctypes.data_as(t)


class Oracle:
    def __init__(self, lib):
        self.lib = lib

    def bfs(self, offsets, cols, source: int):
        """Alg. 1 with a FIFO queue -> (parent_first, depth), int32."""
        off, c = _csr(offsets, cols)
        n = off.size - 1
        parent = np.empty(max(n, 1), np.int32)
        depth = np.empty(max(n, 1), np.int32)
        rc = self.lib.oracle_bfs(n, _p(off, _i64p), _p(c, _i32p), source, _p(parent, _i32p), _p(depth, _i32p))
        if rc:
            raise ValueError(f"oracle_bfs: bad input (code {rc})")
        return parent[:n], depth[:n]

    def bfs_bottom_up(self, offsets, cols, source: int):
        """Alg. 2 (first hit in stored row order) -> (parent, depth)."""
        off, c = _csr(offsets, cols)
        n = off.size - 1
        parent = np.empty(max(n, 1), np.int32)
        depth = np.empty(max(n, 1), np.int32)
        rc = self.lib.oracle_bfs_bottom_up(n, _p(off, _i64p), _p(c, _i32p), source, _p(parent, _i32p),
                                           _p(depth, _i32p))
        if rc:
            raise ValueError(f"oracle_bfs_bottom_up: bad input (code {rc})")
        return parent[:n], depth[:n]

    def min_parent(self, offsets, cols, depth):
        off, c = _csr(offsets, cols)
        n = off.size - 1
        d = np.ascontiguousarray(depth, dtype=np.int32)
        out = np.empty(max(n, 1), np.int32)
        rc = self.lib.oracle_min_parent(n, _p(off, _i64p), _p(c, _i32p), _p(d, _i32p), _p(out, _i32p))
        if rc:
            raise ValueError("oracle_min_parent: bad input")
        return out[:n]

    def bfs_min(self, offsets, cols, source: int):
        """(min-id parent, depth)."""
        _, depth = self.bfs(offsets, cols, source)
        return self.min_parent(offsets, cols, depth), depth

    def validate(self, offsets, cols, source: int, parent, depth):
        """BFS-tree invariants -> (name of the first violated invariant or 'ok', vertex)."""
        off, c = _csr(offsets, cols)
        n = off.size - 1
        p = np.ascontiguousarray(parent, dtype=np.int32)
        d = np.ascontiguousarray(depth, dtype=np.int32)
        bad = ctypes.c_int64()
        rc = self.lib.oracle_validate(n, _p(off, _i64p), _p(c, _i32p), source, _p(p, _i32p), _p(d, _i32p),
                                      ctypes.byref(bad))
        if rc < 0:
            raise ValueError("oracle_validate: bad input")
        return VALIDATE_CODES[rc], bad.value

    def level_stats(self, offsets, depth):
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        n = off.size - 1
        d = np.ascontiguousarray(depth, dtype=np.int32)
        cap = int(d.max()) + 2 if d.size else 1
        nf, mf, mu = (np.zeros(cap, np.int64) for _ in range(3))
        nl = ctypes.c_int64()
        rc = self.lib.oracle_level_stats(n, _p(off, _i64p), _p(d, _i32p), cap, _p(nf, _i64p), _p(mf, _i64p),
                                         _p(mu, _i64p), ctypes.byref(nl))
        if rc:
            raise ValueError("oracle_level_stats failed")
        k = nl.value
        return nf[:k], mf[:k], mu[:k]

    def direction_schedule(self, n, n_f, m_f, m_u, alpha=15.0, beta=18.0, mode=0):
        """dir[d] in {0: top-down, 1: bottom-up}; mode 0 = heuristic, 1 = TD only, 2 = BU only."""
        n_f = np.ascontiguousarray(n_f, np.int64)
        m_f = np.ascontiguousarray(m_f, np.int64)
        m_u = np.ascontiguousarray(m_u, np.int64)
        out = np.zeros(max(n_f.size, 1), np.int32)
        self.lib.oracle_direction_schedule(int(n), n_f.size, _p(n_f, _i64p), _p(m_f, _i64p), _p(m_u, _i64p),
                                           float(alpha), float(beta), int(mode), _p(out, _i32p))
        return out[: n_f.size]

    def bu_scan_lengths(self, offsets, cols, depth, d: int):
        off, c = _csr(offsets, cols)
        n = off.size - 1
        dd = np.ascontiguousarray(depth, dtype=np.int32)
        s, u = ctypes.c_int64(), ctypes.c_int64()
        self.lib.oracle_bu_scan_lengths(n, _p(off, _i64p), _p(c, _i32p), _p(dd, _i32p), d, ctypes.byref(s),
                                        ctypes.byref(u))
        return s.value, u.value

    def block_td(self, nrows, ncols, erow, ecol, col_base, fcols):
        """Alg. 3 local discovery on a block -> (rows, parents) sorted by row."""
        er = np.ascontiguousarray(erow, np.int32)
        ec = np.ascontiguousarray(ecol, np.int32)
        f = np.ascontiguousarray(fcols, np.int32)
        if f.size == 0:
            f = np.zeros(1, np.int32)[:0].copy()
        out_r = np.empty(max(nrows, 1), np.int32)
        out_p = np.empty(max(nrows, 1), np.int32)
        k = ctypes.c_int64()
        fpad = f if f.size else np.zeros(1, np.int32)
        erp = er if er.size else np.zeros(1, np.int32)
        ecp = ec if ec.size else np.zeros(1, np.int32)
        rc = self.lib.oracle_block_td(nrows, ncols, er.size, _p(erp, _i32p), _p(ecp, _i32p), col_base, f.size,
                                      _p(fpad, _i32p), _p(out_r, _i32p), _p(out_p, _i32p), ctypes.byref(k))
        if rc:
            raise ValueError(f"oracle_block_td: bad input (code {rc})")
        return out_r[: k.value].copy(), out_p[: k.value].copy()

    def block_bu(self, nrows, ncols, erow, ecol, col_base, fbits, completed, row_lo, row_hi):
        """Alg. 4 local discovery sub-step -> (rows, parents, completed_after)."""
        er = np.ascontiguousarray(erow, np.int32)
        ec = np.ascontiguousarray(ecol, np.int32)
        fb = np.ascontiguousarray(fbits, np.uint64)
        comp = np.array(completed, dtype=np.uint64, copy=True)
        out_r = np.empty(max(nrows, 1), np.int32)
        out_p = np.empty(max(nrows, 1), np.int32)
        k = ctypes.c_int64()
        erp = er if er.size else np.zeros(1, np.int32)
        ecp = ec if ec.size else np.zeros(1, np.int32)
        fbp = fb if fb.size else np.zeros(1, np.uint64)
        cpp = comp if comp.size else np.zeros(1, np.uint64)
        rc = self.lib.oracle_block_bu(nrows, ncols, er.size, _p(erp, _i32p), _p(ecp, _i32p), col_base,
                                      _p(fbp, _u64p), _p(cpp, _u64p), row_lo, row_hi, _p(out_r, _i32p),
                                      _p(out_p, _i32p), ctypes.byref(k))
        if rc:
            raise ValueError(f"oracle_block_bu: bad input (code {rc})")
        return out_r[: k.value].copy(), out_p[: k.value].copy(), (cpp if comp.size else comp)
