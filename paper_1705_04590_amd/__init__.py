"""Python binding of libbfs (include/bfs.h) -- argument marshalling only.

Every function here has the name of the C entry point it calls and does no
search work of its own: it checks tensor placement, dtype and size, passes raw
device pointers and the current HIP stream, and turns a non-zero status into a
``BfsError``.  PyTorch supplies device memory and streams.  There is no CPU
fallback: if ``libbfs.so`` is missing the first call raises.

torch is imported before libbfs.so is loaded so that both share the HIP
runtime torch already loaded.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfs.so")

BFS_OK = 0
BFS_DIR_DO, BFS_DIR_TD, BFS_DIR_BU = 0, 1, 2
BFS_PARENT_ANY, BFS_PARENT_MIN = 0, 1
BFS_GRAPH_SYMMETRIC, BFS_GRAPH_SORTED, BFS_GRAPH_VALIDATE = 0x1, 0x2, 0x4
KERNEL_KINDS = ["init", "td_scan", "td_expand", "bu_sweep", "convert", "ms_level", "ms_output", "block", "fused"]
STATS_MAX_LEVELS = 64
STATUS_NAMES = {0: "BFS_OK", 1: "BFS_E_INVALID_ARG", 2: "BFS_E_OUT_OF_RANGE", 3: "BFS_E_UNSORTED",
                4: "BFS_E_NOT_SYMMETRIC", 5: "BFS_E_NO_MEMORY", 6: "BFS_E_HIP", 7: "BFS_E_BUDGET",
                8: "BFS_E_UNSUPPORTED"}
EXPORTED = ["bfs_opts_default", "bfs_last_error", "bfs_status_string", "bfs_create_graph_csr",
            "bfs_create_graph_dcsc", "bfs_destroy_graph", "bfs_workspace_bytes", "bfs_run", "bfs_run_multi",
            "bfs_block_td", "bfs_block_bu", "bfs_block_td_noalloc", "bfs_block_set_union"]


class BfsError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class bfs_opts(ctypes.Structure):
    _fields_ = [("dir", ctypes.c_int32), ("parent_mode", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("timing", ctypes.c_int32), ("bu_serial", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("td_claim", ctypes.c_int32), ("small_edges", ctypes.c_int32),
                ("persist_edges", ctypes.c_int32), ("persist_groups", ctypes.c_int32),
                ("bu_head", ctypes.c_int32), ("td_prepass", ctypes.c_int32), ("bu_segments", ctypes.c_int32),
                ("td_segments", ctypes.c_int32), ("td_seg_edges", ctypes.c_int32), ("td_block", ctypes.c_int32),
                ("bu_block", ctypes.c_int32), ("bu_group", ctypes.c_int32), ("fused_max_n", ctypes.c_int32)]


class bfs_stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("td_levels", ctypes.c_int32), ("bu_levels", ctypes.c_int32),
                ("fill_level", ctypes.c_int32), ("reached", ctypes.c_int64), ("isolated", ctypes.c_int64),
                ("edges_examined", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("launches", ctypes.c_int64 * 9), ("kernel_ms", ctypes.c_double * 9),
                ("level_dir", ctypes.c_int8 * STATS_MAX_LEVELS), ("level_nf", ctypes.c_int64 * STATS_MAX_LEVELS),
                ("level_mf", ctypes.c_int64 * STATS_MAX_LEVELS), ("level_mu", ctypes.c_int64 * STATS_MAX_LEVELS),
                ("level_unvisited", ctypes.c_int64 * STATS_MAX_LEVELS),
                ("level_examined", ctypes.c_int64 * STATS_MAX_LEVELS),
                ("level_ms", ctypes.c_float * STATS_MAX_LEVELS), ("td_claims", ctypes.c_int64),
                ("td_duplicates", ctypes.c_int64)]

    def as_dict(self) -> dict:
        L = min(self.levels, STATS_MAX_LEVELS)
        return {
            "levels": self.levels, "td_levels": self.td_levels, "bu_levels": self.bu_levels,
            "fill_level": self.fill_level,
            "reached": self.reached, "isolated": self.isolated, "edges_examined": self.edges_examined, "total_ms": self.total_ms,
            "launches": {k: self.launches[i] for i, k in enumerate(KERNEL_KINDS)},
            "kernel_ms": {k: self.kernel_ms[i] for i, k in enumerate(KERNEL_KINDS)},
            "level_dir": list(self.level_dir[:L]), "level_nf": list(self.level_nf[:L]),
            "level_mf": list(self.level_mf[:L]), "level_mu": list(self.level_mu[:L]),
            "level_unvisited": list(self.level_unvisited[:L]), "level_examined": list(self.level_examined[:L]),
            "level_ms": list(self.level_ms[:L]),
            "td_claims": self.td_claims, "td_duplicates": self.td_duplicates,
        }


_lib = None
_vp = ctypes.c_void_p


def lib():
    """The loaded libbfs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python __graft_entry__.py` or "
                               "`python paper_1705_04590_amd/_build.py` first")
        L = ctypes.CDLL(LIB_PATH)
        L.bfs_opts_default.argtypes = [ctypes.POINTER(bfs_opts)]
        L.bfs_opts_default.restype = None
        L.bfs_last_error.restype = ctypes.c_char_p
        L.bfs_status_string.argtypes = [ctypes.c_int]
        L.bfs_status_string.restype = ctypes.c_char_p
        L.bfs_create_graph_csr.argtypes = [ctypes.c_int64, _vp, ctypes.c_int, _vp, ctypes.c_int64, ctypes.c_uint32,
                                           _vp, ctypes.POINTER(_vp)]
        L.bfs_create_graph_dcsc.argtypes = [ctypes.c_int64] * 4 + [ctypes.c_int64, _vp, _vp, _vp, ctypes.c_int64,
                                                                   _vp, _vp, _vp, ctypes.c_int64, ctypes.c_uint32,
                                                                   _vp, ctypes.POINTER(_vp)]
        L.bfs_destroy_graph.argtypes = [_vp]
        L.bfs_destroy_graph.restype = None
        L.bfs_workspace_bytes.argtypes = [_vp, ctypes.c_int]
        L.bfs_workspace_bytes.restype = ctypes.c_size_t
        L.bfs_run.argtypes = [_vp, ctypes.c_int64, ctypes.POINTER(bfs_opts), _vp, _vp, _vp, ctypes.c_size_t, _vp,
                              ctypes.POINTER(bfs_stats)]
        L.bfs_run_multi.argtypes = [_vp, _vp, ctypes.c_int, ctypes.POINTER(bfs_opts), _vp, _vp, _vp,
                                    ctypes.c_size_t, _vp, ctypes.POINTER(bfs_stats)]
        L.bfs_block_td.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.bfs_block_bu.argtypes = [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int64, _vp, _vp, _vp, _vp,
                                   ctypes.c_size_t, _vp]
        L.bfs_block_td_noalloc.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp, _vp, _vp]
        L.bfs_block_set_union.argtypes = [_vp, ctypes.c_int]
        for name in ("bfs_create_graph_csr", "bfs_create_graph_dcsc", "bfs_run", "bfs_run_multi", "bfs_block_td",
                     "bfs_block_bu", "bfs_block_td_noalloc", "bfs_block_set_union"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != BFS_OK:
        raise BfsError(status, where, lib().bfs_last_error().decode(errors="replace"))


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dev(t: torch.Tensor, dtype, name: str, numel: int | None = None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs {numel} elements, has {t.numel()}")
    return t.data_ptr()


class Graph:
    """Owning wrapper of a bfs_graph* plus the tensors it borrows."""

    def __init__(self, handle, keep, kind, **meta):
        self.handle = handle
        self._keep = keep
        self.kind = kind
        self.__dict__.update(meta)

    def close(self):
        if self.handle:
            lib().bfs_destroy_graph(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bfs_opts_default(**overrides) -> bfs_opts:
    o = bfs_opts()
    lib().bfs_opts_default(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def bfs_status_string(status: int) -> str:
    return lib().bfs_status_string(status).decode()


def bfs_last_error() -> str:
    return lib().bfs_last_error().decode(errors="replace")


def bfs_create_graph_csr(offsets: torch.Tensor, cols: torch.Tensor, flags: int = 0, stream=None) -> Graph:
    if offsets.dtype not in (torch.int32, torch.int64):
        raise TypeError("offsets must be int32 or int64")
    n = offsets.numel() - 1
    po = _dev(offsets, offsets.dtype, "offsets")
    pc = _dev(cols, torch.int32, "cols") if cols.numel() else (cols.data_ptr() if cols.is_cuda else 0)
    h = _vp()
    _check(lib().bfs_create_graph_csr(n, po, offsets.element_size(), pc, cols.numel(), flags, _stream(stream),
                                      ctypes.byref(h)), "bfs_create_graph_csr")
    return Graph(h, (offsets, cols), "csr", n=n, nnz=cols.numel(), flags=flags,
                 offset_bytes=offsets.element_size())


def _opt_ptr(t, dtype, name, numel=None):
    if t is None or t.numel() == 0:
        return None
    return _dev(t, dtype, name, numel)


def bfs_create_graph_dcsc(nrows: int, ncols: int, row_base: int, col_base: int, jc, cp, ir, jr=None, rp=None,
                          ic=None, flags: int = 0, stream=None) -> Graph:
    """Wrap a DCSC block (jc, cp, ir) and optionally its row-compressed copy (jr, rp, ic)."""
    nzc, nnz = jc.numel(), ir.numel()
    pcp = _dev(cp, torch.int64, "cp", nzc + 1)
    nzr, prp = 0, None
    if jr is not None:
        nzr = jr.numel()
        prp = _dev(rp, torch.int64, "rp", nzr + 1)
    h = _vp()
    _check(lib().bfs_create_graph_dcsc(nrows, ncols, row_base, col_base, nzc, _opt_ptr(jc, torch.int32, "jc"), pcp,
                                       _opt_ptr(ir, torch.int32, "ir"), nzr,
                                       _opt_ptr(jr, torch.int32, "jr") if jr is not None else None,
                                       prp, _opt_ptr(ic, torch.int32, "ic") if ic is not None else None, nnz, flags,
                                       _stream(stream), ctypes.byref(h)), "bfs_create_graph_dcsc")
    return Graph(h, (jc, cp, ir, jr, rp, ic), "dcsc", nrows=nrows, ncols=ncols, row_base=row_base,
                 col_base=col_base, nnz=nnz, flags=flags)


def bfs_destroy_graph(g: Graph):
    g.close()


def bfs_workspace_bytes(g: Graph, k: int = 1) -> int:
    return int(lib().bfs_workspace_bytes(g.handle, k))


def workspace(g: Graph, k: int = 1, device=None) -> torch.Tensor:
    """A device byte tensor large enough for bfs_run (k=1), bfs_run_multi (k) or the block calls
    (zero-filled, as the block calls require before first use)."""
    nb = bfs_workspace_bytes(g, k)
    if nb == 0:
        raise BfsError(1, "bfs_workspace_bytes", f"no workspace size for k={k}")
    if g.kind == "dcsc":
        return torch.zeros(nb, dtype=torch.uint8, device=device or "cuda")
    return torch.empty(nb, dtype=torch.uint8, device=device or "cuda")


def bfs_run(g: Graph, source: int, parent: torch.Tensor, depth: torch.Tensor, ws: torch.Tensor,
            opts: bfs_opts | None = None, stream=None, stats: bfs_stats | None = None) -> bfs_stats:
    st = stats if stats is not None else bfs_stats()
    pp = _dev(parent, torch.int32, "parent", g.n)
    pd = _dev(depth, torch.int32, "depth", g.n)
    pw = _dev(ws, torch.uint8, "workspace")
    _check(lib().bfs_run(g.handle, int(source), ctypes.byref(opts) if opts is not None else None, pp, pd, pw,
                         ws.numel(), _stream(stream), ctypes.byref(st)), "bfs_run")
    return st


def bfs_run_multi(g: Graph, sources, parent: torch.Tensor | None, depth: torch.Tensor, ws: torch.Tensor,
                  opts: bfs_opts | None = None, stream=None, stats: bfs_stats | None = None) -> bfs_stats:
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int64))
    k = src.size
    st = stats if stats is not None else bfs_stats()
    pp = _dev(parent, torch.int32, "parent", k * g.n) if parent is not None else None
    pd = _dev(depth, torch.int32, "depth", k * g.n)
    pw = _dev(ws, torch.uint8, "workspace")
    _check(lib().bfs_run_multi(g.handle, src.ctypes.data, k, ctypes.byref(opts) if opts is not None else None, pp,
                               pd, pw, ws.numel(), _stream(stream), ctypes.byref(st)), "bfs_run_multi")
    return st


def bfs_block_td(g: Graph, frontier: torch.Tensor, out_rows: torch.Tensor, out_parents: torch.Tensor,
                 nout: torch.Tensor, ws: torch.Tensor, stream=None):
    """Alg. 3 local discovery on a DCSC block (asynchronous). ws must be zero-filled before its first use."""
    nf = frontier.numel()
    _check(lib().bfs_block_td(g.handle, _opt_ptr(frontier, torch.int32, "frontier"), nf,
                              _dev(out_rows, torch.int32, "out_rows", g.nrows),
                              _dev(out_parents, torch.int32, "out_parents", g.nrows),
                              _dev(nout, torch.int64, "nout", 1), _dev(ws, torch.uint8, "workspace"), ws.numel(),
                              _stream(stream)), "bfs_block_td")


def bfs_block_set_union(g: Graph, mode: int):
    """Union of the frontier columns in bfs_block_td: 0 by density, 1 sorted union when it fits, -1 accumulator."""
    _check(lib().bfs_block_set_union(g.handle, int(mode)), "bfs_block_set_union")


def bfs_block_td_noalloc(g: Graph, frontier: torch.Tensor, out_rows: torch.Tensor, out_parents: torch.Tensor,
                         nout: torch.Tensor, stream=None):
    """bfs_block_td without a caller workspace: the library's static device array is used (asynchronous)."""
    nf = frontier.numel()
    _check(lib().bfs_block_td_noalloc(g.handle, _opt_ptr(frontier, torch.int32, "frontier"), nf,
                                      _dev(out_rows, torch.int32, "out_rows", g.nrows),
                                      _dev(out_parents, torch.int32, "out_parents", g.nrows),
                                      _dev(nout, torch.int64, "nout", 1), _stream(stream)), "bfs_block_td_noalloc")


def bfs_block_bu(g: Graph, fbits: torch.Tensor, completed: torch.Tensor, row_lo: int, row_hi: int,
                 out_rows: torch.Tensor, out_parents: torch.Tensor, nout: torch.Tensor, ws: torch.Tensor, stream=None):
    """Alg. 4 local discovery sub-step on a DCSC block (asynchronous); bitmaps are int64 tensors of words."""
    _check(lib().bfs_block_bu(g.handle, _dev(fbits, torch.int64, "fbits", (g.ncols + 63) // 64),
                              _dev(completed, torch.int64, "completed", (g.nrows + 63) // 64), row_lo, row_hi,
                              _dev(out_rows, torch.int32, "out_rows", g.nrows),
                              _dev(out_parents, torch.int32, "out_parents", g.nrows),
                              _dev(nout, torch.int64, "nout", 1), _dev(ws, torch.uint8, "workspace"), ws.numel(),
                              _stream(stream)), "bfs_block_bu")
