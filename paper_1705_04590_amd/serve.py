"""Python binding of the query server (include/bfs_serve.h) -- argument marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np

from . import BfsError, Graph, bfs_opts, bfs_opts_default, lib

_vp = ctypes.c_void_p


class bfs_server_opts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("want_parent", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("hbm_budget", ctypes.c_size_t), ("batch_wait_us", ctypes.c_double),
                ("opts", bfs_opts)]


class bfs_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("max_inflight", ctypes.c_int64), ("mean_batch", ctypes.c_double), ("p50_us", ctypes.c_double),
                ("p99_us", ctypes.c_double), ("mean_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("first_arrival_s", ctypes.c_double), ("last_completion_s", ctypes.c_double),
                ("queries_per_s", ctypes.c_double), ("device_max_overlap", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_bound = False


def _lib():
    global _bound
    L = lib()
    if not _bound:
        L.bfs_server_opts_default.argtypes = [ctypes.POINTER(bfs_server_opts)]
        L.bfs_server_opts_default.restype = None
        L.bfs_server_create.argtypes = [ctypes.POINTER(bfs_server_opts), ctypes.POINTER(_vp)]
        L.bfs_server_add_graph.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_int32)]
        L.bfs_server_submit.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _vp, _vp]
        L.bfs_server_replay.argtypes = [_vp, ctypes.c_int64, _vp, _vp, _vp, _vp]
        L.bfs_server_drain.argtypes = [_vp]
        L.bfs_server_stats_get.argtypes = [_vp, ctypes.POINTER(bfs_server_stats)]
        L.bfs_server_records.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.bfs_server_destroy.argtypes = [_vp]
        L.bfs_server_destroy.restype = None
        for name in ("bfs_server_create", "bfs_server_add_graph", "bfs_server_submit", "bfs_server_replay",
                     "bfs_server_drain", "bfs_server_stats_get", "bfs_server_records"):
            getattr(L, name).restype = ctypes.c_int
        _bound = True
    return L


def _check(st, where):
    if st != 0:
        raise BfsError(st, where, lib().bfs_last_error().decode(errors="replace"))


def bfs_server_opts_default(**overrides) -> bfs_server_opts:
    o = bfs_server_opts()
    _lib().bfs_server_opts_default(ctypes.byref(o))
    search = overrides.pop("opts", None)
    for k, v in overrides.items():
        setattr(o, k, v)
    if search is not None:
        o.opts = search
    return o


class Server:
    """Owning wrapper of a bfs_server*; keeps registered graphs and host result buffers alive."""

    def __init__(self, opts: bfs_server_opts | None = None):
        self.h = _vp()
        self.opts = opts or bfs_server_opts_default()
        _check(_lib().bfs_server_create(ctypes.byref(self.opts), ctypes.byref(self.h)), "bfs_server_create")
        self.graphs = []
        self._bufs = []

    def bfs_server_add_graph(self, g: Graph) -> int:
        gid = ctypes.c_int32()
        _check(_lib().bfs_server_add_graph(self.h, g.handle, ctypes.byref(gid)), "bfs_server_add_graph")
        self.graphs.append(g)
        return gid.value

    def bfs_server_submit(self, graph_id: int, source: int, request_id: int, depth_out: np.ndarray | None = None,
                          parent_out: np.ndarray | None = None):
        for a in (depth_out, parent_out):
            if a is not None:
                assert a.dtype == np.int32 and a.flags.c_contiguous
                self._bufs.append(a)
        _check(_lib().bfs_server_submit(self.h, graph_id, int(source), int(request_id),
                                        depth_out.ctypes.data if depth_out is not None else None,
                                        parent_out.ctypes.data if parent_out is not None else None),
               "bfs_server_submit")

    def bfs_server_replay(self, arrival_us, graph_ids, sources, request_ids):
        t = np.ascontiguousarray(arrival_us, dtype=np.float64)
        g = np.ascontiguousarray(graph_ids, dtype=np.int32)
        s = np.ascontiguousarray(sources, dtype=np.int64)
        r = np.ascontiguousarray(request_ids, dtype=np.int64)
        self._bufs += [t, g, s, r]
        _check(_lib().bfs_server_replay(self.h, t.size, t.ctypes.data, g.ctypes.data, s.ctypes.data, r.ctypes.data),
               "bfs_server_replay")

    def bfs_server_drain(self):
        _check(_lib().bfs_server_drain(self.h), "bfs_server_drain")
        self._bufs = []

    def bfs_server_stats_get(self) -> dict:
        st = bfs_server_stats()
        _check(_lib().bfs_server_stats_get(self.h, ctypes.byref(st)), "bfs_server_stats_get")
        return st.as_dict()

    def bfs_server_records(self, cap: int = 1 << 20):
        ids = np.empty(cap, np.int64)
        lat = np.empty(cap, np.float64)
        bs = np.empty(cap, np.int32)
        seq = np.empty(cap, np.int64)
        cnt = ctypes.c_int64()
        _check(_lib().bfs_server_records(self.h, ids.ctypes.data, lat.ctypes.data, bs.ctypes.data, seq.ctypes.data,
                                         cap, ctypes.byref(cnt)), "bfs_server_records")
        k = cnt.value
        return ids[:k], lat[:k], bs[:k], seq[:k]

    def bfs_server_destroy(self):
        if self.h:
            _lib().bfs_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.bfs_server_destroy()
        except Exception:
            pass
