"""Seeded synthetic graph inputs shared by the GPU library's tests/bench and the oracle.

This package only draws and lays out graphs (Kronecker/R-MAT, Erdos-Renyi,
2D grids, 2D-decomposition blocks, random sources and frontiers).  It holds
none of the search's arithmetic.  The C part (``graphgen.c``) is built with
gcc/OpenMP into ``libgraphgen.so`` next to this file.

Graph conventions: vertices ``0..n-1``, CSR ``offsets`` int64 ``[n+1]`` and
``cols`` int32 ``[nnz]``; every row sorted ascending, no self-loops, no
duplicate entries, symmetric (each undirected edge stored twice).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

# R-MAT initiator of the paper's data sets (Graph500 parameters)
RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


class _Block(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int64), ("nzc", ctypes.c_int64), ("nzr", ctypes.c_int64),
                ("jc", _i32p), ("ir", _i32p), ("jr", _i32p), ("ic", _i32p),
                ("cp", _i64p), ("rp", _i64p)]


_GPU_SRC = os.path.join(_HERE, "graphgen_gpu.hip")
_GPU_LIB_PATH = os.path.join(_HERE, "libgraphgen_gpu.so")
_gpu_lib = None


def build(force: bool = True) -> str:
    """Compile libgraphgen.so (gcc -O2 -fopenmp) and, where hipcc exists, the
    GPU block generator libgraphgen_gpu.so (gfx950)."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if os.path.exists(hipcc):
        arch = os.environ.get("BFS_OFFLOAD_ARCH", "gfx950")
        tmp = _GPU_LIB_PATH + ".tmp"
        subprocess.run([hipcc, f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-shared",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", tmp, _GPU_SRC],
                       check=True)
        os.replace(tmp, _GPU_LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.gg_free.argtypes = [ctypes.c_void_p]
    lib.gg_kronecker_csr.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int, _i64p, _i64p,
                                     ctypes.POINTER(_i64p), ctypes.POINTER(_i32p)]
    lib.gg_er_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, _i64p,
                              ctypes.POINTER(_i64p), ctypes.POINTER(_i32p)]
    lib.gg_edges_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i64p, ctypes.c_int, _i64p,
                                 ctypes.POINTER(_i64p), ctypes.POINTER(_i32p)]
    lib.gg_grid2d_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p,
                                  ctypes.POINTER(_i64p), ctypes.POINTER(_i32p)]
    lib.gg_kron_edges.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                                  ctypes.c_int64, _i64p, _i64p]
    lib.gg_rand64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    lib.gg_rand64.restype = ctypes.c_uint64
    lib.gg_kron_relabel.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
    lib.gg_kron_relabel.restype = ctypes.c_uint64
    lib.gg_csr_block.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(_Block)]
    lib.gg_kron_block.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(_Block)]
    lib.gg_coo_block.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _i32p, _i32p,
                                 ctypes.POINTER(_Block)]
    lib.gg_block_free.argtypes = [ctypes.POINTER(_Block)]
    _lib = lib
    return lib


def _adopt(ptr, count: int, dtype) -> np.ndarray:
    """Wrap a malloc'ed C buffer as a numpy array freed when the array dies."""
    lib = _load()
    addr = ctypes.cast(ptr, ctypes.c_void_p).value
    if count == 0:
        lib.gg_free(addr)
        return np.zeros(0, dtype=dtype)
    ctype = np.ctypeslib.as_ctypes_type(dtype)
    buf = (ctype * count).from_address(addr)
    weakref.finalize(buf, lib.gg_free, addr)
    return np.frombuffer(buf, dtype=dtype)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"graphgen: {what} failed with code {rc}")


def _csr_out(n, rc, nnz, off, cols, what):
    _check(rc, what)
    return _adopt(off, n + 1, np.int64), _adopt(cols, nnz.value, np.int32)


def kronecker(scale: int, edgefactor: int = 16, seed: int = 1, a: float = RMAT_A, b: float = RMAT_B,
              c: float = RMAT_C, permute: bool = True):
    """Kronecker/R-MAT graph: edgefactor*2^scale draws, cleaned and symmetrised -> (offsets, cols)."""
    lib = _load()
    n, nnz = ctypes.c_int64(), ctypes.c_int64()
    off, cols = _i64p(), _i32p()
    rc = lib.gg_kronecker_csr(scale, edgefactor, seed, a, b, c, int(permute), ctypes.byref(n),
                              ctypes.byref(nnz), ctypes.byref(off), ctypes.byref(cols))
    return _csr_out(n.value, rc, nnz, off, cols, "kronecker")


def erdos_renyi(n: int, avg_degree: float, seed: int = 1):
    """G(n, M) with M = n*avg_degree/2 uniform endpoint draws, cleaned and symmetrised."""
    lib = _load()
    nnz = ctypes.c_int64()
    off, cols = _i64p(), _i32p()
    m = int(round(n * avg_degree / 2))
    rc = lib.gg_er_csr(n, m, seed, ctypes.byref(nnz), ctypes.byref(off), ctypes.byref(cols))
    return _csr_out(n, rc, nnz, off, cols, "erdos_renyi")


def grid2d(h: int, w: int):
    """h x w grid, 4-neighbour, vertex id r*w+c, sorted rows."""
    lib = _load()
    nnz = ctypes.c_int64()
    off, cols = _i64p(), _i32p()
    rc = lib.gg_grid2d_csr(h, w, ctypes.byref(nnz), ctypes.byref(off), ctypes.byref(cols))
    return _csr_out(h * w, rc, nnz, off, cols, "grid2d")


def csr_from_edges(n: int, src, dst, symmetrize: bool = True):
    """CSR from a raw edge list: drops self-loops, (optionally) symmetrises, sorts and dedups rows."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int64)
    dst = np.ascontiguousarray(dst, dtype=np.int64)
    assert src.shape == dst.shape
    nnz = ctypes.c_int64()
    off, cols = _i64p(), _i32p()
    rc = lib.gg_edges_csr(n, src.size, src.ctypes.data_as(_i64p), dst.ctypes.data_as(_i64p),
                          int(symmetrize), ctypes.byref(nnz), ctypes.byref(off), ctypes.byref(cols))
    return _csr_out(n, rc, nnz, off, cols, "csr_from_edges")


def kronecker_edges(scale: int, edgefactor: int = 16, seed: int = 1, start: int = 0, count: int | None = None,
                    a: float = RMAT_A, b: float = RMAT_B, c: float = RMAT_C, permute: bool = True):
    """The raw (u, v) draws of :func:`kronecker` with indices [start, start+count)."""
    lib = _load()
    if count is None:
        count = (edgefactor << scale) - start
    src = np.empty(count, np.int64)
    dst = np.empty(count, np.int64)
    rc = lib.gg_kron_edges(scale, edgefactor, seed, a, b, c, int(permute), start, count,
                           src.ctypes.data_as(_i64p), dst.ctypes.data_as(_i64p))
    _check(rc, "kronecker_edges")
    return src, dst


def _block_out(blk: _Block):
    lib = _load()
    d = {
        "nnz": blk.nnz, "nzc": blk.nzc, "nzr": blk.nzr,
        "jc": np.ctypeslib.as_array(blk.jc, (blk.nzc,)).copy() if blk.nzc else np.zeros(0, np.int32),
        "cp": np.ctypeslib.as_array(blk.cp, (blk.nzc + 1,)).copy(),
        "ir": np.ctypeslib.as_array(blk.ir, (blk.nnz,)).copy() if blk.nnz else np.zeros(0, np.int32),
        "jr": np.ctypeslib.as_array(blk.jr, (blk.nzr,)).copy() if blk.nzr else np.zeros(0, np.int32),
        "rp": np.ctypeslib.as_array(blk.rp, (blk.nzr + 1,)).copy(),
        "ic": np.ctypeslib.as_array(blk.ic, (blk.nnz,)).copy() if blk.nnz else np.zeros(0, np.int32),
    }
    lib.gg_block_free(ctypes.byref(blk))
    return d


def coo_block(nrows: int, ncols: int, rows, cols):
    """Block given as a plain (row, col) list with block-local ids -> DCSC + DCSR (deduplicated)."""
    lib = _load()
    r = np.ascontiguousarray(rows, dtype=np.int32)
    c = np.ascontiguousarray(cols, dtype=np.int32)
    blk = _Block()
    rc = lib.gg_coo_block(nrows, ncols, r.size, r.ctypes.data_as(_i32p), c.ctypes.data_as(_i32p),
                          ctypes.byref(blk))
    _check(rc, "coo_block")
    return _block_out(blk)


def csr_block(offsets, cols, r0: int, nrows: int, c0: int, ncols: int):
    """Block A[r0:r0+nrows, c0:c0+ncols] of a CSR graph in DCSC (jc,cp,ir) and DCSR (jr,rp,ic)
    forms with block-local ids (the paper's 2D checkerboard piece, Eq. 1)."""
    lib = _load()
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    blk = _Block()
    rc = lib.gg_csr_block(offsets.size - 1, offsets.ctypes.data_as(_i64p), cols.ctypes.data_as(_i32p),
                          r0, nrows, c0, ncols, ctypes.byref(blk))
    _check(rc, "csr_block")
    return _block_out(blk)


def kronecker_block(scale: int, r0: int, nrows: int, c0: int, ncols: int, edgefactor: int = 16,
                    seed: int = 1, a: float = RMAT_A, b: float = RMAT_B, c: float = RMAT_C,
                    permute: bool = True):
    """The same block taken straight from the Kronecker draws (no whole-graph CSR needed)."""
    lib = _load()
    blk = _Block()
    rc = lib.gg_kron_block(scale, edgefactor, seed, a, b, c, int(permute), r0, nrows, c0, ncols,
                           ctypes.byref(blk))
    _check(rc, "kronecker_block")
    return _block_out(blk)


def _load_gpu():
    global _gpu_lib
    if _gpu_lib is not None:
        return _gpu_lib
    if not os.path.exists(_GPU_LIB_PATH):
        raise RuntimeError(f"{_GPU_LIB_PATH} is not built (graphgen.build())")
    lib = ctypes.CDLL(_GPU_LIB_PATH)
    lib.ggg_kron_block.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_void_p), _i64p, _i64p, _i64p]
    lib.ggg_block_copy.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 6
    lib.ggg_block_free.argtypes = [ctypes.c_void_p]
    lib.ggg_block_free.restype = None
    _gpu_lib = lib
    return lib


def kronecker_block_gpu(scale: int, r0: int, nrows: int, c0: int, ncols: int, edgefactor: int = 16,
                        seed: int = 1, a: float = RMAT_A, b: float = RMAT_B, c: float = RMAT_C,
                        permute: bool = True, device=None):
    """kronecker_block built on the GPU (same draws, same arrays), returned as
    torch tensors on `device` (default cuda:0): for blocks of graphs too large
    to enumerate on the host."""
    import torch
    dev = torch.device(device or "cuda:0")
    lib = _load_gpu()
    h = ctypes.c_void_p()
    nnz, nzc, nzr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    with torch.cuda.device(dev):
        rc = lib.ggg_kron_block(scale, edgefactor, seed, a, b, c, int(permute), r0, nrows, c0, ncols,
                                ctypes.byref(h), ctypes.byref(nnz), ctypes.byref(nzc), ctypes.byref(nzr))
        if rc != 0:
            raise RuntimeError(f"ggg_kron_block failed ({rc})")
        try:
            out = {"nnz": nnz.value, "nzc": nzc.value, "nzr": nzr.value,
                   "jc": torch.empty(max(nzc.value, 1), dtype=torch.int32, device=dev),
                   "cp": torch.empty(nzc.value + 1, dtype=torch.int64, device=dev),
                   "ir": torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev),
                   "jr": torch.empty(max(nzr.value, 1), dtype=torch.int32, device=dev),
                   "rp": torch.empty(nzr.value + 1, dtype=torch.int64, device=dev),
                   "ic": torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)}
            torch.cuda.synchronize(dev)
            rc = lib.ggg_block_copy(h, *(out[k].data_ptr() for k in ("jc", "cp", "ir", "jr", "rp", "ic")))
            if rc != 0:
                raise RuntimeError(f"ggg_block_copy failed ({rc})")
        finally:
            lib.ggg_block_free(h)
    for k, m in (("jc", nzc.value), ("ir", nnz.value), ("jr", nzr.value), ("ic", nnz.value)):
        out[k] = out[k][:m]
    return out


def rand64(seed: int, stream: int, i: int) -> int:
    return int(_load().gg_rand64(seed, stream, i))


def random_sources(offsets, k: int, seed: int = 2) -> np.ndarray:
    """k distinct vertices of nonzero degree, drawn with the counter-based RNG (stream 3)."""
    offsets = np.asarray(offsets)
    n = offsets.size - 1
    deg = np.diff(offsets)
    nz = int(np.count_nonzero(deg))
    if k > nz:
        raise ValueError(f"only {nz} vertices have nonzero degree, {k} sources requested")
    out, seen, i = [], set(), 0
    while len(out) < k:
        v = int((rand64(seed, 3, i) * n) >> 64)
        i += 1
        if deg[v] > 0 and v not in seen:
            seen.add(v)
            out.append(v)
    return np.array(out, dtype=np.int64)


def random_sorted_subset(universe: int, k: int, seed: int) -> np.ndarray:
    """k distinct ids of [0, universe), sorted ascending (seeded numpy PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if k >= universe:
        return np.arange(universe, dtype=np.int32)
    if k * 4 < universe:
        # union of independent uniform draws, then a uniform k-subset of it
        pool = np.unique(rng.integers(0, universe, size=k + k // 8 + 16))
        while pool.size < k:
            pool = np.union1d(pool, rng.integers(0, universe, size=2 * (k - pool.size) + 16))
        return np.sort(rng.choice(pool, size=k, replace=False)).astype(np.int32)
    return np.sort(rng.choice(universe, size=k, replace=False)).astype(np.int32)


def random_bitmap(nbits: int, density: float, seed: int) -> np.ndarray:
    """Bernoulli(density) bitmap of nbits bits as uint64 words (bit i of word w = id 64*w+i)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    bits = rng.random(nbits) < density
    return bits_to_words(bits)


def bits_to_words(bits) -> np.ndarray:
    bits = np.asarray(bits, dtype=bool)
    nw = (bits.size + 63) // 64
    padded = np.zeros(nw * 64, dtype=bool)
    padded[: bits.size] = bits
    return np.packbits(padded.reshape(nw, 64)[:, ::-1], axis=1).view(">u8").astype(np.uint64).reshape(nw)


def words_to_bits(words, nbits: int) -> np.ndarray:
    words = np.asarray(words, dtype=np.uint64)
    b = np.unpackbits(words.astype(">u8").view(np.uint8).reshape(-1, 8), axis=1)[:, ::-1]
    return b.reshape(-1)[:nbits].astype(bool)
