#!/usr/bin/env python3
"""Benchmark: single-source direction-optimizing BFS on one MI355X.

Workload (default): Kronecker graph, scale 26, edgefactor 16, initiator
(.57,.19,.19,.05), vertex ids permuted, cleaned and symmetrised, int64
offsets + int32 columns resident in HBM; 64 seeded sources of nonzero degree;
alpha = 15, beta = 18.  One step = one search from one source (the sources are
cycled).  value = harmonic-mean GTEPS = m * K / (wall time of the K timed
steps), m = undirected edges after cleanup (nnz / 2), the TEPS convention of
the paper's experimental-design section.

Also reported:
  roofline      the dominant kernel's algorithmic bytes per launch over its
                average HIP-event duration (events recorded by the library on
                the launch stream during the timed steps), against 8 TB/s;
                `traffic` comes from the committed rocprofv3 FETCH_SIZE /
                WRITE_SIZE summary when it was taken on the current kernel source.
  cpu_baseline  the CPU oracle (serial Alg. 1) timed on this host on a bounded
                sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "harmonic-mean GTEPS @ Kronecker scale 26; batched queries/s + p99 latency"
PROFILE_PMC = os.path.join(ROOT, "profiles", "bu_sweep_kron26_pmc.md")
# knob settings found by the autotuner, keyed by device and graph class; a run
# that finds its key reuses them (so profiled runs time the same launches),
# --retune searches again and overwrites the entry
TUNE_CACHE = os.path.join(ROOT, "paper_1705_04590_amd", "autotune_cache.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_1705_04590_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


WORK_TABLE = os.path.join(ROOT, "tests", "golden", "kron{scale}_work_model.json")


def load_work_table(scale, edgefactor, seed, source_seed, n, nnz):
    """The oracle's per-level work counts for this graph and source seed
    (written by tests/golden/make_work_model.py, which runs only the CPU
    oracle), keyed by source id; (None, reason) when no table matches."""
    path = WORK_TABLE.format(scale=scale)
    if not os.path.exists(path):
        return None, f"no work table {os.path.relpath(path, ROOT)}"
    doc = json.load(open(path))
    gr = doc["graph"]
    if (gr["scale"], gr["edgefactor"], gr["seed"], gr["n"], gr["nnz"], doc["source_seed"]) != \
            (scale, edgefactor, seed, n, nnz, source_seed):
        return None, "work table is for another graph or source seed"
    return {"isolated": gr["isolated"], "rows": {r["source"]: r for r in doc["sources"]},
            "path": os.path.relpath(path, ROOT)}, ""


def level_bytes(st: dict, row: dict, n: int, wo: int, iso: int):
    """Algorithmic HBM bytes of every expansion launch of one search, per level.

    top-down level : |F|(4 + 2 W_o) + D_F (4 column + 4 probe) + |N| (4 parent + 4 depth + 4 queue)
    bottom-up level: n/8 visited + 2 W_o |U| + 4 X + n/8 frontier + 8 |N| + n/8 next/visited
                     (+ 8 per entry of the -1 fill of isolated and still unreached
                     vertices, on the sweep that writes it)
    F the frontier, D_F its edges, N the next frontier, U the unvisited
    vertices that have edges, X the adjacency entries a row-order first-hit
    scan examines (Alg. 2).  Every count comes from the oracle's work table
    `row`; only the direction of each level is the library's, and the
    library's own per-level counts must equal the table's.
    """
    lv = row["levels"]
    L = len(st["level_dir"])
    if st["levels"] != len(lv):
        raise ValueError(f"source {row['source']}: {st['levels']} levels, the oracle has {len(lv)}")
    out = []
    for d in range(L):
        nf, mf, mu, u, x = lv[d]
        if (st["level_nf"][d], st["level_mf"][d], st["level_mu"][d]) != (nf, mf, mu):
            raise ValueError(f"source {row['source']} level {d}: library counts differ from the oracle's")
        nn = lv[d + 1][0] if d + 1 < len(lv) else 0
        if st["level_dir"][d] == 0:
            out.append(("td_expand", nf * (4 + 2 * wo) + mf * 8 + nn * 12 if mf > 0 else 0))
        else:
            b = 3 * (n / 8) + 2 * wo * u + 4 * x + 8 * nn
            if st.get("fill_level") == d:
                b += 8 * (iso + u - nn)
            out.append(("bu_sweep", b))
    return out


def ms_level_bytes(st: dict, n: int):
    """Model bytes of each level of a batched (64-source) search, from the
    library's per-level counts: 16 B per vertex touched (its visited and
    frontier masks; a bottom-up level touches every vertex, a top-down level
    its frontier and the vertices it reaches), 12 B per adjacency entry
    scanned (the column and the neighbour's mask), 8 B per next-frontier
    mask.  The 8 B per (vertex, source) output entry belong to the final
    transpose, not to a level."""
    L = len(st["level_dir"])
    out = []
    for d in range(L):
        nn = st["level_nf"][d + 1] if d + 1 < L else 0
        touched = n if st["level_dir"][d] == 1 else st["level_nf"][d] + nn
        out.append(("ms_bu" if st["level_dir"][d] == 1 else "ms_td",
                    16 * touched + 12 * st["level_examined"][d] + 8 * nn))
    return out


def ms_roofline(st: dict, n: int, k: int):
    """Roofline entry of the batched search's bottom-up levels (its dominant
    kernel), from one batch timed with events around every kernel."""
    nbytes, ms, launches = 0.0, 0.0, 0
    for d, (kind, b) in enumerate(ms_level_bytes(st, n)):
        if kind == "ms_bu" and d < len(st["level_ms"]):
            nbytes += b
            ms += st["level_ms"][d]
            launches += 1
    if not launches or ms <= 0:
        return None
    achieved = nbytes / (ms / 1e3) / 1e9
    return {"bound": "hbm", "kernel": "ms_bu_sweep", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "launches": launches,
            "avg_launch_us": round(ms / launches * 1e3, 2), "alg_bytes_per_launch": round(nbytes / launches),
            "alg_bytes_from": "library per-level counts (frontier sizes, entries scanned)", "sources": k}


def read_traffic(kernel: str):
    """Per-launch HBM bytes from the committed PMC summary, if it matches the current kernels."""
    if not os.path.exists(PROFILE_PMC):
        return None
    txt = open(PROFILE_PMC).read()
    m = re.search(r"```json\s*(\{.*?\})\s*```", txt, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_source_hash") != kernel_source_hash() or rec.get("kernel") != kernel:
        return None
    return rec.get("traffic_bytes_per_launch")


def host_cpu():
    """(model name, CPUs this process may run on, CPUs of the machine)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0)), os.cpu_count()


def cpu_baseline(off, cols, sources, m, max_seconds, max_threads=16):
    """The serial oracle (Alg. 1), built -O3 -march=native on this host.

    latency: one thread pinned to one core, sources in order until the
    budget is spent (at least one); throughput: one independent oracle search
    per core at once (up to max_threads cores of this process's affinity
    set), each from its own source, counted as queries/s."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    orc = oracle.load_timing()
    model, nproc, ncpu = host_cpu()
    mask = os.sched_getaffinity(0)
    core = min(mask)
    os.sched_setaffinity(0, {core})
    try:
        t_total, done = 0.0, 0
        for s in sources:
            t0 = time.perf_counter()
            orc.bfs(off, cols, int(s))
            t_total += time.perf_counter() - t0
            done += 1
            if t_total >= max_seconds:
                break
    finally:
        os.sched_setaffinity(0, mask)
    threads = max(1, min(nproc, max_threads, len(sources)))
    with ThreadPoolExecutor(threads) as ex:
        t0 = time.perf_counter()
        list(ex.map(lambda s: orc.bfs(off, cols, int(s)), sources[:threads]))
        wall = time.perf_counter() - t0
    return {"value": m * done / t_total / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{done} of the {len(sources)} sources one after another on one pinned core, full graph, "
                      f"serial Alg. 1 oracle built -O3 -march=native, {t_total:.1f} s",
            "search_s": round(t_total / done, 3),
            "throughput": {"queries_per_s": round(threads / wall, 3), "gteps": round(m * threads / wall / 1e9, 4),
                           "cores": threads,
                           "sample": f"{threads} independent oracle searches at once, one per core, sources "
                                     f"0..{threads - 1}, {wall:.1f} s"},
            "host": {"cpu_model": model, "nproc": nproc, "cpu_count": ncpu}}


SERVE_GRAPHS = [("kron14", "kron", 14, 1), ("kron16", "kron", 16, 1), ("kron18", "kron", 18, 1),
                ("kron20", "kron", 20, 1), ("kron22", "kron", 22, 1), ("kron24", "kron", 24, 1),
                ("er20_deg8", "er", 20, 1), ("grid1024", "grid", 1024, 0), ("grid2048", "grid", 2048, 0),
                ("kron18_s2", "kron", 18, 2), ("kron20_s2", "kron", 20, 2), ("kron22_s2", "kron", 22, 2)]


def serve_graphs(dev):
    """The 12 resident graphs of the serving configuration, with 256 query sources each (seed 6)."""
    import torch

    import graphgen
    import paper_1705_04590_amd as bfs

    graphs, keep = [], []
    for name, kind, p, seed in SERVE_GRAPHS:
        if kind == "kron":
            off, cols = graphgen.kronecker(p, 16, seed=seed)
        elif kind == "er":
            off, cols = graphgen.erdos_renyi(1 << p, 8.0, seed=seed)
        else:
            off, cols = graphgen.grid2d(p, p)
        d_off, d_cols = torch.from_numpy(off).to(dev), torch.from_numpy(cols).to(dev)
        g = bfs.bfs_create_graph_csr(d_off, d_cols, bfs.BFS_GRAPH_SYMMETRIC | bfs.BFS_GRAPH_SORTED)
        srcs = graphgen.random_sources(off, 256, seed=6)
        graphs.append((name, g, srcs, off.size - 1, int(off[-1])))
        keep.append((d_off, d_cols))
    return graphs, keep


def serve_measure(graphs, rates, seconds, max_requests, slots, budget_gib):
    """Poisson arrivals (seed 6) at rates given as multiples of the one-query-per-launch
    capacity; each rate served twice: by continuous batching (up to 64 same-graph
    queries per batch, `slots` batches in flight) and by one query per launch
    (one slot, batches of one).  Returns (capacity one-per-launch, capacity
    batched, per-rate rows)."""
    import numpy as np
    import torch

    from paper_1705_04590_amd import serve

    rng = np.random.default_rng(6)

    def stream(m, rate):
        gaps = rng.exponential(1e6 / rate, m)
        t = np.cumsum(gaps) - gaps[0]
        gi = rng.integers(0, len(graphs), m).astype(np.int32)
        src = np.array([graphs[g][2][rng.integers(0, 256)] for g in gi], dtype=np.int64)
        return t, gi, src

    def run(t, gi, src, nslots, max_batch):
        o = serve.bfs_server_opts_default(slots=nslots, max_batch=max_batch, hbm_budget=budget_gib << 30)
        srv = serve.Server(o)
        for x in graphs:
            srv.bfs_server_add_graph(x[1])
        srv.bfs_server_replay(t, gi, src, np.arange(t.size))
        srv.bfs_server_drain()
        st = srv.bfs_server_stats_get()
        srv.bfs_server_destroy()
        free, total = torch.cuda.mem_get_info()
        log(f"[serve]   server done: {free / 2**30:.1f} of {total / 2**30:.1f} GiB free")
        return st

    m = max_requests
    # capacity of one query per launch: everything arrives at once, FIFO, one
    # slot, batches of one (bfs_run); a short pilot sizes the measured run
    t, gi, src = stream(m, 1e9)
    pilot = run(np.zeros(32), gi[:32], src[:32], 1, 1)["queries_per_s"]
    m1 = int(min(m, max(64, pilot * seconds)))
    log(f"[serve] pilot {pilot:.0f} q/s -> {m1} queries for the one-per-launch capacity run")
    cap1 = run(np.zeros(m1), gi[:m1], src[:m1], 1, 1)["queries_per_s"]
    capb = run(np.zeros(m), gi, src, slots, 64)["queries_per_s"]
    log(f"[serve] capacity: one query per launch {cap1:.0f} q/s, batched {capb:.0f} q/s")
    rows = []
    for f in rates:
        rate = f * cap1
        # arrivals span about `seconds`; the one-per-launch server needs about
        # seconds * max(f, 1) to work through them
        mr = int(min(m, max(64, rate * seconds / max(f, 1.0))))
        t, gi, src = stream(mr, rate)
        single = run(t, gi, src, 1, 1)
        log(f"[serve] {f:>4}x ({mr} queries at {rate:.0f}/s): one-per-launch {single['queries_per_s']:.0f} q/s "
            f"p50 {single['p50_us'] / 1e3:.2f} ms p99 {single['p99_us'] / 1e3:.2f} ms")
        batched = run(t, gi, src, slots, 64)
        rows.append({"rate_x_single_capacity": f, "offered_qps": round(rate, 1), "requests": mr,
                     "batched": {k: round(batched[k], 2) for k in ("queries_per_s", "p50_us", "p99_us",
                                                                    "mean_batch", "max_inflight",
                                                                    "device_max_overlap")},
                     "one_query_per_launch": {k: round(single[k], 2) for k in ("queries_per_s", "p50_us",
                                                                                "p99_us")}})
        log(f"[serve] {f:>4}x: batched {batched['queries_per_s']:.0f} q/s p50 {batched['p50_us'] / 1e3:.2f} ms "
            f"p99 {batched['p99_us'] / 1e3:.2f} ms (batch {batched['mean_batch']:.1f}, inflight "
            f"{batched['max_inflight']}, overlapping on the device {batched['device_max_overlap']})")
    return cap1, capb, rows


def serve_bench(args):
    """Served queries over 12 resident graphs: Poisson arrivals, continuous batching vs one query per launch."""
    import torch

    dev = torch.device("cuda:0")
    t0 = time.time()
    graphs, keep = serve_graphs(dev)
    log(f"[serve] {len(graphs)} graphs resident in {time.time() - t0:.1f}s: " +
        ", ".join(f"{x[0]}(n={x[3]})" for x in graphs))
    cap1, capb, rows = serve_measure(graphs, args.serve_rates, args.serve_seconds, args.serve_requests,
                                     args.serve_slots, args.serve_budget_gib)
    m = args.serve_requests
    out = {"metric": "served BFS queries/s and p50/p99 latency, 12 resident graphs, Poisson arrivals",
           "value": round(capb, 1), "unit": "queries/s", "n_gpus": 1, "steps": m, "warmup": 0,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic",
           "config": {"workload": "serve_12_graphs", "graphs": [x[0] for x in graphs], "max_requests_per_rate": m,
                      "slots": args.serve_slots, "max_batch": 64, "hbm_budget_gib": args.serve_budget_gib,
                      "capacity_one_query_per_launch_qps": round(cap1, 1), "capacity_batched_qps": round(capb, 1)},
           "rates": rows}
    print(json.dumps(out), flush=True)


def block_bench(args):
    """DCSC block local discovery on one block of an 8x8 decomposition of a
    Kronecker graph (default scale 30: a 2^27 x 2^27 block), seeded frontiers."""
    import numpy as np
    import torch

    import graphgen
    import paper_1705_04590_amd as bfs

    dev = torch.device("cuda:0")
    scale = args.block_scale
    n = 1 << scale
    R = C = n // 8
    t0 = time.time()
    blk = graphgen.kronecker_block_gpu(scale, 0, R, C, C, seed=args.seed)
    log(f"[block] scale {scale} 8x8 block (0,1): {R}x{C}, nnz {blk['nnz']}, nzc {blk['nzc']}, nzr {blk['nzr']} "
        f"({time.time() - t0:.1f}s on the GPU)")
    g = bfs.bfs_create_graph_dcsc(R, C, 0, C, blk["jc"], blk["cp"], blk["ir"], blk["jr"], blk["rp"], blk["ic"],
                                  flags=bfs.BFS_GRAPH_SORTED)
    ws = bfs.workspace(g, 1, dev)
    out_r = torch.empty(R, dtype=torch.int32, device=dev)
    out_p = torch.empty(R, dtype=torch.int32, device=dev)
    nout = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    reps = args.block_reps
    nzc = blk["nzc"]

    def timed(fn, before=None):
        ms = []
        for r in range(reps + 1):
            if before:
                before()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            if r:
                ms.append(a.elapsed_time(b))
        return float(np.mean(ms))

    td_rows = []
    for d in (1e-5, 1e-3, 1e-1):
        k = int(round(d * C))
        fr = torch.from_numpy(graphgen.random_sorted_subset(C, k, seed=4)).to(dev)
        ms = timed(lambda: bfs.bfs_block_td(g, fr, out_r, out_p, nout, ws, stream))
        # work of the call: frontier columns present in the block and their entries
        idx = torch.searchsorted(blk["jc"], fr).clamp(max=max(nzc - 1, 0))
        hit = blk["jc"][idx] == fr
        h = int(hit.sum().item())
        eh = int((blk["cp"][idx + 1] - blk["cp"][idx])[hit].sum().item())
        rout = int(nout.item())
        nbytes = 4 * k + 4 * min(nzc, int(k * max(1.0, np.log2(max(nzc, 2))))) + 16 * h + 8 * eh + 8 * rout
        td_rows.append({"density": d, "frontier_cols": k, "cols_in_block": h, "entries": eh, "rows_out": rout,
                        "ms": round(ms, 4), "entries_per_s": round(eh / ms * 1e3, 1),
                        "alg_gb_per_s": round(nbytes / ms / 1e6, 1), "frac": round(nbytes / ms / 1e6 / HBM_PEAK_GBS, 4)})
        log(f"[block] TD density {d}: {k} cols ({h} in block, {eh} entries) -> {rout} rows in {ms:.3f} ms, "
            f"{eh / ms / 1e6:.2f} G entries/s, {nbytes / ms / 1e6:.0f} GB/s algorithmic")
    bu_rows = []
    for d, cd in ((1e-3, 1e-3), (1e-1, 1e-1), (1e-1, 0.5)):
        fb = torch.from_numpy(graphgen.random_bitmap(C, d, seed=4).view(np.int64)).to(dev)
        comp0 = torch.from_numpy(graphgen.random_bitmap(R, cd, seed=5).view(np.int64)).to(dev)
        comp = comp0.clone()
        ms = timed(lambda: bfs.bfs_block_bu(g, fb, comp, 0, R, out_r, out_p, nout, ws, stream),
                   before=lambda: comp.copy_(comp0))
        rout = int(nout.item())
        # lower bound of its traffic: completed and frontier words, the row index
        # and offsets of every non-empty row, parent pairs out
        nbytes = R // 8 + C // 8 + 12 * blk["nzr"] + 8 * rout
        bu_rows.append({"frontier_density": d, "completed_density": cd, "rows_out": rout, "ms": round(ms, 4),
                        "rows_per_s": round(blk["nzr"] / ms * 1e3, 1),
                        "alg_gb_per_s_lower_bound": round(nbytes / ms / 1e6, 1)})
        log(f"[block] BU frontier {d} completed {cd}: {rout} rows found in {ms:.3f} ms")
    top = td_rows[-1]
    out = {"metric": "DCSC block local discovery, top-down SpMSV entries/s (scale-30 8x8 block, density 0.1)",
           "value": top["entries_per_s"], "unit": "entries/s", "n_gpus": 1, "steps": reps, "warmup": 1,
           "ms_per_step": top["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int32", "data": "synthetic",
           "config": {"workload": f"kronecker_s{scale}_8x8_block_0_1", "block_rows": R, "block_cols": C,
                      "nnz": blk["nnz"], "nzc": nzc, "nzr": blk["nzr"]},
           "roofline": {"bound": "hbm", "achieved": top["alg_gb_per_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": top["frac"], "traffic": None, "kernel": "blk_expand"},
           "td": td_rows, "bu": bu_rows}
    print(json.dumps(out), flush=True)


def configs_bench(args):
    """The secondary configurations: Kronecker scale 16 (int32 offsets) and 22
    (int64), top-down only and direction-optimizing; 64-source batches against
    64 single searches on Kronecker scale 24 and on the 4096 x 4096 grid."""
    import numpy as np
    import torch

    import graphgen
    import paper_1705_04590_amd as bfs

    dev = torch.device("cuda:0")
    SYM = bfs.BFS_GRAPH_SYMMETRIC | bfs.BFS_GRAPH_SORTED

    def resident(off, cols, use32):
        d_off = torch.from_numpy(off.astype(np.int32) if use32 else off).to(dev)
        d_cols = torch.from_numpy(cols).to(dev)
        return bfs.bfs_create_graph_csr(d_off, d_cols, SYM), (d_off, d_cols)

    def singles(g, n, srcs, **kw):
        ws = bfs.workspace(g, 1, dev)
        par = torch.empty(n, dtype=torch.int32, device=dev)
        dep = torch.empty(n, dtype=torch.int32, device=dev)
        o = bfs.bfs_opts_default(**kw)
        bfs.bfs_run(g, int(srcs[0]), par, dep, ws, o)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for s_ in srcs:
            bfs.bfs_run(g, int(s_), par, dep, ws, o)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / len(srcs)

    def batch(g, n, srcs, reps):
        k = len(srcs)
        ws = bfs.workspace(g, k, dev)
        par = torch.empty(k * n, dtype=torch.int32, device=dev)
        dep = torch.empty(k * n, dtype=torch.int32, device=dev)
        bfs.bfs_run_multi(g, srcs, par, dep, ws, bfs.bfs_opts_default())
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            bfs.bfs_run_multi(g, srcs, par, dep, ws, bfs.bfs_opts_default())
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    rows = []
    for scale, nsrc in ((16, 16), (22, 64)):
        off, cols = graphgen.kronecker(scale, 16, seed=1)
        n, m = off.size - 1, int(off[-1]) // 2
        g, keep = resident(off, cols, scale < 22)
        srcs = graphgen.random_sources(off, nsrc, seed=2)
        for name, dv in (("top_down", bfs.BFS_DIR_TD), ("direction_optimizing", bfs.BFS_DIR_DO)):
            kw, tuning = dict(dir=dv), "defaults"
            if dv == bfs.BFS_DIR_DO and not args.no_autotune:
                # the knobs tuned on sources of another seed, as for the headline run
                from paper_1705_04590_amd import autotune
                tuned = autotune.tune(g, graphgen.random_sources(off, 16, seed=99), k=1,
                                      cache_path=args.tune_cache, force=args.retune)
                kw = {k: tuned[k] for k in autotune.KNOBS if k in tuned}
                kw["dir"] = dv
                tuning = "autotuned on 16 sources of seed 99" + (" (cached entry)" if tuned.get("cached") else "")
            t = singles(g, n, srcs, **kw)
            rows.append({"workload": f"kronecker_s{scale}", "mode": name, "sources": nsrc,
                         "offsets": "int32" if scale < 22 else "int64", "ms_per_search": round(t * 1e3, 4),
                         "gteps": round(m / t / 1e9, 2), "tuning": tuning})
            log(f"[configs] kronecker s{scale} {name}: {t * 1e3:.3f} ms/search, {m / t / 1e9:.1f} GTEPS ({tuning})")
        bfs.bfs_destroy_graph(g)
        del keep
    for name, gen, nsingle, reps in (("kronecker_s24", lambda: graphgen.kronecker(24, 16, seed=1), 64, 3),
                                     ("grid_4096x4096", lambda: graphgen.grid2d(4096, 4096), 8, 1)):
        off, cols = gen()
        n = off.size - 1
        g, keep = resident(off, cols, False)
        srcs = graphgen.random_sources(off, 64, seed=3 if name.startswith("grid") else 2)
        if name.startswith("grid"):
            srcs = np.r_[0, srcs[:63]]
        t1 = singles(g, n, srcs[:nsingle], parent_mode=bfs.BFS_PARENT_MIN)
        tb = batch(g, n, [int(x) for x in srcs], reps)
        rows.append({"workload": name, "mode": "batched_64_vs_single", "single_ms": round(t1 * 1e3, 3),
                     "single_queries_per_s": round(1 / t1, 1), "batch_ms": round(tb * 1e3, 2),
                     "batch_queries_per_s": round(64 / tb, 1), "speedup": round(64 * t1 / tb, 2),
                     "single_sources_timed": nsingle, "parent_mode": "min"})
        log(f"[configs] {name}: single {t1 * 1e3:.2f} ms ({1 / t1:.0f} q/s), 64-batch {tb * 1e3:.1f} ms "
            f"({64 / tb:.0f} q/s), x{64 * t1 / tb:.2f}")
        bfs.bfs_destroy_graph(g)
        del keep
        torch.cuda.empty_cache()
    out = {"metric": "secondary configurations (GTEPS; batched vs single queries/s)", "value": rows[-1]["speedup"],
           "unit": "x (64-source batch vs 64 single searches, 4096^2 grid)", "n_gpus": 1, "steps": 0, "warmup": 1,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic", "config": {"workload": "configs_1_2_4"}, "rows": rows}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", choices=["single", "serve", "block", "configs"], default="single",
                    help="single: the headline single-source benchmark; serve: the query-server benchmark; "
                         "block: DCSC block local discovery on one block of a 2D decomposition; "
                         "configs: the secondary graph configurations")
    ap.add_argument("--block-scale", type=int, default=30)
    ap.add_argument("--block-reps", type=int, default=10)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[0.3, 1.0, 3.0, 10.0])
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-seconds", type=float, default=8.0,
                    help="approximate span of each serve run (sizes the request count per rate)")
    ap.add_argument("--serve-budget-gib", type=int, default=64)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--edgefactor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--source-seed", type=int, default=2)
    ap.add_argument("--nsources", type=int, default=64)
    ap.add_argument("--dir", choices=["do", "td", "bu"], default="do")
    ap.add_argument("--parent-mode", choices=["any", "min"], default="any")
    ap.add_argument("--alpha", type=float, default=15.0)
    ap.add_argument("--beta", type=float, default=18.0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="time only the given alpha/beta and default knobs (no autotuner pass)")
    ap.add_argument("--tune-sources", type=int, default=16, help="tuning sources (seed 99, distinct from evaluation)")
    ap.add_argument("--retune", action="store_true", help="search again and overwrite the cached entry")
    ap.add_argument("--tune-cache", default=TUNE_CACHE, help="autotune cache file")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="budget of the oracle CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true",
                    help="do not record HIP events around the bottom-up sweeps (no roofline entry)")
    ap.add_argument("--batched-reps", type=int, default=3,
                    help="timed repetitions of the 64-source batched search (0 = skip)")
    ap.add_argument("--no-serve", action="store_true", help="leave the served leg out of the headline line")
    ap.add_argument("--line-serve-rates", type=float, nargs="+", default=[1.0, 3.0],
                    help="offered rates (x the one-query-per-launch capacity) of the headline line's served leg")
    ap.add_argument("--line-serve-seconds", type=float, default=3.0,
                    help="approximate span of each run of the headline line's served leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run three 1 GiB device-to-device copies (the plain copy kernel "
                         "that scales FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the search is built for one GPU, "
              "and no sharded path exists to time on several", file=sys.stderr)
        sys.exit(2)
    if args.workload == "serve":
        serve_bench(args)
        return
    if args.workload == "block":
        block_bench(args)
        return
    if args.workload == "configs":
        configs_bench(args)
        return

    import numpy as np
    import torch

    import graphgen
    import paper_1705_04590_amd as bfs

    t0 = time.time()
    log(f"[bench] generating Kronecker scale {args.scale} edgefactor {args.edgefactor} seed {args.seed}")
    off, cols = graphgen.kronecker(args.scale, args.edgefactor, seed=args.seed)
    n = off.size - 1
    nnz = int(off[-1])
    m = nnz // 2
    log(f"[bench] n={n} nnz={nnz} m={m} generated in {time.time() - t0:.1f}s")
    sources = graphgen.random_sources(off, args.nsources, seed=args.source_seed)
    nsrc = len(sources)
    table, table_note = load_work_table(args.scale, args.edgefactor, args.seed, args.source_seed, n, nnz)
    if table is None:
        log(f"[bench] {table_note}: no roofline entry")

    dev = torch.device("cuda:0")
    use32 = nnz < 2 ** 31 and args.scale < 22
    d_off = torch.from_numpy(off.astype(np.int32) if use32 else off).to(dev)
    d_cols = torch.from_numpy(cols).to(dev)
    g = bfs.bfs_create_graph_csr(d_off, d_cols, bfs.BFS_GRAPH_SYMMETRIC | bfs.BFS_GRAPH_SORTED)
    ws = bfs.workspace(g, 1, dev)
    parent = torch.empty(n, dtype=torch.int32, device=dev)
    depth = torch.empty(n, dtype=torch.int32, device=dev)
    opts = bfs.bfs_opts_default(dir={"do": 0, "td": 1, "bu": 2}[args.dir],
                                parent_mode=1 if args.parent_mode == "min" else 0,
                                alpha=args.alpha, beta=args.beta, timing=0 if args.no_timing else 2)
    stream = torch.cuda.current_stream()
    log(f"[bench] graph resident ({(d_off.numel() * d_off.element_size() + nnz * 4) / 2**30:.2f} GiB), "
        f"workspace {ws.numel() / 2**30:.2f} GiB; warmup {args.warmup}")

    # step i searches from sources[i mod 64]; the warm-up searches take the
    # sources from the end of the list, so K < 64 timed steps still time K
    # distinct sources
    def timed_steps(o, steps):
        for i in range(args.warmup):
            bfs.bfs_run(g, int(sources[(nsrc - 1 - i) % nsrc]), parent, depth, ws, o, stream)
        torch.cuda.synchronize()
        sts = []
        t_begin = time.perf_counter()
        for i in range(steps):
            sts.append(bfs.bfs_run(g, int(sources[i % nsrc]), parent, depth, ws, o, stream))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_begin
        # the per-level records are turned into dicts after the clock stops
        return [st.as_dict() for st in sts], elapsed

    default_params = None
    tuned = None
    if not args.no_autotune and args.dir == "do":
        from paper_1705_04590_amd import autotune
        tsrc = graphgen.random_sources(off, args.tune_sources, seed=99)
        t0 = time.time()
        tuned = autotune.tune(g, tsrc, k=1, cache_path=args.tune_cache, force=args.retune)
        src_note = "cached entry" if tuned.get("cached") else f"{tuned['trials']} trials, {time.time() - t0:.1f}s"
        log(f"[bench] autotune ({src_note}): alpha={tuned['alpha']} beta={tuned['beta']} "
            f"bu_serial={tuned['bu_serial']} grid={tuned['grid_blocks']} claim={tuned['td_claim']} "
            f"engine={tuned.get('small_edges', 0)} ({tuned['default_ms']:.3f} -> {tuned['tuned_ms']:.3f} ms on "
            f"tuning sources)")
        log(f"[bench] timing {args.steps} steps with alpha={args.alpha} beta={args.beta} (defaults)")
        d_stats, d_elapsed = timed_steps(opts, args.steps)
        default_params = {"value": round(m * args.steps / d_elapsed / 1e9, 3), "alpha": args.alpha,
                          "beta": args.beta, "ms_per_step": round(d_elapsed / args.steps * 1e3, 4)}
        log(f"[bench] defaults: {default_params['value']} GTEPS")
        opts = autotune.opts_from(tuned, dir=0, parent_mode=opts.parent_mode, timing=opts.timing)

    log(f"[bench] timing {args.steps} steps (alpha={opts.alpha} beta={opts.beta})")
    stats, elapsed = timed_steps(opts, args.steps)
    gteps = m * args.steps / elapsed / 1e9
    per_source_ms = [s["total_ms"] for s in stats]
    log(f"[bench] {args.steps} searches in {elapsed:.3f}s -> {gteps:.2f} GTEPS "
        f"(per-search ms p50 {np.percentile(per_source_ms, 50):.2f} p99 {np.percentile(per_source_ms, 99):.2f})")

    # ---- roofline of the dominant kernel (HIP events recorded on the launch stream)
    roofline = None
    kernel_totals = {}
    if not args.no_timing:
        for s in stats:
            for k, v in s["kernel_ms"].items():
                kernel_totals[k] = kernel_totals.get(k, 0.0) + v
        log(f"[bench] kernel ms over timed steps: " +
            ", ".join(f"{k}={v:.2f}" for k, v in sorted(kernel_totals.items(), key=lambda x: -x[1]) if v))
    if not args.no_timing and table is not None:
        # events bracket only the bottom-up steps (timing mode 2), the
        # dominant kernel of this workload (see the kernel-trace profile):
        # k_bu_fill on a search's first bottom-up level, k_bu_sweep on the others
        dom = "bu_sweep"
        wo = d_off.element_size()
        nbytes, launches, ms = 0.0, 0, 0.0
        for i, s in enumerate(stats):
            row = table["rows"][int(sources[i % nsrc])]
            for d, (kind, b) in enumerate(level_bytes(s, row, n, wo, table["isolated"])):
                if kind == dom:
                    nbytes += b
                    launches += 1
                    ms += s["level_ms"][d]
        if launches and ms > 0:
            avg_s = ms / launches / 1e3
            achieved = nbytes / launches / avg_s / 1e9
            traffic = read_traffic(dom)
            roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                        "kernels": "k_bu_fill (first bottom-up level of a search), k_bu_sweep (the others)",
                        "launches": launches, "avg_launch_us": round(avg_s * 1e6, 2),
                        "alg_bytes_per_launch": round(nbytes / launches),
                        "alg_bytes_from": f"oracle work table {table['path']} (counts of the timed sources; "
                                          "the -1 fill counted on the sweep that writes it)",
                        "sources_timed": min(args.steps, nsrc)}

    # ---- every source once (outside the K-step timed region)
    all_sources = None
    if args.steps < nsrc:
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        for s_ in sources:
            bfs.bfs_run(g, int(s_), parent, depth, ws, opts, stream)
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t_a
        all_sources = {"sources": nsrc, "gteps": round(m * nsrc / t_all / 1e9, 3),
                       "ms_per_search": round(t_all / nsrc * 1e3, 4)}
        log(f"[bench] all {nsrc} sources once: {m * nsrc / t_all / 1e9:.2f} GTEPS")

    batched = None
    if args.batched_reps > 0:
        from paper_1705_04590_amd import autotune
        k = min(64, nsrc)
        log(f"[bench] batched: {k} sources per bfs_run_multi, {args.batched_reps} timed reps")
        # the same k sources one at a time with minimum parents (the batch's
        # parent mode), with the knobs tuned for single searches
        mino = (autotune.opts_from(tuned, dir=0, parent_mode=1, timing=0) if tuned is not None
                else bfs.bfs_opts_default(parent_mode=1, alpha=args.alpha, beta=args.beta))
        bfs.bfs_run(g, int(sources[0]), parent, depth, ws, mino, stream)
        torch.cuda.synchronize()
        t_s = time.perf_counter()
        for s_ in sources[:k]:
            bfs.bfs_run(g, int(s_), parent, depth, ws, mino, stream)
        torch.cuda.synchronize()
        single_min_qps = k / (time.perf_counter() - t_s)
        wsm = bfs.workspace(g, k, dev)
        bpar = torch.empty(k * n, dtype=torch.int32, device=dev)
        bdep = torch.empty(k * n, dtype=torch.int32, device=dev)
        mopts = bfs.bfs_opts_default(alpha=args.alpha, beta=args.beta, timing=0)
        if tuned is not None:
            mt = autotune.tune(g, graphgen.random_sources(off, k, seed=99), k=k, cache_path=args.tune_cache,
                               force=args.retune)
            mopts = autotune.opts_from(mt, timing=0)
            log(f"[bench] batched autotune: alpha={mt['alpha']} beta={mt['beta']} serial={mt['bu_serial']} "
                f"({mt['default_ms']:.2f} -> {mt['tuned_ms']:.2f} ms)")
        bfs.bfs_run_multi(g, sources[:k], bpar, bdep, wsm, mopts, stream)
        torch.cuda.synchronize()
        # one more batch with events around every kernel: the dominant
        # kernel's (the batched bottom-up sweep's) roofline from the model
        # bytes of its levels
        mt_opts = (autotune.opts_from(mt, timing=1) if tuned is not None
                   else bfs.bfs_opts_default(alpha=args.alpha, beta=args.beta, timing=1))
        ms_roof = ms_roofline(bfs.bfs_run_multi(g, sources[:k], bpar, bdep, wsm, mt_opts, stream).as_dict(), n, k)
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        for _ in range(args.batched_reps):
            bfs.bfs_run_multi(g, sources[:k], bpar, bdep, wsm, mopts, stream)
        torch.cuda.synchronize()
        batch_s = (time.perf_counter() - t_b) / args.batched_reps
        single_any_qps = args.steps / elapsed
        batched = {"sources_per_batch": k, "batch_ms": round(batch_s * 1e3, 3),
                   "queries_per_s": round(k / batch_s, 1), "parent_mode": "min",
                   "single_source_min_queries_per_s": round(single_min_qps, 1),
                   "speedup_vs_single_min": round(k / batch_s / single_min_qps, 3),
                   "single_source_any_queries_per_s": round(single_any_qps, 1),
                   "speedup_vs_single_any": round(k / batch_s / single_any_qps, 3),
                   "roofline": ms_roof}
        log(f"[bench] batched: {batch_s * 1e3:.2f} ms per {k}-source batch -> {k / batch_s:.1f} queries/s "
            f"(single-source: {single_min_qps:.1f} q/s minimum parents, {single_any_qps:.1f} q/s any parents)")
        del wsm, bpar, bdep
        torch.cuda.empty_cache()

    if args.copy_calibration:
        src_t = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst_t = torch.empty_like(src_t)
        for _ in range(3):
            dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t
        log("[bench] copy calibration: 3 x 1 GiB device copies done")

    served = None
    if not args.no_serve:
        t0 = time.time()
        sgraphs, keep = serve_graphs(dev)
        log(f"[bench] serving leg: {len(sgraphs)} graphs resident in {time.time() - t0:.1f}s")
        cap1, capb, rows = serve_measure(sgraphs, args.line_serve_rates, args.line_serve_seconds,
                                         args.serve_requests, args.serve_slots, args.serve_budget_gib)
        served = {"graphs": len(sgraphs), "capacity_one_query_per_launch_qps": round(cap1, 1),
                  "capacity_batched_qps": round(capb, 1), "rates": rows}
        for x in sgraphs:
            x[1].close()
        del keep, sgraphs
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline (latency budget {args.cpu_seconds}s, then one search per core)")
        cpu = cpu_baseline(off, cols, sources, m, args.cpu_seconds)
        log(f"[bench] CPU: {cpu['value']:.4f} GTEPS on one core, {cpu['throughput']['queries_per_s']:.3f} q/s on "
            f"{cpu['throughput']['cores']} cores ({cpu['host']['cpu_model']})")

    out = {
        "metric": METRIC, "value": round(gteps, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"kronecker_s{args.scale}_ef{args.edgefactor}_single_source_{args.dir}",
                   "scale": args.scale, "edgefactor": args.edgefactor, "n": n, "nnz": nnz, "m_undirected": m,
                   "sources": nsrc, "sources_timed": min(args.steps, nsrc),
                   "offsets": "int32" if use32 else "int64",
                   "parent_mode": args.parent_mode, "alpha": opts.alpha, "beta": opts.beta,
                   "bu_serial": opts.bu_serial or 16, "grid_blocks": opts.grid_blocks or 2048,
                   "td_claim": "cas" if opts.td_claim == 1 else "fetch_or",
                   "tuning": ((f"autotuned on {args.tune_sources} sources of seed 99" +
                               (" (cached entry)" if tuned.get("cached") else "")) if tuned else "none"),
                   "levels_p50": int(np.median([s["levels"] for s in stats])),
                   "search_ms_p50": round(float(np.percentile(per_source_ms, 50)), 3),
                   "search_ms_p99": round(float(np.percentile(per_source_ms, 99)), 3),
                   "kernel_ms_total": {k: round(v, 3) for k, v in kernel_totals.items() if v}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "all_sources": all_sources,
        "batched": batched,
        "served": served,
        "default_params": default_params,
    }
    print(json.dumps(out), flush=True)
    g.close()

if __name__ == "__main__":
    main()
