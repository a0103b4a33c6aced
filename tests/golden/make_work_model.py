#!/usr/bin/env python3
"""Writes the per-source, per-level work counts of a Kronecker benchmark graph
from the CPU oracle only (no GPU code is loaded).

For every source and every level d of its search the table stores the counts
the algorithmic-byte model of the benchmark reads, all of them fixed by the
level sets L_d, which are unique (Section 2):

    n_f   = |L_d|                      frontier vertices
    m_f   = sum of deg(u), u in L_d    frontier edges (directed CSR entries)
    m_u   = edges of vertices outside L_0..L_d (the unexplored edges the
            Section 4.4 rule compares m_f with)
    u     = vertices with edges and no parent before level d is expanded
    x     = adjacency entries a first-hit bottom-up expansion of level d
            examines: each of those u vertices scans its sorted row until the
            first member of L_d, inclusive (Alg. 2), else the whole row

x is stored for every level, so any top-down / bottom-up schedule can be
priced; `dir` is the schedule of the Section 4.4 rule at alpha = 15,
beta = 18, from the oracle.

Usage: python tests/golden/make_work_model.py [--scale 26] [--threads 7]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--edgefactor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--source-seed", type=int, default=2)
    ap.add_argument("--nsources", type=int, default=64)
    ap.add_argument("--threads", type=int, default=7)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    out = a.out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                f"kron{a.scale}_work_model.json")
    t0 = time.time()
    off, cols = graphgen.kronecker(a.scale, a.edgefactor, seed=a.seed)
    n = off.size - 1
    iso = int((np.diff(off) == 0).sum())
    print(f"graph: n={n} nnz={int(off[-1])} isolated={iso} ({time.time() - t0:.0f}s)", flush=True)
    sources = [int(s) for s in graphgen.random_sources(off, a.nsources, seed=a.source_seed)]
    orc = oracle.load()

    def one(i_s):
        i, s = i_s
        t = time.time()
        _, depth = orc.bfs(off, cols, s)
        n_f, m_f, m_u = orc.level_stats(off, depth)
        sched = orc.direction_schedule(n, n_f, m_f, m_u, 15.0, 18.0)
        levels = []
        for d in range(len(n_f)):
            x, un = orc.bu_scan_lengths(off, cols, depth, d)
            levels.append([int(n_f[d]), int(m_f[d]), int(m_u[d]), int(un - iso), int(x)])
        print(f"source {i} ({s}): {len(levels)} levels, {time.time() - t:.0f}s", flush=True)
        return {"source": s, "levels": levels, "dir": [int(v) for v in sched]}

    with ThreadPoolExecutor(a.threads) as ex:
        rows = list(ex.map(one, enumerate(sources)))
    doc = {
        "what": "per-level work counts of single-source BFS from the CPU oracle (see make_work_model.py)",
        "graph": {"kind": "kronecker", "scale": a.scale, "edgefactor": a.edgefactor, "seed": a.seed,
                  "n": n, "nnz": int(off[-1]), "isolated": iso},
        "source_seed": a.source_seed,
        "level_fields": ["n_f", "m_f", "m_u", "u", "x"],
        "alpha": 15.0, "beta": 18.0,
        "sources": rows,
    }
    with open(out, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
        f.write("\n")
    print(f"wrote {out} ({time.time() - t0:.0f}s)", flush=True)


if __name__ == "__main__":
    main()
