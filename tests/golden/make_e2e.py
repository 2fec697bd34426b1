"""Writes tests/golden/e2e_oracle.json: the FP64 oracle's whole layouts of
three configurations and the objectives of its results, for the end-to-end
GPU tests (whose own runs take well under a second, while the oracle needs
minutes per layout and its full stress over all pairs up to ~10 minutes).

Only oracle/ (the method) and synth/ (seeded input generators) are used:

* rgg17: random geometric graph, 2^17 points, mean degree 6, largest
  component (graph seed 1); k = 3, Barnes-Hut theta = 0.5 on every level,
  alpha decay 0.5, hierarchy down to <= 100 vertices; layout seeds 1, 2, 3;
* rmat16: R-MAT scale 16, 8 * 2^16 draws (a, b, c) = (.57, .19, .19), largest
  component, ids permuted (graph seed 1); k = 2, theta = 0.5, decay 0.5,
  hierarchy to <= 100 vertices; layout seeds 1, 2, 3;
* snapshots: RGG 2^16 (mean degree 6, graph seed 1) and three churned
  snapshots of it (1% of the edges replaced, new edges at hop distance 2);
  snapshot 0 laid out from scratch (k = 3, theta = 0.5, decay 0.5, <= 100
  vertices, seed 1), each later one warm-started from the previous layout
  at alpha_min on the finest level (Sec. 4.3).

Per layout: maxent-stress M_S at alpha_min over the k-hop sets (Eq. 1), its
stress and entropy parts, full stress F at the optimal scale s* (Sec. 4,
"Methodology"), level sizes, iterations and cap hits per level.

Run: python tests/golden/make_e2e.py [case ...]   (about 45 minutes on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "e2e_oracle.json")


def params(k, seed):
    return oracle.Params(k=k, theta=0.5, alpha_decay=0.5, coarsest_n=100, seed=seed)


def summarize(g, k, x, st, p):
    kh = oracle.khop_build(g.row_ptr, g.col, k)
    o = oracle.objective(kh, x, p.alpha_min, p.q)
    fs = oracle.full_stress(g.row_ptr, g.col, x)
    lv = sorted(st["levels"], key=lambda r: r["level"])
    return {"M_S": o["M"], "stress": o["stress"], "entropy": o["ent"],
            "coincident": int(o["coincident"]), "F": fs["F"], "s_opt": fs["s_opt"],
            "level_n": [int(r["n"]) for r in lv], "level_iters": [int(r["iters"]) for r in lv],
            "level_cap_hit": [bool(r["final_iters"] == p.max_final_iters
                                   and r["hist"][-1][1] >= p.eps_final) for r in lv]}


def layouts(name, graph, k):
    g = synth.config_graph(graph, 1)
    res = {"graph": graph, "n": int(g.n), "m": int(g.m), "k": k, "theta": 0.5,
           "alpha_decay": 0.5, "coarsest_n": 100, "seeds": {}}
    for seed in (1, 2, 3):
        t0 = time.time()
        p = params(k, seed)
        x, st = oracle.layout(g, p)
        r = summarize(g, k, x, st, p)
        r["seconds"] = time.time() - t0
        res["seeds"][str(seed)] = r
        print(f"[{name}] seed {seed}: M_S {r['M_S']:.6e} F {r['F']:.6e} "
              f"({r['seconds']:.0f} s)", flush=True)
    return res


def snapshots():
    k = 3
    g = synth.config_graph("rgg16", 1)
    snaps = [g]
    for i in range(1, 4):
        snaps.append(synth.churn_snapshot(snaps[-1], 1000 + i, 0.01, 2))
    res = {"graph": "rgg16", "n": int(g.n), "k": k, "theta": 0.5, "alpha_decay": 0.5,
           "coarsest_n": 100, "seed": 1, "churn_seeds": [1001, 1002, 1003], "snapshots": []}
    p = params(k, 1)
    x = None
    for i, s in enumerate(snaps):
        t0 = time.time()
        x, st = oracle.layout(s, p, init_xy=x)
        r = summarize(s, k, x, st, p)
        r["m"] = int(s.m)
        r["seconds"] = time.time() - t0
        res["snapshots"].append(r)
        print(f"[snapshots] {i}: M_S {r['M_S']:.6e} F {r['F']:.6e} ({r['seconds']:.0f} s)",
              flush=True)
    return res


CASES = {"rgg17": lambda: layouts("rgg17", "rgg17", 3),
         "rmat16": lambda: layouts("rmat16", "rmat16", 2),
         "snapshots": snapshots}


def main():
    want = sys.argv[1:] or list(CASES)
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data["_about"] = ("FP64 oracle layouts and objectives written by tests/golden/make_e2e.py "
                      "(oracle/ and synth/ only); see that script for the configurations")
    for name in want:
        data[name] = CASES[name]()
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
            fh.write("\n")


if __name__ == "__main__":
    main()
