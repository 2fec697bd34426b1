"""Benchmark: multilevel maxent-stress layout on one MI355X.

A step is one complete layout of the workload (every stage: coarsening,
k-hop sets on every level, Barnes-Hut far field, Jacobi sweeps with the
alpha schedule, prolongation), with the graph already resident in HBM.

Default workload: R-MAT, 2^20 vertices, 8*2^20 edge draws (a, b, c) =
(0.57, 0.19, 0.19), duplicates/self-loops removed, largest component (546,036
vertices, 8.04M edges), ids permuted by the seed; k = 2, theta = 0.5, q = 0,
alpha 1 -> x0.5 -> 0.008, a = 2, eps 1e-4, <= 200 final iterations, hierarchy
down to <= 100 vertices.  Synthetic data, random initial layout from the seed.

Prints one JSON line.  value = vertex updates (n of a level x iterations on
it, summed over levels) per second of layout wall time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "vertex-updates/s of maxent-stress sweep at 2^20 verts; time-to-layout at fixed stress"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "rmat20": dict(graph="rmat20", k=2, theta=0.5, alpha_decay=0.5, coarsest_n=100,
                   desc="R-MAT scale 20 (8*2^20 draws, a=.57 b=c=.19), LCC, k=2, theta=0.5, "
                        "full hierarchy to <=100 vertices"),
    "rgg17": dict(graph="rgg17", k=3, theta=0.5, alpha_decay=0.5, coarsest_n=100,
                  desc="RGG 2^17 points, mean degree ~6, LCC, k=3, theta=0.5"),
    "grid32": dict(graph="grid32", k=3, theta=-1.0, alpha_decay=0.5, max_levels=3,
                   desc="32x32 grid, k=3, exact far field, 3 coarsening levels"),
    "rgg22": dict(graph="rgg22", k=3, theta=0.5, alpha_decay=0.5, coarsest_n=100,
                  desc="RGG 2^22 points, mean degree ~8, LCC, k=3, theta=0.5"),
    # the paper's configuration (S = E, decay 0.3, coarsening to 2 vertices) on a
    # Delaunay triangulation of the shape of its del20 instance (context only)
    "del20": dict(graph="del20", k=1, theta=0.5, alpha_decay=0.3, coarsest_n=2,
                  desc="Delaunay triangulation of 2^20 uniform points, k=1 (S=E), theta=0.5, "
                       "decay 0.3, hierarchy to 2 vertices"),
}


def batch_comparison(args):
    """4096 uneven graphs (64..8192 vertices; grids, random trees, RGGs) laid
    out in one batch vs one at a time (a uniform random sample of the same
    graphs, scaled to the batch), k = 3, theta = 0.5, hierarchy to <= 100
    vertices per graph.  Prints one JSON line."""
    import numpy as np
    import torch

    import paper_1506_04383_amd as mm
    import synth

    ctx = mm.Context(0)
    t0 = time.perf_counter()
    gs = synth.batch_graphs(args.batch_graphs, args.seed)
    rp, col, offs = synth.concat(gs)
    print(f"[batch] {len(gs)} graphs, n={int(offs[-1])}, generated in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    P = dict(k=3, theta=0.5, alpha_decay=0.5, coarsest_n=100, seed=args.seed, validate=0)
    dg = ctx.graph(rp, col)
    if args.warmup:
        mm.layout_batch(ctx, dg, None, offs, mm.Params(**P))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xy, lev, st = mm.layout_batch(ctx, dg, None, offs, mm.Params(**P))
    torch.cuda.synchronize()
    T_batch = time.perf_counter() - t0
    print(f"[batch] batched layout {T_batch:.2f}s, {st['levels']} union levels",
          file=sys.stderr, flush=True)
    rng = np.random.default_rng(args.seed)
    sample = rng.choice(len(gs), size=min(args.batch_sample, len(gs)), replace=False)
    times, rel = [], []
    for j, i in enumerate(sample):
        g = gs[int(i)]
        dgi = ctx.graph(g.row_ptr, g.col)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x1, _ = mm.layout(ctx, dgi, mm.Params(**P))
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        kh = mm.khop_build(ctx, dgi, 3)
        Mb = mm.objective(ctx, kh, xy[int(offs[i]):int(offs[i + 1])], 0.008)["M"]
        M1 = mm.objective(ctx, kh, x1, 0.008)["M"]
        kh.free()
        rel.append((Mb - M1) / abs(M1))
        if j % 16 == 15:
            print(f"[batch] {j + 1} single layouts timed", file=sys.stderr, flush=True)
    times = np.array(times)
    T_seq = float(times.mean() * len(gs))
    T_seq_se = float(times.std(ddof=1) / np.sqrt(times.size) * len(gs))
    rel = np.array(rel)
    out = {"metric": "time to lay out 4096 uneven graphs, batched vs one at a time",
           "value": T_seq / T_batch, "unit": "speedup (x)", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(gs)} graphs, n log-uniform in [64, 8192], grids / "
                      "random recursive trees / RGG (deg 6, LCC); k=3, theta=0.5, hierarchy "
                      "to <=100 vertices per graph", "graphs": len(gs), "n": int(offs[-1]),
                      "m": int(rp[-1]) // 2, "seed": args.seed},
           "batched_s": T_batch, "one_at_a_time_s_estimate": T_seq,
           "one_at_a_time_s_stderr": T_seq_se,
           "one_at_a_time_sample": int(times.size),
           "batched_graphs_per_s": len(gs) / T_batch,
           "union_levels": st["levels"], "union_iters_per_level":
               [l["iters"] for l in st["per_level"]],
           "stress_rel_diff_batched_vs_single": {"mean": float(rel.mean()),
                                                 "max_abs": float(np.abs(rel).max())}}
    print(json.dumps(out))
    ctx.close()


def snapshot_comparison(args):
    """64 snapshots of RGG 2^16 (mean degree 6), each with 1% of its edges
    replaced (non-tree edges dropped, new edges to vertices 2 hops away); each
    snapshot warm-started from the previous layout at alpha_min on the finest
    level, vs laying it out from scratch.  Prints one JSON line."""
    import numpy as np
    import torch

    import paper_1506_04383_amd as mm
    import synth

    ctx = mm.Context(0)
    g = synth.config_graph("rgg16", args.seed)
    snaps = [g]
    t0 = time.perf_counter()
    for i in range(1, args.snapshots):
        snaps.append(synth.churn_snapshot(snaps[-1], args.seed * 1000 + i, 0.01, 2))
        if i % 8 == 0:
            print(f"[snap] generated {i} snapshots ({time.perf_counter() - t0:.0f}s)",
                  file=sys.stderr, flush=True)
    dgs = [ctx.graph(s.row_ptr, s.col) for s in snaps]
    P = dict(k=3, theta=0.5, alpha_decay=0.5, coarsest_n=100, seed=args.seed, validate=0)
    x0, _ = mm.layout(ctx, dgs[0], mm.Params(**P))
    torch.cuda.synchronize()
    # chain A: the default stopping rule at alpha_min (relative change < 1e-4);
    # chain B: the same chain run to the iteration cap (relative change < 1e-7)
    warm_t, warm_M, tight_t, tight_M, scratch_t, scratch_M, idx = [], [], [], [], [], [], []
    x, xt = x0, x0
    for i in range(1, len(snaps)):
        t1 = time.perf_counter()
        x, st = mm.layout(ctx, dgs[i], mm.Params(**P), init_xy=x)
        torch.cuda.synchronize()
        warm_t.append(time.perf_counter() - t1)
        t1 = time.perf_counter()
        xt, _ = mm.layout(ctx, dgs[i], mm.Params(**{**P, "eps_final": 1e-7}), init_xy=xt)
        torch.cuda.synchronize()
        tight_t.append(time.perf_counter() - t1)
        if i % args.snapshot_scratch_every == 0:
            kh = mm.khop_build(ctx, dgs[i], 3)
            t1 = time.perf_counter()
            xs, _ = mm.layout(ctx, dgs[i], mm.Params(**P))
            torch.cuda.synchronize()
            scratch_t.append(time.perf_counter() - t1)
            warm_M.append(mm.objective(ctx, kh, x, 0.008)["M"])
            tight_M.append(mm.objective(ctx, kh, xt, 0.008)["M"])
            scratch_M.append(mm.objective(ctx, kh, xs, 0.008)["M"])
            kh.free()
            idx.append(i)
    # spread of scratch layouts over seeds (noise floor of "equal stress")
    kh = mm.khop_build(ctx, dgs[-1], 3)
    seedM = [mm.objective(ctx, kh, mm.layout(ctx, dgs[-1], mm.Params(**{**P, "seed": args.seed + j}))[0],
                          0.008)["M"] for j in range(3)]
    kh.free()
    warm_t = np.array(warm_t)
    ratio = np.array(warm_M) / np.array(scratch_M)
    ratio_t = np.array(tight_M) / np.array(scratch_M)
    out = {"metric": "time per snapshot at equal maxent-stress, warm-started dynamic update "
                     "(run to the iteration cap at alpha_min) vs layout from scratch",
           "value": float(np.mean(scratch_t) / np.mean(tight_t)), "unit": "speedup (x)",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(snaps)} snapshots of RGG 2^16 (deg 6, LCC), 1% edge "
                      "churn per snapshot (D=2); warm start at alpha_min on the finest level; "
                      "k=3, theta=0.5", "n": g.n, "m": g.m, "seed": args.seed},
           "default_rule_chain": {"s_per_snapshot": float(warm_t.mean()),
                                  "speedup": float(np.mean(scratch_t) / warm_t.mean())},
           "scratch_s_per_snapshot": float(np.mean(scratch_t)),
           "scratch_sample": idx,
           "default_rule_stress_ratio_vs_scratch": {"mean": float(ratio.mean()),
                                                    "min": float(ratio.min()),
                                                    "max": float(ratio.max())},
           "tight_chain": {"s_per_snapshot": float(np.mean(tight_t)),
                           "stress_ratio_vs_scratch": {"mean": float(ratio_t.mean()),
                                                       "min": float(ratio_t.min()),
                                                       "max": float(ratio_t.max())}},
           "M_warm": warm_M, "M_tight": tight_M, "M_scratch": scratch_M,
           "scratch_seed_spread": float((max(seedM) - min(seedM)) / abs(np.mean(seedM)))}
    print(json.dumps(out))
    ctx.close()


def dynamic_comparison(args):
    """The update algorithm of Sec. 4.3 against layouts from scratch, on the
    paper's grid: x in {1, 5} % of the edges replaced, new edges to vertices
    1 < d <= D hops away with D in {2, 16}, MulMent_h with h in {0, 7} (h = 0:
    exact far field; h = 7: Eq. 3 with the graph 7 levels beneath, the update
    cutting the hierarchy after 7 levels).  Graphs: RGG 2^16 and a Delaunay
    triangulation of 2^16 points, the paper's configuration otherwise (S = E,
    decay 0.3).  Prints one JSON line."""
    import numpy as np
    import torch

    import paper_1506_04383_amd as mm
    import synth

    ctx = mm.Context(0)
    base = dict(k=1, alpha_decay=0.3, coarsest_n=2, seed=args.seed, validate=0)
    graphs = [("rgg16", synth.config_graph("rgg16", args.seed)),
              ("del16", synth.delaunay(1 << 16, args.seed))]
    rows = []
    for gname, g in graphs:
        dg = ctx.graph(g.row_ptr, g.col)
        churned = {}
        for x in (1, 5):
            for D in (2, 16):
                t0 = time.perf_counter()
                churned[(x, D)] = synth.churn_snapshot(g, args.seed * 100 + x * 10 + D, x / 100.0, D)
                print(f"[dyn] {gname} churn x={x}% D={D} in {time.perf_counter() - t0:.1f}s",
                      file=sys.stderr, flush=True)
        for h in (0, 7):
            P = dict(base, theta=-1.0) if h == 0 else dict(base, theta=0.5, approx_h=h)
            xg, _ = mm.layout(ctx, dg, mm.Params(**P))
            for (x, D), q in churned.items():
                dq = ctx.graph(q.row_ptr, q.col)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                xd, _ = mm.layout(ctx, dq, mm.Params(**P), init_xy=xg)
                torch.cuda.synchronize()
                t_dyn = time.perf_counter() - t0
                t0 = time.perf_counter()
                xs, _ = mm.layout(ctx, dq, mm.Params(**P))
                torch.cuda.synchronize()
                t_scr = time.perf_counter() - t0
                kh = mm.khop_build(ctx, dq, 1)
                Md = mm.objective(ctx, kh, xd, 0.008)["M"]
                Ms = mm.objective(ctx, kh, xs, 0.008)["M"]
                kh.free()
                Fd = mm.full_stress(ctx, dq, xd)["F"]
                Fs = mm.full_stress(ctx, dq, xs)["F"]
                rows.append({"graph": gname, "x_pct": x, "D": D, "h": h, "t_dyn_s": t_dyn,
                             "t_scratch_s": t_scr, "speedup": t_scr / t_dyn,
                             "F_dyn_over_scratch": Fd / Fs, "M_dyn": Md, "M_scratch": Ms})
                print(f"[dyn] {gname} x={x} D={D} h={h}: dyn {t_dyn:.3f}s scratch {t_scr:.3f}s "
                      f"F ratio {Fd / Fs:.3f} M dyn {Md:.6g} scratch {Ms:.6g}", file=sys.stderr,
                      flush=True)

    def gmean(v):
        return float(np.exp(np.mean(np.log(v))))

    by_h = {h: [r for r in rows if r["h"] == h] for h in (0, 7)}
    out = {"metric": "time of the update algorithm vs scratch on the paper's dynamic protocol "
                     "(Sec. 4.3)",
           "value": gmean([r["speedup"] for r in rows]), "unit": "speedup (x, geometric mean)",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "RGG 2^16 and Delaunay 2^16; x in {1,5}%, D in {2,16}, "
                                  "h in {0,7}; k=1, decay 0.3", "seed": args.seed},
           "speedup_by_h": {str(h): gmean([r["speedup"] for r in v]) for h, v in by_h.items()},
           "F_ratio_mean": float(np.mean([r["F_dyn_over_scratch"] for r in rows])),
           # M can change sign (k = 1 has few stress pairs), so no ratio: the
           # share of runs where the update ends at no higher maxent-stress
           "M_dyn_not_above_scratch": float(np.mean([r["M_dyn"] <= r["M_scratch"] for r in rows])),
           "runs": rows}
    print(json.dumps(out))
    ctx.close()


def caps_comparison(args):
    """Time against stress: the RGG 2^17 (k = 3) and R-MAT 2^20 (k = 2)
    layouts with the cap on the iterations at alpha_min set to 25, 50, 100 and
    200 (the paper stops at a relative change below 1e-4 and names no cap).
    Per cap: layout time, maxent-stress M_S, full stress F at the optimal
    scale, levels stopped by the cap.  Prints one JSON line."""
    import numpy as np
    import torch

    import paper_1506_04383_amd as mm
    import synth

    ctx = mm.Context(0)
    if args.tune_db and os.path.exists(args.tune_db):
        recs = json.load(open(args.tune_db))["records"]
        ctx.tune_import(np.array(recs, dtype=np.int64).reshape(-1, mm.TUNE_FIELDS))
    rows = []
    for wname in ("rgg17", "rmat20"):
        wl = WORKLOADS[wname]
        g = synth.config_graph(wl["graph"], args.seed)
        dg = ctx.graph(g.row_ptr, g.col)
        kh = mm.khop_build(ctx, dg, wl["k"])
        for cap in (25, 50, 100, 200):
            p = mm.Params(k=wl["k"], theta=wl["theta"], alpha_decay=wl["alpha_decay"],
                          coarsest_n=wl["coarsest_n"], seed=args.seed, validate=0,
                          autotune=1, exact_below=args.exact_below, max_final_iters=cap)
            mm.layout(ctx, dg, p)  # warm-up (tunes levels the table lacks)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xy, st = mm.layout(ctx, dg, p)
            torch.cuda.synchronize()
            T = time.perf_counter() - t0
            M = mm.objective(ctx, kh, xy, p.alpha_min, p.q)["M"]
            F = mm.full_stress(ctx, dg, xy)["F"]
            caps = [l["cap_hit"] for l in st["per_level"]]
            rows.append({"workload": wname, "cap": cap, "time_s": T, "M_S": M, "F": F,
                         "levels_stopped_by_cap": int(sum(caps)), "levels": len(caps),
                         "vertex_updates": st["vertex_updates"]})
            print(f"[caps] {wname} cap {cap}: {T:.2f} s, M_S {M:.6e}, F {F:.6e}, "
                  f"{sum(caps)}/{len(caps)} levels at the cap", file=sys.stderr, flush=True)
        kh.free()
    print(json.dumps({"metric": "time-to-layout and final stress vs the cap on final iterations",
                      "unit": "s", "n_gpus": 1, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "RGG 2^17 (k=3) and R-MAT 2^20 (k=2), theta=0.5, "
                                 "decay 0.5, hierarchy to <=100 vertices, exact far field "
                                 f"at <= {args.exact_below} vertices", "seed": args.seed},
                      "rows": rows}))
    ctx.close()


def learned_comparison(args):
    """Learned far field vs plain Barnes-Hut on RGG 2^22 (k = 3), searched over
    the opening angle: plain theta = 0.5 (the reference), then plain and
    learned at theta = 1, 1.5, 2, 3.  For each theta the network is trained on
    the GPU on exact residuals of the cells that theta accepts in layouts of
    RGG 2^14 (mean degree 8) made by the method (so its inputs cover the cell
    sizes that theta admits).  A configuration is at equal stress when its
    final maxent-stress M_S is within 1% of the reference's; the line reports
    the cheapest equal-stress configuration of each form and value = time of
    the cheapest plain one / time of the cheapest learned one (null if no
    learned configuration reaches equal stress).  Prints one JSON line."""
    import numpy as np
    import torch

    import paper_1506_04383_amd as mm
    import synth

    ctx = mm.Context(0)
    base = dict(k=3, alpha_decay=0.5, coarsest_n=100, seed=args.seed, validate=0)
    thetas = [float(t) for t in args.learned_thetas.split(",")]
    # layouts of the training graphs (made by the method, plain theta = 0.5)
    t0 = time.perf_counter()
    train_xy = []
    for s in range(101, 101 + args.train_graphs):
        g = synth.config_graph("rgg14", s)
        xy, _ = mm.layout(ctx, ctx.graph(g.row_ptr, g.col), mm.Params(theta=0.5, **{**base, "seed": s}))
        train_xy.append(xy)
    t_layouts = time.perf_counter() - t0
    nets, training = {}, {}
    for th in thetas:
        t0 = time.perf_counter()
        feats, tgts = [], []
        for xy in train_xy:
            S = mm.far_samples(ctx, xy, th)
            feats.append(S["feat"])
            tgts.append(S["target"])
        feat, tgt = torch.cat(feats), torch.cat(tgts)
        torch.cuda.synchronize()
        t_samples = time.perf_counter() - t0
        w = mm.mlp_init(ctx, 11, out_scale=0.1)
        adam = torch.zeros(2 * mm.MLP_PARAMS, dtype=torch.float32, device="cuda")
        t0 = time.perf_counter()
        losses = mm.mlp_train(ctx, feat, tgt, w, adam, args.train_steps, 4096, 2e-3, 5)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        losses = losses.cpu().numpy()
        nets[th] = w
        training[str(th)] = {"samples": int(feat.shape[0]), "sample_s": t_samples,
                             "train_s": t_train, "loss_first": float(losses[:20].mean()),
                             "loss_last": float(losses[-100:].mean())}
        print(f"[learned] theta {th}: {feat.shape[0]} samples in {t_samples:.1f}s, "
              f"{args.train_steps} Adam steps in {t_train:.2f}s, loss {losses[:20].mean():.3e} -> "
              f"{losses[-100:].mean():.3e}", file=sys.stderr, flush=True)
        del feat, tgt

    g = synth.config_graph("rgg22", args.seed)
    dg = ctx.graph(g.row_ptr, g.col)
    print(f"[learned] rgg22 n={g.n} m={g.m}", file=sys.stderr, flush=True)
    kh = mm.khop_build(ctx, dg, 3)
    configs = [("plain", 0.5)] + [(form, th) for th in thetas for form in ("plain", "learned")]
    runs = []
    for form, th in configs:
        p = mm.Params(theta=th, mlp_weights=nets[th] if form == "learned" else None, **base)
        if args.warmup:
            mm.layout(ctx, dg, p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xy, st = mm.layout(ctx, dg, p)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        o = mm.objective(ctx, kh, xy, 0.008)
        L0 = st["per_level"][0]
        runs.append({"form": form, "theta": th, "time_to_layout_s": T,
                     "final_maxent_stress": o["M"], "stress_part": o["stress"],
                     "far_field_ms": sum(l["far_ms"] for l in st["per_level"]),
                     "iterations_ms": st["t_iterate_ms"], "finest_iters": L0["iters"],
                     "finest_far_ms_per_iter": L0["far_ms"] / max(L0["iters"], 1)})
        print(f"[learned] {form} theta {th}: {T:.2f}s M_S={o['M']:.6e} stress part "
              f"{o['stress']:.6e}", file=sys.stderr, flush=True)
    kh.free()
    ref = runs[0]
    for r in runs:
        r["stress_ratio_vs_plain_theta0.5"] = r["final_maxent_stress"] / ref["final_maxent_stress"]
        r["equal_stress"] = bool(abs(r["final_maxent_stress"] - ref["final_maxent_stress"])
                                 <= 0.01 * abs(ref["final_maxent_stress"]))

    def cheapest(form):
        ok = [r for r in runs if r["form"] == form and r["equal_stress"]]
        return min(ok, key=lambda r: r["time_to_layout_s"]) if ok else None

    best_plain, best_learned = cheapest("plain"), cheapest("learned")
    out = {"metric": "time-to-layout at equal maxent-stress, learned far field vs plain Barnes-Hut",
           "value": (best_plain["time_to_layout_s"] / best_learned["time_to_layout_s"]
                     if best_learned else None),
           "unit": "speedup (x)", "n_gpus": 1, "higher_is_better": True, "dtype": "f32+bf16",
           "data": "synthetic",
           "config": {"workload": "RGG 2^22 points, mean degree ~8, LCC, k=3; plain Barnes-Hut "
                      "at theta 0.5 (reference) and " + ", ".join(str(t) for t in thetas) +
                      "; learned: the same thetas + MLP 8-64-64-2 (BF16 MFMA) trained per theta "
                      "on RGG 2^14 layouts", "n": g.n, "m": g.m, "seed": args.seed,
                      "equal_stress": "M_S within 1% of plain theta 0.5"},
           "cheapest_plain": {"theta": best_plain["theta"], "time_s": best_plain["time_to_layout_s"]},
           "cheapest_learned": ({"theta": best_learned["theta"],
                                 "time_s": best_learned["time_to_layout_s"]} if best_learned else None),
           "training": {"graphs": args.train_graphs, "layouts_s": t_layouts,
                        "steps": args.train_steps, "batch": 4096, "per_theta": training},
           "runs": runs}
    print(json.dumps(out))
    ctx.close()


def sweep_bytes(n: int, k: int, entries: int, coarse: bool) -> int:
    """Algorithmic HBM bytes of one sweep launch: 4 B per stress-set entry,
    per vertex 8 B row offset + 4k B hop ends + 8 B x_u + 8 B F_u + 8 B x'_u
    (+ 4 B sqrt c on coarse levels), and the coordinate array once (8n B)."""
    per_v = 8 + 4 * k + 8 + 8 + 8 + (4 if coarse else 0)
    return 4 * entries + n * per_v + 8 * n


# copy-calibrated HBM traffic of the finest-level sweep step, per sweep kernel
TRAFFIC_PROFILES = {"sliced": os.path.join(ROOT, "profiles", "k_sweep_sliced_rmat20_traffic.md"),
                    "tiled": os.path.join(ROOT, "profiles", "k_sweep_tiled_rmat20_traffic.md")}
SLICED_GROUP = 64  # lanes code of the sliced layout in the per-level statistics
# Autotuner choices measured on MI355X for the bench workloads (written by
# --save-tune-db); loading them makes the timed layouts use a fixed, known
# sweep configuration per level.
TUNE_DB = os.path.join(ROOT, "paper_1506_04383_amd", "tune_mi355x.json")


def measured_traffic(workload: str, tile_bits: int, group: int, blocks: int):
    """HBM bytes per finest-level sweep step from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE passes (copy-calibrated), or None when the workload
    or the sweep configuration (tile bits, lanes per chunk, blocks per step) differs or the
    kernel source changed since the counters were taken."""
    import hashlib

    prof = TRAFFIC_PROFILES["sliced" if group == SLICED_GROUP else "tiled"]
    if workload != "rmat20" or not os.path.exists(prof):
        return None
    kv = {}
    for line in open(prof):
        if ":" in line and not line.startswith(("|", "#", " ", "`")):
            key, _, val = line.partition(":")
            kv[key.strip()] = val.strip()
    src = os.path.join(ROOT, kv.get("kernel_source", "-"))
    if not os.path.exists(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != kv.get("kernel_source_sha256"):
        return None
    if kv.get("sweep_config") != f"{tile_bits},{group},{blocks}":
        return None
    return int(kv["traffic_bytes_per_launch"])


def host_cpu() -> dict:
    """Model, sockets and logical CPUs of the host (lscpu), as far as readable."""
    import subprocess

    info = {"model": None, "sockets": None, "logical_cpus": os.cpu_count()}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            key, _, val = line.partition(":")
            key, val = key.strip(), val.strip()
            if key == "Model name":
                info["model"] = val
            elif key == "Socket(s)":
                info["sockets"] = int(val) if val.isdigit() else val
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(g, k, x, F, alpha, seconds=15.0, seed=0, seconds_1t=6.0):
    """The FP64 oracle's update of sampled rows (each row's stress set found by
    BFS, then Eq. 2), timed on the host cores: all threads, then one thread."""
    import numpy as np

    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rng = np.random.default_rng(seed)

    def timed(nrows):
        rows = rng.choice(g.n, size=nrows, replace=False).astype(np.int32)
        t0 = time.perf_counter()
        _, sizes = oracle.sweep_rows(g.row_ptr, g.col, k, x, F, alpha, rows)
        return rows.size, time.perf_counter() - t0, sizes

    prev = oracle.set_threads(threads)
    n1, dt, _ = timed(min(g.n, 256))
    target = max(256, min(g.n, int(n1 * seconds / max(dt, 1e-3))))
    nrows, dt, sizes = timed(target)
    oracle.set_threads(1)
    n1, dt1, _ = timed(min(g.n, 64))
    target1 = max(64, min(g.n, int(n1 * seconds_1t / max(dt1, 1e-3))))
    nrows1, dt1, sizes1 = timed(target1)
    oracle.set_threads(prev)
    return {"value": nrows / dt, "unit": "vertex-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{nrows} random rows of the finest level (mean |S| "
                      f"{float(sizes.mean()):.0f}), FP64 update of Eq. 2 with each row's "
                      f"k-hop set found by BFS, far field given, {dt:.1f} s; the same "
                      f"on 1 thread: {nrows1} rows in {dt1:.1f} s",
            "value_1_thread": nrows1 / dt1, "host": host_cpu()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat20", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-objective", action="store_true")
    ap.add_argument("--full-stress", action="store_true",
                    help="also compute the full stress F(x) over all pairs at the optimal scale "
                         "(breadth-first searches on the GPU: bit-parallel over all vertices for "
                         "low diameters, banded otherwise)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: the sweep configuration of every level is timed and chosen during "
                         "the first layout (the warm-up) and reused by the timed ones")
    ap.add_argument("--exact-below", type=int, default=49152,
                    help="levels with at most this many vertices use the exact all-pairs far "
                         "field (cheaper there than the tree on this GPU); 0 = Barnes-Hut on "
                         "every level")
    ap.add_argument("--approx-h", type=int, default=0,
                    help="h > 0: MulMent_h, the paper's cluster far field (Eq. 3) with the "
                         "graph h levels beneath, on every level with a coarser one")
    ap.add_argument("--tune-db", default=TUNE_DB,
                    help="JSON file of autotuner choices (per level shape) loaded into the "
                         "context before the first layout; levels it does not cover are tuned")
    ap.add_argument("--save-tune-db", default="",
                    help="write the context's autotuner choices here after the run")
    ap.add_argument("--mode", default="layout",
                    choices=["layout", "learned", "batch", "snapshots", "dynamic", "caps"],
                    help="layout: the layout benchmark; learned: learned far field vs plain "
                         "Barnes-Hut on RGG 2^22; batch: 4096 graphs batched vs one at a "
                         "time; snapshots: warm-started dynamic snapshots vs scratch; dynamic: "
                         "the paper's update protocol (x, D, h grid) vs scratch; caps: time "
                         "and stress against the cap on the final iterations")
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--batch-sample", type=int, default=96)
    ap.add_argument("--snapshots", type=int, default=64)
    ap.add_argument("--snapshot-scratch-every", type=int, default=8)
    ap.add_argument("--train-graphs", type=int, default=4)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--learned-thetas", default="1,1.5,2,3",
                    help="opening angles of the learned/plain comparison (besides plain 0.5)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the layout library "
              "does not shard a layout across GPUs", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        a = torch.ones(args.calibrate_copy * (1 << 18), dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4}))
        return

    if args.mode == "learned":
        learned_comparison(args)
        return
    if args.mode == "batch":
        batch_comparison(args)
        return
    if args.mode == "snapshots":
        snapshot_comparison(args)
        return
    if args.mode == "dynamic":
        dynamic_comparison(args)
        return
    if args.mode == "caps":
        caps_comparison(args)
        return

    import paper_1506_04383_amd as mm
    import synth

    wl = WORKLOADS[args.workload]
    t0 = time.time()
    g = synth.config_graph(wl["graph"], args.seed)
    print(f"[bench] generated {wl['graph']} n={g.n} m={g.m} in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    ctx = mm.Context(0)
    dg = ctx.graph(g.row_ptr, g.col)
    p = mm.Params(k=wl["k"], theta=wl["theta"], alpha_decay=wl["alpha_decay"],
                  coarsest_n=wl.get("coarsest_n", 2), max_levels=wl.get("max_levels", 62),
                  seed=args.seed, validate=0, autotune=args.autotune,
                  exact_below=args.exact_below if wl["theta"] >= 0 else 0,
                  approx_h=args.approx_h)

    tune_loaded = 0
    if args.autotune and args.tune_db and os.path.exists(args.tune_db):
        recs = json.load(open(args.tune_db))["records"]
        ctx.tune_import(np.array(recs, dtype=np.int64).reshape(-1, mm.TUNE_FIELDS))
        tune_loaded = len(recs)

    for i in range(args.warmup):
        t = time.time()
        mm.layout(ctx, dg, p)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i} {time.time() - t:.2f}s", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    xy = None
    for i in range(args.steps):
        xy, st = mm.layout(ctx, dg, p)
        stats.append(st)
        print(f"[bench] step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0

    updates = sum(s["vertex_updates"] for s in stats)
    st = stats[-1]
    L0 = st["per_level"][0]
    n0, e0 = L0["n"], L0["khop_entries"]
    sweep_avg_ms = L0["sweep_ms"] / max(L0["iters"], 1)
    bytes0 = sweep_bytes(n0, wl["k"], e0, False)
    achieved = bytes0 / (sweep_avg_ms * 1e-3) / 1e9
    far_avg_ms = L0["far_ms"] / max(L0["iters"], 1)
    total_sweep_ms = sum(l["sweep_ms"] for l in st["per_level"])
    total_far_ms = sum(l["far_ms"] for l in st["per_level"])
    traffic = measured_traffic(args.workload, L0["tile_bits"], L0["group"], L0["blocks"])
    caps = [l["cap_hit"] for l in st["per_level"]]

    out = {
        "metric": METRIC,
        "value": updates / T,
        "unit": "vertex-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": g.n, "m": g.m, "k": wl["k"],
                   "theta": wl["theta"], "alpha_decay": wl["alpha_decay"], "seed": args.seed,
                   "exact_far_field_below_n": p.exact_below,
                   "far_field": (f"MulMent_{p.approx_h} (Eq. 3)" if p.approx_h > 0
                                 else "Barnes-Hut" if wl["theta"] >= 0 else "exact"),
                   "levels": st["levels"]},
        "time_to_layout_s": T / args.steps,
        "finest_sweep_updates_per_s": n0 / (sweep_avg_ms * 1e-3),
        "finest_iteration_updates_per_s": n0 / (L0["wall_ms"] / max(L0["iters"], 1) * 1e-3),
        "finest_iters": L0["iters"],
        "vertex_updates_per_step": updates // args.steps,
        # iterations: elapsed time of all Jacobi iterations; sweep and
        # far_field are the kernel times inside them, which overlap (the far
        # field runs on a second stream beside the sweep's stress sums)
        "time_split_ms": {"iterations": st["t_iterate_ms"], "sweep": total_sweep_ms,
                          "far_field": total_far_ms, "khop": st["t_khop_ms"],
                          "coarsen": st["t_coarsen_ms"], "other": st["t_other_ms"]},
        "per_level_fields": ["n", "stress_entries", "iters", "final_iters", "cap_hit",
                             "final_rel_change", "iterations_ms", "sweep_ms", "far_ms",
                             "tile_bits", "lanes", "blocks"],
        "per_level": [[l["n"], l["khop_entries"], l["iters"], l["final_iters"], l["cap_hit"],
                       float(f"{l['delta']:.3e}"), round(l["wall_ms"], 1),
                       round(l["sweep_ms"], 1), round(l["far_ms"], 1), l["tile_bits"],
                       l["group"], l["blocks"]] for l in st["per_level"]],
        # stopping rule at alpha_min: relative change < eps_final, or the cap
        "convergence": {"eps_final": p.eps_final, "max_final_iters": p.max_final_iters,
                        "levels_stopped_by_cap": int(sum(caps)), "levels": len(caps),
                        "finest_final_rel_change": L0["delta"],
                        "finest_stopped_by_cap": bool(L0["cap_hit"])},
        "autotune": {"enabled": args.autotune, "tuning_ms_in_timed_step": st["t_tune_ms"],
                     "records_loaded": tune_loaded},
        "roofline": {"bound": "hbm",
                     "kernel": ("k_sweep_sliced" if L0["group"] == SLICED_GROUP and L0["tile_bits"]
                                else "k_sweep_tiled" if L0["tile_bits"] else "k_sweep")
                               + (" + k_combine" if L0["tile_bits"] else "")
                               + " (finest-level sweep step)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "bytes_per_launch": bytes0, "avg_ms": sweep_avg_ms,
                     # achieved/frac count the algorithmic bytes (4 B per stress-set
                     # id); the kernel reads 16-bit tile-major ids, so the bytes HBM
                     # actually moves (traffic, from the counters) are fewer
                     "measured_GBps": (traffic / (sweep_avg_ms * 1e-3) / 1e9
                                       if traffic else None),
                     "measured_frac": (traffic / (sweep_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                       if traffic else None),
                     "limiter": "vector-instruction issue (SQ counters)"},
    }
    if not args.no_objective:
        t1 = time.perf_counter()
        kh = mm.khop_build(ctx, dg, wl["k"])
        o = mm.objective(ctx, kh, xy, p.alpha_min, p.q)
        kh.free()
        out["final_maxent_stress"] = o["M"]
        out["objective_s"] = time.perf_counter() - t1
    if args.full_stress:
        t1 = time.perf_counter()
        fs = mm.full_stress(ctx, dg, xy)
        out["full_stress"] = {"F": fs["F"], "s_opt": fs["s_opt"], "pairs": g.n * (g.n - 1) // 2,
                              "seconds": time.perf_counter() - t1}
    if not args.no_cpu_baseline:
        x = xy.cpu().numpy().astype(np.float64)
        F = mm.repulsion(ctx, xy, p.q, p.theta)["F"].cpu().numpy().astype(np.float64)
        out["cpu_baseline"] = cpu_baseline(g, wl["k"], x, F, p.alpha_min)
    if args.save_tune_db:
        old = []
        if os.path.exists(args.save_tune_db):
            old = json.load(open(args.save_tune_db))["records"]
        recs = {tuple(r[:4]): list(r) for r in old}
        recs.update({tuple(int(v) for v in r[:4]): [int(v) for v in r]
                     for r in ctx.tune_export()})
        rows = ",\n".join("  " + json.dumps(r) for r in sorted(recs.values()))
        with open(args.save_tune_db, "w") as fh:
            fh.write('{"fields": ["coarse", "n", "stress_entries", "k", "tile_bits", "lanes", '
                     '"blocks"],\n'
                     f' "records": [\n{rows}\n]}}\n')
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
