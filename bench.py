#!/usr/bin/env python
"""EXCMG benchmark on one MI355X.

A step is one pass of the whole path on the 512^3-cell workload (8 grids from 4^3, CG tolerance 1e-10, FP64, seeded
smooth field u = sum_k a_k sin sin sin + exp(x+y+z)/10): level data, direct solves on the two coarsest grids,
EXP_finite + tri-quartic initial guesses, the fused stencil-CG relaxation on every grid, the sixth-order EXP_true
extrapolation and the compact gradient.  Inputs f and g are resident in HBM before the timed region.

value = sum over grids of (interior unknowns x CG iterations) / step time, in G unknown-iterations/s.

Also reported: the FP32-in-FP64 iterative-refinement solve of the same workload (time, error vs the FP64 result),
the roofline of the dominant CG sweep (HIP events around every launch in the timed steps), and the CPU oracle timed on
the same inputs on this host (a bounded number of repeats).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "stencil-CG Gunknown-iters/s (%HBM peak); EXCMG solve time 512³ FP64 vs mixed"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per interior unknown of one launch (FP64; halve for FP32)
# a grid's first CG iteration (p = r): pass A reads r only, pass B reads r once for both of its operands
BYTES_PER_UNKNOWN = {"cg_a": 24, "cg_b": 40, "cg_a0": 8, "cg_b0": 32, "cg_a32": 12, "cg_b32": 20}
# algorithmic bytes of the other finest-grid steps: per interior unknown (residual: reads u, f; writes r) or per node
# (EXP_finite: writes w, reads u_2h and u_4h; EXP_true: reads u_h and u_2h, writes u~ and the caller's copy of u_h;
# gradient: per axis reads u and writes one component)
BYTES_PER_NODE = {"exp_finite": 8 * (1 + 1 / 8 + 1 / 64), "exp_true": 8 * (2 + 1 + 1 / 8), "gradient": 48}


def unknown_iters(st):
    tot = 0
    for (nx, ny, nz), it in zip(st["n"], st["iters"]):
        tot += (nx - 1) * (ny - 1) * (nz - 1) * it
    return tot


def trace_summary(db, top=30):
    """Per-kernel summary of a rocprofv3 database (kernel trace and/or counters), grouped by kernel and grid size.
    A CG launch made after its grid converged returns at once; launches shorter than half the longest of their group
    (early exits, or a coarser grid's launches of the same shape) are left out of the 'working' average, and for the
    CG passes those shorter than 0.9 of it (also a grid's first iteration, whose passes move 8 and 32 B per unknown
    instead of 24 and 40)."""
    import re
    import sqlite3

    c = sqlite3.connect(db)

    def clean(nm):
        nm = nm.replace("excmg::(anonymous namespace)::", "").replace("void ", "")
        return re.sub(r"\(.*", "", nm)[:44]

    rows = c.execute("select name, grid_x, workgroup_x, duration from kernels").fetchall()
    if rows:
        groups = {}
        for nm, gx, wx, d in rows:
            groups.setdefault((clean(nm), gx, wx), []).append(d)
        tot = sum(d for _, _, _, d in rows)
        print(f"kernel trace: {len(rows)} dispatches, {tot / 1e6:.3f} ms of kernel time")
        print(f"{'kernel':44s} {'grid':>9s} {'wg':>5s} {'calls':>6s} {'total_ms':>9s} {'avg_us':>9s} "
              f"{'working':>7s} {'work_avg_us':>11s}")
        def line(nm, gx, wx, ds):
            w = [d for d in ds if d >= (0.9 if nm.startswith("cg_pass") else 0.5) * max(ds)]
            print(f"{nm:44s} {gx:9d} {wx:5d} {len(ds):6d} {sum(ds) / 1e6:9.3f} {sum(ds) / len(ds) / 1e3:9.2f} "
                  f"{len(w):7d} {sum(w) / len(w) / 1e3:11.2f}")
            return sum(w) / len(w)

        for (nm, gx, wx), ds in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]:
            line(nm, gx, wx, ds)
        print()
        print("The other kernels of a step (not the CG passes, the autotuner's, the bandwidth probe's or the runtime's; "
              "working average at least 50 us):")
        print(f"{'kernel':44s} {'grid':>9s} {'wg':>5s} {'calls':>6s} {'total_ms':>9s} {'avg_us':>9s} "
              f"{'working':>7s} {'work_avg_us':>11s}")
        skip = ("cg_pass_", "cg_selfred_", "tune_", "delay_", "probe_", "__amd", "finalize_")
        for (nm, gx, wx), ds in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
            if nm.startswith(skip):
                continue
            w = [d for d in ds if d >= 0.5 * max(ds)]
            if sum(w) / len(w) >= 50e3:
                line(nm, gx, wx, ds)
    pm = c.execute("select kernel_name, grid_size, counter_name, value from counters_collection").fetchall()
    if pm:
        groups = {}
        for nm, gx, cn, v in pm:
            groups.setdefault((clean(nm), gx, cn), []).append(v)
        print("counters (per dispatch; 'working' = dispatches with at least half of the group's largest value)")
        print(f"{'kernel':44s} {'grid':>9s} {'counter':>12s} {'calls':>6s} {'working':>7s} {'work_avg':>14s}")
        for (nm, gx, cn), vs in sorted(groups.items(), key=lambda kv: -max(kv[1]))[:top]:
            w = [v for v in vs if v >= 0.5 * max(vs)]
            print(f"{nm:44s} {gx:9d} {cn:>12s} {len(vs):6d} {len(w):7d} {sum(w) / max(len(w), 1):14.1f}")


def solve_trace_summary(db):
    """The CG launches of the solves in a rocprofv3 kernel trace of the benchmark (the dispatches after the
    autotuner's last trial), grouped by kernel and grid size (which tells the grids apart): calls, average duration
    of the launches that did a sweep (at least half the group's longest: launches made after convergence return at
    once), and the average idle time from the end of a launch to the start of the next dispatch."""
    import re
    import sqlite3

    c = sqlite3.connect(db)

    def clean(nm):
        nm = nm.replace("excmg::(anonymous namespace)::", "").replace("void ", "")
        return re.sub(r"\(.*", "", nm)[:44]

    rows = c.execute("select name, grid_x, workgroup_x, start, end from kernels order by start").fetchall()
    names = [clean(r[0]) for r in rows]
    last = max((i for i, nm in enumerate(names) if nm.startswith(("tune_", "delay_"))), default=-1)
    groups = {}
    for i in range(last + 1, len(rows) - 1):
        nm, (_, gx, wx, t0, t1) = names[i], rows[i]
        if not nm.startswith(("cg1_", "cg_selfred_", "cg_pass_", "small_cg", "finalize_")):
            continue
        groups.setdefault((nm, gx, wx), []).append((t1 - t0, rows[i + 1][3] - t1))
    print(f"solve launches after the autotuner: {len(rows) - last - 1} dispatches")
    print(f"{'kernel':44s} {'grid':>9s} {'wg':>5s} {'calls':>6s} {'working':>7s} {'work_avg_us':>11s} {'gap_us':>7s}")
    for (nm, gx, wx), v in sorted(groups.items(), key=lambda kv: kv[0][1]):
        top = max(d for d, _ in v)
        w = [d for d, _ in v if d >= 0.5 * top]
        print(f"{nm:44s} {gx:9d} {wx:5d} {len(v):6d} {len(w):7d} {sum(w) / len(w) / 1e3:11.2f} "
              f"{sum(g for _, g in v) / len(v) / 1e3:7.2f}")


def _timed(torch, fn, reps):
    """Median wall time (ms) of reps calls of fn after one warm-up call."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts)), r


def bench_aniso(ex, synth, torch, args):
    """1024 x 512 x 256 cells (hx : hy : hz = 1 : 2 : 4), 8 grids from 8 x 4 x 2, tol 1e-10: FP64 against the FP32
    refinement, both against the exact field."""
    n = (1024, 512, 256)
    p = synth.smooth(0)
    f_np, g_np, u_np = synth.sample(p, n)
    f, g = torch.from_numpy(f_np).cuda(), torch.from_numpy(g_np).cuda()
    del f_np, g_np
    res = {"cells": list(n), "n_coarse": [8, 4, 2]}
    sol = {}
    for name, prec in (("fp64", ex.FP64), ("fp32_ir", ex.FP32_IR)):
        s = ex.Solver(n, p.box, args.tol, n_coarse=(8, 4, 2), precision=prec)
        s.autotune()
        u = s.empty()
        ms, (_, _, st) = _timed(torch, lambda: s.solve(f, g, u=u), max(2, args.steps // 2))
        uh = u.cpu().numpy()
        sol[name] = uh
        res[name] = {"solve_ms": round(ms, 3), "iters": st["iters"], "ir_outer": st["ir_outer"],
                     "max_error_vs_exact": float(np.max(np.abs(uh - u_np)))}
        del s, u
    res["rel_l2_fp32_ir_vs_fp64"] = float(np.linalg.norm(sol["fp32_ir"] - sol["fp64"]) / np.linalg.norm(sol["fp64"]))
    res["speedup_fp32_ir"] = round(res["fp64"]["solve_ms"] / res["fp32_ir"]["solve_ms"], 3)
    return res


def bench_mixed4(ex, synth, torch, args, f, g, u_exact):
    """FP64 against FP32 refinement where the error is the scheme's discretisation error: the benchmark's 512^3
    workload at tol 1e-13 and 1e-14 (default stopping norm), and 1024x512x256 cells (8 grids from 8x4x2) at 1e-13.
    Per form: the solve time (median of 3 after a warm-up, autotuned), the finest grid's iterations (FP32 refinement:
    inner iterations and outer steps) and the error against the exact field (L2 = RMS over all nodes, and max); per
    case the relative L2 difference of the two solutions.  (The error against the FP64 oracle of the same solves is
    checked node by node in the GPU tests, tests/test_gpu_mixed.py.)"""
    res = {}

    def one_case(name, n, nc, tol, fd, gd, ue):
        out = {"cells": list(n), "tol": tol}
        sol = {}
        for form, prec in (("fp64", ex.FP64), ("fp32_ir", ex.FP32_IR)):
            sv = ex.Solver(n, (1.0, 1.0, 1.0), tol, n_coarse=nc, precision=prec)
            sv.autotune()
            uu = sv.empty()
            ms, (_, _, st) = _timed(torch, lambda: sv.solve(fd, gd, u=uu), 3)
            d = uu - ue
            out[form] = {"solve_ms": round(ms, 2), "finest_iters": st["iters"][-1],
                         "finest_outer": st["ir_outer"][-1], "L2": float(torch.sqrt(torch.mean(d * d))),
                         "max": float(torch.max(torch.abs(d)))}
            sol[form] = uu
            del sv, d
        out["rel_l2_fp32_ir_vs_fp64"] = float(torch.linalg.vector_norm(sol["fp32_ir"] - sol["fp64"]) /
                                              torch.linalg.vector_norm(sol["fp64"]))
        out["speedup_fp32_ir"] = round(out["fp64"]["solve_ms"] / out["fp32_ir"]["solve_ms"], 3)
        res[name] = out

    ue = torch.from_numpy(u_exact).cuda()
    for tol in (1e-13, 1e-14):
        one_case(f"512_tol{tol:g}", (args.n,) * 3, (4, 4, 4), tol, f, g, ue)
    del ue
    n = (1024, 512, 256)
    p = synth.smooth(0)
    f_np, g_np, u_np = synth.sample(p, n)
    fd, gd, ue = (torch.from_numpy(a).cuda() for a in (f_np, g_np, u_np))
    del f_np, g_np, u_np
    one_case("1024x512x256_tol1e-13", n, (8, 4, 2), 1e-13, fd, gd, ue)
    return res


def bench_batch(ex, synth, torch, args):
    """96 problems (master seed 4), cells per axis from {32, 64, 96, 128, 192}, box edges U(0.5, 2), coarsest N/16,
    FP32 refinement, tol 1e-10, one batched call per step (after the batched autotuner; the same problems solved
    one at a time and batched with the default chunks, both before it, for comparison)."""
    cases = synth.batch(4, 96)
    solvers, fs, gs = [], [], []
    for n, p in cases:
        f, g, _ = synth.sample(p, n)
        solvers.append(ex.Solver(n, p.box, args.tol, n_coarse=tuple(v // 16 for v in n), precision=ex.FP32_IR))
        fs.append(torch.from_numpy(f).cuda())
        gs.append(torch.from_numpy(g).cuda())
    us = [s.empty() for s in solvers]
    ws = torch.empty(ex.batch_workspace_bytes(len(solvers)), dtype=torch.uint8, device="cuda")
    # one at a time and batched with the default chunks first, then batched with the batched autotuner's chunks
    seq_ms, _ = _timed(torch, lambda: [s.solve(f, g, u=u) for s, f, g, u in zip(solvers, fs, gs, us)], 1)
    ms_default, _ = _timed(torch, lambda: ex.solve_batched(solvers, fs, gs, us=us, workspace=ws), 2)
    t0 = time.perf_counter()
    zc = ex.autotune_batched(solvers, workspace=ws)
    tune_s = time.perf_counter() - t0
    ms, (_, stats, per) = _timed(torch, lambda: ex.solve_batched(solvers, fs, gs, us=us, workspace=ws), args.steps)
    unknowns = sum((n[0] - 1) * (n[1] - 1) * (n[2] - 1) for n, _ in cases)
    ui = sum(sum((a - 1) * (b - 1) * (c - 1) * it for (a, b, c), it in zip(st["n"], st["iters"])) for st in stats)
    per = np.array(per)
    return {"problems": len(cases), "finest_unknowns": unknowns, "batch_ms": round(ms, 3),
            "problems_per_s": round(len(cases) / (ms * 1e-3), 1),
            "p50_ms": round(float(np.percentile(per, 50)), 3), "p99_ms": round(float(np.percentile(per, 99)), 3),
            "gunknown_iters_per_s": round(ui / (ms * 1e-3) / 1e9, 3),
            "one_at_a_time_ms": round(seq_ms, 3), "speedup_vs_one_at_a_time": round(seq_ms / ms, 2),
            "batch_ms_default_chunks": round(ms_default, 3), "autotune_s": round(tune_s, 2),
            "round_graphs_replayed_captured": list(solvers[0].batch_graph_counts()),
            "autotuned_z_chunks_fp64_fp32_by_grid_from_finest": {str(k): list(v) for k, v in zc.items()},
            "autotuned_tile_heights": batch_heights(solvers),
            "autotuned_batch_shape_fp64_fp32": dict(zip(("tile_height", "depth"),
                                                        [list(solvers[0].get_batch_shape()[:2]),
                                                         list(solvers[0].get_batch_shape()[2:])]))}


def batch_heights(solvers):
    """Tile heights of the batched CG passes after the batched autotuner, per precision: read from the grids that
    relax in it (grids of more than 8000 interior unknowns; FP32 refinement from 2^20 on)."""
    seen = {"fp64": set(), "fp32": set()}
    for s in solvers:
        for l in range(2, s.levels):
            m = [c << l for c in s.n_coarse]
            interior = (m[0] - 1) * (m[1] - 1) * (m[2] - 1)
            if interior <= 8000:
                continue
            if interior >= 1 << 20:
                seen["fp32"].add(s.get_sweep(l, "a32")[3])
            else:
                seen["fp64"].add(s.get_sweep(l, "a")[3])
    return {k: sorted(v) for k, v in seen.items()}


def bench_adjoint(ex, synth, torch, args):
    """256^3 cells, FP64, tol 1e-10: forward solve and the adjoint (backward) solve with the two transposes."""
    n = (256, 256, 256)
    p = synth.smooth(0)
    f_np, g_np, _ = synth.sample(p, n)
    _, _, ut_np = synth.sample(synth.smooth(5), n)
    f, g, ut = (torch.from_numpy(a).cuda() for a in (f_np, g_np, ut_np))
    s = ex.Solver(n, p.box, args.tol)
    s.autotune()
    u = s.empty()
    fwd_ms, _ = _timed(torch, lambda: s.solve(f, g, u=u), args.steps)
    G = u - ut
    bwd_ms, (_, _, _, st) = _timed(torch, lambda: s.adjoint(G), args.steps)
    return {"cells": list(n), "forward_ms": round(fwd_ms, 3), "adjoint_ms": round(bwd_ms, 3),
            "adjoint_iters": st["iters"]}


def bench_r25(ex, synth, torch, args):
    """The low-regularity field u = r^2.5 (r the distance to the box centre; u is in H^(4-e), below every example of the
    paper): errors of u_h, of the extrapolated solution and of the compact gradient against the exact field on 32^3 to
    256^3 cells at tol 1e-13 (so that the algebraic error stays below the discretisation error), FP64, and their
    orders between consecutive grids.  L2 is the root mean square over all nodes (for the gradient, of the three
    components together), max the largest absolute error."""
    p = synth.r25()
    grids = [32, 64, 128, 256]
    keys = ("u_L2", "u_max", "ext_L2", "ext_max", "grad_L2", "grad_max")
    res = {k: [] for k in keys}
    res["finest_iters"] = []
    for N in grids:
        n = (N, N, N)
        f_np, g_np, u_np = synth.sample(p, n)
        f, g, ue = (torch.from_numpy(a).cuda() for a in (f_np, g_np, u_np))
        s = ex.Solver(n, p.box, 1e-13)
        ug, ut, st = s.solve(f, g, want_ext=True)
        gr = s.gradient(ug)
        gex = [torch.from_numpy(a).cuda() for a in synth.exact_gradient(p, n)]
        e, et = ug - ue, ut - ue
        eg = [a - b for a, b in zip(gr, gex)]
        res["u_L2"].append(float(torch.sqrt(torch.mean(e * e))))
        res["u_max"].append(float(torch.max(torch.abs(e))))
        res["ext_L2"].append(float(torch.sqrt(torch.mean(et * et))))
        res["ext_max"].append(float(torch.max(torch.abs(et))))
        res["grad_L2"].append(float(torch.sqrt(sum(torch.mean(d * d) for d in eg))))
        res["grad_max"].append(float(max(torch.max(torch.abs(d)) for d in eg)))
        res["finest_iters"].append(st["iters"][-1])
        del s, ug, ut, gr, gex, e, et, eg, f, g, ue
    for k in keys:
        v = res[k]
        res[k.replace("_L2", "_order_L2").replace("_max", "_order_max")] = [
            round(float(np.log2(v[i] / v[i + 1])), 2) for i in range(len(v) - 1)]
    res["grids"] = grids
    res["tol"] = 1e-13
    return res


# Table 13: EXCMG on the paper's examples at their finest grids (example: cells, eps, total CPU seconds of the paper's
# serial FP64 Fortran code on an Intel Core i7-4790K at 4.0 GHz, finest-grid CG iterations).  Context only.
PAPER_TABLE13 = {1: ((256, 256, 256), 1e-14, 12.9, 8), 2: ((256, 256, 256), 1e-14, 12.6, 9),
                 3: ((256, 256, 256), 1e-11, 11.8, 8), 4: ((512, 256, 128), 1e-9, 10.8, 8),
                 5: ((256, 256, 256), 1e-12, 13.8, 9), 6: ((256, 256, 256), 1e-13, 13.3, 9)}


def bench_paper(ex, synth, torch, args):
    """The paper's six examples at the grids and tolerances of its timing table (Table 13), FP64 on this GPU: the EXCMG
    solve with EXP_true (median of 3 after a warm-up), the finest grid's CG iterations and u_h's L2 error (RMS over
    all nodes), under the default reading of the stopping norm and under the reading that reproduces the printed
    tables (tables_reading_*: (R f, g) below the finest grid; for Example 4, whose finest meshes that reading misses,
    also ex4_reading_*: every grid below the finest at eps/100, tol_coarse), beside the paper's CPU time and
    iteration count (its hardware, context only)."""
    res = {}
    for e, (n, tol, paper_s, paper_it) in PAPER_TABLE13.items():
        p = synth.example(e)
        f_np, g_np, u_np = synth.sample(p, n)
        f, g, uex = (torch.from_numpy(a).cuda() for a in (f_np, g_np, u_np))
        out = {"cells": list(n), "tol": tol, "paper_cpu_s": paper_s, "paper_finest_iters": paper_it}
        # the default reading of the stopping norm, and the one that reproduces the printed tables ((R f, g) below the
        # finest grid, b on it)
        readings = [("", "b", 0.0), ("tables_reading_", "fg_coarse", 0.0)]
        if e == 4:
            readings.append(("ex4_reading_", "b", tol / 100))
        for tag, sn, tc in readings:
            s = ex.Solver(n, p.box, tol, n_coarse=(8, 4, 2) if e == 4 else (4, 4, 4), stop_norm=sn, tol_coarse=tc)
            s.autotune()
            u, ue = s.empty(), s.empty()
            ms, (_, _, st) = _timed(torch, lambda: s.solve(f, g, u=u, want_ext=True), 3)
            d = u - uex
            out[tag + "solve_ms"] = round(ms, 2)
            out[tag + "finest_iters"] = st["iters"][-1]
            out[tag + "u_L2"] = float(torch.sqrt(torch.mean(d * d)))
            del s, u, ue, d
        res[f"ex{e}"] = out
        del f, g, uex
    res["paper_hardware"] = "Intel Core i7-4790K 4.0 GHz, serial FP64 Fortran (the paper's Table 13)"
    return res


def bench_slab(ex, synth, torch, args):
    """One GPU's share of the z-slab decomposition of the benchmark's grid over G GPUs: the finest-grid CG sweeps on an
    N x N x N/G slab (h as in the cube), timed per launch with HIP events.  The halo exchange and the all-reduces of a
    real multi-GPU run are not in these figures."""
    N = args.n
    res = {}
    for G in (2, 4, 8):
        n = (N, N, N // G)
        box = (1.0, 1.0, 1.0 / G)
        p = synth.smooth(0, box)
        f_np, g_np, _ = synth.sample(p, n)
        f, g = torch.from_numpy(f_np).cuda(), torch.from_numpy(g_np).cuda()
        s = ex.Solver(n, box, args.tol, timing=True)
        s.autotune()
        u = s.empty()
        s.solve(f, g, u=u)
        tot = {"cg_a": 0.0, "cg_b": 0.0}
        calls = {"cg_a": 0, "cg_b": 0}
        for _ in range(3):
            _, _, st = s.solve(f, g, u=u)
            for k in tot:
                tot[k] += st["kernel_ms_finest"][k]
                calls[k] += st["kernel_calls_finest"][k]
        unknowns = (n[0] - 1) * (n[1] - 1) * (n[2] - 1)
        out = {"cells": list(n), "finest_iters": st["iters"][-1]}
        for k, b in (("cg_a", 24), ("cg_b", 40)):
            if calls[k]:
                ms = tot[k] / calls[k]
                out[k + "_ms"] = round(ms, 4)
                out[k + "_GBs"] = round(b * unknowns / (ms * 1e-3) / 1e9, 1)
        out["vector_MB"] = round(8 * (n[0] + 1) * (n[1] + 1) * (n[2] + 1) / 1e6, 1)
        res[f"G{G}"] = out
        del s, u, f, g
    return res


def bench_guess(ex, synth, torch, args, f, g, u_ref):
    """The paper's initial guess against the two it compares with (tri-quadratic after the same extrapolation; CMG's
    trilinear interpolation of u_2h), FP64 on the benchmark's workload: finest-grid CG iterations and solve time per
    guess, and ||w_h - u_h|| (the guess against the converged solution) at N and N/2.  The grids N/2, N/4, N/8 of the
    cascade are the finest data sampled at strides 2, 4, 8 and are solved here as problems of their own."""
    N = args.n
    p = synth.smooth(0)
    h3 = (1.0 / N) ** 3
    sub = {}
    for m in (N // 2, N // 4, N // 8):
        st_ = N // m
        s_ = ex.Solver((m, m, m), p.box, args.tol)
        sub[m], _, _ = s_.solve(f[::st_, ::st_, ::st_].contiguous(), g[::st_, ::st_, ::st_].contiguous())
        del s_
    sub[N] = u_ref

    def werr(kind, m):  # the guess on grid m from the solutions on m/2 and m/4, against the solution on m
        st_ = N // m
        gm = g[::st_, ::st_, ::st_].contiguous()
        w = ex.op_initial_guess(kind, sub[m // 2], sub[m // 4] if kind != "linear" else None, gm, (m, m, m))
        e = w - sub[m]
        return (float(torch.sqrt(torch.sum(e * e) * h3 * (N // m) ** 3)), float(torch.max(torch.abs(e))))

    res = {}
    for kind in ("quartic", "quadratic", "linear"):
        s = ex.Solver((N, N, N), p.box, args.tol, guess=kind)
        s.autotune()
        u = s.empty()
        ms, (_, _, st) = _timed(torch, lambda: s.solve(f, g, u=u), 3)
        eN, eH = werr(kind, N), werr(kind, N // 2)
        res[kind] = {"solve_ms": round(ms, 3), "iters": st["iters"], "w_minus_u_L2": [eH[0], eN[0]],
                     "w_minus_u_max": [eH[1], eN[1]], "order_L2": round(float(np.log2(eH[0] / eN[0])), 2)}
        del s, u
    res["grids_of_w_minus_u"] = [N // 2, N]
    return res


def bench_tolerance(ex, synth, torch, args, f, g, u_exact):
    """Accuracy of the extrapolated solution u~_h against the tolerance, on the benchmark's workload: its L2 error at
    N/2 and N (the N/2 problem is the finest data at stride 2), the order between them, the finest grid's CG
    iterations and the solve time at N, for the benchmark's setting, a tolerance of 1e-15 under either stopping norm,
    and the level-dependent tolerance (tol_order 6: every coarser grid 64 times looser)."""
    N = args.n
    p = synth.smooth(0)
    ue_d = torch.from_numpy(u_exact).cuda()
    cfgs = [("bench", args.tol, "b", 0.0), ("b_1e-15", 1e-15, "b", 0.0), ("fg_1e-15", 1e-15, "fg", 0.0),
            ("fg_1e-15_p6", 1e-15, "fg", 6.0)]
    res = {}
    for name, tol, sn, po in cfgs:
        errs = []
        for m in (N // 2, N):
            q = N // m
            fm = f[::q, ::q, ::q].contiguous() if q > 1 else f
            gm = g[::q, ::q, ::q].contiguous() if q > 1 else g
            s = ex.Solver((m, m, m), p.box, tol, stop_norm=sn, tol_order=po, max_iters=5000)
            if m == N:
                s.autotune()
            _, ue, st = s.solve(fm, gm, want_ext=True)
            d = ue - (ue_d[::q, ::q, ::q] if q > 1 else ue_d)
            errs.append(float(torch.sqrt(torch.mean(d * d))))
            if m == N:
                u = s.empty()
                ms, (_, _, st) = _timed(torch, lambda: s.solve(fm, gm, u=u), 2)
                res[name] = {"tol": tol, "stop_norm": sn, "tol_order": po, "solve_ms": round(ms, 2),
                             "iters": st["iters"]}
                del u
            del s, ue, d
        res[name]["ext_L2"] = errs
        res[name]["ext_order"] = round(float(np.log2(errs[0] / errs[1])), 2)
    res["grids"] = [N // 2, N]
    return res


PROBE_BYTES = 2 << 30  # buffer of the streaming probe: its copy kernel reads PROBE_BYTES/2 and writes PROBE_BYTES/2
COUNTERS_FILE = os.path.join(ROOT, "profiles", "excmg_512_fp64_hbm_counters.txt")
KERNEL_SOURCES = ["paper_1507_05063_amd/csrc/kernels_cg.hip", "paper_1507_05063_amd/csrc/excmg_internal.h"]


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_summary(fetch_db, write_db, min_bytes=512 << 20):
    """HBM bytes per dispatch from a FETCH_SIZE run and a WRITE_SIZE run (KiB per dispatch), each scaled so that the
    probe's copy kernel (PROBE_BYTES/2 read, PROBE_BYTES/2 written) reads its known size.  One JSON line per
    (kernel, grid size) that moves at least min_bytes, for the working dispatches (at least 0.9 of the group's
    largest value: this drops launches that return at once, a coarser grid's launches of the same shape, and a grid's
    first CG iteration, whose passes move 8 and 32 B per unknown instead of 24 and 40)."""
    import re
    import sqlite3

    def load(db, counter):
        c = sqlite3.connect(db)
        g = {}
        for nm, gx, cn, v in c.execute("select kernel_name, grid_size, counter_name, value from counters_collection"):
            if cn != counter:
                continue
            nm = re.sub(r"\(.*", "", nm.replace("excmg::(anonymous namespace)::", "").replace("void ", ""))
            g.setdefault((nm, gx), []).append(v)
        return {k: [x for x in v if x >= 0.9 * max(v)] for k, v in g.items() if max(v) > 0}

    fetch, write = load(fetch_db, "FETCH_SIZE"), load(write_db, "WRITE_SIZE")
    probe = [k for k in fetch if k[0] == "probe_copy_kernel"]
    fk = (PROBE_BYTES / 2) / (np.mean(fetch[probe[0]]) * 1024)
    wk = (PROBE_BYTES / 2) / (np.mean(write[probe[0]]) * 1024)
    print(json.dumps({"calibration": "probe_copy_kernel", "known_read_bytes": PROBE_BYTES // 2,
                      "known_write_bytes": PROBE_BYTES // 2, "fetch_KiB": float(np.mean(fetch[probe[0]])),
                      "write_KiB": float(np.mean(write[probe[0]])), "fetch_scale": round(fk, 4),
                      "write_scale": round(wk, 4), "kernel_source_hash": kernel_source_hash()}))
    for k in sorted(set(fetch) & set(write)):
        fb = float(np.mean(fetch[k])) * 1024 * fk
        wb = float(np.mean(write[k])) * 1024 * wk
        if fb + wb < min_bytes:
            continue
        print(json.dumps({"kernel": k[0], "grid": k[1], "n": len(fetch[k]), "read": round(fb), "write": round(wb),
                          "hbm_bytes": round(fb + wb)}))


def measured_traffic(kernel, grid):
    """HBM bytes per launch of (kernel, grid) from the committed counter summary, if it was taken on the current
    kernel sources; else None."""
    try:
        lines = [json.loads(x) for x in open(COUNTERS_FILE) if x.startswith("{")]
    except OSError:
        return None
    cal = [x for x in lines if "calibration" in x]
    if not cal or cal[0]["kernel_source_hash"] != kernel_source_hash():
        return None
    for x in lines:
        if x.get("kernel") == kernel and x.get("grid") == grid:
            return x["hbm_bytes"]
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace-summary", metavar="DB", help="print a summary of a rocprofv3 database and exit")
    ap.add_argument("--solve-trace-summary", metavar="DB",
                    help="print the solves' CG launches of a rocprofv3 kernel trace (durations, gaps) and exit")
    ap.add_argument("--counter-summary", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="print HBM bytes per dispatch from a FETCH_SIZE and a WRITE_SIZE rocprofv3 run and exit")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512, help="cells per axis of the finest grid")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="CPU work of the oracle's timed sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-aniso", action="store_true", help="skip the 1024x512x256 FP64 / FP32-refinement section")
    ap.add_argument("--no-batch", action="store_true", help="skip the 96-problem batched section")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the 256^3 adjoint section")
    ap.add_argument("--no-guess", action="store_true", help="skip the initial-guess ablation (three 512^3 solves)")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the paper's six examples at the grids of its timing table (six solves)")
    ap.add_argument("--no-slab", action="store_true",
                    help="skip one GPU's z-slab share of the grid for 2, 4 and 8 GPUs (three solves)")
    ap.add_argument("--no-tolerance", action="store_true",
                    help="skip the accuracy of u~_h against the tolerance (eight solves at N/2 and N)")
    args = ap.parse_args()
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.solve_trace_summary:
        solve_trace_summary(args.solve_trace_summary)
        return
    if args.counter_summary:
        counter_summary(*args.counter_summary)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU z-slab form of this "
              "solver is a design, not a build", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1507_05063_amd as ex
    import synth

    torch.cuda.set_device(0)
    N = args.n
    n = (N, N, N)
    p = synth.smooth(0)
    f_np, g_np, u_exact = synth.sample(p, n)
    f = torch.from_numpy(f_np).cuda()
    g = torch.from_numpy(g_np).cuda()
    print(f"# workload {N}^3 cells, inputs resident: {f.numel() * 16 / 1e9:.2f} GB", file=sys.stderr, flush=True)

    probe, probe_shapes = ex.bandwidth_probe(PROBE_BYTES, with_shapes=True)
    print("# streaming probe (GB/s): " + ", ".join(f"{k} {v:.0f}" for k, v in probe.items()), file=sys.stderr,
          flush=True)
    s = ex.Solver(n, p.box, args.tol, timing=True)
    t_tune = time.perf_counter()
    zc64, dp64 = s.autotune(with_depth=True)
    tune_s = time.perf_counter() - t_tune
    print(f"# autotuned z chunks (A, B) per grid: {[z[:2] for z in zc64]}, depths {[d[:2] for d in dp64]}",
          file=sys.stderr, flush=True)
    u = s.empty()
    ue = s.empty()
    grads = (s.empty(), s.empty(), s.empty())

    grad_events = []

    def one():
        uu, uext, st = s.solve(f, g, u=u, want_ext=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.gradient(uu, out=grads)
        e1.record(s.stream)
        grad_events.append((e0, e1))
        return st, uext

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    # the headline: the steps without per-launch timing events
    s.set_timing(False)
    plain = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, _ = one()
        plain.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1e3 / args.steps
    ui = unknown_iters(plain[-1])
    value = ui / (ms_step * 1e-3) / 1e9
    print(f"# fp64 step {ms_step:.2f} ms, iters {plain[-1]['iters']}", file=sys.stderr, flush=True)
    # the same number of steps again with HIP events around every finest-grid launch (on the solver's stream): the
    # per-kernel times of the roofline and of the finest-grid table
    s.set_timing(True)
    grad_events.clear()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, _ = one()
        stats.append(st)
    torch.cuda.synchronize()
    ms_step_timed = (time.perf_counter() - t0) * 1e3 / args.steps

    # roofline of the dominant finest-grid CG sweep, from the HIP events of the timed steps
    tot = {k: sum(st["kernel_ms_finest"][k] for st in stats) for k in ("cg_a", "cg_b")}
    calls = {k: sum(st["kernel_calls_finest"][k] for st in stats) for k in ("cg_a", "cg_b")}
    dom = max(tot, key=lambda k: tot[k])
    nI = (N - 1) ** 3
    avg_ms = tot[dom] / max(calls[dom], 1)
    achieved = BYTES_PER_UNKNOWN[dom] * nI / (avg_ms * 1e-3) / 1e9
    # measured HBM bytes of the same kernel and launch shape (z chunk) from the committed counter runs
    zc_dom = zc64[-1][0 if dom == "cg_a" else 1]
    dvar = dp64[-1][0 if dom == "cg_a" else 1]  # prefetch depth + 10 (non-temporal policy) + 100 * tile height
    ty = dvar // 100
    grid_threads = -(-(N - 1) // 64) * -(-(N - 1) // ty) * -(-(N - 1) // zc_dom) * 64 * ty
    kname = (f"cg_pass_{dom[-1]}_kernel<double, {dvar % 10}, {'true' if (dvar // 10) % 10 else 'false'}, "
             f"{dvar // 100}>")
    traffic = measured_traffic(kname, grid_threads)
    # stencil-CG sweeps of the finest grid alone: unknown-iterations per second of pass A + pass B kernel time
    fin_iters = stats[-1]["iters"][-1]
    cg_ms_fin = sum(sum(st["kernel_ms_finest"][k] for k in ("cg_a0", "cg_b0", "cg_a", "cg_b", "finalize"))
                    for st in stats) / args.steps
    guis_fin_sweeps = nI * fin_iters / (cg_ms_fin * 1e-3) / 1e9 if cg_ms_fin > 0 else None

    # every finest-grid step against the HBM peak: HIP-event time per launch (per call for the residual, which is the
    # boundary-term kernel, the sweep and its reduction), algorithmic bytes as above
    nodes = (N + 1) ** 3
    kernels = {}
    for k, b in [("cg_a0", BYTES_PER_UNKNOWN["cg_a0"] * nI), ("cg_b0", BYTES_PER_UNKNOWN["cg_b0"] * nI),
                 ("cg_a", BYTES_PER_UNKNOWN["cg_a"] * nI), ("cg_b", BYTES_PER_UNKNOWN["cg_b"] * nI),
                 ("resid", 24 * nI), ("exp_finite", BYTES_PER_NODE["exp_finite"] * nodes),
                 ("exp_true", BYTES_PER_NODE["exp_true"] * nodes)]:
        c = sum(st["kernel_calls_finest"][k] for st in stats)
        if c:
            ms_k = sum(st["kernel_ms_finest"][k] for st in stats) / c
            kernels[k] = {"ms": round(ms_k, 4), "calls_per_step": c / args.steps, "GB": round(b / 1e9, 3),
                          "GBs": round(b / (ms_k * 1e-3) / 1e9, 1),
                          "frac": round(b / (ms_k * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    ms_g = float(np.mean([a.elapsed_time(b) for a, b in grad_events[-args.steps:]]))
    bg = BYTES_PER_NODE["gradient"] * nodes
    kernels["gradient"] = {"ms": round(ms_g, 4), "calls_per_step": 1, "GB": round(bg / 1e9, 3),
                           "GBs": round(bg / (ms_g * 1e-3) / 1e9, 1),
                           "frac": round(bg / (ms_g * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    u_np = u.cpu().numpy()
    err_fp64 = float(np.max(np.abs(u_np - u_exact)))

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gunknown-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"EXCMG {N}^3 cells FP64, 8 grids from 4^3, tol {args.tol:g}, seeded smooth field "
                               "(seed 0), incl. EXP_true and compact gradient",
                   "cells": list(n), "levels": stats[-1]["levels"], "tol": args.tol},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": round(traffic / (avg_ms * 1e-3) / 1e9, 1) if traffic else None,
                     "traffic_bytes_per_launch": traffic, "traffic_kernel": kname, "traffic_grid": grid_threads,
                     "avg_launch_ms": round(avg_ms, 4), "bytes_per_launch": BYTES_PER_UNKNOWN[dom] * nI,
                     "probe_GBs": {k: round(v, 1) for k, v in probe.items()},
                     "probe_shapes": probe_shapes,
                     "frac_of_probe_mix": round(achieved / max(probe["mix"], probe["mix_nt"]), 4),
                     "traffic_frac_of_probe_mix": (round(traffic / (avg_ms * 1e-3) / 1e9 /
                                                         max(probe["mix"], probe["mix_nt"]), 4) if traffic else None)},
        "finest_grid_kernels": kernels,
        "iters_per_grid": stats[-1]["iters"],
        "autotuned_z_chunks": [list(z[:2]) for z in zc64],
        "autotuned_depths": [[x % 100 for x in d[:2]] for d in dp64],
        "autotuned_tile_heights": [[x // 100 for x in d[:2]] for d in dp64],
        "autotune_s": round(tune_s, 2),
        "ms_per_grid": [round(v, 3) for v in plain[-1]["ms_level"]],
        "solve_ms_fp64": round(float(np.median([st["ms_total"] for st in plain])), 3),  # median over the timed steps
        "ms_per_step_with_kernel_events": round(ms_step_timed, 3),
        "finest_cg_sweeps_gunknown_iters_s": round(guis_fin_sweeps, 2) if guis_fin_sweeps else None,
        "max_error_vs_exact_fp64": err_fp64,
    }

    if not args.no_mixed:
        sm = ex.Solver(n, p.box, args.tol, precision=ex.FP32_IR, timing=False)
        zc32 = sm.autotune()
        um = sm.empty()
        for _ in range(max(1, args.warmup)):
            sm.solve(f, g, u=um)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, _, stm = sm.solve(f, g, u=um)
        torch.cuda.synchronize()
        ms_m = (time.perf_counter() - t0) * 1e3 / args.steps
        um_np = um.cpu().numpy()
        out["mixed"] = {
            "solve_ms": round(ms_m, 3),
            "inner_iters_per_grid": stm["iters"],
            "ms_per_grid": [round(v, 3) for v in stm["ms_level"]],
            "outer_steps_per_grid": stm["ir_outer"],
            "max_error_vs_exact": float(np.max(np.abs(um_np - u_exact))),
            "rel_l2_vs_fp64_solution": float(np.linalg.norm(um_np - u_np) / np.linalg.norm(u_np)),
            "speedup_vs_fp64_solve": round(float(np.median([st["ms_total"] for st in plain])) / ms_m, 3),
        }
        del sm
        print(f"# mixed solve {ms_m:.2f} ms", file=sys.stderr, flush=True)

    if not args.no_mixed:
        out["mixed_4th_order"] = bench_mixed4(ex, synth, torch, args, f, g, u_exact)
        print(f"# mixed at fourth-order accuracy: {out['mixed_4th_order']}", file=sys.stderr, flush=True)
    if not args.no_aniso:
        out["aniso"] = bench_aniso(ex, synth, torch, args)
        print(f"# aniso: {out['aniso']}", file=sys.stderr, flush=True)
    if not args.no_batch:
        out["batch"] = bench_batch(ex, synth, torch, args)
        print(f"# batch: {out['batch']}", file=sys.stderr, flush=True)
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(ex, synth, torch, args)
        print(f"# adjoint: {out['adjoint']}", file=sys.stderr, flush=True)
        out["r25"] = bench_r25(ex, synth, torch, args)
        print(f"# r25: {out['r25']}", file=sys.stderr, flush=True)
    if not args.no_guess:
        out["guess_ablation"] = bench_guess(ex, synth, torch, args, f, g, u)
        print(f"# guess ablation: {out['guess_ablation']}", file=sys.stderr, flush=True)
    if not args.no_paper:
        out["paper_examples"] = bench_paper(ex, synth, torch, args)
        print(f"# paper examples: {out['paper_examples']}", file=sys.stderr, flush=True)
    if not args.no_slab:
        out["slab"] = bench_slab(ex, synth, torch, args)
        print(f"# slab: {out['slab']}", file=sys.stderr, flush=True)
    if not args.no_tolerance:
        out["tolerance"] = bench_tolerance(ex, synth, torch, args, f, g, u_exact)
        print(f"# tolerance: {out['tolerance']}", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        # the oracle timed on the same step (solve with EXP_true, then the gradient) of the same inputs, repeated
        # until about --cpu-seconds of CPU work have run (at least two runs; the median run is reported)
        import oracle

        threads = max(1, min(len(os.sched_getaffinity(0)), 64))
        oracle.set_threads(threads)
        runs = []
        while len(runs) < 2 or sum(runs) < args.cpu_seconds:
            t0 = time.perf_counter()
            r = oracle.excmg(f_np, g_np, p.box, stats[-1]["n"][0], args.tol, want_ext=True)
            oracle.gradient(r["u"], p.box)
            runs.append(time.perf_counter() - t0)
            print(f"# oracle step {len(runs)}: {runs[-1]:.2f} s on {oracle.get_threads()} threads", file=sys.stderr,
                  flush=True)
        secs = float(np.median(runs))
        ui_c = sum((nx - 1) * (ny - 1) * (nz - 1) * int(it) for (nx, ny, nz), it in zip(stats[-1]["n"], r["iters"]))
        out["cpu_baseline"] = {"value": round(ui_c / secs / 1e9, 4), "unit": "Gunknown-iters/s",
                               "cores": oracle.get_threads(), "kind": "oracle",
                               "sample": f"the whole step ({N}^3 cells, solve with EXP_true + gradient) on the same "
                                         f"inputs, {len(runs)} runs, median {secs:.2f} s; oracle iterations "
                                         f"{[int(v) for v in r['iters']]}"}
        # and on one thread, the same step at half the cells per axis (one run)
        n1 = (N // 2,) * 3
        f1, g1, _ = synth.sample(p, n1)
        oracle.set_threads(1)
        t0 = time.perf_counter()
        r1 = oracle.excmg(f1, g1, p.box, stats[-1]["n"][0], args.tol, want_ext=True)
        oracle.gradient(r1["u"], p.box)
        secs1 = time.perf_counter() - t0
        oracle.set_threads(threads)
        L1 = len(r1["iters"])
        cells1 = [tuple(v // 2 ** (L1 - 1 - q) for v in n1) for q in range(L1)]
        ui_1 = sum((a - 1) * (b - 1) * (c - 1) * int(it) for (a, b, c), it in zip(cells1, r1["iters"]))
        out["cpu_baseline"]["one_thread"] = {
            "value": round(ui_1 / secs1 / 1e9, 4), "unit": "Gunknown-iters/s", "cores": 1,
            "sample": f"the whole step at {N // 2}^3 cells (solve with EXP_true + gradient), one run, {secs1:.2f} s; "
                      f"oracle iterations {[int(v) for v in r1['iters']]}"}
        print(f"# oracle on one thread at {N // 2}^3: {secs1:.2f} s", file=sys.stderr, flush=True)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
