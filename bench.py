#!/usr/bin/env python
"""Benchmark: FMM matvecs/s and GMRES solve seconds at 1,024,000 nodes.

Workload: 2000 star islands r0 (1 + 0.3 cos k t), r0 ~ U[0.01, 0.03] rad,
k ~ U{3..7}, 512 nodes each (seed 5), density sigma ~ N(0, 1) (seed 51).
A step is one application of (I + K) sigma with the FP32 far field and FP32
near field (p = 16), FP64 assembly.  Also reported: the FP64 FMM (p = 30)
matvec rate, GMRES solve seconds to a preconditioned relative residual of
1e-10 with mixed-precision refinement and with FP64 only (data of the
paper's examples), the error of the solved u at 1e5 sphere targets against
the exact solution, per-stage GPU times, the roofline position of the
dominant kernel and the CPU oracle timed on sampled rows.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("FMM matvecs/s & GMRES solve s at 1M nodes, FP32-mixed vs FP64, "
          "1e-10 err")
WORKLOAD = "stars2000x512"
PEAK_FP32_TFLOPS = 157.3
# FP32 vector peak without packed (two-wide) FP32 instructions, which the
# HIP sources are compiled without: 256 CUs x 64 lanes x 2 FLOP x 2.4 GHz
PEAK_FP32_NOPK_TFLOPS = 78.6
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# algorithmic FLOP counts (see the roofline section of the design notes)
FLOP_P2P_PAIR = 11        # Re(p/(z - w)): 2 sub, |d|^2 (3), p.d (3), div, acc
FLOP_CMAC = 8             # one complex multiply-add


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_matvecs(torch, sol, x, prec, steps, warmup):
    """Two timed regions of `steps` matvecs each: the first without any
    event (the rate), the second with HIP events around every stage on the
    library's stream (per-stage averages)."""
    y = torch.empty_like(x)
    for _ in range(warmup):
        sol.matvec(x, "iplusk", prec, out=y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sol.matvec(x, "iplusk", prec, out=y)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sol.stage_times()
    sol.stage_timing(True)
    torch.cuda.synchronize()
    for _ in range(steps):
        sol.matvec(x, "iplusk", prec, out=y)
    torch.cuda.synchronize()
    sol.stage_timing(False)
    st = sol.stage_times()
    return dt, y, {k: v[0] / steps for k, v in st.items() if v[1]}


def stage_work(tree, n_nodes, P, fp64):
    """Algorithmic work of one operator application per stage: FLOPs for
    the arithmetic-bound stages, HBM bytes for the streaming ones."""
    boxes = tree["boxes"]
    sb = 16 if fp64 else 8                 # bytes of one complex strength
    return {
        "strengths": ("hbm", (8 + 16 + 8) * n_nodes + sb * n_nodes),
        "upward": ("alu", FLOP_CMAC * P * n_nodes
                   + FLOP_CMAC * P * (P + 1) // 2 * (boxes - 1)),
        "l2l": ("alu", FLOP_CMAC * P * (P + 1) // 2 * (boxes - 1)),
        "m2l": ("mfma" if not fp64 else "alu",
                (4 * P * P + 14 * P) * tree["v_pairs"]),
        "p2l": ("alu", FLOP_CMAC * P * tree["p2l_evals"]),
        "leaf": ("alu", FLOP_P2P_PAIR * tree["p2p_interactions"]
                 + FLOP_CMAC * P * (n_nodes + tree["m2p_evals"])),
        "gamma": ("hbm", 16 * n_nodes),
    }


def stage_roofline(tree, n_nodes, P, stages_ms, fp64):
    """Achieved rate per timed stage.  A stage the library folds into
    another launch has no time of its own: the FP32 M2L kernel also forms
    the P2L sums and the correction sums, so its work then counts the P2L
    FLOPs as well (the correction's 16 B per node are left out of a FLOP
    figure) and the entry lists what it includes."""
    peak_flops = PEAK_FP64_TFLOPS if fp64 else PEAK_FP32_TFLOPS
    work = stage_work(tree, n_nodes, P, fp64)
    folded = {}
    if "m2l" in stages_ms:
        for name in ("p2l", "gamma"):
            if name not in stages_ms:
                folded[name] = work[name]
    if "p2l" in folded:
        work["m2l"] = (work["m2l"][0], work["m2l"][1] + folded["p2l"][1])
    out = {}
    for name, (bound, work) in work.items():
        ms = stages_ms.get(name)
        if not ms:
            continue
        if bound == "hbm":
            ach = work / (ms * 1e-3) / 1e9
            out[name] = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                         "avg_ms": ms, "bytes_per_launch": work}
        else:
            ach = work / (ms * 1e-3) / 1e12
            out[name] = {"bound": bound, "achieved": ach, "peak": peak_flops,
                         "unit": "TFLOP/s", "frac": ach / peak_flops,
                         "avg_ms": ms, "flop_per_launch": work}
    if folded and "m2l" in out:
        out["m2l"]["includes"] = sorted(folded)
    return out


def measured_traffic(kernel):
    """(HBM bytes, fetched HBM bytes) per launch of `kernel` from the
    committed counter summary; None for what it lacks, and both None when
    it is missing or was taken on other kernel sources than the ones built
    now."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_stars2000x512.txt")
    src = os.path.join(ROOT, "paper_1306_0612_amd", "csrc", "fmm.hip")
    if not os.path.exists(path):
        return None, None
    rec, sha = {}, None
    with open(path) as f:
        for line in f:
            if line.startswith("source_sha256 "):
                sha = line.split()[1]
            if line.startswith("kernel "):
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                rec[kv["name"]] = kv
    with open(src, "rb") as f:
        now = hashlib.sha256(f.read()).hexdigest()
    kv = rec.get(kernel)
    if sha != now or kv is None:
        return None, None
    total = kv.get("bytes_per_launch")
    fetch = kv.get("fetch_bytes_per_launch")
    return (None if total is None else float(total),
            None if fetch is None else float(fetch))


def adjoint_leg(torch, sol, islands, dev, n_targets):
    """Gradient of L = 1/2 |u - u*|^2 at 1e5 sphere targets with respect to
    the node data and the 16 shape coefficients of every island: forward
    solve (mixed, 1e-10) and evaluation, then the transposed evaluation,
    the transposed solve (mixed, 1e-10) and the shape VJP."""
    M = sol.n_islands
    xyz = sol.nodes().cpu().numpy()
    import synth
    g = torch.tensor(synth.exact_harmonic(xyz, islands.center,
                                          synth.paper_data_coeffs(M)),
                     dtype=torch.float64, device=dev)
    tg = synth.sphere_targets(56, n_targets, islands)
    ustar = synth.exact_harmonic(tg, islands.center,
                                 synth.random_data_coeffs(57, islands))
    tgd = torch.tensor(tg, dtype=torch.float64, device=dev)
    usd = torch.tensor(ustar, dtype=torch.float64, device=dev)
    res = {}

    def timed(name, f):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = f()
        torch.cuda.synchronize()
        res[name + "_s"] = time.perf_counter() - t0
        return r

    sig, A, info = timed("forward_solve", lambda: sol.solve(
        g, tol=1e-10, precision="mixed", check=False))
    u = timed("forward_eval", lambda: sol.eval(sig, A, tgd))
    w = (u - usd).contiguous()
    gs, ga = timed("eval_T", lambda: sol.eval_T(w, tgd))
    ls, la, infoT = timed("solve_T", lambda: sol.solve_T(
        gs, ga, tol=1e-10, precision="mixed", check=False))
    dc = timed("shape_vjp", lambda: sol.shape_vjp(sig, A, ls, w, tgd))
    res["backward_s"] = res["eval_T_s"] + res["solve_T_s"] + res["shape_vjp_s"]
    res["solve_T"] = {k: infoT[k] for k in ("status", "iters", "outer_steps",
                                            "rel_resid", "fp32_matvecs")}
    # u is linear in g: w . u = (2 lambda_sigma) . g up to the tolerances
    J = float(w @ u)
    res["duality_rel"] = abs(J - float(2.0 * ls @ g)) / float(
        (w.abs() * u.abs()).sum())
    res["grad_g_norm"] = float((2.0 * ls).norm())
    res["grad_coef_norm"] = float(dc.norm())
    res["n_targets"] = n_targets
    return res


def batch_leg(torch, lbs, dev, n_geoms, n_rhs, steps):
    """64 geometries of 10-400 islands (4k-100k nodes each) with 16
    right-hand sides each in one handle: mixed-precision operator
    applications per second over all systems, and one mixed solve of all
    systems to 1e-10."""
    import synth
    geoms = synth.batch_geometries(n_geoms)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol = lbs.Solver(geoms)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    N, no = sol.n_nodes, sol.node_offsets
    xyz = sol.nodes().cpu().numpy()
    xi = (xyz[:, 0] + 1j * xyz[:, 1]) / (1.0 - xyz[:, 2])
    rng = np.random.default_rng(58)
    G = np.empty((n_rhs, N))
    for q, gm in enumerate(geoms):
        sl = slice(no[q], no[q + 1])
        for r in range(n_rhs):
            k = rng.integers(gm.m)
            c = gm.center[k]
            eta = (c[0] + 1j * c[1]) / (1.0 - c[2])
            a = rng.standard_normal() + 1j * rng.standard_normal()
            G[r, sl] = np.real(a / (xi[sl] - eta))
    Gd = torch.tensor(G, dtype=torch.float64, device=dev)
    X = torch.tensor(rng.standard_normal((n_rhs, N)), dtype=torch.float64,
                     device=dev)
    Y = torch.empty_like(X)
    sol.matvec(X, "iplusk", "mixed", out=Y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sol.matvec(X, "iplusk", "mixed", out=Y)
    torch.cuda.synchronize()
    mv = (time.perf_counter() - t0) / steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, info = sol.solve(Gd, tol=1e-10, precision="mixed", check=False)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    out = {"geometries": n_geoms, "rhs": n_rhs, "nodes": N,
           "islands": sol.n_islands, "setup_s": setup,
           "matvec_ms_all_systems": 1e3 * mv,
           "system_matvecs_per_s": n_geoms * n_rhs / mv,
           "node_rhs_per_s": N * n_rhs / mv,
           "solve_s_mixed": ts,
           "solve": {k: info[k] for k in ("status", "iters", "outer_steps",
                                          "rel_resid")}}
    sol.close()
    return out


def cpu_baseline(islands, sigma, rows_n, y64, y32):
    from threadpoolctl import threadpool_limits
    from oracle import nystrom
    from oracle.geometry import Curves
    cv = Curves(islands)
    rows = np.sort(np.random.default_rng(52).choice(cv.n, rows_n,
                                                    replace=False))
    with threadpool_limits(1):
        t0 = time.perf_counter()
        ref = nystrom.apply_iplusk(cv, sigma, rows)
        dt = time.perf_counter() - t0
    scale = np.abs(ref).max()
    return {
        "value": rows_n / cv.n / dt, "unit": "matvecs/s", "cores": 1,
        "kind": "oracle",
        "sample": "%d sampled rows of the direct O(N^2) sum of (I+K) sigma "
                  "at %d nodes (%.1f s, one thread), scaled to full "
                  "matvecs" % (rows_n, cv.n, dt),
    }, {
        "fmm64_rows_rel_err": float(np.abs(y64[rows] - ref).max() / scale),
        "fmm32_rows_rel_err": float(np.abs(y32[rows] - ref).max() / scale),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="default FMM schedule instead of lbs_autotune's")
    ap.add_argument("--leaf-max", type=int, default=0,
                    help="fixed schedule (skips the tuner): leaf size")
    ap.add_argument("--p32", type=int, default=0)
    ap.add_argument("--p64", type=int, default=0)
    ap.add_argument("--batch-geoms", type=int, default=64)
    ap.add_argument("--batch-rhs", type=int, default=16)
    ap.add_argument("--cpu-rows", type=int, default=512)
    ap.add_argument("--targets", type=int, default=100000)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain elementwise copy kernel that "
                    "reads and writes BYTES each (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs the solver on one GPU; --gpus %d is not "
              "supported (the multi-GPU design is documented, not built)"
              % args.gpus, file=sys.stderr)
        return 2

    import torch
    if args.copy_probe:
        n = args.copy_probe // 8
        a = torch.rand(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 8 * n,
                          "copy_probe_bytes_written": 8 * n,
                          "dispatches": 3}))
        return 0
    import synth
    from paper_1306_0612_amd import lbs
    lbs.load()
    dev = torch.device("cuda:0")

    log("generating islands", args.workload)
    islands = synth.config_islands(args.workload)
    t0 = time.perf_counter()
    tuned = None
    opts = lbs.default_options()
    fixed = {k: v for k, v in (("leaf_max", args.leaf_max), ("p32", args.p32),
                               ("p64", args.p64)) if v}
    if fixed:
        opts = lbs.default_options(**fixed)
    elif not args.no_tune:
        tt = time.perf_counter()
        opts, entries = lbs.autotune(islands, tol_mixed=1e-6, tol_fp64=1e-10)
        tuned = {"leaf_max": opts.leaf_max, "p32": opts.p32, "p64": opts.p64,
                 "tune_s": time.perf_counter() - tt,
                 "settings_timed": len(entries)}
        log("autotune", tuned)
        t0 = time.perf_counter()
    sol = lbs.Solver(islands, options=opts)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    N, M = sol.n_nodes, sol.n_islands
    tree = sol.tree_info()
    log("setup %.2f s, N=%d M=%d tree=%s" % (setup_s, N, M, tree))
    sigma = synth.random_vector(51, N)
    x = torch.tensor(sigma, dtype=torch.float64, device=dev)

    dt32, y32, st32 = timed_matvecs(torch, sol, x, "mixed", args.steps,
                                    args.warmup)
    log("mixed matvec %.3f ms" % (1e3 * dt32 / args.steps), st32)
    k64 = max(1, args.steps // 2)
    dt64, y64, st64 = timed_matvecs(torch, sol, x, "fp64", k64,
                                    max(1, args.warmup // 2))
    log("fp64 matvec %.3f ms" % (1e3 * dt64 / k64), st64)
    y32n, y64n = y32.cpu().numpy(), y64.cpu().numpy()
    mixed_vs_fp64 = float(np.abs(y32n - y64n).max() / np.abs(y64n).max())

    P32, P64 = sol.options.p32, sol.options.p64
    rl32 = stage_roofline(tree, N, P32, st32, False)
    rl64 = stage_roofline(tree, N, P64, st64, True)
    dom = max(st32, key=st32.get)
    kname = {"leaf": "k_leaf32<%d,1>" % P32,
             "m2l": "k_m2l_mfma16" if P32 == 16 else "k_m2l<float,%d>" % P32,
             "p2l": "k_p2l<float,%d>" % P32,
             "upward": "k_m2m3<float,%d>" % P32,
             "l2l": "k_l2l3<float,%d>" % P32}.get(dom, dom)
    r = rl32.get(dom, {})
    roofline = {"bound": r.get("bound", "alu"), "kernel": kname,
                "achieved": r.get("achieved"),
                "peak": r.get("peak", PEAK_FP32_TFLOPS),
                "unit": r.get("unit", "TFLOP/s"), "frac": r.get("frac"),
                "traffic": None, "avg_ms": st32[dom]}
    roofline["traffic"], fetched = measured_traffic(kname)
    if fetched is not None:
        roofline["hbm_fetch_bytes"] = fetched
    if roofline["unit"] == "TFLOP/s" and roofline["achieved"]:
        roofline["peak_no_packed_fp32"] = PEAK_FP32_NOPK_TFLOPS
        roofline["frac_no_packed_fp32"] = (roofline["achieved"]
                                           / PEAK_FP32_NOPK_TFLOPS)

    out = {
        "metric": METRIC,
        "value": args.steps / dt32,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2000 star islands x 512 nodes (1,024,000 "
                               "nodes), (I+K) sigma by FMM, FP32 far and "
                               "near field, FP64 assembly",
                   "islands": M, "nodes": N, "p32": P32, "p64": P64,
                   "leaf_max": sol.options.leaf_max},
        "fp64_matvecs_per_s": k64 / dt64,
        "fp64_ms_per_matvec": 1e3 * dt64 / k64,
        "mixed_vs_fp64_matvec_rel": mixed_vs_fp64,
        "setup_s": setup_s,
        "stages_ms_mixed": st32,
        "stages_ms_fp64": st64,
        "tree": tree,
        "tuned": tuned,
        "roofline": roofline,
        "roofline_stages_mixed": rl32,
        "roofline_stages_fp64": rl64,
    }

    if not args.no_solve:
        xyz = sol.nodes().cpu().numpy()
        coeffs = synth.paper_data_coeffs(M)
        g = torch.tensor(synth.exact_harmonic(xyz, islands.center, coeffs),
                         dtype=torch.float64, device=dev)
        tg = synth.sphere_targets(55, args.targets, islands)
        exact = synth.exact_harmonic(tg, islands.center, coeffs)
        tgd = torch.tensor(tg, dtype=torch.float64, device=dev)
        for prec in ("mixed", "fp64"):
            # the first solve captures the GMRES iterations as HIP graphs;
            # the second, timed one replays them
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sol.solve(g, tol=1e-10, precision=prec, check=False)
            torch.cuda.synchronize()
            out["solve_s_cold_" + prec] = time.perf_counter() - t0
            t0 = time.perf_counter()
            s, a, info = sol.solve(g, tol=1e-10, precision=prec, check=False)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
            t0 = time.perf_counter()
            u = sol.eval(s, a, tgd)
            torch.cuda.synchronize()
            te = time.perf_counter() - t0
            err = np.abs(u.cpu().numpy() - exact).max() / np.abs(exact).max()
            out["solve_s_" + prec] = ts
            out["solve_" + prec] = {k: info[k] for k in (
                "status", "iters", "outer_steps", "rel_resid",
                "fp64_matvecs", "fp32_matvecs")}
            out["u_rel_err_" + prec] = float(err)
            out["eval_s_" + prec] = te
            log(prec, "solve %.3f s" % ts, info, "u err %.2e" % err)

    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(torch, sol, islands, dev, args.targets)
        log("adjoint", out["adjoint"])
    sol.close()
    if not args.no_batch:
        out["batch"] = batch_leg(torch, lbs, dev, args.batch_geoms,
                                 args.batch_rhs, max(3, args.steps // 5))
        log("batch", out["batch"])

    if not args.no_cpu_baseline:
        cb, acc = cpu_baseline(islands, sigma, args.cpu_rows, y64n, y32n)
        out["cpu_baseline"] = cb
        out.update(acc)
        log("cpu baseline", cb, acc)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
