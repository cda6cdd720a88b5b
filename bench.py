#!/usr/bin/env python
"""Benchmark: FMM matvecs/s and GMRES solve seconds at 1,024,000 nodes.

Workload: 2000 star islands r0 (1 + 0.3 cos k t), r0 ~ U[0.01, 0.03] rad,
k ~ U{3..7}, 512 nodes each (seed 5), density sigma ~ N(0, 1) (seed 51).
A step is one application of (I + K) sigma with the FP32 far field and FP32
near field (p = 16), FP64 assembly.  Also reported: the FP64 FMM (p = 30)
matvec rate; GMRES solve seconds with mixed-precision refinement and with
FP64 only at the tolerance (1e-12) that puts the solved u within 1e-10 of
the exact solution at 1e5 sphere targets (data of the paper's examples),
with that error, and the same at the residual tolerance 1e-10; the
preconditioned and unpreconditioned solves of 15 islands as the node count
grows (the paper's Table 1 experiment); per-stage GPU times and roofline
positions; the adjoint leg; the batch of 64 geometries x 16 right-hand
sides; and the CPU oracle timed on sampled rows on the host's cores.

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
# Algorithmic FLOP per near-field source-target pair.  The reference count
# is 17 (complex difference 2, complex division written out: |d|^2 3,
# numerator 6, two quotients 2, Re of the strength product 2, accumulate
# 2); the minimal count of Re(p conj(d)) / |d|^2 is 11 (2 sub, |d|^2 3,
# Re(p conj d) 3, division 1, accumulate 1, with the quotient's imaginary
# part never formed).  `frac` uses 17, `frac_11flop` the minimal count.
FLOP_P2P_PAIR = 17
FLOP_P2P_PAIR_MIN = 11
FLOP_CMAC = 8             # one complex multiply-add
MAX_HOST_WORKERS = 16     # the host share of one GPU


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------- CPU oracle
_POOL_STATE = {}


def _oracle_rows(rows):
    from threadpoolctl import threadpool_limits
    from oracle import nystrom
    with threadpool_limits(1):
        return nystrom.apply_iplusk(_POOL_STATE["cv"], _POOL_STATE["sigma"],
                                    rows)


def _oracle_pool_rows(cv, sigma, rows, workers):
    """(I + K) sigma at `rows` by the oracle's direct sum, the rows split
    over `workers` forked processes (one BLAS thread each)."""
    import multiprocessing as mp
    _POOL_STATE["cv"], _POOL_STATE["sigma"] = cv, sigma
    chunks = np.array_split(rows, max(1, 4 * workers))
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        parts = pool.map(_oracle_rows, chunks)
    return np.concatenate(parts)


def host_workers():
    return max(1, min(MAX_HOST_WORKERS, os.cpu_count() or 1))


def cpu_baseline(islands, sigma, rows_n):
    """The oracle's direct O(N^2) (I + K) sigma on rows_n sampled rows on the
    host's cores (before the GPU is touched), scaled to full matvecs."""
    from threadpoolctl import threadpool_info
    from oracle.geometry import Curves
    cv = Curves(islands)
    rows = np.sort(np.random.default_rng(52).choice(cv.n, rows_n,
                                                    replace=False))
    workers = host_workers()
    t0 = time.perf_counter()
    ref = _oracle_pool_rows(cv, sigma, rows, workers)
    dt = time.perf_counter() - t0
    blas = sorted({(d.get("internal_api"), d.get("num_threads"))
                   for d in threadpool_info()})
    return {
        "value": rows_n / cv.n / dt, "unit": "matvecs/s", "cores": workers,
        "kind": "oracle",
        "sample": "%d sampled rows of the direct O(N^2) sum of (I+K) sigma "
                  "at %d nodes (%.1f s on %d processes of one BLAS thread "
                  "each; os.cpu_count() = %s), scaled to full matvecs"
                  % (rows_n, cv.n, dt, workers, os.cpu_count()),
        "os_cpu_count": os.cpu_count(),
        "blas_threads_per_process": 1,
        "blas_libraries": [list(b) for b in blas],
    }, rows, ref


def cpu_configs(workers):
    """The oracle on the smaller workloads: dense assembly + LU of the cap
    (256 nodes) and of 40 islands x 512 nodes (20,480 nodes), and the
    direct matvec of 1000 islands x 256 nodes on sampled rows (its GMRES
    time is that matvec times the iteration count, both reported)."""
    import synth
    from threadpoolctl import threadpool_limits
    from oracle import nystrom
    from oracle.geometry import Curves
    out = {"workers": workers}
    for name in ("cap256", "stars40x512"):
        isl = synth.config_islands(name)
        cv = Curves(isl)
        g = synth.exact_harmonic(cv.x, isl.center,
                                 synth.paper_data_coeffs(cv.m))
        with threadpool_limits(workers):
            t0 = time.perf_counter()
            A = nystrom.system_matrix(cv)
            t1 = time.perf_counter()
            import scipy.linalg as sla
            lu = sla.lu_factor(A, check_finite=False)
            rhs = np.concatenate([2.0 * g, np.zeros(cv.m)])
            sla.lu_solve(lu, rhs, check_finite=False)
            t2 = time.perf_counter()
        out[name] = {"nodes": cv.n, "assembly_s": t1 - t0, "lu_solve_s": t2 - t1,
                     "blas_threads": workers}
        del A, lu
    isl = synth.config_islands("stars1000x256")
    cv = Curves(isl)
    sigma = synth.random_vector(8, cv.n)
    rows = np.sort(np.random.default_rng(9).choice(cv.n, 4096, replace=False))
    t0 = time.perf_counter()
    _oracle_pool_rows(cv, sigma, rows, workers)
    dt = time.perf_counter() - t0
    out["stars1000x256"] = {"nodes": cv.n,
                            "matvec_s_extrapolated": dt * cv.n / rows.size,
                            "rows_timed": int(rows.size)}
    return out


# -------------------------------------------------------------- GPU legs
def timed_matvecs(torch, sol, x, prec, steps, warmup, reps):
    """The rate over `steps` back-to-back matvecs (no events), the median
    of `reps` single matvecs bracketed by HIP events on the library's
    stream, and per-stage averages from the library's stage timer."""
    y = torch.empty_like(x)
    for _ in range(warmup):
        sol.matvec(x, "iplusk", prec, out=y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sol.matvec(x, "iplusk", prec, out=y)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ev = [(torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        sol.matvec(x, "iplusk", prec, out=y)
        b.record()
    torch.cuda.synchronize()
    med = float(np.median([a.elapsed_time(b) for a, b in ev]))
    sol.stage_times()
    sol.stage_timing(True)
    torch.cuda.synchronize()
    for _ in range(steps):
        sol.matvec(x, "iplusk", prec, out=y)
    torch.cuda.synchronize()
    sol.stage_timing(False)
    st = sol.stage_times()
    return dt, med, y, {k: v[0] / steps for k, v in st.items() if v[1]}


def stage_work(tree, n_nodes, P, fp64, pair_flop=FLOP_P2P_PAIR, nrhs=1):
    """Algorithmic work of one operator application per stage: FLOPs for
    the arithmetic-bound stages, HBM bytes for the streaming ones."""
    boxes = tree["boxes"]
    sb = 16 if fp64 else 8                 # bytes of one complex strength
    w = {
        "strengths": ("hbm", (8 + 16 + 8) * n_nodes + sb * n_nodes),
        "upward": ("alu", FLOP_CMAC * P * n_nodes
                   + FLOP_CMAC * P * (P + 1) // 2 * (boxes - 1)),
        "l2l": ("alu", FLOP_CMAC * P * (P + 1) // 2 * (boxes - 1)),
        "m2l": ("mfma" if not fp64 else "alu",
                (4 * P * P + 14 * P) * tree["v_pairs"]),
        "p2l": ("alu", FLOP_CMAC * P * tree["p2l_evals"]),
        "leaf": ("alu", pair_flop * tree["p2p_interactions"]
                 + FLOP_CMAC * P * (n_nodes + tree["m2p_evals"])),
        "gamma": ("hbm", 16 * n_nodes),
    }
    return {k: (b, v * nrhs) for k, (b, v) in w.items()}


def stage_roofline(tree, n_nodes, P, stages_ms, fp64, nrhs=1, fetched=None):
    """Achieved rate per timed stage.  A stage the library folds into
    another launch has no time of its own: the FP32 M2L kernel also forms
    the P2L sums and the correction sums, so its work then counts the P2L
    FLOPs as well (the correction's 16 B per node are left out of a FLOP
    figure) and the entry lists what it includes.  `fetched` maps a stage
    to the HBM bytes its kernels fetch per application (counter profile)."""
    peak_flops = PEAK_FP64_TFLOPS if fp64 else PEAK_FP32_TFLOPS
    work = stage_work(tree, n_nodes, P, fp64, nrhs=nrhs)
    wmin = stage_work(tree, n_nodes, P, fp64, FLOP_P2P_PAIR_MIN, nrhs)
    folded = {}
    if "m2l" in stages_ms:
        for name in ("p2l", "gamma"):
            if name not in stages_ms:
                folded[name] = work[name]
    if "p2l" in folded:
        work["m2l"] = (work["m2l"][0], work["m2l"][1] + folded["p2l"][1])
    out = {}
    for name, (bound, wk) in work.items():
        ms = stages_ms.get(name)
        if not ms:
            continue
        if bound == "hbm":
            ach = wk / (ms * 1e-3) / 1e9
            out[name] = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                         "avg_ms": ms, "bytes_per_launch": wk}
        else:
            ach = wk / (ms * 1e-3) / 1e12
            out[name] = {"bound": bound, "achieved": ach, "peak": peak_flops,
                         "unit": "TFLOP/s", "frac": ach / peak_flops,
                         "avg_ms": ms, "flop_per_launch": wk}
            if name == "leaf":
                a11 = wmin[name][1] / (ms * 1e-3) / 1e12
                out[name]["frac_11flop"] = a11 / peak_flops
        if fetched and fetched.get(name):
            out[name]["hbm_fetch_GBs"] = fetched[name] / (ms * 1e-3) / 1e9
    if folded and "m2l" in out:
        out["m2l"]["includes"] = sorted(folded)
    return out


def traffic_profile():
    """Per-kernel counter records of the committed HBM traffic summary and
    whether they were taken on the kernel sources built now."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_stars2000x512.txt")
    if not os.path.exists(path):
        return {}, False
    rec, sha = {}, {}
    with open(path) as f:
        for line in f:
            if line.startswith("source_sha256 "):
                p = line.split()
                if len(p) == 3:        # source_sha256 <path> <sha256>
                    sha[p[1]] = p[2]
                else:
                    sha["paper_1306_0612_amd/csrc/fmm.hip"] = p[1]
            if line.startswith("kernel "):
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                rec[kv["name"]] = kv
    fresh = bool(sha)
    for rel, h in sha.items():
        src = os.path.join(ROOT, rel)
        if not os.path.exists(src):
            fresh = False
            continue
        with open(src, "rb") as f:
            fresh &= hashlib.sha256(f.read()).hexdigest() == h
    return rec, fresh


STAGE_KERNELS32 = {  # stage -> kernels of one mixed application
    "upward": ["k_p2m_pair<16>", "k_pass<float,16,false>"],
    "m2l": ["k_m2l_mfma16"],
    "l2l": ["k_pass<float,16,true>"],
    "leaf": ["k_leaf32<16,1>"],
}


def stage_fetch(rec, fresh):
    """HBM bytes each stage's kernels fetch per application: a kernel's
    mean per launch times its launches per application (the summary's
    `per_app`, its dispatches over those of the leaf kernel, which runs
    once per application)."""
    if not fresh:
        return None
    out = {}
    for st, ks in STAGE_KERNELS32.items():
        tot = 0.0
        for k in ks:
            kv = rec.get(k)
            if kv is None or "fetch_bytes_per_launch" not in kv:
                tot = None
                break
            tot += float(kv.get("per_app", 1)) * float(kv["fetch_bytes_per_launch"])
        if tot:
            out[st] = tot
    return out


def solve_leg(torch, sol, islands, dev, n_targets, out):
    import synth
    xyz = sol.nodes().cpu().numpy()
    coeffs = synth.paper_data_coeffs(sol.n_islands)
    g = torch.tensor(synth.exact_harmonic(xyz, islands.center, coeffs),
                     dtype=torch.float64, device=dev)
    tg = synth.sphere_targets(55, n_targets, islands)
    exact = synth.exact_harmonic(tg, islands.center, coeffs)
    tgd = torch.tensor(tg, dtype=torch.float64, device=dev)
    keys = ("status", "iters", "outer_steps", "rel_resid", "true_rel_resid",
            "fp64_matvecs", "fp32_matvecs")
    # tol 1e-12: the headline (u within 1e-10 of the exact solution);
    # tol 1e-10: the same solves stopped at a 1e-10 residual, for reference
    for tol, suffix in ((1e-12, ""), (1e-10, "_tol1e-10")):
        for prec in ("mixed", "fp64"):
            # the first solve captures the GMRES iterations as HIP graphs;
            # the second, timed one replays them
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sol.solve(g, tol=tol, precision=prec, check=False)
            torch.cuda.synchronize()
            cold = time.perf_counter() - t0
            t0 = time.perf_counter()
            s, a, info = sol.solve(g, tol=tol, precision=prec, check=False)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
            t0 = time.perf_counter()
            u = sol.eval(s, a, tgd)
            torch.cuda.synchronize()
            te = time.perf_counter() - t0
            err = float(np.abs(u.cpu().numpy() - exact).max()
                        / np.abs(exact).max())
            out["solve_s_" + prec + suffix] = ts
            out["solve_s_cold_" + prec + suffix] = cold
            out["solve_" + prec + suffix] = {k: info[k] for k in keys}
            out["u_rel_err_" + prec + suffix] = err
            out["eval_s_" + prec + suffix] = te
            log(prec, "tol %g solve %.4f s" % (tol, ts), info,
                "u err %.2e" % err)
    out["solve_tol"] = 1e-12
    out["u_err_targets"] = n_targets


def table1_leg(torch, lbs, dev):
    """The paper's Table 1 experiment on 15 star islands: GMRES iterations,
    solve time and the error at sphere targets with and without the block
    preconditioner as the nodes per curve grow (FP64, tol 1e-11, restart
    50)."""
    import synth
    base = synth.star_islands(15, 15, (0.1, 0.3), nodes=512)
    coeffs = synth.paper_data_coeffs(15)
    # targets clear of every curve by ten node spacings of the finest grid
    tg = synth.sphere_targets(16, 75, base)
    exact = synth.exact_harmonic(tg, base.center, coeffs)
    tgd = torch.tensor(tg, dtype=torch.float64, device=dev)
    rows = []
    for n in (32, 64, 128, 256, 512):
        isl = base.with_nodes(n)
        for pre in (0, 1):
            sol = lbs.Solver(isl, leaf_max=32, precond=pre, max_iter=4000)
            xyz = sol.nodes().cpu().numpy()
            g = torch.tensor(synth.exact_harmonic(xyz, isl.center, coeffs),
                             dtype=torch.float64, device=dev)
            sol.solve(g, tol=1e-11, precision="fp64", check=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s, a, info = sol.solve(g, tol=1e-11, precision="fp64",
                                   check=False)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
            u = sol.eval(s, a, tgd).cpu().numpy()
            rows.append({"N": n, "precond": pre, "iters": info["iters"],
                         "status": info["status"], "solve_ms": 1e3 * ts,
                         "true_rel_resid": info["true_rel_resid"],
                         "u_rel_err": float(np.abs(u - exact).max()
                                            / np.abs(exact).max())})
            log("table1", rows[-1])
            sol.close()
    return rows


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
    applications per second over all systems, the leaf kernel's roofline
    position, and one mixed solve of all systems to 1e-10."""
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
    dt, med, _, st = timed_matvecs(torch, sol, X, "mixed", steps, 1, steps)
    mv = dt / steps
    tree = sol.tree_info()
    rl = stage_roofline(tree, N, sol.options.p32, st, False, nrhs=n_rhs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, info = sol.solve(Gd, tol=1e-10, precision="mixed", check=False)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    out = {"geometries": n_geoms, "rhs": n_rhs, "nodes": N,
           "islands": sol.n_islands, "setup_s": setup,
           "matvec_ms_all_systems": 1e3 * mv,
           "matvec_ms_all_systems_median": med,
           "system_matvecs_per_s": n_geoms * n_rhs / mv,
           "node_rhs_per_s": N * n_rhs / mv,
           "stages_ms": st, "roofline_stages": rl,
           "solve_s_mixed": ts,
           "solve": {k: info[k] for k in ("status", "iters", "outer_steps",
                                          "rel_resid", "true_rel_resid")}}
    sol.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--reps", type=int, default=100,
                    help="single matvecs timed by events (median)")
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="also time the oracle on the smaller workloads")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-table1", action="store_true")
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
    ap.add_argument("--cpu-rows", type=int, default=4096)
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
    log("generating islands", args.workload)
    islands = synth.config_islands(args.workload)
    sigma = synth.random_vector(51, islands.n_total)
    extra = {}
    cb = None
    if not args.no_cpu_baseline:
        # the oracle runs in forked processes before the GPU is touched
        cb, cb_rows, cb_ref = cpu_baseline(islands, sigma, args.cpu_rows)
        log("cpu baseline", cb)
        if args.cpu_configs:
            extra["cpu_configs"] = cpu_configs(host_workers())
            log("cpu configs", extra["cpu_configs"])

    from paper_1306_0612_amd import lbs
    lbs.load()
    dev = torch.device("cuda:0")
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
    log("setup")
    sol = lbs.Solver(islands, options=opts)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    N, M = sol.n_nodes, sol.n_islands
    tree = sol.tree_info()
    log("setup %.2f s, N=%d M=%d tree=%s" % (setup_s, N, M, tree))
    x = torch.tensor(sigma, dtype=torch.float64, device=dev)

    dt32, med32, y32, st32 = timed_matvecs(torch, sol, x, "mixed", args.steps,
                                           args.warmup, args.reps)
    log("mixed matvec %.3f ms (median %.3f)" % (1e3 * dt32 / args.steps,
                                                med32), st32)
    k64 = max(1, args.steps // 2)
    dt64, med64, y64, st64 = timed_matvecs(torch, sol, x, "fp64", k64,
                                           max(1, args.warmup // 2),
                                           max(1, args.reps // 2))
    log("fp64 matvec %.3f ms (median %.3f)" % (1e3 * dt64 / k64, med64), st64)
    y32n, y64n = y32.cpu().numpy(), y64.cpu().numpy()
    mixed_vs_fp64 = float(np.abs(y32n - y64n).max() / np.abs(y64n).max())

    P32, P64 = sol.options.p32, sol.options.p64
    rec, fresh = traffic_profile()
    rl32 = stage_roofline(tree, N, P32, st32, False,
                          fetched=stage_fetch(rec, fresh))
    rl64 = stage_roofline(tree, N, P64, st64, True)
    dom = max(st32, key=st32.get)
    kname = {"leaf": "k_leaf32<%d,1>" % P32,
             "m2l": "k_m2l_mfma16" if P32 == 16 else "k_m2l<float,%d>" % P32,
             "p2l": "k_p2l<float,%d>" % P32,
             "upward": "k_pass<float,%d,false>" % P32,
             "l2l": "k_pass<float,%d,true>" % P32}.get(dom, dom)
    r = rl32.get(dom, {})
    roofline = {"bound": r.get("bound", "alu"), "kernel": kname,
                "achieved": r.get("achieved"),
                "peak": r.get("peak", PEAK_FP32_TFLOPS),
                "unit": r.get("unit", "TFLOP/s"), "frac": r.get("frac"),
                "traffic": None, "avg_ms": st32[dom],
                "flop_per_pair": FLOP_P2P_PAIR}
    if "frac_11flop" in r:
        roofline["frac_11flop"] = r["frac_11flop"]
    kv = rec.get(kname) if fresh else None
    if kv is not None:
        if "bytes_per_launch" in kv:
            roofline["traffic"] = float(kv["bytes_per_launch"])
        if "fetch_bytes_per_launch" in kv:
            roofline["hbm_fetch_bytes"] = float(kv["fetch_bytes_per_launch"])
        if "write_bytes_per_launch" in kv:
            roofline["hbm_write_bytes"] = float(kv["write_bytes_per_launch"])
    elif rec:
        roofline["traffic_note"] = ("counter summary taken on other kernel "
                                    "sources than the ones built now")
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
        "ms_per_matvec_median_mixed": med32,
        "ms_per_matvec_median_fp64": med64,
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
    out.update(extra)
    if cb is not None:
        out["cpu_baseline"] = cb
        scale = np.abs(cb_ref).max()
        out["fmm64_rows_rel_err"] = float(np.abs(y64n[cb_rows] - cb_ref).max()
                                          / scale)
        out["fmm32_rows_rel_err"] = float(np.abs(y32n[cb_rows] - cb_ref).max()
                                          / scale)

    if not args.no_solve:
        solve_leg(torch, sol, islands, dev, args.targets, out)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(torch, sol, islands, dev, args.targets)
        log("adjoint", out["adjoint"])
    sol.close()
    if not args.no_table1:
        out["table1"] = table1_leg(torch, lbs, dev)
        log("table1", out["table1"])
    if not args.no_batch:
        out["batch"] = batch_leg(torch, lbs, dev, args.batch_geoms,
                                 args.batch_rhs, max(3, args.steps // 5))
        log("batch", out["batch"])
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
