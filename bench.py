"""Benchmark: factor + solve throughput of the recursive-skeletonisation
direct solver on one MI355X.

One step = build the compressed inverse of the Nystrom matrix for the
workload's grid (inputs already in HBM) + solve all its right-hand sides +
release the factor.  value = unknowns per second = N * steps / time.

    python bench.py [--steps K] [--warmup W] [--workload laplace256]
                    [--precision fp64|fp32] [--no-cpu-baseline]

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6e12, "f32": 157.3e12}   # dense MFMA, MI355X
HBM_PEAK = 8.0e12
PROF_EVERY = 5   # one timed step in PROF_EVERY carries the roofline kernel's events


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(pts, a, f, budget_s=30.0, max_cols=None):
    """The CPU reference as it stands: GMRES on the exact FFT product, column by
    column, with BLAS limited to one thread.  Returns the record and the
    reference solutions of the columns it solved (column index -> vector)."""
    from oracle import krylov
    try:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        ctx = None
    done = 0
    sols = {}
    t0 = time.perf_counter()
    for c in range(f.shape[1] if max_cols is None else min(max_cols, f.shape[1])):
        sols[c], _ = krylov.solve(pts, f[:, c], a, tol=1e-13)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    if ctx is not None:
        ctx.unregister() if hasattr(ctx, "unregister") else None
    n = pts.shape[0]
    # unknowns/s for a full step (all right-hand sides), from the sampled columns
    per_step = dt / done * f.shape[1]
    return {"value": n / per_step, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"GMRES(50) to 1e-13 with the exact FFT product on the full {n}-point "
                      f"system, {done} of {f.shape[1]} right-hand sides timed ({dt:.1f} s), "
                      f"scaled to all {f.shape[1]}; a dense solver, not the paper's method"}, sols


def err_vs_oracle(x, sols):
    """Relative error of each GPU result column against the oracle's solution
    of the same right-hand side (the columns the CPU leg solved)."""
    return {str(c): float(np.linalg.norm(x[:, c] - r) / np.linalg.norm(r)) for c, r in sols.items()}


def batched_measure(torch, rsd, W, reps=2):
    """64 grids of uneven size (side 32..256), float32 factors + float64
    refinement to 1e-8, one right-hand side each: build all (batched call) +
    solve all (batched call); inputs resident in HBM.  Returns a dict for the
    JSON line."""
    pts, coefs, rhs, tol = W.make_batch()
    dev = torch.device("cuda:0")
    d_pts = [torch.from_numpy(p).to(dev) for p in pts]
    d_a = [torch.from_numpy(a).to(dev) for a in coefs]
    d_f = [torch.from_numpy(np.ascontiguousarray(f)).to(dev) for f in rhs]
    d_x = [torch.empty_like(f) for f in d_f]
    n_tot = sum(p.shape[0] for p in pts)
    lib = rsd.load()
    worst = 0.0

    def once():
        nonlocal worst
        facs = rsd.build_batched(d_pts, d_a, tol=tol, precision=rsd.RSD_PREC_FP32_REFINE)
        st, infos = rsd.solve_batched_raw(facs, [f.data_ptr() for f in d_f], 1, [x.data_ptr() for x in d_x])
        if st != rsd.RSD_OK:
            raise rsd.RsdError(st, lib.rsd_last_error().decode())
        worst = max([worst] + [i.rel_residual for i in infos])
        for fac in facs:
            fac.close()

    def timed():
        once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            once()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    rsd.tune_clear()
    dt_rule = timed()
    # the project's autotuner on this batch: every candidate tile / split-K
    # choice timed per launch-shape bucket on the batch's own builds
    t0 = time.perf_counter()
    n_buckets = rsd.autotune(d_pts, d_a, tol=tol, precision=rsd.RSD_PREC_FP32_REFINE, reps=1)
    t_tune = time.perf_counter() - t0
    dt = timed()
    rsd.tune_clear()
    return {"workload": "batch of 64 grids, side U{32..256}, bump coefficients, tol 1e-8, 1 RHS each",
            "precision": "fp32+refine", "n_instances": len(pts), "n_unknowns": n_tot,
            "ms_per_batch": dt * 1e3, "unknowns_per_s": n_tot / dt, "max_rel_residual": worst,
            "tiles": "autotuned", "ms_per_batch_builtin_rule": dt_rule * 1e3,
            "tuned_buckets": n_buckets, "tuning_s": t_tune}


def serving_measure(torch, rsd, W, seconds=3.0, rate=200.0, seed=4):
    """Resident Laplace factors of sides 128 and 256 (float64, tol 1e-10);
    single-RHS solve requests arrive as a Poisson process (rate per second)
    on uniformly chosen factors, device buffers; returns latency percentiles
    and throughput from the server's own statistics."""
    rng = np.random.default_rng(seed)
    dev = torch.device("cuda:0")
    srv = rsd.Server(n_workers=2, max_coalesce=64)
    sides = (128, 256)
    fids, sizes = [], []
    for n in sides:
        pts = W.grid_points(n)
        fids.append(srv.submit_factor(torch.from_numpy(pts).to(dev), torch.from_numpy(W.coef_sine(pts)).to(dev),
                                      tol=1e-10))
        sizes.append(pts.shape[0])
    # request pool prepared up front (inputs resident in HBM)
    pool = []
    for i in range(64):
        g = i % len(sides)
        f = torch.from_numpy(rng.standard_normal((1, sizes[g]))).to(dev)
        pool.append((g, f, torch.empty_like(f)))
    torch.cuda.synchronize()
    tickets = []
    t0 = time.perf_counter()
    t_next = t0
    k = 0
    while t_next - t0 < seconds:
        now = time.perf_counter()
        if now < t_next:
            time.sleep(min(t_next - now, 0.002))
            continue
        g, f, x = pool[k % len(pool)]
        tickets.append(srv.submit_solve(fids[g], f, x))
        k += 1
        t_next += rng.exponential(1.0 / rate)
    bad = 0
    for tk in tickets:
        st, _ = srv.wait(tk)
        bad += st != rsd.RSD_OK
    st = srv.stats()
    srv.close()
    return {"workload": f"Poisson arrivals {rate:.0f}/s for {seconds:.0f} s, 1 RHS each, resident Laplace "
                        f"factors of sides {list(sides)} (float64, tol 1e-10)",
            "requests": st["n_done"], "failed": bad, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
            "mean_batch_rhs": st["mean_batch_rhs"], "rhs_per_s": st["rhs_per_s"]}


def serving_scatter_measure(torch, rsd, W, seconds=3.0, rate=200.0, seed=4, sides=(128, 256), bulk="c64"):
    """The served scattering workload: Lippmann-Schwinger factors (Helmholtz
    kernel, wavenumber 20, Gaussian contrast bump) of the given sides, with
    complex128 refinement to 1e-8; bulk "c64": complex64 factors (float32 J
    form, three layers, root block in float64, at most eight refinement
    steps), "c128": complex128 factors (float64 J form, at most two steps).
    The factors are submitted while single-RHS complex solve requests arrive
    as a Poisson process on the factors already resident; returns latency
    percentiles, throughput and the worst residual."""
    c64 = bulk == "c64"
    rng = np.random.default_rng(seed)
    dev = torch.device("cuda:0")
    srv = rsd.Server(n_workers=2, max_coalesce=64, mem_budget=64 << 30)
    fids, sizes = [], []
    t0 = time.perf_counter()
    for n in sides:
        pts = W.grid_points(n)
        b = W.contrast_bump(pts)
        fids.append(srv.submit_factor(torch.from_numpy(pts).to(dev), None, tol=1e-8,
                                      precision=rsd.RSD_PREC_FP32_REFINE if c64 else rsd.RSD_PREC_FP64,
                                      max_refine=8 if c64 else 2, refine_tol=1e-8,
                                      kernel=rsd.RSD_KERNEL_HELMHOLTZ, wavenumber=W.SCATTER_K,
                                      contrast=torch.from_numpy(b).to(dev), wait=False))
        sizes.append(pts.shape[0])
    pools = []
    for g in range(len(sides)):
        pools.append([])
        for i in range(16):
            z = rng.standard_normal((1, sizes[g])) + 1j * rng.standard_normal((1, sizes[g]))
            f = torch.from_numpy(z).to(dev)
            pools[g].append((f, torch.empty_like(f)))
    torch.cuda.synchronize()
    srv.wait_factor(fids[0])            # arrivals start once the first factor is resident
    tickets = []
    t_start = time.perf_counter()
    t_next = t_start
    k = 0
    ready = [False] * len(fids)
    while t_next - t_start < seconds:
        now = time.perf_counter()
        if now < t_next:
            time.sleep(min(t_next - now, 0.002))
            continue
        # requests go to the factors resident so far (the others are still
        # being admitted and built beside the solves)
        for i, fid in enumerate(fids):
            ready[i] = ready[i] or srv.wait_factor(fid, 0) == rsd.RSD_OK
        live = [i for i in range(len(fids)) if ready[i]]
        g = live[int(rng.integers(len(live)))]
        f, x = pools[g][k % 16]
        tickets.append(srv.submit_solve(fids[g], f, x))
        k += 1
        t_next += rng.exponential(1.0 / rate)
    bad, worst = 0, 0.0
    for tk in tickets:
        st, info = srv.wait(tk)
        bad += st != rsd.RSD_OK
        worst = max(worst, info.rel_residual)
    st = srv.stats()
    t_all = time.perf_counter() - t0
    srv.close()
    return {"workload": f"Lippmann-Schwinger, Helmholtz k={W.SCATTER_K:g}, contrast bump 0.5/0.15, sides {list(sides)}; "
                        f"factors submitted at t=0 ("
                        + ("complex64 bulk: float32 J form" if c64 else "complex128 bulk: float64 J form")
                        + ", tol 1e-8, complex128 refinement), "
                        f"Poisson arrivals {rate:.0f}/s for {seconds:.0f} s, 1 complex RHS each",
            "requests": st["n_done"], "failed": bad, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
            "mean_batch_rhs": st["mean_batch_rhs"], "rhs_per_s": st["rhs_per_s"], "max_rel_residual": worst,
            "factors_built": st["n_built"], "wall_s": t_all}


def compressed_product_measure(torch, rsd, W, reps=10):
    """The factor's compressed forward product (recursive-skeleton form of A,
    O(N) work) against the exact FFT product on the 256^2 workload's factor:
    device buffers, 1 and 16 right-hand sides, median over reps; relative
    difference of the two products."""
    pts, a, f, tol = W.make_workload("laplace256")
    dev = torch.device("cuda:0")
    fac = rsd.Factor(torch.from_numpy(pts).to(dev), torch.from_numpy(a).to(dev), tol)
    out = {"workload": "laplace256 factor (float64, tol 1e-10), x ~ N(0,1)"}
    for nrhs in (1, 16):
        x = torch.from_numpy(np.ascontiguousarray(W.rhs_normal(len(pts), nrhs, 3).T)).to(dev)
        ye, yc = torch.empty_like(x), torch.empty_like(x)
        times = {}
        for key, fn, y in (("exact_ms", fac.matvec_raw, ye), ("compressed_ms", fac.matvec_compressed_raw, yc)):
            fn(x.data_ptr(), nrhs, y.data_ptr())
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = fn(x.data_ptr(), nrhs, y.data_ptr())
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                if st != rsd.RSD_OK:
                    raise rsd.RsdError(st, rsd.load().rsd_last_error().decode())
            times[key] = 1e3 * float(np.median(ts))
        rel = float(torch.linalg.norm(yc - ye) / torch.linalg.norm(ye))
        out[f"nrhs{nrhs}"] = {**times, "rel_diff": rel}
    fac.close()
    return out


def measure(torch, rsd, W, workload, precision, steps, warmup, fp32_interp=False, latency_solves=30,
            tol=None, with_breakdown=True):
    """Timed factor + solve steps of one workload (inputs resident in HBM).
    Returns (record, last solution as an (N, nrhs) array, stats of the last
    factor)."""
    pts, a, f, wtol = W.make_workload(workload)
    tol = wtol if tol is None else tol
    n, nrhs = f.shape
    dev = torch.device("cuda:0")
    prec = rsd.RSD_PREC_FP64 if precision == "fp64" else rsd.RSD_PREC_FP32_REFINE
    flags = rsd.RSD_FLAG_FP32_INTERP if fp32_interp else 0
    d_pts = torch.from_numpy(pts).to(dev)
    d_a = torch.from_numpy(a).to(dev)
    d_f = torch.from_numpy(np.ascontiguousarray(f.T)).to(dev)      # column-major N x nrhs
    d_x = torch.empty_like(d_f)
    torch.cuda.synchronize()
    lib = rsd.load()

    def step():
        fac = rsd.Factor(d_pts, d_a, tol, precision=prec, flags=flags)
        st, info = fac.solve_raw(d_f.data_ptr(), nrhs, d_x.data_ptr())
        if st != rsd.RSD_OK:
            raise rsd.RsdError(st, lib.rsd_last_error().decode())
        stats = fac.stats()
        fac.close()
        return stats, info

    log(f"workload {workload}: N={n}, nrhs={nrhs}, precision={precision}, tol={tol:g}")
    dt = "f64" if precision == "fp64" else "f32"
    gemm_cls = "factor_gemm_f64" if dt == "f64" else "factor_gemm_f32"
    # the timed steps bracket only the roofline kernel's launches with HIP
    # events (on the stream each runs on), in every PROF_EVERY-th step: the
    # kernel's average duration is sampled across the timed region while the
    # other steps run without events; the warmup creates those events
    rsd.profile_enable(True, classes=[gemm_cls])
    for i in range(warmup):
        stats, info = step()
        log(f"warmup {i}: build {stats['build_ms']:.2f} ms (device)")
    torch.cuda.synchronize()
    rsd.profile_enable(True, classes=[gemm_cls])
    prof_steps = 0
    t0 = time.perf_counter()
    for i in range(steps):
        sampled = i % PROF_EVERY == 0
        rsd.profile_pause(not sampled)
        prof_steps += sampled
        stats, info = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rsd.profile_pause(False)
    g = rsd.profile_query()[gemm_cls]
    rsd.profile_enable(False)
    ms_step = (t1 - t0) * 1e3 / steps
    value = n * steps / (t1 - t0)
    log(f"timed {steps} steps: {ms_step:.2f} ms/step, {value:.4g} unknowns/s")
    prof = {}
    n_prof = 2
    if with_breakdown:
        # per-class breakdown from separate, untimed steps with every class bracketed
        rsd.profile_enable(True)
        for i in range(n_prof):
            step()
        torch.cuda.synchronize()
        prof = rsd.profile_query()
        rsd.profile_enable(False)
        for k, v in prof.items():
            if v["launches"]:
                log(f"  {k:16s} {v['ms'] / n_prof:9.3f} ms/step  {v['launches'] // n_prof:5d} launches/step"
                    f"  {v['flops'] / max(v['ms'], 1e-9) / 1e9:9.1f} TF/s")
    # accuracy of the last step against the exact operator (FP64 residual on device)
    fac = rsd.Factor(d_pts, d_a, tol, precision=prec, flags=flags)
    x = d_x.cpu().numpy().T
    r = f - fac.matvec(np.asfortranarray(x))
    rel_res = float((np.linalg.norm(r, axis=0) / np.linalg.norm(f, axis=0)).max())
    log(f"max relative residual |f - A x| / |f| = {rel_res:.3e}")
    # solve latency (factor resident)
    lat = []
    for i in range(latency_solves):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        fac.solve_raw(d_f.data_ptr(), nrhs, d_x.data_ptr())
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - s0) * 1e3)
    fac.close()
    lat = np.array(lat[2:] if len(lat) > 4 else lat)
    p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
    log(f"solve latency ({nrhs} rhs): p50 {p50:.3f} ms, p99 {p99:.3f} ms")
    achieved = g["flops"] / (g["ms"] * 1e-3) if g["ms"] > 0 else 0.0
    cls_time = {k: v["ms"] for k, v in prof.items()}
    # HBM bytes per launch from the committed counter summary, valid only while
    # the GEMM source is the one the counters were taken with
    traffic = None
    if workload == "laplace256" and dt == "f64":
        from paper_1303_5466_amd import profsum
        rec = profsum.read_traffic(os.path.join(ROOT, "profiles", "gemm_kernel_laplace256_traffic.md"))
        if rec is not None and rec[1] == profsum.gemm_source_digest():
            traffic = rec[0]
    roof = {"bound": "mfma", "kernel": "gemm_kernel<" + ("double" if dt == "f64" else "float") + ", 0, *>",
            "class": gemm_cls, "achieved": achieved / 1e12, "peak": PEAK[dt] / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK[dt], "traffic": traffic,
            "launches_per_step": g["launches"] // max(prof_steps, 1),
            "sampled_steps": prof_steps,
            "flops_per_launch": g["flops"] / max(g["launches"], 1),
            "algorithmic_bytes_per_launch": g["bytes"] / max(g["launches"], 1),
            "avg_launch_us": g["ms"] * 1e3 / max(g["launches"], 1),
            "dominant_class_by_time": max(cls_time, key=cls_time.get) if cls_time else None}
    rec = {"workload": workload, "n_unknowns": n, "nrhs": nrhs, "tol": tol, "precision": precision,
           "dtype": dt, "layers": stats["layers"], "ms_per_step": ms_step, "unknowns_per_s": value,
           "solve_p50_ms": p50, "solve_p99_ms": p99, "max_rel_residual": rel_res,
           "factor_bytes": stats["factor_bytes"], "factor_flops_model": stats["factor_flops"],
           "kernels_ms_per_step": {k: v["ms"] / n_prof for k, v in prof.items() if v["launches"]},
           "roofline": roof}
    return rec, x, (pts, a, f)


def accuracy_ratio(torch, rsd, W, sides=(64, 128, 256, 512)):
    """Low-accuracy mode against the full one (Sec. 5.2): for each grid, the
    factor time (device build), factor memory and 1-RHS solve time at tol
    1e-5 (one layer) and 1e-10 (two layers), and their ratios."""
    dev = torch.device("cuda:0")
    out = []
    for n in sides:
        pts = W.grid_points(n)
        d_pts = torch.from_numpy(pts).to(dev)
        f = torch.from_numpy(W.rhs_normal(pts.shape[0], 1, 5).T.copy()).to(dev)
        x = torch.empty_like(f)
        row = {"side": n, "n_unknowns": pts.shape[0]}
        for tol in (1e-5, 1e-10):
            builds, solves = [], []
            for rep in range(4):
                t0 = time.perf_counter()
                fac = rsd.Factor(d_pts, None, tol)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                fac.solve_raw(f.data_ptr(), 1, x.data_ptr())
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                if rep:
                    builds.append(t1 - t0)
                    solves.append(t2 - t1)
                st = fac.stats()
                if rep < 3:
                    fac.close()
            xr = x.cpu().numpy().T
            r = f.cpu().numpy().T - fac.matvec(np.asfortranarray(xr))
            res = float(np.linalg.norm(r) / np.linalg.norm(f.cpu().numpy()))
            fac.close()
            key = "lo" if tol > 1e-8 else "hi"
            row[key] = {"tol": tol, "layers": st["layers"], "build_ms": 1e3 * float(np.median(builds)),
                        "solve_ms": 1e3 * float(np.median(solves)), "factor_bytes": st["factor_bytes"],
                        "factor_flops_model": st["factor_flops"], "rel_residual": res}
        lo, hi = row["lo"], row["hi"]
        row["ratio_time"] = hi["build_ms"] / lo["build_ms"]
        row["ratio_memory"] = hi["factor_bytes"] / lo["factor_bytes"]
        row["ratio_solve"] = hi["solve_ms"] / lo["solve_ms"]
        row["ratio_flops_model"] = hi["factor_flops_model"] / lo["factor_flops_model"]
        log(f"  {n}^2: 1e-5 build {lo['build_ms']:.2f} ms, {lo['factor_bytes'] / 1e6:.1f} MB, res {lo['rel_residual']:.1e};"
            f" 1e-10 build {hi['build_ms']:.2f} ms, {hi['factor_bytes'] / 1e6:.1f} MB; ratios time "
            f"{row['ratio_time']:.2f} memory {row['ratio_memory']:.2f} solve {row['ratio_solve']:.2f}"
            f" flops {row['ratio_flops_model']:.2f}")
        out.append(row)
    return {"workload": "Laplace, a = 1, 1 RHS N(0,1); tol 1e-5 (one layer) vs 1e-10 (two layers)",
            "grids": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="laplace256")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--fp32-interp", action="store_true",
                    help="fp32 factors: solve the interpolation problems in float32 as well")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-solves", type=int, default=30)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched many-grid measurement")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--no-fp32", action="store_true", help="skip the 512^2 float32 + refinement record")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the 1e-5 vs 1e-10 ratio study")
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1303_5466_amd import rsd, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.pmc_calibration:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)      # one elementwise kernel: reads and writes nbytes
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes}), flush=True)
        return
    main_rec, x, (pts, a, f) = measure(torch, rsd, W, args.workload, args.precision, args.steps, args.warmup,
                                       fp32_interp=args.fp32_interp, latency_solves=args.latency_solves)
    n, nrhs = f.shape
    out = {
        "metric": "unknowns/sec factor+solve at 1e-10, FP64 vs FP32+refine; solve p50/p99 ms",
        "value": main_rec["unknowns_per_s"], "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": main_rec["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": main_rec["dtype"], "data": "synthetic",
        "config": {"workload": args.workload, "grid": f"{int(round(n ** 0.5))}x{int(round(n ** 0.5))}",
                   "n_unknowns": n, "nrhs": nrhs, "tol": main_rec["tol"], "precision": args.precision,
                   "interp": "fp32" if args.fp32_interp and args.precision == "fp32" else "fp64",
                   "kernel": "laplace (1/2pi) log r", "leaf": "8x8", "layers": main_rec["layers"]},
        "solve_p50_ms": main_rec["solve_p50_ms"], "solve_p99_ms": main_rec["solve_p99_ms"],
        "max_rel_residual": main_rec["max_rel_residual"],
        "factor_flops_model": main_rec["factor_flops_model"],
        "kernels_ms_per_step": main_rec["kernels_ms_per_step"],
        "roofline": main_rec["roofline"],
    }
    fp32_x = None
    if not args.no_fp32 and args.workload == "laplace256":
        log("float32 factor + float64 refinement on the 512^2 workload ...")
        rec32, fp32_x, fp32_in = measure(torch, rsd, W, "laplace512", "fp32", 3, 2, latency_solves=12)
        out["fp32_refine"] = rec32
    if not args.no_accuracy and args.workload == "laplace256":
        log("accuracy ratio study: tol 1e-5 vs 1e-10 ...")
        out["accuracy_ratio"] = accuracy_ratio(torch, rsd, W)
        log("compressed forward product vs the exact product ...")
        out["compressed_product"] = compressed_product_measure(torch, rsd, W)
        for key in ("nrhs1", "nrhs16"):
            r = out["compressed_product"][key]
            log(f"  {key}: compressed {r['compressed_ms']:.3f} ms, exact {r['exact_ms']:.3f} ms, "
                f"difference {r['rel_diff']:.1e}")
    if not args.no_batched and args.workload == "laplace256":
        log("batched builds: 64 grids of uneven size ...")
        out["batched"] = batched_measure(torch, rsd, W)
        log(f"  {out['batched']['ms_per_batch']:.1f} ms per batch, "
            f"{out['batched']['unknowns_per_s']:.4g} unknowns/s, residual {out['batched']['max_rel_residual']:.2e}")
    if not args.no_serving and args.workload == "laplace256":
        log("serving loop: Poisson solve requests on resident factors ...")
        out["serving"] = serving_measure(torch, rsd, W)
        sv = out["serving"]
        log(f"  {sv['requests']} requests, p50 {sv['p50_ms']:.2f} ms, p99 {sv['p99_ms']:.2f} ms, "
            f"{sv['mean_batch_rhs']:.2f} RHS per coalesced solve")
        for key, bulk, sides in (("serving_scatter", "c64", (128, 256)), ("serving_scatter_c128", "c128", (128, 256, 512))):
            log(f"served scattering workload ({bulk} factors, sides {sides}): Helmholtz Lippmann-Schwinger factors "
                f"+ Poisson solves ...")
            out[key] = serving_scatter_measure(torch, rsd, W, bulk=bulk, sides=sides)
            sv = out[key]
            log(f"  {sv['requests']} requests ({sv['failed']} failed), p50 {sv['p50_ms']:.2f} ms, "
                f"p99 {sv['p99_ms']:.2f} ms, residual {sv['max_rel_residual']:.1e}")
    if not args.no_cpu_baseline:
        log("timing the CPU reference on a bounded sample ...")
        out["cpu_baseline"], sols = cpu_baseline(pts, a, f)
        # the error of each GPU result against the oracle's solution of the same column
        out["err_vs_oracle"] = err_vs_oracle(x, sols)
        log(f"  error vs oracle, max over {len(sols)} columns: {max(out['err_vs_oracle'].values()):.2e}")
        if fp32_x is not None:
            _, sols32 = cpu_baseline(fp32_in[0], fp32_in[1], fp32_in[2], budget_s=10.0, max_cols=1)
            out["fp32_refine"]["err_vs_oracle"] = err_vs_oracle(fp32_x, sols32)
            log(f"  512^2 float32 + refinement, error vs oracle: {out['fp32_refine']['err_vs_oracle']}")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
