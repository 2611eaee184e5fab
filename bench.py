#!/usr/bin/env python3
"""Benchmark of the finite-volume hot path on one MI355X.

One step = one 3-stage Runge-Kutta finite-volume step of the convection-
diffusion problem followed by one Poisson solve (Jacobi-CG to 1e-10 relative
true residual, warm-started from the previous solution, right-hand side =
the transported scalar; the operator applied matrix-free, the stored-matrix
CG is reported beside it), on a synthetic jittered-tetrahedron unit cube:

  cube120 (default): 120^3 hexes x 6 tets = 10,368,000 cells, seed 2
  cube20:             20^3 hexes x 6 tets =     48,000 cells, seed 1
  cube60:             60^3 hexes x 6 tets =  1,296,000 cells, seed 2 (an eighth of cube120)

Fields: Gaussian pulse (sigma 0.1, centre 0.5,0.5,0.5), velocity
(sin pi y, sin pi z, sin pi x), diffusivity 1e-3, zero-flux walls for the
scalar, Dirichlet 0 for the potential, dt from CFL 0.4.

Prints one JSON line.  `value` is FV cell-updates per second (cells x RK3
steps / FV time); the Poisson solve time per step is reported beside it.
Per-kernel durations come from HIP events the library records around its
own launches on the launch stream: in the timed region around the solve's
dominant kernel only (named by the last warm-up step's fully timed solve,
which gives the other solve kernels' durations); the FV kernels' from the
same steps launched directly after the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FV cell-updates/s + Poisson solve ms @1e-10 rel; plain vs mixed/learned"

# HBM bytes per dispatch measured with rocprofv3 FETCH_SIZE + WRITE_SIZE on the
# cube120 workload, scaled by a known-size copy (profiles/*_hbm_traffic.md).
# Each is valid only for the kernel source it was taken on: the bench reports
# it when that source (the kernel's file and the reduction headers) still
# hashes to the recorded prefix, else null.
MEASURED_TRAFFIC = {"cube120": {
    "k_mf_cg_cell": {"src": "8fdb010b17804213", "bytes": 1215810467},
    "k_mf_vertex": {"src": "8fdb010b17804213", "bytes": 623188346},
    "k_cg_axpy": {"src": "50d641f414878f07", "bytes": 668804504},
    "k_cg_dir": {"src": "50d641f414878f07", "bytes": 248844609},
    "k_grad_moments": {"src": "7212ca82332031bf", "bytes": 3720635711},
    "k_cell_step": {"src": "7212ca82332031bf", "bytes": 2159479857},
}}
# timing id -> the FP64 kernel it times
KERNEL_NAMES = {"grad_limiter": "k_grad_moments", "mf_gather": "k_mf_cg_cell", "fv_cell": "k_cell_step"}
KERNEL_FILES = {
    "grad_limiter": "fv_kernels.hip", "fv_cell": "fv_kernels.hip",
    "cg_spmv": "solve_kernels.hip", "cg_axpy": "solve_kernels.hip", "cg_dir": "solve_kernels.hip",
    "mf_vertex": ("mf_kernels.hip", "mf_cell.h"), "mf_gather": ("mf_kernels.hip", "mf_cell.h"),
}


def measure_copy_peak(gib=1, reps=10):
    """Achievable HBM bandwidth, the better of two streams over `gib` GiB
    vectors (torch's kernels): b = a (read + write) and c = a + b (two reads,
    one write); bytes moved per second, best of `reps` each."""
    import torch
    n = (gib << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    c = torch.empty_like(a)

    def best(fn, nbytes):
        fn()
        t = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            t = min(t, e0.elapsed_time(e1) / 1e3)
        return nbytes / t / 1e9

    copy = best(lambda: b.copy_(a), 2 * n * 8)
    add = best(lambda: torch.add(a, b, out=c), 3 * n * 8)
    del a, b, c
    return max(copy, add), {"copy": round(copy, 1), "add": round(add, 1)}


def kernel_source_hash(name):
    import hashlib
    h = hashlib.sha256()
    files = KERNEL_FILES[name] if isinstance(KERNEL_FILES[name], tuple) else (KERNEL_FILES[name],)
    for f in files + ("reduce.h", "seg.h", "cg_scalars.h", "halo_stage.h"):
        with open(os.path.join(ROOT, "paper_2203_00925_amd", "csrc", f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]
HBM_PEAK_GBS = 8000.0
# strength threshold and Jacobi weight of the W-cycle forms: the best of a
# sweep theta in {0.1 .. 0.6} x omega in {0.6 .. 1.0} on cube120 (cold solves)
AMG_W_OPTS = dict(theta=0.4, omega=0.8)
WORKLOADS = {
    "cube120": dict(n=120, seed=2),
    "cube20": dict(n=20, seed=1),
    "cube60": dict(n=60, seed=2),     # one GPU's share of cube120 split 8 ways
    "batch64": None,          # 64 uneven meshes, see run_batch
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(info):
    """Bytes each kernel must move per launch: every stored array it reads or
    writes counted once (gathered neighbour data counted once per array, not
    once per reference; padding of the 64-row slices not counted)."""
    nc, nf, nb, nv = info.nc, info.nf, info.nb, info.nv
    offdiag = info.matrix_nnz - nc
    halo = info.halo_entries
    return {
        # star-moment gradient on LDS tiles: tile halo list 4/entity; x, y,
        # z, u of cells and ghosts 32; own vertex lists: 16-bit local index 2
        # + weight 8 per entry, list length 4 and value written 8 per vertex;
        # foreign vertex lists: index 2 per entry, length 4 per row; per cell
        # c2f 16, local face neighbours 8, local vertices 8, M^-1 48, the
        # four face values written 32; edge-only neighbours: index 2 per
        # entry; face centroids 24/face
        "grad_limiter": halo * 4 + (nc + nb) * 32 + info.node_entries * 10 + nv * 12
        + info.foreign_entries * 2 + info.foreign_rows * 4 + nc * (16 + 8 + 8 + 48 + 32)
        + info.edge_nbr_entries * 2 + nf * 24,
        # the FP64 stage in one pass per cell: per cell outward phi 32, c2n
        # 16, face slots 1, vertex ids 16, vertex weights 32, kRL weights 32,
        # its four face values 32 (the neighbours' gathered, counted once),
        # u_in 8, u^n 8, vol 8, src 8, u written 8; the vertex values 8 per
        # vertex, gathered once; per ghost: its value read and written 16,
        # its face's kAC, kBC, kRL, A, B, C, area, tag, value and distance 64
        "fv_cell": nc * 201 + nv * 8 + nb * 80,
        # value 8 + 16-bit local index 2 per off-diagonal entry; tile halo
        # list 4/entity; p 8, diagonal 8, q written 8 per row
        "cg_spmv": offdiag * 10 + halo * 4 + nc * 24,
        # x,p,r,q,dinv read 40; x,r,z written 24
        "cg_axpy": nc * 64,
        # z,p read, p written
        "cg_dir": nc * 24,
        # matrix-free product: vertex lists (weight 8 + index 4 per entry, a
        # ghost entry folded onto its owner), x gathered once, vertex values
        # written
        "mf_vertex": info.node_entries * 12 + nc * 8 + nv * 8,
        # the per-cell product: per cell 4 vertex ids 16, 4 vertex weights 32,
        # 4 face neighbours 16, 4 face weights 32, p 8 (neighbours' p counted
        # once), q written 8; vertex values gathered once
        "mf_gather": nc * 112 + nv * 8,
    }


def cpu_baseline(seconds_target=15.0):
    """The FP64 oracle on the host (single thread), on the 48,000-cell cube of
    the same recipe: RK3 steps for about `seconds_target` seconds."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import synth
    from oracle import fv, poisson
    from oracle.geometry import build_geometry, ZERO_FLUX, DIRICHLET
    with threadpool_limits(limits=1):
        m = synth.jittered_cube(20, 1)
        geo = build_geometry(m.xyz, m.tets, m.btris, m.btags)
        pf = synth.problem_fields(m)
        kinds = [ZERO_FLUX] * 6
        phi = fv.face_velocity_flux(geo, pf.vel)
        dt = fv.cfl_dt(geo, phi, pf.diffusivity, pf.cfl, kinds)
        u = pf.u0
        steps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds_target or steps == 0:
            u = fv.rk3_step(geo, u, dt, phi, pf.diffusivity, kinds, [0.0] * 6)
            steps += 1
        t_fv = time.perf_counter() - t0
        K, c = poisson.assemble(geo, [DIRICHLET] * 6, [0.0] * 6)
        t1 = time.perf_counter()
        _, its, _ = poisson.jacobi_cg(K, poisson.rhs(geo, u, c), tol=1e-10)
        t_solve = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    try:
        host_cores = len(os.sched_getaffinity(0))
    except AttributeError:
        host_cores = os.cpu_count()
    return {"value": geo.nc * steps / t_fv, "unit": "cell-updates/s", "cores": 1,
            "host_cores": host_cores, "host_cpu": model,
            "kind": "oracle",
            "sample": f"single thread (1 core of the {host_cores} this process may use); "
                      f"48,000-cell cube of the same recipe (n=20, seed 1), {steps} RK3 steps "
                      f"in {t_fv:.1f} s; one cold Jacobi-CG solve to 1e-10: {its} iterations, "
                      f"{t_solve * 1e3:.0f} ms",
            "poisson_solve_ms": t_solve * 1e3}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="cube120")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--forms", default="all",
                    help="comma-separated forms to run after the main steps (fp32_refined, stored_matrix_cg, "
                         "fgmres30, multigrid_fcg, multigrid_w_fcg, streamer, learned, cube20, batch64), or all; "
                         "each runs min(--steps, 5) steps (batch64: 4; cube20: its own 10)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the reduced-precision (FP32 + refined solve) run")
    ap.add_argument("--learned-samples", type=int, default=0,
                    help="training samples of the learned form (default 2000; fewer only to shorten "
                         "profiled runs, whose network is then trained less)")
    ap.add_argument("--log", default=None,
                    help="append per-step and per-solve JSON-lines records of the main run to this file "
                         "(adds one conservation sum and a host synchronisation per timed step)")
    ap.add_argument("--calibrate-copy-gb", type=float, default=0.0,
                    help="first run one device-to-device copy of this many GB (a kernel of "
                         "known traffic, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.learned_samples > 0:
        LEARNED["samples"] = args.learned_samples
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the method's "
                          "multi-GPU decomposition is not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2203_00925_amd import binding as B

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(3)
    torch.cuda.set_device(0)
    if args.workload == "batch64":
        print(json.dumps(run_batch(args)), flush=True)
        return
    if args.calibrate_copy_gb > 0:
        n = int(args.calibrate_copy_gb * 1e9 / 8)
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: {n * 8} bytes read, {n * 8} bytes written")
        del a, b
    wl = WORKLOADS[args.workload]
    t = time.perf_counter()
    mesh = synth.jittered_cube(wl["n"], wl["seed"])
    pf = synth.problem_fields(mesh)
    log(f"mesh n={wl['n']} cells={mesh.nc} generated in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    M = B.Mesh.from_cube(mesh)
    info = M.info
    log(f"preprocessed in {time.perf_counter() - t:.1f}s; workspace {info.ws_bytes / 1e9:.2f} GB")
    st = B.State(M, diffusivity=pf.diffusivity)
    st.set_bcs(B.VAR_SCALAR, [B.ZERO_FLUX] * 6)
    st.set_bcs(B.VAR_POTENTIAL, [B.DIRICHLET] * 6)
    st.set_field(B.FIELD_VEL, torch.from_numpy(np.ascontiguousarray(pf.vel.T.ravel())))
    st.set_field(B.FIELD_U, torch.from_numpy(pf.u0))
    del mesh
    st.poisson_assemble()
    dt = st.cfl_dt(pf.cfl)
    total0 = st.conservation()
    log(f"state ready; dt={dt:.6g}")

    stream = torch.cuda.current_stream()
    # the FV step replays the library's captured step graph (the time step,
    # one ghost fill, 3 stages of 2 launches); capture it here, outside
    # warm-up and timing, and undo the
    # step it runs so that the state stays in step with the forms' runs
    u_keep = st.get_field(B.FIELD_U).clone()
    st.step_graph(1, dt)
    st.set_field(B.FIELD_U, u_keep)
    del u_keep

    def one_step(evs=None):
        if evs is not None:
            evs[0].record(stream)
        st.step_graph(1, dt)
        if evs is not None:
            evs[1].record(stream)
        info_s = st.poisson_solve(None, tol=1e-10, restart=500, matrix_free=True)
        if evs is not None:
            evs[2].record(stream)
        return info_s

    # the last warm-up step's solve runs with every kernel timed: it names
    # the solve's dominant kernel, the only one the timed region brackets
    # with events (an event pair around each of the seven launches of a CG
    # iteration costs about 6% of the solve), and gives the other kernels'
    # durations
    cg_names = ("mf_vertex", "mf_gather", "cg_axpy", "cg_dir")
    wstats = None
    for w in range(args.warmup):
        last = w == args.warmup - 1
        if last:
            st.kernel_timing(True)
        s = one_step()
        if last:
            wstats = st.kernel_stats()
            st.kernel_timing(False)
        log(f"warmup {w}: solve {s['iterations']} it, {s['ms']:.1f} ms")
    torch.cuda.synchronize()
    dominant = max(cg_names, key=lambda k: wstats[k][0]) if wstats else None
    if dominant:
        st.kernel_timing(True, only=[dominant])
    else:
        st.kernel_timing(True)
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    solves = []
    totals = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        solves.append(one_step(events[k]))
        if args.log:
            totals.append(st.conservation())
        log(f"step {k}: solve {solves[-1]['iterations']} it, rel {solves[-1]['rel_residual']:.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kstats = st.kernel_stats()
    st.kernel_timing(False)
    fv_ms = [e[0].elapsed_time(e[1]) for e in events]
    # per-kernel durations of the FV kernels (replayed without events in the
    # timed region): the same number of steps launched directly, then the
    # state restored
    u_keep = st.get_field(B.FIELD_U).clone()
    st.kernel_timing(True)
    for _ in range(args.steps):
        st.step(1, dt)
    fv_stats = st.kernel_stats()
    st.kernel_timing(False)
    st.set_field(B.FIELD_U, u_keep)
    del u_keep
    for k in ("ghost_fill", "grad_limiter", "fv_cell"):
        kstats[k] = fv_stats[k]
    solve_ms = [e[1].elapsed_time(e[2]) for e in events]
    total1 = st.conservation()

    copy_gbs, streams = measure_copy_peak()
    log(f"measured streams: {streams} GB/s")
    fv_total_s = sum(fv_ms) / 1e3
    value = info.nc * args.steps / fv_total_s
    nbytes = algorithmic_bytes(info)

    measured = MEASURED_TRAFFIC.get(args.workload, {})

    def roof(name, stats=None):
        ms, n = (stats or kstats)[name]
        avg_s = ms / max(n, 1) / 1e3
        gbs = nbytes[name] / avg_s / 1e9
        kname = KERNEL_NAMES.get(name, f"k_{name}")
        rec = measured.get(kname)
        traffic = rec["bytes"] if rec and rec["src"] == kernel_source_hash(name) else None
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
                "copy_peak": round(copy_gbs, 1), "frac_of_copy": round(gbs / copy_gbs, 4),
                "avg_us": round(avg_s * 1e6, 2), "launches": n,
                "bytes_per_launch": nbytes[name],
                "traffic_GBps": round(traffic / avg_s / 1e9, 1) if traffic else None}

    iters = [s["iterations"] for s in solves]
    if args.log:
        from paper_2203_00925_amd.runlog import RunLog
        mf_bytes = nbytes["mf_vertex"] + nbytes["mf_gather"] + nbytes["cg_axpy"] + \
            nbytes["cg_dir"]
        with RunLog(args.log, cells=info.nc, conservation0=total0) as rl:
            rl.run(workload=args.workload, cells=info.nc, faces=info.nf, steps=args.steps,
                   warmup=args.warmup, dt=dt, conservation_initial=total0)
            for k in range(args.steps):
                rl.step(args.warmup + k + 1, dt, conservation=totals[k], ms=fv_ms[k])
                rl.solve(args.warmup + k + 1, solves[k], method=0, ms=solve_ms[k],
                         bytes_per_iteration=mf_bytes, matrix_free=True)
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: jittered 6-tet cube n={wl['n']} seed {wl['seed']}, "
                               f"{info.nc} cells; RK3 step (CFL 0.4, D=1e-3, zero-flux) + "
                               "warm-started Jacobi-CG Poisson solve to 1e-10",
                   "cells": info.nc, "faces": info.nf, "matrix_nnz": info.matrix_nnz,
                   "parallelism": "single GPU"},
        "fv_ms_per_step": sum(fv_ms) / args.steps,
        "poisson_solve_ms": sum(solve_ms) / args.steps,
        "poisson_iterations": iters,
        "poisson_rel_residual": max(s["rel_residual"] for s in solves),
        "conservation_rel_drift": abs(total1 - total0) / abs(total0),
        # the kernel with the most GPU time in the timed region
        "roofline": roof(dominant or max(cg_names + ("grad_limiter",), key=lambda k: kstats[k][0])),
        "roofline_fv": {k: roof(k) for k in ("grad_limiter", "fv_cell")},
        "roofline_cg": {k: roof(k, kstats if (k == dominant or not wstats) else wstats) for k in cg_names},
        "kernel_timing": {"timed_region": dominant or "all",
                          "others": "last warm-up step" if dominant else "timed region"},
        "measured_streams_GBps": streams,
    }
    if not args.no_forms:
        u64 = st.get_field(B.FIELD_U)
        p64 = st.get_field(B.FIELD_P)
        torch.cuda.synchronize()
        del st
        torch.cuda.empty_cache()
        want = None if args.forms == "all" else set(args.forms.split(","))
        run = lambda name: want is None or name in want
        result["forms"] = {}
        main_args = args
        args = argparse.Namespace(**vars(main_args))      # the forms run at most 5 steps
        args.steps = min(main_args.steps, 5)
        args.warmup = min(main_args.warmup, 1)
        if run("fp32_refined"):
            # as many steps as the FP64 run: its errors are against that run's end state
            result["forms"]["fp32_refined"] = run_fp32_form(main_args, M, pf, u64, p64, result["poisson_solve_ms"])
            torch.cuda.empty_cache()
        plain_ms = sum(solve_ms) / len(solve_ms)
        if run("stored_matrix_cg"):
            result["forms"]["stored_matrix_cg"] = run_solver_form(
                args, M, pf, "Jacobi-CG on the stored matrix", dict(matrix_free=False), plain_ms, p64)
            form_cg = result["forms"]["stored_matrix_cg"]
            form_cg["roofline_cg_spmv"] = {
                "bytes_per_launch": nbytes["cg_spmv"], "avg_us": form_cg["kernel_avg_ms"]["cg_spmv"] * 1e3,
                "achieved_GBps": round(nbytes["cg_spmv"] / (form_cg["kernel_avg_ms"]["cg_spmv"] * 1e-3) / 1e9, 1)}
            torch.cuda.empty_cache()
        if run("fgmres30"):
            result["forms"]["fgmres30"] = run_solver_form(
                args, M, pf, "FGMRES(30) + Jacobi, matrix-free", dict(method=B.SOLVE_FGMRES, matrix_free=True),
                plain_ms, p64, fgmres_m=30)
            torch.cuda.empty_cache()
        if run("multigrid_fcg"):
            result["forms"]["multigrid_fcg"] = run_solver_form(
                args, M, pf, "flexible CG + aggregation multigrid V(1,1), matrix-free, graph-replayed chunks of 8",
                dict(method=B.SOLVE_AMG, matrix_free=True, graph=1, chunk=8), plain_ms, p64, amg=True,
                kernel_times=False)
            torch.cuda.empty_cache()
        if run("multigrid_w_fcg"):
            result["forms"]["multigrid_w_fcg"] = run_solver_form(
                args, M, pf, "flexible CG + aggregation multigrid W(1,1), theta 0.4, omega 0.8, matrix-free, "
                "graph-replayed chunks of 8",
                dict(method=B.SOLVE_AMG, matrix_free=True, graph=1, chunk=8), plain_ms, p64, amg=True,
                cycle=B.CYCLE_W, kernel_times=False, amg_opts=AMG_W_OPTS)
            torch.cuda.empty_cache()
        if run("streamer"):
            result["forms"]["streamer"] = run_streamer_form(args, M, pf)
            torch.cuda.empty_cache()
        if run("learned"):
            result["forms"]["learned"] = run_learned_form(args, M, pf, iters, solve_ms)
            torch.cuda.empty_cache()
        if run("cube20"):
            result["forms"]["cube20"] = run_small_form()
            torch.cuda.empty_cache()
        if run("batch64"):
            del M
            b = run_batch(args, steps=min(args.steps, 4), warmup=args.warmup)
            result["forms"]["batch64"] = {k: b[k] for k in (
                "value", "unit", "config", "fv_ms_per_step", "step_plus_solve_ms", "poisson_solve_ms",
                "poisson_iterations_max_per_solve", "poisson_iterations_mean_per_solve",
                "poisson_rel_residual_max", "per_launch_solve_ms", "per_launch_iterations_max",
                "persistent_same_solve_ms", "autotune",
                "preprocess_s", "workspace_GB", "steps", "warmup")}
            torch.cuda.empty_cache()
        args = main_args
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(result), flush=True)


def timed_kernels(st, dt, solve_kw, p):
    """Per-kernel durations of a form, outside its timed solves (whose
    durations carry no event records): one more step and solve with every
    kernel timed, then u and P restored (P to `p`)."""
    from paper_2203_00925_amd import binding as B
    u_keep = st.get_field(B.FIELD_U).clone()
    st.kernel_timing(True)
    st.step(1, dt)
    st.poisson_solve(None, **solve_kw)
    kstats = st.kernel_stats()
    st.kernel_timing(False)
    st.set_field(B.FIELD_U, u_keep)
    st.set_field(B.FIELD_P, p)
    return kstats


def run_fp32_form(args, M, pf, u64, p64, plain_ms):
    """The same steps in the reduced-precision form: FP32 step kernels and the
    FP32-inner, FP64-refined Poisson solve (inner CG on the FP32 matrix-free
    product).  Errors are against the FP64 run after the same number of steps
    (same inputs, same dt); one cold solve each with the matrix-free and the
    stored FP32 operator."""
    import numpy as np
    import torch
    from paper_2203_00925_amd import binding as B
    st = B.State(M, diffusivity=pf.diffusivity, precision=B.FP32)
    st.set_bcs(B.VAR_SCALAR, [B.ZERO_FLUX] * 6)
    st.set_bcs(B.VAR_POTENTIAL, [B.DIRICHLET] * 6)
    st.set_field(B.FIELD_VEL, torch.from_numpy(np.ascontiguousarray(pf.vel.T.ravel())))
    st.set_field(B.FIELD_U, torch.from_numpy(pf.u0))
    st.poisson_assemble()
    dt = st.cfl_dt(pf.cfl)
    stream = torch.cuda.current_stream()
    solve_kw = dict(tol=1e-10, restart=500, method=B.SOLVE_IR_FP32, inner_tol=1e-2, matrix_free=True)
    for w in range(args.warmup):
        st.step(1, dt)
        s = st.poisson_solve(None, **solve_kw)
        log(f"fp32 form warmup {w}: solve {s['iterations']} it, {s['outer']} outer, {s['ms']:.1f} ms")
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    solves = []
    for k in range(args.steps):
        ev[k][0].record(stream)
        st.step(1, dt)
        ev[k][1].record(stream)
        solves.append(st.poisson_solve(None, **solve_kw))
        ev[k][2].record(stream)
        log(f"fp32 form step {k}: solve {solves[-1]['iterations']} it, {solves[-1]['outer']} outer")
    torch.cuda.synchronize()
    fv_ms = sum(e[0].elapsed_time(e[1]) for e in ev)
    solve_ms = sum(e[1].elapsed_time(e[2]) for e in ev)
    u = st.get_field(B.FIELD_U)
    p = st.get_field(B.FIELD_P)
    torch.cuda.synchronize()
    uerr = float((u - u64).abs().max() / u64.abs().max())
    perr = float((p - p64).norm() / p64.norm())
    cold = {}
    for name, mf in (("matrix_free", True), ("stored_fp32_matrix", False)):
        st.set_field(B.FIELD_P, torch.zeros(M.info.nc, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        c = st.poisson_solve(None, **dict(solve_kw, matrix_free=mf))
        cold[name] = {"inner_iterations": c["iterations"], "outer": c["outer"], "ms": round(c["ms"], 3)}
        log(f"fp32 form cold solve ({name}): {c['iterations']} inner it, {c['outer']} outer, {c['ms']:.1f} ms")
    del st
    return {"fv_cell_updates_per_s": M.info.nc * args.steps / (fv_ms / 1e3),
            "fv_ms_per_step": fv_ms / args.steps,
            "poisson_solve_ms": solve_ms / args.steps,
            "poisson_inner_iterations": [s["iterations"] for s in solves],
            "poisson_outer_steps": [s["outer"] for s in solves],
            "poisson_rel_residual": max(s["rel_residual"] for s in solves),
            "speedup_vs_plain_fp64_solve": plain_ms / (solve_ms / args.steps),
            "u_max_rel_err_vs_fp64": uerr, "P_rel_err_vs_fp64": perr, "cold": cold,
            "dtype": "f32 step; f32 inner CG (matrix-free) with f64 residual, dots and refinement"}



def run_solver_form(args, M, pf, name, solve_kw, plain_ms, p64, fgmres_m=0, amg=False, cycle=0,
                    kernel_times=True, amg_opts=None):
    """The FP64 run's steps with another solver of the same system: solve time
    and iterations per step, the last solution's difference from plain
    Jacobi-CG continued to 1e-12, and one cold solve (P = 0).  amg: build and attach the multigrid
    hierarchy first (its host setup time is reported, outside the timings);
    cycle: its cycle type (0 V, CYCLE_W); amg_opts: its theta / omega.
    kernel_times: time each kernel
    (per-kernel events, which keep solves from replaying captured graphs);
    off for the forms timed on graph replay."""
    import numpy as np
    import torch
    from paper_2203_00925_amd import binding as B
    st = B.State(M, diffusivity=pf.diffusivity)
    st.set_bcs(B.VAR_SCALAR, [B.ZERO_FLUX] * 6)
    st.set_bcs(B.VAR_POTENTIAL, [B.DIRICHLET] * 6)
    st.set_field(B.FIELD_VEL, torch.from_numpy(np.ascontiguousarray(pf.vel.T.ravel())))
    st.set_field(B.FIELD_U, torch.from_numpy(pf.u0))
    st.poisson_assemble()
    if fgmres_m:
        st.fgmres_attach(fgmres_m)
    amg_info = st.amg_build(cycle=cycle, **(amg_opts or {})) if amg else None
    if amg:
        log(f"{name}: {amg_info['levels']} levels {amg_info['rows']}, setup {amg_info['setup_ms'] / 1e3:.1f} s")
    dt = st.cfl_dt(pf.cfl)
    kw = dict(tol=1e-10, restart=500, **solve_kw)
    if solve_kw.get("graph") == 1:         # capture the chunk graph outside the cold timing
        st.poisson_solve(None, **kw)
        st.set_field(B.FIELD_P, torch.zeros(M.info.nc, dtype=torch.float64, device="cuda"))
    cold = st.poisson_solve(None, **kw)
    st.set_field(B.FIELD_P, torch.zeros(M.info.nc, dtype=torch.float64, device="cuda"))
    stream = torch.cuda.current_stream()
    for w in range(args.warmup):
        st.step(1, dt)
        st.poisson_solve(None, **kw)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    solves = []
    for k in range(args.steps):
        st.step(1, dt)
        ev[k][0].record(stream)
        solves.append(st.poisson_solve(None, **kw))
        ev[k][1].record(stream)
        log(f"{name} step {k}: {solves[-1]['iterations']} it, rel {solves[-1]['rel_residual']:.2e}")
    torch.cuda.synchronize()
    p = st.get_field(B.FIELD_P).clone()
    torch.cuda.synchronize()
    ms = sum(e[0].elapsed_time(e[1]) for e in ev) / args.steps
    kstats = timed_kernels(st, dt, kw, p) if kernel_times else {}
    # the last solution against plain Jacobi-CG taken on to 1e-12 from it
    st.poisson_solve(None, tol=1e-12, restart=500, matrix_free=True)
    p_ref = st.get_field(B.FIELD_P)
    perr = float((p - p_ref).norm() / p_ref.norm())
    del st
    extra = {"multigrid": {"levels": amg_info["levels"], "rows": amg_info["rows"], "nnz": amg_info["nnz"],
                           "host_setup_s": amg_info["setup_ms"] / 1e3}} if amg else {}
    return {**extra, "solver": name, "poisson_solve_ms": ms, "speedup_vs_main_solve": plain_ms / ms,
            "poisson_iterations": [s["iterations"] for s in solves],
            "poisson_rel_residual": max(s["rel_residual"] for s in solves),
            "P_rel_diff_vs_plain_cg_1e-12": perr,
            "cold": {"iterations": cold["iterations"], "ms": cold["ms"]},
            "kernel_avg_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in kstats.items() if v[1]},
            "dtype": "f64"}


# Learned-preconditioner form: training data from config-1-style runs on
# meshes of 1.05M-1.97M cells (unseen by the test), 2,000 samples.
LEARNED = dict(train_n=(56, 60, 64, 69), train_seed0=7000, samples=2000, epochs=4, lr=3e-3,
               lr_min=3e-4, snapshots=(0, 1, 2, 4, 8, 16, 32, 64, 128, 256), data_seed=77)


def learned_training_data(B, net, log_prefix="learned"):
    """Samples of true residuals along the plain solver's runs: per right-hand
    side, a Gaussian pulse (random centre in [0.3, 0.7]^3, sigma in [0.05,
    0.2]) advanced 0-10 RK3 steps in the rotating flow, then restarted
    Jacobi-CG from P = 0 with a sample at each snapshot iteration."""
    import numpy as np
    import torch
    import synth
    rng = np.random.default_rng(LEARNED["data_seed"])
    states, samples, owner = [], [], []
    per = LEARNED["samples"] // len(LEARNED["train_n"])
    for k, n in enumerate(LEARNED["train_n"]):
        m = synth.jittered_cube(n, LEARNED["train_seed0"] + k)
        pf = synth.problem_fields(m)
        st = B.State(B.Mesh.from_cube(m), diffusivity=pf.diffusivity)
        st.set_bcs(B.VAR_SCALAR, [B.ZERO_FLUX] * 6)
        st.set_bcs(B.VAR_POTENTIAL, [B.DIRICHLET] * 6)
        st.set_field(B.FIELD_VEL, torch.from_numpy(np.ascontiguousarray(pf.vel.T.ravel())))
        st.poisson_assemble()
        net.attach(st, training=True)
        dt = st.cfl_dt(pf.cfl)
        zero = torch.zeros(m.nc, dtype=torch.float64, device="cuda")
        got = 0
        while got < per:
            c = rng.uniform(0.3, 0.7, 3)
            st.set_field(B.FIELD_U, torch.from_numpy(synth.gaussian_field(m, c, rng.uniform(0.05, 0.2))))
            st.step(int(rng.integers(0, 11)), dt)
            st.set_field(B.FIELD_P, zero)
            done = 0
            for it in LEARNED["snapshots"]:
                if it > done:
                    st.poisson_solve(None, tol=1e-14, maxit=it - done, restart=0, allow_not_converged=True)
                    done = it
                else:
                    st.poisson_rhs(None)
                smp, rms = st.nn_sample()
                if rms > 0:
                    samples.append(smp)
                    owner.append(k)
                    got += 1
                if got >= per:
                    break
        states.append(st)
        log(f"{log_prefix}: training mesh n={n} ({m.nc} cells): {got} samples")
    return states, samples, owner


def run_small_form():
    """The small configuration on the GPU: the 48,000-cell cube (n = 20, seed
    1) with the same fields, 10 RK3 steps at CFL 0.4 (one captured graph),
    then one cold Jacobi-CG solve to 1e-10 (Dirichlet 0, right-hand side =
    the stepped scalar), matrix-free and on the stored matrix.  At this size
    the step is bound by its launches, not by HBM."""
    import numpy as np
    import torch
    import synth
    from paper_2203_00925_amd import binding as B
    wl = WORKLOADS["cube20"]
    m = synth.jittered_cube(wl["n"], wl["seed"])
    pf = synth.problem_fields(m)
    st = B.State(B.Mesh.from_cube(m), diffusivity=pf.diffusivity)
    st.set_bcs(B.VAR_SCALAR, [B.ZERO_FLUX] * 6)
    st.set_bcs(B.VAR_POTENTIAL, [B.DIRICHLET] * 6)
    st.set_field(B.FIELD_VEL, torch.from_numpy(np.ascontiguousarray(pf.vel.T.ravel())))
    st.set_field(B.FIELD_U, torch.from_numpy(pf.u0))
    st.poisson_assemble()
    dt = st.cfl_dt(pf.cfl)
    u0 = st.get_field(B.FIELD_U).clone()
    st.step_graph(10, dt)                               # capture (and one untimed run)
    st.set_field(B.FIELD_U, u0)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    st.step_graph(10, dt)
    e1.record(stream)
    torch.cuda.synchronize()
    fv_ms = e0.elapsed_time(e1)
    solves = {}
    for name, mf in (("matrix_free", True), ("stored_matrix", False)):
        st.set_field(B.FIELD_P, torch.zeros(m.nc, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        e0.record(stream)
        s = st.poisson_solve(None, tol=1e-10, restart=500, matrix_free=mf)
        e1.record(stream)
        torch.cuda.synchronize()
        solves[name] = {"iterations": s["iterations"], "ms": round(e0.elapsed_time(e1), 3),
                        "rel_residual": s["rel_residual"]}
    log(f"cube20: 10 steps {fv_ms:.2f} ms, solves {solves}")
    del st
    return {"cells": m.nc, "fv_cell_updates_per_s": m.nc * 10 / (fv_ms / 1e3), "fv_ms_per_step": fv_ms / 10,
            "poisson_solve": solves, "dtype": "f64"}


def run_streamer_form(args, M, pf):
    """The coupled streamer-type loop (eq. (10)) on the same mesh, set up as
    the paper's streamer run: potential 1 at x = 0 and 0 at x = 1 with
    homogeneous Neumann elsewhere, homogeneous Neumann for n_e, n_p = n_e
    at the start (a Gaussian pulse on a background); constant mobility and
    Townsend-type ionisation (the paper's fits are not usable).  Each step:
    the warm-started matrix-free Jacobi-CG solve for the charge, E, v_e and
    S_e, the CFL step of n_e and the ion update."""
    import numpy as np
    import torch
    from paper_2203_00925_amd import binding as B
    st = B.State(M, diffusivity=pf.diffusivity)
    st.set_bcs(B.VAR_SCALAR, [B.NEUMANN] * 6, [0.0] * 6)
    st.set_bcs(B.VAR_POTENTIAL, [B.DIRICHLET, B.DIRICHLET] + [B.NEUMANN] * 4, [1.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    st.poisson_assemble()
    ne = torch.from_numpy(pf.u0 + 1e-2)
    st.set_field(B.FIELD_U, ne)
    st.set_field(B.FIELD_ION, ne)
    params = dict(mobility=1.0, charge_scale=40.0, alpha_a=2.0, alpha_b=0.3, cfl=0.4, tol=1e-10,
                  matrix_free=True)
    first = st.streamer_step(1, **params)                  # cold solve
    log(f"streamer: first step {first['iterations_max']} CG iterations")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    info = st.streamer_step(args.steps, **params)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    ion = st.get_field(B.FIELD_ION)
    torch.cuda.synchronize()
    log(f"streamer: {args.steps} steps, {ms:.1f} ms per step, CG {info['iterations_sum']} iterations")
    out = {"ms_per_coupled_step": ms, "cg_iterations_per_step": info["iterations_sum"] / args.steps,
           "first_step_cg_iterations": first["iterations_max"], "dt": info["last_dt"],
           "ion_gain_rel": float(ion.sum().item() / float(ne.sum()) - 1.0),
           "model": "eq. (10) with v = -mu E (mu 1), alpha = 2 exp(-0.3/|E|), kappa 40, D 1e-3",
           "dtype": "f64"}
    del st
    return out


def run_learned_form(args, M, pf, plain_iters, plain_solve_ms):
    """The learned preconditioner: generate the training data with the
    library's own solver on smaller unseen meshes, train the network with the
    library's kernels, then run the same steps as the FP64 run with the
    flexible-CG solve; plus one cold solve (P = 0) with each method."""
    import numpy as np
    import torch
    from paper_2203_00925_amd import binding as B
    net = B.Network(seed=1)
    t0 = time.perf_counter()
    tstates, samples, owner = learned_training_data(B, net)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    tr = net.train(tstates, samples, owner, epochs=LEARNED["epochs"], lr=LEARNED["lr"],
                   lr_min=LEARNED["lr_min"], seed=3, loss=B.LOSS_RESIDUAL)
    log(f"learned: {len(samples)} samples in {t_data:.1f}s; trained {tr['steps']} steps in "
        f"{tr['ms'] / 1e3:.1f}s; epoch losses {np.round(tr['epoch_loss'], 4).tolist()}")
    del samples, tstates
    torch.cuda.empty_cache()
    st = B.State(M, diffusivity=pf.diffusivity)
    st.set_bcs(B.VAR_SCALAR, [B.ZERO_FLUX] * 6)
    st.set_bcs(B.VAR_POTENTIAL, [B.DIRICHLET] * 6)
    st.set_field(B.FIELD_VEL, torch.from_numpy(np.ascontiguousarray(pf.vel.T.ravel())))
    st.set_field(B.FIELD_U, torch.from_numpy(pf.u0))
    st.poisson_assemble()
    net.attach(st)
    form, ms_layers, ms_fused = st.nn_form()
    form_info = {"form": {B.NN_FORM_LAYERS: "layers", B.NN_FORM_FUSED: "fused"}.get(form, str(form)),
                 "attach_ms_layers": round(ms_layers, 4), "attach_ms_fused": round(ms_fused, 4)}
    log(f"learned: network forward {form_info}")
    dt = st.cfl_dt(pf.cfl)
    kw = dict(tol=1e-10, restart=500, method=B.SOLVE_LEARNED, allow_fell_back=True, matrix_free=True)
    kw_csr = dict(kw, matrix_free=False)
    # cold solves of the initial right-hand side, both methods
    zero = torch.zeros(M.info.nc, dtype=torch.float64, device="cuda")
    st.set_field(B.FIELD_P, zero)
    cold_plain = st.poisson_solve(None, tol=1e-10, restart=500, matrix_free=True)
    st.set_field(B.FIELD_P, zero)
    cold = st.poisson_solve(None, **kw)
    log(f"learned: cold solve {cold['iterations']} it {cold['ms']:.0f} ms vs Jacobi-CG "
        f"{cold_plain['iterations']} it {cold_plain['ms']:.0f} ms (matrix-free product)")
    st.set_field(B.FIELD_P, zero)
    cold_csr = st.poisson_solve(None, **kw_csr)
    st.set_field(B.FIELD_P, zero)
    cold_plain_csr = st.poisson_solve(None, tol=1e-10, restart=500)
    log(f"learned, stored matrix: cold solve {cold_csr['iterations']} it {cold_csr['ms']:.0f} ms vs "
        f"Jacobi-CG {cold_plain_csr['iterations']} it {cold_plain_csr['ms']:.0f} ms")
    st.set_field(B.FIELD_P, zero)
    stream = torch.cuda.current_stream()
    for w in range(args.warmup):
        st.step(1, dt)
        st.poisson_solve(None, **kw)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    solves = []
    for k in range(args.steps):
        st.step(1, dt)
        ev[k][0].record(stream)
        solves.append(st.poisson_solve(None, **kw))
        ev[k][1].record(stream)
        log(f"learned step {k}: {solves[-1]['iterations']} it, rel {solves[-1]['rel_residual']:.2e}, "
            f"fell back {solves[-1]['fell_back']}")
    torch.cuda.synchronize()
    solve_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / args.steps
    kstats = timed_kernels(st, dt, kw, st.get_field(B.FIELD_P).clone())
    plain_ms = sum(plain_solve_ms) / len(plain_solve_ms)
    layer_ms = {k: round(v[0] / max(v[1], 1), 4) for k, v in kstats.items() if v[1]}
    # the trained network as the finest-level smoother of the multigrid W-cycle:
    # cold solves of one right-hand side with each smoother and plain
    # Jacobi-CG, then stepped (warm) solves
    amg_info = st.amg_build(cycle=B.CYCLE_W, **AMG_W_OPTS)
    kw_mg = dict(tol=1e-10, restart=500, method=B.SOLVE_AMG, matrix_free=True)
    cold_mg = {}
    for name, extra in (("jacobi_smoother", {}), ("learned_smoother", dict(learned_smoother=True, chunk=8))):
        st.set_field(B.FIELD_P, zero)
        c = st.poisson_solve(None, **kw_mg, **extra)
        cold_mg[name] = {"iterations": c["iterations"], "ms": round(c["ms"], 3)}
    st.set_field(B.FIELD_P, zero)
    c = st.poisson_solve(None, tol=1e-10, restart=500, matrix_free=True)
    cold_mg["jacobi_cg"] = {"iterations": c["iterations"], "ms": round(c["ms"], 3)}
    log(f"learned smoother in the multigrid cycle, cold: {cold_mg}")
    ev2 = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    mg_solves = []
    for k in range(args.steps):
        st.step(1, dt)
        ev2[k][0].record(stream)
        mg_solves.append(st.poisson_solve(None, **kw_mg, learned_smoother=True, chunk=8))
        ev2[k][1].record(stream)
    torch.cuda.synchronize()
    mg_ms = sum(e[0].elapsed_time(e[1]) for e in ev2) / args.steps
    log(f"learned smoother in the multigrid cycle, warm: {[s['iterations'] for s in mg_solves]} it, {mg_ms:.1f} ms")
    del st
    return {"poisson_solve_ms": solve_ms,
            "poisson_iterations": [s["iterations"] for s in solves],
            "poisson_rel_residual": max(s["rel_residual"] for s in solves),
            "fell_back": [s["fell_back"] for s in solves],
            "speedup_vs_jacobi_cg": plain_ms / solve_ms,
            "jacobi_cg_iterations": plain_iters, "jacobi_cg_solve_ms": plain_ms,
            "cold": {"learned_iterations": cold["iterations"], "learned_ms": cold["ms"],
                     "jacobi_cg_iterations": cold_plain["iterations"], "jacobi_cg_ms": cold_plain["ms"],
                     "stored_matrix": {"learned_iterations": cold_csr["iterations"], "learned_ms": cold_csr["ms"],
                                       "jacobi_cg_iterations": cold_plain_csr["iterations"],
                                       "jacobi_cg_ms": cold_plain_csr["ms"]}},
            "kernel_avg_ms": layer_ms,
            "network_forward": form_info,
            "as_multigrid_smoother": {"poisson_solve_ms": mg_ms,
                                      "poisson_iterations": [s["iterations"] for s in mg_solves],
                                      "poisson_rel_residual": max(s["rel_residual"] for s in mg_solves),
                                      "speedup_vs_jacobi_cg": plain_ms / mg_ms, "cold": cold_mg,
                                      "levels": amg_info["rows"]},
            "training": {"meshes_n": list(LEARNED["train_n"]), "samples": LEARNED["samples"],
                         "epochs": LEARNED["epochs"], "loss": "residual",
                         "epoch_loss": [round(float(x), 5) for x in tr["epoch_loss"]],
                         "data_s": t_data, "train_s": tr["ms"] / 1e3},
            "dtype": "bf16 network (fp32 accumulation), f64 flexible CG"}


def run_batch(args, steps=None, warmup=None):
    """Batched form: 64 jittered cubes with log-uniform cell counts in
    [5e4, 2e6] (33.8M cells in all), per-mesh diffusivity and Gaussian
    centre, all advanced in one state without the stored Poisson matrix:
    each step an RK3 step of every mesh at its own CFL time step (one launch
    per kernel for all meshes), then every mesh's warm-started matrix-free
    Jacobi-CG in the persistent batch kernel (schedule from its autotuner),
    the whole run captured in one graph.  Also timed: the FV steps alone
    (cell-updates/s) and one step with the per-launch solver for comparison."""
    import numpy as np
    import torch
    import synth
    from paper_2203_00925_amd import binding as B
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    recipe = synth.batch_recipe()
    t = time.perf_counter()
    meshes = [synth.jittered_cube(r.n, r.seed) for r in recipe]
    u0 = np.concatenate([synth.gaussian_field(m, r.center, 0.1) for m, r in zip(meshes, recipe)])
    vel = [synth.rotating_velocity(m) for m in meshes]
    vel = np.concatenate([np.concatenate([v[:, k] for v in vel]) for k in range(3)])
    log(f"batch: {len(meshes)} meshes, {sum(m.nc for m in meshes)} cells generated in "
        f"{time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    M = B.Mesh.from_batch(meshes, no_matrix=True)
    del meshes
    t_pre = time.perf_counter() - t
    log(f"batch preprocessed in {t_pre:.1f}s; workspace {M.info.ws_bytes / 1e9:.2f} GB (no stored matrix)")
    st = B.State(M)
    st.set_mesh_diffusivity([r.diffusivity for r in recipe])
    st.set_bcs(B.VAR_SCALAR, [B.ZERO_FLUX] * 6)
    st.set_bcs(B.VAR_POTENTIAL, [B.DIRICHLET] * 6)
    st.set_field(B.FIELD_VEL, torch.from_numpy(vel))
    st.set_field(B.FIELD_U, torch.from_numpy(u0))
    st.cfl_dt(0.4)
    bt = B.Batch(st)
    tune = bt.autotune(os.path.join(ROOT, "paper_2203_00925_amd", "_lib", "batch_tune.json"))
    log(f"batch autotune: {tune}")

    stream = torch.cuda.current_stream()
    if warmup > 0:
        w = bt.run(warmup)
        log(f"batch warmup: {warmup} steps, solve max {w['iterations_max']} it, {w['ms']:.0f} ms")
    nc = M.info.nc
    # the FV steps alone (captured step graph), restored afterwards
    u_keep = st.get_field(B.FIELD_U).clone()
    st.step_graph(steps, 0.0)                        # capture outside the timing
    st.set_field(B.FIELD_U, u_keep)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    st.step_graph(steps, 0.0)
    e1.record(stream)
    torch.cuda.synchronize()
    fv_ms = e0.elapsed_time(e1) / steps
    st.set_field(B.FIELD_U, u_keep)
    del u_keep
    # the timed run: steps and persistent solves, one graph (captured by the
    # first call, so run once untimed with the same arguments)
    p_keep = st.get_field(B.FIELD_P).clone()
    u_keep = st.get_field(B.FIELD_U).clone()
    bt.run(steps)
    st.set_field(B.FIELD_U, u_keep)
    st.set_field(B.FIELD_P, p_keep)
    torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    info = bt.run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    run_ms = e0.elapsed_time(e1) / steps
    its = st.mesh_values("iterations")
    log(f"batch run: {steps} steps, {run_ms:.0f} ms per step (FV {fv_ms:.1f} ms); solve iterations per mesh "
        f"max {info['iterations_max']} mean {info['iterations_mean']:.0f} over the run, rel max "
        f"{info['rel_residual_max']:.2e}")
    # one more step, then its solve twice from the same start: the per-launch
    # solver (chunks of iterations for all meshes, host checks between them)
    # and the persistent kernel
    st.step_graph(1, 0.0)
    p_keep = st.get_field(B.FIELD_P).clone()
    e2 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    s_l = st.poisson_solve(None, tol=1e-10, restart=500, matrix_free=True)
    e2.record(stream)
    torch.cuda.synchronize()
    launch_ms = e0.elapsed_time(e2)
    st.set_field(B.FIELD_P, p_keep)
    chosen = bt.schedule()
    # the persistent kernel at its best schedule from the tuner
    bt.set_schedule(item_rows=tune["p_item_rows"], grid=tune["p_grid"], policy=tune["p_policy"],
                    vertex_batch=tune["p_vertex_batch"])
    torch.cuda.synchronize()
    e0.record(stream)
    bt_one = bt.solve(tol=1e-10)
    e2.record(stream)
    torch.cuda.synchronize()
    persistent_ms = e0.elapsed_time(e2)
    bt.set_schedule(**{k: chosen[k] for k in ("item_rows", "grid", "policy", "vertex_batch", "chunk")})
    log(f"batch: one step's solve per-launch {launch_ms:.0f} ms ({s_l['iterations']} it max) vs persistent "
        f"{persistent_ms:.0f} ms ({bt_one['iterations_max']} it max)")
    out = {"metric": METRIC, "value": nc / (fv_ms / 1e3), "unit": "cell-updates/s",
           "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": wall * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batch64: 64 jittered 6-tet cubes, cells log-uniform in [5e4, 2e6] "
                                  f"({nc} in all), per-mesh D and centre; RK3 step with per-mesh CFL "
                                  "dt + per-mesh warm-started Jacobi-CG (matrix-free product) to 1e-10, "
                                  "persistent batch kernel, one graph",
                      "cells": nc, "meshes": M.info.nmeshes, "parallelism": "single GPU"},
           "fv_ms_per_step": fv_ms, "step_plus_solve_ms": run_ms, "poisson_solve_ms": run_ms - fv_ms,
           "poisson_iterations_max_per_solve": int(its.max()),
           "poisson_iterations_mean_per_solve": float(info["iterations_mean"] / max(info["solves"], 1)),
           "poisson_rel_residual_max": info["rel_residual_max"],
           "per_launch_solve_ms": launch_ms, "per_launch_iterations_max": s_l["iterations"],
           "persistent_same_solve_ms": persistent_ms,
           "autotune": tune, "preprocess_s": t_pre, "workspace_GB": M.info.ws_bytes / 1e9}
    del bt, st
    return out


if __name__ == "__main__":
    main()
