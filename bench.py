#!/usr/bin/env python3
"""Benchmark of the EMD misfit hot path on one MI355X.

A step is the whole path over one batch of synthetic gathers already resident in
HBM: emd_decompose -> the PDHG-with-linesearch solve, started coarse-to-fine (the
multi-grid strategy the paper applies to the EMD: the data restricted to coarser
grids are solved first, and each solution, interpolated, starts the next finer
solve; every level runs to the relative-residual stop rule) -> emd_adjoint_source.
The metric is PDHG cell-updates per second over all levels (sum of nr * nt *
iterations, divided by the step time) for the batched FP32 solve; the EMD of the
first gathers is checked against FP64 solves of them taken far past the stop rule
(the accuracy the metric is quoted at), and the plain FP64 solve of the same gathers,
one gather per plan, is timed beside it.  Further legs: the solve without the
coarse start, the same linesearch solve started from coarse levels solved by plain
fixed-step PDHG, plain fixed-step PDHG with three iterations per sweep on every
level, the 16 x 4000 x 1600 batch at a fixed budget and its whole misfit to the stop
rule (also from fixed-step coarse levels), the one-pass kernels and grid transfers,
and the CPU oracle.

Default workload: 64 gathers, nt ~ U{1500..3000}, nr ~ U{200..500}, 4-8 hyperbolic
events (seed 3).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
C5_FULL_MAX_ITER = 1000000
BYTES_PER_CELL_ITER = {"f32": 36, "f64": 72}  # read u, phi, s, R; write u, phi, R
# Bytes crossing the L2 boundary per sweep over the algorithmic bytes, from the
# FETCH_SIZE / WRITE_SIZE profiler runs (scaled by a plain copy's readings) of the
# sweep source with this digest, per kernel; the traffic figure is null for any other
# source.
MEASURED_TRAFFIC = {"sweep_source_sha256_16": "4b79b79f83f54e78",
                    "ratio": {"k_sweep<float, false>": 1.0734, "k_sweep2<float>": 1.0630,
                              "k_sweep3<float>": 1.0420}}


def sweep_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("emd_sweep.hip", "emd_internal.h", "emd_abi.hip", "emd_tiling.h"):
        with open(os.path.join(ROOT, "paper_1808_07284_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from synth import config2_gather, config3_batch, config4_batch, config5_batch
    if name == "c3":
        return config3_batch(), "64 gathers, nt~U{1500..3000} x nr~U{200..500}, 4-8 hyperbolic events, seed 3"
    if name == "c2":
        return [config2_gather()], "1 gather, nt=2000 x nr=400, 6 hyperbolic events, seed 2"
    if name == "c4":
        return config4_batch(), "32 gathers, nt=2000 x nr=300, seed 4"
    if name == "c5":
        return config5_batch(), "16 gathers, nt=4000 x nr=1600, 10 events + direct arrival, seed 5"
    raise SystemExit(f"unknown workload {name}")


def run_step(E, plan, pcal, pobs, bufs, mg=None):
    """decompose -> solve (coarse-to-fine when mg is given) -> adjoint source."""
    if mg is None:
        s, mass = E.emd_decompose(plan, pcal, pobs, s_out=bufs["s"], mass_out=bufs["mass"])
        emd, phi, _, info = E.emd_pdhg_solve(plan, s, phi=bufs["phi"], mass=mass,
                                             emd_out=bufs["emd"], info_out=bufs["info"])
    else:
        emd, phi, _, info, mass = mg.solve(pcal, pobs, emd_out=bufs["emd"], info_out=bufs["info"])
    E.emd_adjoint_source(plan, phi, pcal, pobs, mass, psi_out=bufs["psi"])
    return emd, info


def step_stats(plan, mg=None):
    """Cell updates, sweep time (HIP events the library records) and sweeps of the
    last step, over the fine plan and its coarse levels."""
    plans = [plan] + ([lv[0] for lv in mg.levels] if mg is not None else [])
    qs = [p.query() for p in plans]
    return (sum(q["last_cell_updates"] for q in qs), sum(q["last_sweep_ms"] for q in qs),
            sum(q["last_sweeps"] for q in qs))


def parse_levels(spec, workload_name):
    if spec == "auto":
        # a single small gather's coarse sweeps are as latency-bound as its fine ones,
        # so it is solved without a coarse start
        spec = {"c5": "1x4,2x4", "c2": "none"}.get(workload_name, "1x2,1x2,1x2")
    if spec == "none":
        return []
    return [tuple(int(v) for v in f.split("x")) for f in spec.split(",")]


def fp64_reference(E, torch, pcal, pobs, desc, idx, tol, leg):
    """EMD of gathers `idx` solved in FP64 far past the benchmark's stop rule (to the
    residual `tol`), in resumed legs of `leg` iterations so that progress shows.
    Returns (emd per gather, iterations, seconds, EMD change over the last leg)."""
    import dataclasses
    descs, parts_c, parts_o, off = [], [], [], 0
    for k in idx:
        nr, nt, dx, dt, o = desc[k]
        descs.append((nr, nt, dx, dt, off))
        parts_c.append(pcal[o:o + nr * nt])
        parts_o.append(pobs[o:o + nr * nt])
        off += nr * nt
    a = torch.cat(parts_c).double().contiguous()
    b = torch.cat(parts_o).double().contiguous()
    p = E.SolverParams(precision=E.F64, tol_res=tol, max_iter=leg, sweeps_per_sync=256)
    plan = E.Plan(descs, off, p)
    t0 = time.perf_counter()
    s, mass = E.emd_decompose(plan, a, b)
    u = plan.empty(2)
    emd, phi, u, info = E.emd_pdhg_solve(plan, s, u=u, mass=mass)
    done, prev = leg, None
    while True:
        torch.cuda.synchronize()
        inf = E.info_numpy(info)
        cur = emd.cpu().numpy().copy()
        log(f"fp64 reference: {done} iterations, statuses {inf['status'].tolist()}, "
            f"residual max {inf['rel_res'].max():.2e}")
        if not (inf["status"] == E.GATHER_STATUS.index("MAX_ITER")).any() or done >= 8 * leg:
            break
        prev = cur
        state = E.solver_state(plan)
        done += leg
        plan.set_params(dataclasses.replace(p, max_iter=done))
        emd, phi, u, info = E.emd_pdhg_solve_resume(plan, s, state, u, phi, mass=mass)
    el = time.perf_counter() - t0
    change = float(np.max(np.abs(cur / prev - 1))) if prev is not None else None
    plan.close()
    return cur, inf, el, change


def cpu_baseline(gathers, iters, threads):
    """The FP64 oracle, as it stands, on a bounded sample: `threads` gathers of the
    workload, `iters` fixed iterations each, one gather per host thread."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.build()
    sample = gathers[:threads]
    srcs = []
    for g in sample:
        s, _, _, _ = oracle.decompose(g.pcal.astype(np.float64), g.pobs.astype(np.float64), g.dx, g.dt)
        srcs.append((s, g))
    p = oracle.Params(max_iter=iters, tol_res=0.0, check_every=iters)

    def one(item):
        s, g = item
        r = oracle.solve(s, g.dx, g.dt, p)
        return g.cells * r.iters

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        cu = sum(ex.map(one, srcs))
    el = time.perf_counter() - t0
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": cu / el, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sample)} gathers of the workload ({sum(g.cells for g in sample)} cells), "
                      f"{iters} fixed PDHG-linesearch iterations each, one gather per thread, "
                      f"{el:.1f} s wall",
            "host": f"{model}, {os.cpu_count()} logical CPUs"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)  # each step solves the batch to the stop rule
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--tol", type=float, default=1e-5, help="relative residual stop rule")
    ap.add_argument("--max-iter", type=int, default=100000)
    ap.add_argument("--rows", type=int, default=0, help="rows per tile for every gather (0: autotune)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile height")
    ap.add_argument("--heights-from", default="", metavar="JSON",
                    help="take the per-gather tile heights from an earlier bench line")
    ap.add_argument("--ls", choices=["l2", "l1"], default="l2",
                    help="linesearch test: Euclidean (default) or the l1 norms of Algorithm 1")
    ap.add_argument("--no-f64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--f64-gathers", type=int, default=4,
                    help="gathers of the workload solved by the plain FP64 path (bounded sample)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--coarse", default="auto", metavar="FRxFT[,FRxFT...]",
                    help="coarse levels that start the timed solve, finest first, each grouping FR "
                         "receivers by FT samples of the level above ('none': a plain solve; 'auto': "
                         "1x4,2x4 for c5, none for c2, else 1x2,1x2,1x2)")
    ap.add_argument("--coarse-rows", default="8", metavar="ROWS[,ROWS...]",
                    help="tile height of the coarse levels: one for all, or one per level, finest first")
    ap.add_argument("--coarse-fixed-ips", type=int, default=3, choices=(0, 2, 3),
                    help="iterations per sweep of the fixed-step coarse levels in the legs that start "
                         "the linesearch solve from them (0: skip those legs)")
    ap.add_argument("--coarse-tol-factor", type=float, default=1.0,
                    help="stop rule of the coarse levels over the fine one's")
    ap.add_argument("--fine-only-steps", type=int, default=1,
                    help="timed steps of the same solve without the coarse start (0: skip)")
    ap.add_argument("--cpu-iters", type=int, default=60)
    ap.add_argument("--gate-gathers", type=int, default=4,
                    help="gathers whose FP32 EMD is checked against an FP64 reference (0: skip)")
    ap.add_argument("--gate-ref-tol", type=float, default=2e-7,
                    help="residual the FP64 reference is solved to")
    ap.add_argument("--fixed-steps", type=int, default=1,
                    help="timed steps of plain fixed-step PDHG, several iterations per sweep (0: skip)")
    ap.add_argument("--fixed-ips", type=int, default=3, choices=[2, 3],
                    help="iterations per sweep of the fixed-step leg")
    ap.add_argument("--fixed-rows", type=int, default=24, help="tile height of the fixed-step leg's fine plan")
    ap.add_argument("--c5-iters", type=int, default=300,
                    help="fixed-budget leg on 16 gathers of 4000 x 1600 (0: skip)")
    ap.add_argument("--c5-full", type=int, default=1,
                    help="with the fixed-budget leg, also solve that batch to the stop rule once (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (read + write) 5 times, "
                         "to scale the HBM byte counters of a profiler run")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_mib": args.copy_calibration, "launches": 5}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 (a batch "
                                   "would shard by gather across GPUs; no multi-GPU path exists)"}))
        sys.exit(2)

    import torch
    import paper_1808_07284_amd as E
    from synth import pack_batch

    gathers, wdesc = workload(args.workload)
    cells = sum(g.cells for g in gathers)
    log(f"workload {args.workload}: {len(gathers)} gathers, {cells} cells")
    pcal_h, pobs_h, desc = pack_batch(gathers, np.float32)
    dev = torch.device("cuda", 0)
    pcal = torch.from_numpy(pcal_h).to(dev)
    pobs = torch.from_numpy(pobs_h).to(dev)
    params = E.SolverParams(precision=E.F32, tol_res=args.tol, max_iter=args.max_iter,
                            ls_mode=E.LS_L1 if args.ls == "l1" else E.LS_L2)
    plan = E.Plan(desc, len(pcal_h), params)
    heights = None
    rows = None
    if args.rows:
        plan.set_tiling(args.rows)
    elif args.heights_from:
        # the per-gather heights an earlier (autotuned) run chose, to profile that run's
        # configuration without the autotuner's own sweeps
        with open(args.heights_from) as fh:
            rows = json.load(fh)["config"]["tile_rows_per_gather"]
        plan.set_gather_tiling(rows)
        heights = {str(h): rows.count(h) for h in sorted(set(rows))}
    elif not args.no_autotune:
        # tile heights per size bucket, picked by the library's autotuner (untimed setup)
        s0, _ = E.emd_decompose(plan, pcal, pobs)
        t_at = time.perf_counter()
        rows = plan.autotune(s0)
        del s0
        heights = {str(h): rows.count(h) for h in sorted(set(rows))}
        log(f"autotuned tile heights {heights} in {time.perf_counter() - t_at:.1f} s")
    bufs = {"s": plan.empty(), "phi": plan.empty(), "psi": plan.empty(),
            "mass": torch.empty(len(gathers), 3, dtype=torch.float64, device=dev),
            "emd": torch.empty(len(gathers), dtype=torch.float64, device=dev),
            "info": torch.empty(len(gathers) * E.INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)}
    levels = parse_levels(args.coarse, args.workload)
    crows = [int(v) for v in args.coarse_rows.split(",")]
    crows = crows[0] if len(crows) == 1 else crows
    mg = (E.Multigrid(plan, levels, coarse_rows=crows, coarse_tol_factor=args.coarse_tol_factor)
          if levels else None)

    # Accuracy gate (untimed): the FP32 EMD of the first gathers at the stop rule
    # against FP64 solves of them taken far past it.  If the gate fails, the stop rule
    # is tightened before the timed steps, so the rate is measured where it holds.
    GATE = 1e-5
    gate = None
    ref = None
    if args.gate_gathers > 0:
        idx = list(range(min(args.gate_gathers, len(gathers))))
        ref, ref_inf, ref_s, ref_change = fp64_reference(E, torch, pcal, pobs, desc, idx,
                                                         args.gate_ref_tol, 250000)
        gate = {"gathers": idx, "gate": GATE, "ref": "FP64 solve of the same gathers",
                "ref_tol_res": args.gate_ref_tol, "ref_iters": ref_inf["iters"].tolist(),
                "ref_seconds": round(ref_s, 1), "ref_change_last_leg": ref_change}

    def check_gate(emd_t, info_t):
        e = emd_t.cpu().numpy()[:len(ref)]
        pr = E.info_numpy(info_t)["primal"][:len(ref)]
        err = np.abs(e / ref - 1)
        perr = np.abs(pr / ref - 1)
        return float(err.max()), float(perr.max()), err

    for w in range(max(args.warmup, 1 if gate is not None else 0)):
        emd_w, info_w = run_step(E, plan, pcal, pobs, bufs, mg)
        torch.cuda.synchronize()
        log(f"warmup {w} done")
    tightened = []
    if gate is not None:
        for _ in range(3):
            err, perr, _ = check_gate(emd_w, info_w)
            log(f"gate at residual {params.tol_res:g}: EMD rel err max {err:.2e} "
                f"(objective of the flux alone {perr:.2e})")
            if err <= GATE:
                break
            tightened.append({"tol_res": params.tol_res, "emd_rel_err_max": err})
            params = dataclasses.replace(params, tol_res=params.tol_res * 0.3)
            plan.set_params(params)
            emd_w, info_w = run_step(E, plan, pcal, pobs, bufs, mg)
            torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    cell_updates = 0
    sweep_ms = 0.0
    sweeps = 0
    torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    for k in range(args.steps):
        emd, info = run_step(E, plan, pcal, pobs, bufs, mg)
        cu_k, ms_k, sw_k = step_stats(plan, mg)
        cell_updates += cu_k
        sweep_ms += ms_k
        sweeps += sw_k
        log(f"step {k}: {sw_k} sweeps, {ms_k:.1f} ms in sweeps")
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    value = cell_updates / (ms / 1e3)
    # the last step's time in sweeps per level, the fine grid first, then the coarse
    # levels finest first (HIP events the library records)
    level_ms = [round(p.query()["last_sweep_ms"], 1)
                for p in [plan] + ([lv[0] for lv in mg.levels] if mg is not None else [])]
    inf = E.info_numpy(info)
    emd32 = emd.cpu().numpy().copy()
    if gate is not None:
        err, perr, errs = check_gate(emd, info)
        gate.update({"stop_rule": f"||div u + s||/||s|| <= {params.tol_res:g}",
                     "emd_rel_err_vs_ref": [float(x) for x in errs], "emd_rel_err_vs_ref_max": err,
                     "objective_rel_err_vs_ref_max": perr, "passed": err <= GATE,
                     "tightened_from": tightened})
        log(f"gate (timed solves): EMD rel err max {err:.2e}, objective {perr:.2e}")
    log(f"f32: {value:.3e} cell-updates/s, {ms_per_step:.1f} ms/step (wall {wall:.1f} s), "
        f"iters min/mean/max {inf['iters'].min()}/{inf['iters'].mean():.0f}/{inf['iters'].max()}, "
        f"statuses {np.bincount(inf['status'], minlength=7).tolist()}")

    # dominant kernel: the fused sweep; algorithmic bytes per launch = 36 B x cells
    # updated in that launch, timed with HIP events the library records on this stream
    algo_bytes = BYTES_PER_CELL_ITER["f32"] * cell_updates
    achieved = algo_bytes / (sweep_ms / 1e3) / 1e9 if sweep_ms > 0 else 0.0
    traffic = None
    measured = sweep_source_digest() == MEASURED_TRAFFIC["sweep_source_sha256_16"]
    if args.ls == "l2" and measured:
        traffic = round(MEASURED_TRAFFIC["ratio"]["k_sweep<float, false>"] * achieved, 1)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"k_sweep<float, {'true' if args.ls == 'l1' else 'false'}>", "launches": int(sweeps),
                # one sweep = one launch per chain (the graph runs the chains
                # concurrently); the figures are per sweep of the whole batch
                "avg_launch_us": round(sweep_ms * 1e3 / max(sweeps, 1), 2),
                "algo_bytes_per_launch": int(algo_bytes / max(sweeps, 1))}

    extra = {}
    # the one-pass kernels around the solve, timed on their own: decompose (reads
    # Pcal and Pobs, writes s: 12 B per cell at least; it makes two passes, 20 B) and
    # the adjoint source (reads phi, writes psi: 8 B; two passes, 12 B); and a plain
    # device copy of 1 GiB as the measured bandwidth ceiling
    reps = 5
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    big = torch.ones((1 << 30) // 4, dtype=torch.float32, device=dev)
    big2 = torch.empty_like(big)
    big2.copy_(big)
    torch.cuda.synchronize()
    ev[0].record(stream)
    for _ in range(reps):
        E.emd_decompose(plan, pcal, pobs, s_out=bufs["s"], mass_out=bufs["mass"])
    ev[1].record(stream)
    for _ in range(reps):
        E.emd_adjoint_source(plan, bufs["phi"], pcal, pobs, bufs["mass"], psi_out=bufs["psi"])
    ev[2].record(stream)
    for _ in range(reps):
        big2.copy_(big)
    ev[3].record(stream)
    torch.cuda.synchronize()
    t_dec = ev[0].elapsed_time(ev[1]) / reps
    t_adj = ev[1].elapsed_time(ev[2]) / reps
    copy_gbs = 2 * big.numel() * 4 / (ev[2].elapsed_time(ev[3]) / reps / 1e3) / 1e9
    del big, big2
    extra["one_pass_kernels"] = {
        "decompose": {"ms": round(t_dec, 3), "GB/s_at_12B_per_cell": round(12 * cells / t_dec / 1e6, 1)},
        "adjoint": {"ms": round(t_adj, 3), "GB/s_at_8B_per_cell": round(8 * cells / t_adj / 1e6, 1)}}
    if mg is not None:
        # the grid transfers between the fine grid and its first coarse level: the
        # restriction of one field (reads the fine field, writes the coarse one: 4 B per
        # fine and per coarse cell) and the prolongation of u and phi (12 B per coarse
        # and per fine cell)
        cp, fr, ft = mg.levels[0]
        nc = cp.batch_len
        xr = cp.empty()
        uc, pc = cp.empty(2).normal_(), cp.empty().normal_()
        uf, pf = plan.empty(2), plan.empty()
        evt = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        E.restrict(plan, cp, fr, ft, pcal, out=xr)
        E.prolong(cp, plan, fr, ft, uc, pc, u_out=uf, phi_out=pf)
        evt[0].record(stream)
        for _ in range(reps):
            E.restrict(plan, cp, fr, ft, pcal, out=xr)
        evt[1].record(stream)
        for _ in range(reps):
            E.prolong(cp, plan, fr, ft, uc, pc, u_out=uf, phi_out=pf)
        evt[2].record(stream)
        torch.cuda.synchronize()
        t_res = evt[0].elapsed_time(evt[1]) / reps
        t_pro = evt[1].elapsed_time(evt[2]) / reps
        extra["one_pass_kernels"]["restrict_fine_level"] = {
            "ms": round(t_res, 3), "GB/s_at_4B_per_fine_and_coarse_cell": round(4 * (cells + nc) / t_res / 1e6, 1)}
        extra["one_pass_kernels"]["prolong_fine_level"] = {
            "ms": round(t_pro, 3), "GB/s_at_12B_per_fine_and_coarse_cell": round(12 * (cells + nc) / t_pro / 1e6, 1)}
        del xr, uc, pc, uf, pf
    roofline["measured_copy_GBs"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(achieved / copy_gbs, 4)
    log(f"decompose {t_dec:.3f} ms, adjoint {t_adj:.3f} ms, 1 GiB copy {copy_gbs:.0f} GB/s")

    if not args.no_f64:
        # the plain FP64 solve: one gather per plan (its own launch sequence), to the
        # same stop rule, on a bounded sample of the workload's gathers
        p64 = E.SolverParams(precision=E.F64, tol_res=params.tol_res, max_iter=args.max_iter)
        pc64 = pcal.double()
        po64 = pobs.double()
        sample = list(range(min(args.f64_gathers, len(gathers))))
        emd64 = np.zeros(len(sample))
        cu64 = 0
        el64 = 0.0
        for j, k in enumerate(sample):
            nr, nt, dx, dt, off = desc[k]
            pl = E.Plan([(nr, nt, dx, dt, 0)], nr * nt, p64)
            mg64 = E.Multigrid(pl, levels, coarse_tol_factor=args.coarse_tol_factor) if levels else None
            a = pc64[off:off + nr * nt]
            b = po64[off:off + nr * nt]
            b64 = {"s": pl.empty(), "phi": pl.empty(), "psi": pl.empty(),
                   "mass": torch.empty(1, 3, dtype=torch.float64, device=dev),
                   "emd": torch.empty(1, dtype=torch.float64, device=dev),
                   "info": torch.empty(E.INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)}
            torch.cuda.synchronize()
            t64 = time.perf_counter()
            e, _ = run_step(E, pl, a, b, b64, mg64)
            torch.cuda.synchronize()
            el64 += time.perf_counter() - t64
            cu64 += step_stats(pl, mg64)[0]
            emd64[j] = float(e.cpu()[0])
            if mg64 is not None:
                mg64.close()
            pl.close()
        rel = np.abs(emd32[sample] - emd64) / np.abs(emd64)
        extra["plain_f64"] = {"what": "the same solve (coarse start, fused sweep) in FP64, one gather per "
                                      "plan and launch sequence, on the first gathers of the workload",
                              "value": cu64 / el64, "unit": "cell-updates/s", "seconds": round(el64, 2),
                              "gathers": len(sample), "stop_rule": f"{params.tol_res:g}",
                              "speedup_f32_batched": round(value / (cu64 / el64), 2),
                              "emd_rel_diff_f32_vs_f64_max": float(rel.max())}
        if ref is not None:
            m = min(len(ref), len(sample))
            extra["plain_f64"]["emd_rel_err_vs_ref_max"] = float(np.max(np.abs(emd64[:m] / ref[:m] - 1)))
        log(f"plain f64 ({len(sample)} gathers): {cu64 / el64:.3e} cell-updates/s in {el64:.1f} s; "
            f"EMD rel diff f32 vs f64 max {rel.max():.2e}")

    cpu = None
    if not args.no_cpu:
        threads = max(1, min(16, os.cpu_count() or 1))
        cpu = cpu_baseline(gathers, args.cpu_iters, threads)
        log(f"cpu oracle: {cpu['value']:.3e} cell-updates/s on {threads} threads")

    if args.fixed_steps > 0:
        # Plain PDHG with the fixed steps alpha_1, beta_1 = delta alpha_1 (Section 2.2
        # before the linesearch): no per-iteration decision, so one sweep runs K
        # iterations (read u, phi, s; write u, phi: 28 B per cell per sweep, 28 / K per
        # iteration), to the same stop rule, checked every 3K iterations, with its own
        # roofline and accuracy against the reference
        K = args.fixed_ips
        pf = dataclasses.replace(params, ls_mode=E.LS_FIXED, iters_per_sweep=K, check_every=3 * K,
                                 max_iter=4 * args.max_iter)
        planf = E.Plan(desc, len(pcal_h), pf)
        planf.set_tiling(args.fixed_rows)
        mgf = E.Multigrid(planf, levels, coarse_rows=16,
                          coarse_tol_factor=args.coarse_tol_factor) if levels else None
        run_step(E, planf, pcal, pobs, bufs, mgf)  # captures the graphs
        torch.cuda.synchronize()
        cuf, msf, swf = 0, 0.0, 0
        e0.record(stream)
        for _ in range(args.fixed_steps):
            emd_f, info_f = run_step(E, planf, pcal, pobs, bufs, mgf)
            cu_k, ms_k, sw_k = step_stats(planf, mgf)
            cuf += cu_k
            msf += ms_k
            swf += sw_k
        e1.record(stream)
        torch.cuda.synchronize()
        stepf = e0.elapsed_time(e1) / args.fixed_steps
        inff = E.info_numpy(info_f)
        kname = f"k_sweep{K}<float>"
        achf = 28.0 / K * cuf / (msf / 1e3) / 1e9
        extra["plain_pdhg_fixed_steps"] = {
            "what": f"plain PDHG with fixed steps, {K} iterations per HBM pass, FP32, same coarse start "
                    "and stop rule",
            "iterations_per_sweep": K, "tile_rows": args.fixed_rows,
            "value": cuf / args.fixed_steps / (stepf / 1e3), "unit": "cell-updates/s",
            "ms_per_step": round(stepf, 3), "speedup_vs_linesearch_step": round(ms_per_step / stepf, 3),
            "iters_mean": float(inff["iters"].mean()), "iters_max": int(inff["iters"].max()),
            "statuses": np.bincount(inff["status"], minlength=7).tolist(),
            "roofline": {"bound": "hbm", "achieved": round(achf, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achf / HBM_PEAK_GBS, 4), "kernel": kname,
                         "traffic": round(MEASURED_TRAFFIC["ratio"][kname] * achf, 1)
                         if measured and kname in MEASURED_TRAFFIC["ratio"] else None,
                         "launches": int(swf), "avg_launch_us": round(msf * 1e3 / max(swf, 1), 2),
                         "algo_bytes_per_launch": int(28.0 / K * cuf / max(swf, 1))}}
        if ref is not None:
            ef = emd_f.cpu().numpy()[:len(ref)]
            extra["plain_pdhg_fixed_steps"]["emd_rel_err_vs_ref_max"] = float(np.max(np.abs(ef / ref - 1)))
        log(f"fixed steps, {K} iterations per sweep: {stepf:.1f} ms/step ({ms_per_step / stepf:.2f}x the "
            f"linesearch), iters mean {inff['iters'].mean():.0f}, sweeps at {achf:.0f} GB/s")
        if mgf is not None:
            mgf.close()
        planf.close()

    if args.c5_iters > 0 and args.workload != "c5":
        # the >2 GB workload at a fixed budget (the paper's experiments run 100-200
        # iterations per gather): 16 gathers of 4000 x 1600, decompose -> solve ->
        # adjoint per step, with the sweep's own roofline
        g5, w5 = workload("c5")
        pc5_h, po5_h, desc5 = pack_batch(g5, np.float32)
        del g5
        pc5 = torch.from_numpy(pc5_h).to(dev)
        po5 = torch.from_numpy(po5_h).to(dev)
        del pc5_h, po5_h
        p5 = E.SolverParams(precision=E.F32, tol_res=0.0, max_iter=args.c5_iters, check_every=args.c5_iters)
        plan5 = E.Plan(desc5, pc5.numel(), p5)
        b5 = {"s": plan5.empty(), "phi": plan5.empty(), "psi": plan5.empty(),
              "mass": torch.empty(len(desc5), 3, dtype=torch.float64, device=dev),
              "emd": torch.empty(len(desc5), dtype=torch.float64, device=dev),
              "info": torch.empty(len(desc5) * E.INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)}
        run_step(E, plan5, pc5, po5, b5)  # captures the graph
        torch.cuda.synchronize()
        reps5, cu5, ms5, sw5 = 3, 0, 0.0, 0
        e0.record(stream)
        for _ in range(reps5):
            run_step(E, plan5, pc5, po5, b5)
            q5 = plan5.query()
            cu5 += q5["last_cell_updates"]
            ms5 += q5["last_sweep_ms"]
            sw5 += q5["last_sweeps"]
        e1.record(stream)
        torch.cuda.synchronize()
        step5 = e0.elapsed_time(e1) / reps5
        ach5 = BYTES_PER_CELL_ITER["f32"] * cu5 / (ms5 / 1e3) / 1e9
        extra["large_fixed_budget"] = {
            "workload": w5, "iterations": args.c5_iters, "steps": reps5,
            "value": cu5 / reps5 / (step5 / 1e3), "unit": "cell-updates/s", "ms_per_step": round(step5, 3),
            "roofline": {"bound": "hbm", "achieved": round(ach5, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach5 / HBM_PEAK_GBS, 4), "kernel": "k_sweep<float, false>",
                         "launches": int(sw5), "avg_launch_us": round(ms5 * 1e3 / max(sw5, 1), 2),
                         "algo_bytes_per_launch": int(BYTES_PER_CELL_ITER["f32"] * cu5 / max(sw5, 1))}}
        log(f"16 x 4000 x 1600, {args.c5_iters} iterations: {step5:.1f} ms/step, sweeps at "
            f"{ach5:.0f} GB/s ({ach5 / HBM_PEAK_GBS:.3f} of peak)")
        plan5.close()
        del b5
        if args.c5_full:
            # the whole misfit of that batch and its adjoint source, to the stop rule,
            # started coarse-to-fine (1 x 4, then 2 x 4): one run, its graph captures
            # included (they are a few ms of it).  Its coarsest level needs up to ~330k
            # iterations, hence a budget of its own.
            p5f = E.SolverParams(precision=E.F32, tol_res=args.tol, max_iter=C5_FULL_MAX_ITER)
            plan5f = E.Plan(desc5, pc5.numel(), p5f)
            lv5 = parse_levels("auto", "c5")
            mg5 = E.Multigrid(plan5f, lv5, coarse_tol_factor=args.coarse_tol_factor)
            b5f = {"s": plan5f.empty(), "phi": plan5f.empty(), "psi": plan5f.empty(),
                   "mass": torch.empty(len(desc5), 3, dtype=torch.float64, device=dev),
                   "emd": torch.empty(len(desc5), dtype=torch.float64, device=dev),
                   "info": torch.empty(len(desc5) * E.INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)}
            torch.cuda.synchronize()
            e0.record(stream)
            _, info5 = run_step(E, plan5f, pc5, po5, b5f, mg5)
            e1.record(stream)
            torch.cuda.synchronize()
            ms5f = e0.elapsed_time(e1)
            cu5f, msw5f, sw5f = step_stats(plan5f, mg5)
            inf5 = E.info_numpy(info5)
            ach5f = BYTES_PER_CELL_ITER["f32"] * cu5f / (msw5f / 1e3) / 1e9
            extra["large_full_misfit"] = {
                "workload": w5, "what": "decompose -> solve to the stop rule -> adjoint source, one run",
                "stop_rule": f"||div u + s||/||s|| <= {args.tol:g}",
                "coarse_levels": ",".join(f"{a}x{b}" for a, b in lv5),
                "coarse_stop_rule": f"{args.tol * args.coarse_tol_factor:g}",
                "ms": round(ms5f, 1), "value": cu5f / (ms5f / 1e3), "unit": "cell-updates/s",
                "fine_iters_mean": float(inf5["iters"].mean()), "fine_iters_max": int(inf5["iters"].max()),
                "coarse_iters_max": [int(E.info_numpy(i)["iters"].max()) for i in mg5.last_info],
                "statuses": np.bincount(inf5["status"], minlength=7).tolist(),
                "roofline": {"bound": "hbm", "achieved": round(ach5f, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(ach5f / HBM_PEAK_GBS, 4), "kernel": "k_sweep<float, false>",
                             "launches": int(sw5f), "avg_launch_us": round(msw5f * 1e3 / max(sw5f, 1), 2),
                             "algo_bytes_per_launch": int(BYTES_PER_CELL_ITER["f32"] * cu5f / max(sw5f, 1))}}
            log(f"16 x 4000 x 1600 to the stop rule: {ms5f / 1e3:.2f} s, {cu5f / (ms5f / 1e3):.3e} cell-updates/s, "
                f"fine iters mean {inf5['iters'].mean():.0f} max {inf5['iters'].max()}, "
                f"statuses {np.bincount(inf5['status'], minlength=7).tolist()}")
            mg5.close()
            if args.coarse_fixed_ips > 0:
                # the same misfit with the coarse levels solved by plain fixed-step PDHG
                emd5 = b5f["emd"].cpu().numpy().copy()
                mg5h = E.Multigrid(plan5f, lv5, coarse_tol_factor=args.coarse_tol_factor,
                                   coarse_iters_per_sweep=args.coarse_fixed_ips)
                torch.cuda.synchronize()
                e0.record(stream)
                _, info5h = run_step(E, plan5f, pc5, po5, b5f, mg5h)
                e1.record(stream)
                torch.cuda.synchronize()
                ms5h = e0.elapsed_time(e1)
                inf5h = E.info_numpy(info5h)
                rel5 = np.abs(b5f["emd"].cpu().numpy() / emd5 - 1)
                extra["large_full_misfit_fixed_step_coarse"] = {
                    "what": f"the same misfit, the coarse levels solved by plain PDHG with fixed steps, "
                            f"{args.coarse_fixed_ips} iterations per sweep, one run",
                    "ms": round(ms5h, 1), "speedup_vs_linesearch_coarse": round(ms5f / ms5h, 3),
                    "fine_iters_mean": float(inf5h["iters"].mean()), "fine_iters_max": int(inf5h["iters"].max()),
                    "coarse_iters_max": [int(E.info_numpy(i)["iters"].max()) for i in mg5h.last_info],
                    "statuses": np.bincount(inf5h["status"], minlength=7).tolist(),
                    "emd_rel_diff_vs_linesearch_coarse_max": float(rel5.max())}
                log(f"16 x 4000 x 1600, fixed-step coarse levels: {ms5h / 1e3:.2f} s ({ms5f / ms5h:.2f}x), "
                    f"EMD rel diff max {rel5.max():.2e}")
                mg5h.close()
            plan5f.close()
            del b5f
        del pc5, po5

    if args.fine_only_steps > 0 and mg is not None:
        # the same step with the solve started cold on the fine grid: the residual rule
        # certifies feasibility, not optimality, and without the coarse start a few
        # gathers stop feasible but above the optimum (see the accuracy notes)
        run_step(E, plan, pcal, pobs, bufs)
        torch.cuda.synchronize()
        cuo, mso = 0, 0.0
        e0.record(stream)
        for _ in range(args.fine_only_steps):
            emd_o, info_o = run_step(E, plan, pcal, pobs, bufs)
            cu_k, ms_k, _ = step_stats(plan)
            cuo += cu_k
            mso += ms_k
        e1.record(stream)
        torch.cuda.synchronize()
        stepo = e0.elapsed_time(e1) / args.fine_only_steps
        io = E.info_numpy(info_o)
        rel_o = np.abs(emd_o.cpu().numpy() / emd32 - 1)
        extra["fine_only_start"] = {
            "what": "the same solve started cold on the fine grid", "ms_per_step": round(stepo, 3),
            "value": cuo / args.fine_only_steps / (stepo / 1e3), "unit": "cell-updates/s",
            "coarse_start_speedup": round(stepo / ms_per_step, 3),
            "iters_mean": float(io["iters"].mean()), "iters_max": int(io["iters"].max()),
            "emd_rel_diff_vs_coarse_start_max": float(rel_o.max())}
        if ref is not None:
            extra["fine_only_start"]["emd_rel_err_vs_ref_max"] = float(
                np.max(np.abs(emd_o.cpu().numpy()[:len(ref)] / ref - 1)))
        log(f"cold fine start: {stepo:.1f} ms/step (the coarse start is {stepo / ms_per_step:.2f}x faster), "
            f"iters mean {io['iters'].mean():.0f}, EMD rel diff vs coarse start max {rel_o.max():.2e}")

    if args.coarse_fixed_ips > 0 and mg is not None:
        # the same linesearch solve on the fine grid, started from coarse levels solved
        # by plain PDHG with fixed steps, K iterations per sweep: a coarse level only
        # supplies a start, and the fixed-step sweeps move fewer bytes per iteration
        Kc = args.coarse_fixed_ips
        # coarse levels at the rule the headline's coarse levels use (a failed gate
        # tightens only the fine plan's)
        mgh = E.Multigrid(plan, levels, params=dataclasses.replace(params, tol_res=args.tol),
                          coarse_tol_factor=args.coarse_tol_factor, coarse_iters_per_sweep=Kc)
        run_step(E, plan, pcal, pobs, bufs, mgh)  # captures the coarse plans' graphs
        torch.cuda.synchronize()
        e0.record(stream)
        emd_h, info_h = run_step(E, plan, pcal, pobs, bufs, mgh)
        e1.record(stream)
        torch.cuda.synchronize()
        steph = e0.elapsed_time(e1)
        ih = E.info_numpy(info_h)
        rel_h = np.abs(emd_h.cpu().numpy() / emd32 - 1)
        extra["fixed_step_coarse_start"] = {
            "what": f"the same linesearch solve on the fine grid, its coarse levels solved by plain PDHG "
                    f"with fixed steps, {Kc} iterations per sweep", "ms_per_step": round(steph, 3),
            "speedup_vs_linesearch_coarse": round(ms_per_step / steph, 3),
            "sweep_ms_per_level": [round(p.query()["last_sweep_ms"], 1)
                                   for p in [plan] + [lv[0] for lv in mgh.levels]],
            "fine_iters_mean": float(ih["iters"].mean()), "fine_iters_max": int(ih["iters"].max()),
            "coarse_iters_mean": [float(E.info_numpy(i)["iters"].mean()) for i in mgh.last_info],
            "statuses": np.bincount(ih["status"], minlength=7).tolist(),
            "emd_rel_diff_vs_linesearch_coarse_max": float(rel_h.max())}
        if ref is not None:
            extra["fixed_step_coarse_start"]["emd_rel_err_vs_ref_max"] = float(
                np.max(np.abs(emd_h.cpu().numpy()[:len(ref)] / ref - 1)))
        log(f"fixed-step coarse start: {steph:.1f} ms/step ({ms_per_step / steph:.2f}x), "
            f"EMD rel diff vs linesearch coarse levels max {rel_h.max():.2e}")
        mgh.close()

    out = {"metric": "PDHG cell-updates/s to 1e-5 rel EMD err, batched FP32 vs plain FP64; % HBM peak",
           "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": wdesc, "gathers": len(gathers), "cells": cells,
                      "stop_rule": f"||div u + s||/||s|| <= {params.tol_res:g}", "max_iter": args.max_iter,
                      "linesearch": args.ls,
                      "coarse_levels": ",".join(f"{a}x{b}" for a, b in levels) or "none",
                      "coarse_stop_rule": f"{args.tol * args.coarse_tol_factor:g}" if levels else None,
                      "coarse_tile_rows": crows if levels else None,
                      "sweep_ms_per_level": level_ms,
                      "fine_iters_mean": float(inf["iters"].mean()), "fine_iters_max": int(inf["iters"].max()),
                      "coarse_iters_mean": [float(E.info_numpy(i)["iters"].mean()) for i in mg.last_info]
                      if mg is not None else [],
                      "tile_rows": heights if heights else (args.rows or plan.query()["rows_per_tile"]),
                      "tile_rows_per_gather": plan.gather_tiling()},
           "roofline": roofline, "cpu_baseline": cpu}
    if gate is not None:
        out["emd_rel_err_vs_ref_max"] = gate["emd_rel_err_vs_ref_max"]
        out["accuracy_gate"] = gate
    out.update(extra)
    print(json.dumps(out))
    if mg is not None:
        mg.close()
    plan.close()


if __name__ == "__main__":
    main()
