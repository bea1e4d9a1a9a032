#!/usr/bin/env python3
"""Throughput of the PIC-MCC step on one MI355X.

One step is the whole hot path: Fowler-Nordheim emission, gather + leapfrog
push + boundary removal + fixed-point deposit + binning, Monte Carlo
collisions (elastic, impact ionization, charge exchange), field ionization,
products, and the Poisson solve to a relative residual of 1e-8 followed by the
node field. The workload is the GPU-scale configuration: a 128 x 128 x 512
node grid at 1 nm around a Cu tip (r = 10 nm, H = 100 nm, 10 GV/m at the
apex) with 20 M particles stored as FP32 SoA (16 M electrons at kT = 5 eV,
1 M Cu+ at 1 eV, 3 M Cu at 0.1 eV, uniform over the vacuum box), synthetic
256-node cross-section tables, dt = 5e-17 s. Inputs are generated on the host,
copied to the GPU and resident in HBM before timing starts.

Prints one JSON line: the throughput (value, ms_per_step), the roofline of
the dominant kernel (k_pcg_b: HIP-event time against the 8 TB/s HBM peak,
with the HBM bytes measured by rocprofv3 counters when a summary is present),
the CPU oracle's rate on a bounded sample, and the learned warm start's
iteration counts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (push+deposit+MCC) + CG iters to 1e-8: learned vs plain"
HBM_PEAK_GBS = 8000.0


def workload(name, load=None):
    """Configuration, counts, temperatures and load region of a workload;
    load overrides the region ("box": uniform over the vacuum box, the
    default of gpu_scale; "near_tip": clustered in rho <= 3 r, z < H + 2 r)."""
    import numpy as np
    from paper_2402_08404_amd import workloads as W
    if name == "gpu_scale":
        cfg = W.gpu_scale()
        counts = (16_000_000, 1_000_000, 3_000_000)
        kT = (5.0, 1.0, 0.1)
        region = load or "box"
    elif name == "tiny":
        cfg = W.tiny()
        counts = (20000, 200, 2000)
        kT = None
        region = "near_tip"
    else:
        raise SystemExit("unknown workload " + name)
    return cfg, counts, kT, region, np


def push_bytes(n_particles, n_nodes, fp32=True):
    """Algorithmic bytes of one push launch: per particle read x, v and the id,
    write x, v, the cell key and the slot; per node one read of the field
    (4 values) and one write of the int64 charge."""
    t = 4 if fp32 else 8
    per_p = 6 * t + 4 + 6 * t + 8
    per_n = 4 * t + 8
    return per_p * n_particles + per_n * n_nodes


# Algorithmic bytes per node of the solver kernels on the finest level: FP64
# Krylov vectors (x, r, p, q), FP32 multigrid vectors (z and the smoother's
# iterates), uint8 node type; what each launch must read and write once.
SOLVER_BYTES_PER_NODE = {
    "cg_a": 29,           # read z (4), p_old (8), type (1); write p_new (8), q (8)
    "cg_b": 48,           # read p, x, r, q (32); write x, r (16)
    "mg_first": 13,       # read b (8), type (1); write x (4)
    "mg_restrict": 17,    # residual: read x (4), b (8), type (1); write r (4)
    "mg_corr": 9.5,       # prolongation: read x (4), type (1), coarse x (4 per 8 nodes); write x (4)
    "mg_last": 17,        # read x (4), b (8), type (1); write z (4)
}


# Device symbol of each timed kernel (for the rocprofv3 traffic summary).
KERNEL_SYMBOLS = {
    "push_electrons": "k_push<float, 0, true>",
    "cg_a": "k_pcg_a2",
    "cg_b": "k_pcg_b<double>",
    "mg_first": "k_mg_fine_sweep<1, false, double>",
    "mg_restrict": "k_mg_fine_sweep<3, false, double>",
    "mg_corr": "k_mg_prolong2",
    "mg_last": "k_mg_fine_sweep<0, true, double>",
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_gpu_scale.json")


def pmc_summary(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_mib, out_path):
    """HBM bytes per dispatch of every kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch, median over dispatches of the
    largest grid of each kernel), each scaled by what the same counter reads
    for a plain device copy of copy_mib MiB."""
    import csv
    import statistics

    def per_kernel(path):
        d = {}
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").strip()
            d.setdefault((name, int(r["Grid_Size"])), []).append(float(r["Counter_Value"]))
        best, grids = {}, {}
        for (name, grid), v in d.items():
            grids.setdefault(name, {})[grid] = statistics.median(v)
            if name not in best or grid > best[name][0]:
                best[name] = (grid, statistics.median(v), len(v))
        return best, grids

    def copy_kib(path):
        v = [float(r["Counter_Value"]) for r in csv.DictReader(open(path)) if "copyBuffer" in r["Kernel_Name"]
             or "copy" in r["Kernel_Name"].lower()]
        return statistics.median(v)

    f_fetch = copy_mib * 1024.0 / copy_kib(copy_fetch_csv)
    f_write = copy_mib * 1024.0 / copy_kib(copy_write_csv)
    (fe, fe_g), (wr, wr_g) = per_kernel(fetch_csv), per_kernel(write_csv)
    out = {"fetch_scale": f_fetch, "write_scale": f_write, "copy_mib": copy_mib, "kernels": {}}
    for name in sorted(set(fe) & set(wr)):
        by_grid = {str(gr): 1024.0 * (fe_g[name][gr] * f_fetch + wr_g[name][gr] * f_write)
                   for gr in sorted(set(fe_g[name]) & set(wr_g[name]))}
        out["kernels"][name] = {"grid": fe[name][0], "fetch_kib": fe[name][1], "write_kib": wr[name][1],
                                "dispatches": fe[name][2],
                                "bytes": 1024.0 * (fe[name][1] * f_fetch + wr[name][1] * f_write),
                                "bytes_by_grid": by_grid}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    return out


def trace_summary(trace_csv, min_us=10.0):
    """Per-launch durations of the step kernels from a rocprofv3 --kernel-trace
    CSV: average over all launches and over the launches longer than min_us
    (a solve replays its iterations in captured chunks, so some launches of the
    solver kernels come after convergence and return at once)."""
    import csv
    import statistics
    rows = list(csv.DictReader(open(trace_csv)))
    res = {}
    for sym in list(KERNEL_SYMBOLS.values()) + ["k_mcc_small<float>", "k_mcc_cells<float>", "k_mg_sweep_z<false>",
                                                  "k_mg_restrict2z"]:
        name = "pic::" + sym
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows
             if r["Kernel_Name"].replace("void ", "").startswith(name + "(") or
             r["Kernel_Name"].replace("void ", "") == name]
        w = [x for x in d if x > min_us]
        res[name] = {"launches": len(d), "avg_us": sum(d) / max(len(d), 1), "working": len(w),
                     "working_avg_us": sum(w) / max(len(w), 1), "working_median_us": statistics.median(w) if w else 0.0}
    return res


def measured_traffic(kernel: str):
    """Scaled HBM bytes per launch of a kernel from the committed summary, or None."""
    sym = KERNEL_SYMBOLS.get(kernel)
    if not sym or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    for name, v in t["kernels"].items():
        if name.endswith(sym):
            return v["bytes"]
    return None


def _cpu_worker(arg):
    """One single-threaded oracle process of the CPU baseline: set up its
    sample, wait for the others, then time its steps."""
    cfg_name, load, sub, steps, seed, barrier = arg
    import oracle
    from paper_2402_08404_amd import workloads as W
    cfg, counts, kT, region, _ = workload(cfg_name, load)
    o = oracle.Oracle(cfg, laplace=False)
    o.load(W.initial_load(cfg, counts=sub, kT_eV=kT, region=region, seed=seed))
    o.set_phi(W.synthetic_potential(cfg, o.V0))
    n = sum(s.n for s in o.sp)
    barrier.wait()
    t0 = time.perf_counter()
    for _ in range(steps):
        o.push()
        o.collide()
        o.deposit()
        o.step_no += 1
    return n, time.perf_counter() - t0


def cpu_baseline(cfg_name, sample, steps, np, procs=0, load=None):
    """The CPU oracle (FP64, single-threaded C) on a bounded sample of the same
    workload, run as `procs` concurrent processes (default: every host core
    up to 16), each on its own sample of `sample` particles with the same
    species mix and distributions on the same grid, timed over `steps` steps
    of push, collisions and deposit; the rate is the total of the processes
    over the slowest one's time. The oracle's Poisson solve is left out (a
    solve of the 128 x 128 x 512 grid takes minutes on one core); a smooth
    synthetic potential stands in for the field. Runs before the GPU is
    touched (the processes are forked)."""
    import multiprocessing as mp
    cfg, counts, kT, region, _ = workload(cfg_name, load)
    ncpu = os.cpu_count() or 1
    procs = procs or min(16, ncpu)
    frac = sample / sum(counts)
    sub = tuple(int(round(c * frac)) for c in counts)
    ctx = mp.get_context("fork")
    barrier = ctx.Manager().Barrier(procs)
    with ctx.Pool(procs) as pool:
        res = pool.map(_cpu_worker, [(cfg_name, load, sub, steps, cfg.seed + 7 + k, barrier) for k in range(procs)])
    n_tot = sum(n for n, _ in res)
    t_max = max(t for _, t in res)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n_tot * steps / t_max, "unit": "particle-steps/s", "cores": procs, "kind": "oracle",
            "host": {"nproc": ncpu, "model": model},
            "sample": f"{procs} processes of the single-threaded oracle, each {res[0][0]} particles ({sub[0]} e, "
                      f"{sub[1]} Cu+, {sub[2]} Cu) of the same workload on the same grid, {steps} steps of "
                      f"push+collisions+deposit, synthetic potential, solve excluded; slowest process "
                      f"{t_max:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gpu_scale", choices=["gpu_scale", "tiny"])
    ap.add_argument("--load", default=None, choices=["box", "near_tip"],
                    help="gpu_scale's load: uniform over the box (default) or clustered near the tip")
    ap.add_argument("--solver", default="mgcg", choices=["cg", "mgcg", "mixed"])
    ap.add_argument("--sort-every", type=int, default=0,
                    help="reorder period of the particle arrays (0: the tuned value for this grid, else 16)")
    ap.add_argument("--stencil-blocks", type=int, default=0, help="override the tuned block count of the solver kernels")
    ap.add_argument("--step-guess", type=int, default=1, choices=[0, 1],
                    help="step-solve guess: 0 previous potential, 1 linear extrapolation in time")
    ap.add_argument("--cpu-sample", type=int, default=1_500_000, help="particles per oracle process")
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--cpu-procs", type=int, default=0, help="oracle processes of the CPU baseline (0: cores, <= 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-zero-solve", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned warm-start leg (training on pairs of this run, then iteration counts)")
    ap.add_argument("--learned-pairs", type=int, default=16)
    ap.add_argument("--learned-iters", type=int, default=300)
    ap.add_argument("--prof-steps", type=int, default=0,
                    help="steps of the profiled replay (per-phase and per-kernel HIP-event timings; 0: as many as "
                         "the timed steps)")
    ap.add_argument("--unet", action="store_true",
                    help="time the warm-start network (forward, and forward + backward + Adam) at 1 x 512 x 128 x 128")
    ap.add_argument("--learned-experiment", action="store_true",
                    help="the learned warm-start experiment on the tiny workload's shape: pairs from plain runs at "
                         "6 ... 14 GV/m, 7 and 13 GV/m held out, then iterations to 1e-8 from each guess")
    ap.add_argument("--le-pairs", type=int, default=20000, help="training and held-out pairs of the experiment")
    ap.add_argument("--le-iters", type=int, default=4000, help="Adam steps of the experiment")
    ap.add_argument("--le-batch", type=int, default=16, help="mini-batch of the experiment")
    ap.add_argument("--batch", action="store_true",
                    help="the batched field sweep (16 instances at 6.0 ... 13.5 GV/m, 1 M - 40 M particles) instead")
    ap.add_argument("--batch-scale", type=float, default=1.0, help="scale factor of the sweep's particle counts")
    ap.add_argument("--autotune", action="store_true", help="with --batch: autotune first and store the choices")
    ap.add_argument("--batch-compare", action="store_true",
                    help="with --batch: also time the same steps with the instances stepped one after another")
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_2402_08404_amd", "tuning.json"))
    ap.add_argument("--rz", action="store_true",
                    help="the axisymmetric variant on the paper's geometry: every stage of its step")
    ap.add_argument("--rz-scale", type=float, default=1.0, help="scale factor of the axisymmetric particle counts")
    ap.add_argument("--rz-iters", action="store_true", help="with --rz: read the CG iterations after every step")
    ap.add_argument("--rz-sort-every", type=int, default=16, help="with --rz: reorder period of the particles")
    ap.add_argument("--pmc-out", default=TRAFFIC_FILE, help="where --pmc-summary writes its JSON")
    ap.add_argument("--pmc-summary", nargs=5, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV",
                                                        "COPY_MIB"),
                    help="write the HBM traffic summary of rocprofv3 --pmc runs to profiles/ and exit")
    ap.add_argument("--trace-summary", metavar="KERNEL_TRACE_CSV",
                    help="print the per-launch durations of the step kernels in a rocprofv3 kernel trace and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (the reference kernel that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters to bytes) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); a multi-GPU run is not built "
              "(the intended layout: one process per GPU, the grid split into z-slabs)", file=sys.stderr)
        sys.exit(2)

    if args.pmc_summary:
        a = args.pmc_summary
        out = pmc_summary(a[0], a[1], a[2], a[3], float(a[4]), args.pmc_out)
        print(json.dumps({k: round(v["bytes"] / 1e6, 1) for k, v in out["kernels"].items()}, indent=1))
        return
    if args.trace_summary:
        print(json.dumps(trace_summary(args.trace_summary), indent=1))
        return
    cpu_base = None
    if not (args.no_cpu_baseline or args.calibrate_copy or args.batch or args.unet or args.learned_experiment
            or args.rz):
        print("[bench] cpu baseline (oracle processes)", file=sys.stderr, flush=True)
        cpu_base = cpu_baseline(args.workload, args.cpu_sample, args.cpu_steps, __import__("numpy"), args.cpu_procs,
                                args.load)
    import torch
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}), flush=True)
        return
    from paper_2402_08404_amd import pic
    from paper_2402_08404_amd import workloads as W

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    if args.learned_experiment:
        return learned_experiment(args, log)
    if args.batch:
        return batch_main(args, log)
    if args.rz:
        return rz_main(args, log)
    if args.unet:
        return unet_main(args, log)

    cfg, counts, kT, region, np = workload(args.workload, args.load)
    solver = {"cg": pic.PIC_SOLVER_CG, "mgcg": pic.PIC_SOLVER_MGCG, "mixed": pic.PIC_SOLVER_MIXED}[args.solver]
    fp32 = args.workload == "gpu_scale"
    caps = (counts[0] + counts[2] + max(counts[0] // 8, 4096), counts[1] + counts[2] + max(counts[1] // 8, 4096),
            counts[2] + 1024)
    t_setup = time.perf_counter()
    # launch settings chosen by the autotuner for this grid shape, if it has run
    from paper_2402_08404_amd import batch as B
    tune = B.load_tuning(args.tuning).get(B.shape_key(cfg), {})
    stencil_blocks = int(args.stencil_blocks or tune.get("stencil_blocks", 0))
    args.sort_every = int(args.sort_every or tune.get("sort_every", 16))
    def new_instance():
        """An instance with the workload's load (the same seeded load every
        time) and its deposit."""
        s_ = pic.Simulation(cfg, caps=caps, precision=pic.PIC_F32 if fp32 else pic.PIC_F64, solver=solver,
                            step_rtol=1e-8, step_maxit=20000, sort_every=args.sort_every,
                            stencil_blocks=stencil_blocks, step_guess=args.step_guess)
        ld = W.initial_load(cfg, counts=counts, kT_eV=kT, region=region, dtype=np.float32 if fp32 else np.float64)
        s_.load(ld)
        del ld
        s_.step(1, pic.STEP_DEPOSIT)
        return s_

    sim = new_instance()
    log(f"[bench] instance ready ({time.perf_counter() - t_setup:.1f} s), {sum(counts)} particles")
    nn = cfg.nx * cfg.ny * cfg.nz
    # CG iterations to 1e-8 from a zero guess (plain CG) and from V0 phi1
    cg_info = {}
    if not args.skip_zero_solve:
        saved = sim.phi.clone()
        r0 = sim.solve(solver=pic.PIC_SOLVER_CG, guess=pic.PIC_GUESS_ZERO, rtol=1e-8, maxit=200000)
        cg_info["plain_zero_guess_iters"] = r0["iterations"]
        sim.phi.copy_(saved)
    r1 = sim.solve(solver=solver, guess=pic.PIC_GUESS_PREVIOUS, rtol=1e-8, maxit=200000)
    cg_info["initial_solve_iters"] = r1["iterations"]
    log(f"[bench] setup {time.perf_counter() - t_setup:.1f} s; warmup {args.warmup} steps")
    sim.step(args.warmup, pic.STEP_FULL)
    m0 = sim.moments()
    it0 = m0["cg_iters_total"]

    # timed region: the production path (no profiling events, solver
    # iterations as captured graphs, collisions concurrent with the solve)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps, pic.STEP_FULL)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m1 = sim.moments()
    log(f"[bench] timed {args.steps} steps in {wall:.3f} s")
    n_avg = 0.5 * (m0["n_alive"].sum() + m1["n_alive"].sum())
    ms_step = 1e3 * wall / args.steps
    value = n_avg * args.steps / wall
    learned = learned_leg(sim, pic, args, log) if not args.no_learned else None
    sim.close()

    # profiled replay: a second instance from the same initial state runs the
    # same warm-up and the same steps with HIP events on the library stream
    # around each phase and each hot kernel (phases one after another, the
    # same kernels launched one by one), so the per-phase times belong to the
    # particle populations of the timed steps
    simp = new_instance()
    simp.solve(solver=solver, guess=pic.PIC_GUESS_PREVIOUS, rtol=1e-8, maxit=200000)
    simp.step(args.warmup, pic.STEP_FULL)
    psteps = args.prof_steps if args.prof_steps > 0 else args.steps
    pic.pic_profile(simp.ctx, True)
    pic.pic_timers(simp.ctx, reset=True)
    mp = simp.moments()
    it_p0 = mp["cg_iters_total"]
    alive_steps = []
    for _ in range(psteps):
        a0 = int(mp["n_alive"].sum())
        simp.step(1, pic.STEP_FULL)
        mp = simp.moments()
        alive_steps.append(0.5 * (a0 + int(mp["n_alive"].sum())))
    tm = pic.pic_timers(simp.ctx, reset=True)
    pic.pic_profile(simp.ctx, False)
    iters_prof = int(mp["cg_iters_total"] - it_p0)
    m2 = mp
    simp.close()
    log(f"[bench] profiled replay of {psteps} steps")

    def avg(name):
        ms, cnt = tm[name]
        return ms / cnt if cnt else float("nan")

    # the particle path (push + deposit + binning + collisions + emission):
    # algorithmic bytes per particle-step 60 B (read x, v, id; write x, v;
    # write and read the cell key) and per node-step 32 B (read the field,
    # clear and write the int64 charge)
    particle_ms = tm["inject"][0] + tm["particles"][0] + tm["collide"][0]
    p_bytes = sum(60.0 * a + 32.0 * nn for a in alive_steps)
    p_gbs = p_bytes / (particle_ms * 1e-3) / 1e9 if particle_ms else float("nan")
    particle_path = {
        "value": float(sum(alive_steps) / (particle_ms * 1e-3)) if particle_ms else None,
        "unit": "particle-steps/s", "ms_per_step": particle_ms / psteps,
        "alive_mean": float(np.mean(alive_steps)),
        "roofline": {"bound": "hbm", "achieved": round(p_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(p_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_step": p_bytes / psteps},
        "phases_ms_per_step": {k2: tm[k2][0] / psteps for k2 in
                               ("inject", "particles", "push", "bin", "deposit", "collide", "mcc")},
        "what": "emission + push/deposit/binning + collisions, HIP-event time on the library stream, profiled "
                "replay of the timed steps (60 B per particle-step + 32 B per node-step algorithmic)"}
    solve_ms = tm["solve"][0] / psteps
    poisson = {"solves_per_s": 1e3 / solve_ms if solve_ms else None, "ms_per_solve": solve_ms,
               "iters_per_solve": iters_prof / psteps, "solver": args.solver,
               "what": "MG-preconditioned CG to a relative residual of 1e-8 plus the node field, HIP-event time"}
    k_push_e = avg("push_e")
    ne_avg = 0.5 * (m1["n_alive"][0] + m2["n_alive"][0])
    pb = push_bytes(float(np.mean(alive_steps)) * 0.8, nn, fp32)
    kernels = {"push_electrons": {"avg_ms": k_push_e, "launches": tm["push_e"][1], "bytes": pb,
                                  "gbs": pb / (k_push_e * 1e-3) / 1e9}}
    # A solve launches its iterations in chunks, so some launches of the
    # solver kernels come after convergence and return at once: each kernel's
    # total event time is divided by the iterations that did work (the
    # returning launches' few microseconds stay in the total, so the average
    # errs high and the bandwidth low).
    for name, per_node in SOLVER_BYTES_PER_NODE.items():
        b = per_node * nn
        n_work = iters_prof if 0 < iters_prof <= tm[name][1] else tm[name][1]
        a_ms = tm[name][0] / n_work if n_work else float("nan")
        kernels[name] = {"avg_ms": a_ms, "launches": n_work, "launches_total": tm[name][1], "bytes": b,
                         "gbs": b / (a_ms * 1e-3) / 1e9}
    # dominant kernel: largest time summed over its launches in the profiled pass
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"]
              if kernels[k]["launches"] else -1.0)
    k = kernels[dom]
    traffic = measured_traffic(dom)
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(k["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(k["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
            "bytes_per_launch": k["bytes"], "avg_launch_ms": k["avg_ms"]}

    out = {
        "metric": METRIC,
        "value": float(value),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": [cfg.nx, cfg.ny, cfg.nz], "h_m": cfg.h,
                   "particles": list(counts), "load": region, "particle_state": "fp32" if fp32 else "fp64",
                   "poisson": f"{args.solver} fp64 rtol 1e-8, guess "
                              + ("extrapolated from the two previous steps" if args.step_guess else "previous step"),
                   "sort_every": args.sort_every,
                   "stencil_blocks": stencil_blocks or 1024},
        "roofline": roof,
        "particle_path": particle_path,
        "poisson": poisson,
        "profiled_pass_ms_per_step": {k2: tm[k2][0] / psteps for k2 in
                                      ("inject", "particles", "push", "collide", "mcc", "solve", "step")},
        "kernels": kernels,
        "cg": dict(cg_info, step_iters_avg=(m1["cg_iters_total"] - it0) / args.steps,
                   profiled_iters_avg=iters_prof / psteps),
        "alive": [int(x) for x in m1["n_alive"]],
        "events_total": [int(x) for x in m1["events"]],
    }
    if learned is not None:
        out["cg"]["learned"] = learned
    out["cpu_baseline"] = cpu_base
    print(json.dumps(out), flush=True)


def unet_flops(d: int, h: int, w: int, base: int = 16) -> float:
    """Multiply-add FLOPs (2 per MAC) of one forward pass over d x h x w: each
    layer costs taps x cin x cout MACs per output voxel of its GEMM rows (the
    8-channel input counts its 8 channels, as the kernels compute them)."""
    c = [base, 2 * base, 4 * base, 8 * base]
    vox = [d * h * w / 8 ** l for l in range(4)]
    layers = [(27, 8, c[0], 0), (27, c[0], c[0], 0)]
    for lv in (1, 2, 3):
        layers += [(8, c[lv - 1], c[lv], lv), (27, c[lv], c[lv], lv), (27, c[lv], c[lv], lv)]
    for lv in (2, 1, 0):
        layers += [(8, c[lv + 1], c[lv], lv), (27, 2 * c[lv], c[lv], lv), (27, c[lv], c[lv], lv)]
    macs = sum(t * ci * co * vox[lv] for t, ci, co, lv in layers)
    # the transposed convolutions: 8 taps over coarse voxels = 1 tap over fine voxels
    macs -= sum(7 * c[lv + 1] * c[lv] * vox[lv] for lv in (2, 1, 0))
    return 2.0 * macs + 2.0 * base * vox[0]


def unet_main(args, log):
    """Throughput of the warm-start network's bf16 MFMA kernels."""
    import torch
    from paper_2402_08404_amd import pic
    D, H, Wd = 512, 128, 128
    net = pic.UNet(1, D, H, Wd, seed=1)
    x = torch.randn(1, D, H, Wd, device="cuda")
    t = torch.randn(1, D, H, Wd, device="cuda")
    for _ in range(args.warmup):
        net.forward(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.forward(x)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / args.steps
    for _ in range(args.warmup):
        net.train_step(x, t, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.train_step(x, t, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    trn = (time.perf_counter() - t0) / args.steps
    fl = unet_flops(D, H, Wd)
    peak = 2500.0
    out = {"metric": "warm-start network throughput (bf16 MFMA, fp32 accumulate)", "value": fl / fwd / 1e12,
           "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * fwd,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "unet_1x512x128x128", "params": net.n_params},
           "roofline": {"bound": "mfma", "achieved": fl / fwd / 1e12, "peak": peak, "unit": "TFLOP/s",
                        "frac": fl / fwd / 1e12 / peak, "traffic": None},
           "forward_ms": 1e3 * fwd, "train_step_ms": 1e3 * trn, "forward_tflop": fl / 1e12,
           "train_tflops_est": 3 * fl / trn / 1e12}
    net.close()
    print(json.dumps(out), flush=True)


def learned_leg(sim, pic, args, log):
    """The learned warm start on this workload: training pairs from the
    running simulation (a tight solve, then pic_training_sample, every two
    steps), Adam on the library's network kernels, then on a later state the
    iterations to 1e-8 of plain CG and of MG-PCG from a zero guess, from the
    previous step's potential, from V0 phi1 and from the learned guess (the
    raw network output and its energy-norm projection)."""
    import torch
    from paper_2402_08404_amd import warmstart
    cfg = sim.cfg
    shape = (cfg.nz, cfg.ny, cfg.nx)
    t0 = time.perf_counter()
    xs, ys = [], []
    for k in range(args.learned_pairs):
        if k:
            sim.step(2, pic.STEP_FULL)
        sim.solve(solver=pic.PIC_SOLVER_MGCG, guess=pic.PIC_GUESS_PREVIOUS, rtol=1e-12, maxit=100000)
        x = torch.empty(shape, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        pic.pic_training_sample(sim.ctx, x.data_ptr(), y.data_ptr())
        xs.append(x)
        ys.append(y)
    X, Y = torch.stack(xs), torch.stack(ys)
    net = pic.UNet(1, *shape, seed=7)
    losses = warmstart.train(net, X, Y, iters=args.learned_iters, lr=3e-4, lr_final=5e-5)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    sim.step(3, pic.STEP_FULL)  # a state the network has not seen
    # one more step without its solve: phi is then the previous step's
    # potential (the "previous" guess of the step solve)
    sim.step(1, pic.STEP_FULL & ~pic.STEP_SOLVE)
    net.sync()
    res = {}
    for sname, solver in (("plain", pic.PIC_SOLVER_CG), ("mgcg", pic.PIC_SOLVER_MGCG)):
        for gname, guess, project in (("zero", pic.PIC_GUESS_ZERO, True), ("previous", pic.PIC_GUESS_PREVIOUS, True),
                                      ("laplace", pic.PIC_GUESS_LAPLACE, True),
                                      ("learned_raw", pic.PIC_GUESS_LEARNED, False),
                                      ("learned", pic.PIC_GUESS_LEARNED, True)):
            pic.pic_set_learned_guess(sim.ctx, net.net, 2, project)
            saved = sim.phi.clone()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = sim.solve(solver=solver, guess=guess, rtol=1e-8, maxit=200000)
            res[f"{sname}_{gname}"] = {"iters": r["iterations"], "relres0": r["relres0"],
                                       "ms": 1e3 * (time.perf_counter() - t1)}
            sim.phi.copy_(saved)
    pic.pic_set_learned_guess(sim.ctx, None)
    net.close()
    log(f"[bench] learned leg: {args.learned_pairs} pairs, {args.learned_iters} Adam steps, {t_train:.1f} s")
    m = min(10, len(losses))
    return {"pairs": args.learned_pairs, "adam_steps": args.learned_iters,
            "loss_first10": sum(losses[:m]) / m, "loss_last10": sum(losses[-m:]) / m, "train_s": t_train,
            "solves": res,
            "plain_gain_vs_zero": res["plain_zero"]["iters"] / max(res["plain_learned"]["iters"], 1),
            "plain_gain_vs_laplace": res["plain_laplace"]["iters"] / max(res["plain_learned"]["iters"], 1)}


def learned_experiment(args, log):
    """The learned warm start at the tiny workload's shape (32 x 32 x 64
    nodes): (x, y) pairs from plain FP64 runs of the tiny workload at apex
    fields 6, 7, ..., 14 GV/m (one run per field, a pair every 5 steps after a
    tight solve), the runs at 7 and 13 GV/m held out of training; the network
    trained on the others by the library's kernels; then, on fresh runs at the
    held-out fields, the iterations to a relative residual of 1e-8 of plain CG
    and of MG-PCG from a zero guess, the previous step's potential, V0 phi1
    and the learned guess (projected, judged by plain CG)."""
    import dataclasses
    import numpy as np
    import torch
    from paper_2402_08404_amd import pic, warmstart
    from paper_2402_08404_amd import workloads as W
    base = W.tiny()
    fields = [6e9, 7e9, 8e9, 9e9, 10e9, 11e9, 12e9, 13e9, 14e9]
    held = {7e9, 13e9}
    per_field = max(1, args.le_pairs // len(fields))
    shape = (base.nz, base.ny, base.nx)
    t0 = time.perf_counter()
    xs, ys, xh, yh = [], [], [], []
    for i, F in enumerate(fields):
        X, Y = warmstart.collect_samples(base, fields=[F], per_field=per_field, steps_between=5,
                                         counts=(20000, 200, 2000), seed=11 + 97 * i)
        (xh if F in held else xs).append(X)
        (yh if F in held else ys).append(Y)
        log(f"[learned] field {F / 1e9:.0f} GV/m: {X.shape[0]} pairs ({time.perf_counter() - t0:.0f} s)")
    Xt, Yt = torch.cat(xs), torch.cat(ys)
    Xh, Yh = torch.cat(xh), torch.cat(yh)
    t_data = time.perf_counter() - t0
    net = pic.UNet(args.le_batch, *shape, seed=7)
    t1 = time.perf_counter()
    losses = warmstart.train(net, Xt, Yt, iters=args.le_iters, lr=1e-3, lr_final=3e-5, log_every=500)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    log(f"[learned] trained {args.le_iters} steps on {Xt.shape[0]} pairs in {t_train:.0f} s")
    guess_net = pic.UNet(1, *shape, params=net.params)
    guess_net.sync()
    # held-out pairs: relative L2 error of the network's charge response
    errs = []
    for k in range(0, Xh.shape[0], max(1, Xh.shape[0] // 64)):
        y = guess_net.forward(Xh[k:k + 1])
        errs.append(float((y - Yh[k:k + 1]).norm() / Yh[k:k + 1].norm().clamp_min(1e-30)))
    res = {}
    for F in sorted(held):
        cfg = dataclasses.replace(base, apex_field=F, seed=5000 + int(F / 1e9))
        sim = pic.Simulation(cfg, caps=(200000, 20000, 8000), precision=pic.PIC_F64, solver=pic.PIC_SOLVER_MGCG,
                             step_rtol=1e-10)
        sim.load(W.initial_load(cfg, counts=(20000, 200, 2000), seed=6000 + int(F / 1e9)))
        sim.step(1, pic.STEP_DEPOSIT)
        sim.solve(solver=pic.PIC_SOLVER_MGCG, rtol=1e-10)
        sim.step(60, pic.STEP_FULL)
        rows = {}
        for state in range(8):
            sim.step(9, pic.STEP_FULL)
            sim.step(1, pic.STEP_FULL & ~pic.STEP_SOLVE)   # phi is the previous step's potential
            for sname, solver in (("plain", pic.PIC_SOLVER_CG), ("mgcg", pic.PIC_SOLVER_MGCG)):
                for gname, guess in (("zero", pic.PIC_GUESS_ZERO), ("previous", pic.PIC_GUESS_PREVIOUS),
                                     ("laplace", pic.PIC_GUESS_LAPLACE), ("learned", pic.PIC_GUESS_LEARNED)):
                    pic.pic_set_learned_guess(sim.ctx, guess_net.net, 0, True)
                    saved = sim.phi.clone()
                    torch.cuda.synchronize()
                    t2 = time.perf_counter()
                    r = sim.solve(solver=solver, guess=guess, rtol=1e-8, maxit=200000)
                    ms = 1e3 * (time.perf_counter() - t2)
                    d = rows.setdefault(f"{sname}_{gname}", {"iters": [], "relres0": [], "ms": [], "fell_back": 0})
                    d["iters"].append(r["iterations"])
                    d["relres0"].append(r["relres0"])
                    d["ms"].append(ms)
                    d["fell_back"] += int(r["fell_back"])
                    sim.phi.copy_(saved)
            sim.solve(solver=pic.PIC_SOLVER_MGCG, guess=pic.PIC_GUESS_PREVIOUS, rtol=1e-10)
        pic.pic_set_learned_guess(sim.ctx, None)
        sim.close()
        res[f"{F / 1e9:.0f}GVm"] = {k: {"iters_mean": float(np.mean(v["iters"])), "iters": v["iters"],
                                        "relres0_mean": float(np.mean(v["relres0"])), "ms_mean": float(np.mean(v["ms"])),
                                        "fell_back": v["fell_back"]} for k, v in rows.items()}
        log(f"[learned] held-out {F / 1e9:.0f} GV/m: " +
            ", ".join(f"{k} {np.mean(v['iters']):.1f}" for k, v in rows.items()))
    gains = {f: {"plain_vs_zero": v["plain_zero"]["iters_mean"] / v["plain_learned"]["iters_mean"],
                 "plain_vs_previous": v["plain_previous"]["iters_mean"] / v["plain_learned"]["iters_mean"],
                 "mgcg_vs_zero": v["mgcg_zero"]["iters_mean"] / v["mgcg_learned"]["iters_mean"]}
             for f, v in res.items()}
    m = min(20, len(losses))
    out = {"metric": "CG iterations to 1e-8: learned vs plain (held-out fields)", "value":
           float(np.mean([g["plain_vs_zero"] for g in gains.values()])), "unit": "x fewer plain-CG iterations",
           "higher_is_better": True, "data": "synthetic", "dtype": "bf16",
           "config": {"workload": "tiny_32x32x64", "fields_GVm": [f / 1e9 for f in fields],
                      "held_out_GVm": sorted(f / 1e9 for f in held), "train_pairs": int(Xt.shape[0]),
                      "held_out_pairs": int(Xh.shape[0]), "adam_steps": args.le_iters, "batch": args.le_batch},
           "data_s": t_data, "train_s": t_train, "loss_first": sum(losses[:m]) / m, "loss_last": sum(losses[-m:]) / m,
           "held_out_relative_error": {"mean": float(np.mean(errs)), "max": float(np.max(errs)), "n": len(errs)},
           "solves": res, "gains": gains}
    net.close()
    guess_net.close()
    print(json.dumps(out), flush=True)


def batch_main(args, log):
    """The batched sweep: concurrent instances, whole-job particle-steps/s."""
    import torch
    from paper_2402_08404_amd import batch, pic
    items = batch.sweep_configs(16, scale=args.batch_scale)
    tuning = batch.load_tuning(args.tuning)
    if args.autotune:
        tuning = batch.autotune(items, log=log)
        batch.save_tuning(tuning, args.tuning)
    t0 = time.perf_counter()
    b = batch.Batch(items, tuning=tuning, log=log)
    log(f"[bench] batch of {len(items)} instances ready ({time.perf_counter() - t0:.1f} s), "
        f"{sum(sum(c) for _, c in items)} particles")
    b.step(args.warmup)
    n0 = b.alive()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # in chunks of 100 steps with a progress line after each
    done = 0
    while done < args.steps:
        k = min(100, args.steps - done)
        b.step(k)
        done += k
        if done < args.steps:
            log(f"[bench] batch step {done} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n1 = b.alive()
    value = 0.5 * (n0 + n1) * args.steps / wall
    serial = None
    if args.batch_compare:
        # the same number of steps with one instance at a time (no overlap)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for s in b.sims:
            s.step(args.steps, pic.STEP_FULL)
            torch.cuda.synchronize()
        serial = 1e3 * (time.perf_counter() - t1) / args.steps
    out = {
        "metric": "particle-steps/s (batched field sweep, push+deposit+MCC+solve)",
        "value": float(value), "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "field_sweep_16", "fields_GVm": [round(c.apex_field / 1e9, 2) for c, _ in items],
                   "grids": [[c.nx, c.ny, c.nz] for c, _ in items], "particles": [sum(n) for _, n in items],
                   "tuning": tuning},
        "alive": [n0, n1],
        "serial_ms_per_step": serial,
    }
    b.close()
    print(json.dumps(out), flush=True)


def rz_cpu_baseline(geo, per_species, steps):
    """The axisymmetric oracle on a bounded sample: per_species particles of
    each species drawn like the GPU load, whole steps with every stage (its
    solve is a direct sparse factorization of the same grid)."""
    import numpy as np
    from oracle.rz import RZ
    from paper_2402_08404_amd import workloads as W
    load = W.rz_load(geo, (per_species,) * 3, rng=np.random.default_rng(11))
    o = RZ(geo["nr"], geo["nz"], geo["h"], geo["tip_r"], geo["tip_h"], geo["apex_field"], geo["dt"], geo["m_ion"],
           seed=geo["seed"], xs=geo["xs"], fn_rings=geo["fn_rings"], cu2=geo["cu2"])
    nid = 0
    for s in range(3):
        o.load(s, load[s], np.arange(nid, nid + per_species))
        nid += per_species
    t0 = time.perf_counter()
    n = 0
    for _ in range(steps):
        n += sum(len(o.sp[s]["id"]) for s in range(3))
        o.step(emit=True, collide=True)
    wall = time.perf_counter() - t0
    return {"value": n / wall, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{per_species} particles per species on the same grid, {steps} whole steps "
                      f"({wall:.1f} s, one thread; the direct solve of the grid dominates)"}


kBlockRz = 256  # threads per block of the axisymmetric particle kernels (grid = capacity rounded up)


def rz_main(args, log):
    """The axisymmetric variant on the paper's geometry: emission, push,
    collisions, field ionization, deposit and the CG solve in every step."""
    import numpy as np
    import torch
    from paper_2402_08404_amd import rz
    from paper_2402_08404_amd import workloads as W
    geo = W.rz_context()
    counts = tuple(int(c * args.rz_scale) for c in (4_000_000, 4_000_000, 4_000_000))
    t0 = time.perf_counter()
    load = W.rz_load(geo, counts)
    caps = [int(1.25 * counts[0]) + 65536, int(1.25 * counts[1]) + 4096, counts[2] + 1]
    keys = ("nr", "nz", "h", "tip_r", "tip_h", "apex_field", "dt", "m_ion")
    sim = rz.RZSimulation(**{k: geo[k] for k in keys}, load=load, caps=caps, step_rtol=1e-8, seed=geo["seed"],
                          xs=geo["xs"], fn_rings=geo["fn_rings"], cu2=geo["cu2"], sort_every=args.rz_sort_every)
    del load
    log(f"[bench] rz instance ready ({time.perf_counter() - t0:.1f} s), {sum(counts)} particles")
    sim.step(1, rz.PIC_RZ_DEPOSIT | rz.PIC_RZ_SOLVE)
    sim.step(args.warmup, rz.PIC_RZ_ALL)
    m0 = sim.moments()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, iters = 0, 0
    while done < args.steps:
        k = min(10, args.steps - done)
        if args.rz_iters:
            for _ in range(k):
                sim.step(1, rz.PIC_RZ_ALL)
                iters += sim.moments()["last_cg_iters"]
        else:
            sim.step(k, rz.PIC_RZ_ALL)  # one call: the library checks its sticky errors once per call
        done += k
        log(f"[bench] rz step {done} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m1 = sim.moments()
    n0, n1 = int(m0["n_alive"].sum()), int(m1["n_alive"].sum())
    value = 0.5 * (n0 + n1) * args.steps / wall
    # the push of every species, timed alone with HIP events on the library's
    # stream: algorithmic bytes = 84 B per alive particle (r, z, vr, vt, vz
    # and the id read, the five written) + the node field read once
    nn = geo["nr"] * geo["nz"]
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 10
    alive = int(sim.moments()["n_alive"].sum())
    ev[0].record(stream)
    for _ in range(reps):
        sim.step(1, rz.PIC_RZ_PUSH)
    ev[1].record(stream)
    torch.cuda.synchronize()
    t_push = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
    push_bytes = 84.0 * alive + 16.0 * nn
    ach = push_bytes / t_push / 1e9
    # HBM bytes of one pass (the three species' launches) from the counters
    # in profiles/traffic_rz_context.json, where they were taken
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic_rz_context.json")
    if os.path.exists(tf):
        with open(tf) as f:
            kp = json.load(f)["kernels"].get("pic_rz::k_push")
        grids = [str(kBlockRz * ((c + kBlockRz - 1) // kBlockRz)) for c in caps]
        if kp and all(g in kp["bytes_by_grid"] for g in grids):
            traffic = sum(kp["bytes_by_grid"][g] for g in grids)
    cpu = None if args.no_cpu_baseline else rz_cpu_baseline(geo, 2000, 2)
    out = {
        "metric": "particle-steps/s (axisymmetric variant: emission, push, collisions with Cu2+, field "
                  "ionization, deposit, CG solve)",
        "value": float(value), "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "rz_context", "grid": [geo["nr"], geo["nz"]], "h_nm": geo["h"] * 1e9,
                   "sort_every": args.rz_sort_every,
                   "tip_r_nm": geo["tip_r"] * 1e9, "tip_h_um": geo["tip_h"] * 1e6, "particles": list(counts)},
        "roofline": {"bound": "hbm", "kernel": "k_push (all species, one pass)", "achieved": ach, "peak": 8000.0,
                     "unit": "GB/s", "frac": ach / 8000.0, "traffic": traffic,
                     "launch_us": t_push * 1e6, "bytes": push_bytes},
        "cpu_baseline": cpu,
        "alive": [n0, n1], "events": m1["events"].tolist(), "injected": int(m1["injected"]),
        "n_cu2": int(m1["n_cu2"]),
        "cg_iterations_per_step": (iters / args.steps) if args.rz_iters else None,
    }
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
