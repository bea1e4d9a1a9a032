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


def workload(name):
    import numpy as np
    from paper_2402_08404_amd import workloads as W
    if name == "gpu_scale":
        cfg = W.gpu_scale()
        counts = (16_000_000, 1_000_000, 3_000_000)
        kT = (5.0, 1.0, 0.1)
        region = "box"
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
        best = {}
        for (name, grid), v in d.items():
            if name not in best or grid > best[name][0]:
                best[name] = (grid, statistics.median(v), len(v))
        return best

    def copy_kib(path):
        v = [float(r["Counter_Value"]) for r in csv.DictReader(open(path)) if "copyBuffer" in r["Kernel_Name"]
             or "copy" in r["Kernel_Name"].lower()]
        return statistics.median(v)

    f_fetch = copy_mib * 1024.0 / copy_kib(copy_fetch_csv)
    f_write = copy_mib * 1024.0 / copy_kib(copy_write_csv)
    fe, wr = per_kernel(fetch_csv), per_kernel(write_csv)
    out = {"fetch_scale": f_fetch, "write_scale": f_write, "copy_mib": copy_mib, "kernels": {}}
    for name in sorted(set(fe) & set(wr)):
        out["kernels"][name] = {"grid": fe[name][0], "fetch_kib": fe[name][1], "write_kib": wr[name][1],
                                "dispatches": fe[name][2],
                                "bytes": 1024.0 * (fe[name][1] * f_fetch + wr[name][1] * f_write)}
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


def cpu_baseline(cfg_name, sample, steps, np):
    """The CPU oracle (single thread, FP64) on a bounded sample of the same
    workload: `sample` particles with the same species mix and distributions
    on the same grid, timed over `steps` steps of push, collisions and
    deposit. The oracle's Poisson solve is left out (a solve of the
    128 x 128 x 512 grid takes minutes on one core); a smooth synthetic
    potential stands in for the field."""
    import oracle
    from paper_2402_08404_amd import workloads as W
    cfg, counts, kT, region, _ = workload(cfg_name)
    frac = sample / sum(counts)
    sub = tuple(int(round(c * frac)) for c in counts)
    o = oracle.Oracle(cfg, laplace=False)
    o.load(W.initial_load(cfg, counts=sub, kT_eV=kT, region=region, seed=cfg.seed + 7))
    o.set_phi(W.synthetic_potential(cfg, o.V0))
    n = sum(s.n for s in o.sp)
    t0 = time.perf_counter()
    for _ in range(steps):
        o.push()
        o.collide()
        o.deposit()
        o.step_no += 1
    dt = time.perf_counter() - t0
    return {"value": n * steps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} particles ({sub[0]} e, {sub[1]} Cu+, {sub[2]} Cu) of the same workload, {steps} steps "
                      f"of push+collisions+deposit on the same grid, synthetic potential, solve excluded; "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gpu_scale", choices=["gpu_scale", "tiny"])
    ap.add_argument("--solver", default="mgcg", choices=["cg", "mgcg", "mixed"])
    ap.add_argument("--sort-every", type=int, default=0,
                    help="reorder period of the particle arrays (0: the tuned value for this grid, else 16)")
    ap.add_argument("--stencil-blocks", type=int, default=0, help="override the tuned block count of the solver kernels")
    ap.add_argument("--step-guess", type=int, default=1, choices=[0, 1],
                    help="step-solve guess: 0 previous potential, 1 linear extrapolation in time")
    ap.add_argument("--cpu-sample", type=int, default=3_000_000)
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-zero-solve", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned warm-start leg (training on pairs of this run, then iteration counts)")
    ap.add_argument("--learned-pairs", type=int, default=16)
    ap.add_argument("--learned-iters", type=int, default=300)
    ap.add_argument("--prof-steps", type=int, default=5,
                    help="steps of the profiled pass after the timed region (per-kernel HIP-event timings)")
    ap.add_argument("--unet", action="store_true",
                    help="time the warm-start network (forward, and forward + backward + Adam) at 1 x 512 x 128 x 128")
    ap.add_argument("--batch", action="store_true",
                    help="the batched field sweep (16 instances at 6.0 ... 13.5 GV/m, 1 M - 40 M particles) instead")
    ap.add_argument("--batch-scale", type=float, default=1.0, help="scale factor of the sweep's particle counts")
    ap.add_argument("--autotune", action="store_true", help="with --batch: autotune first and store the choices")
    ap.add_argument("--batch-compare", action="store_true",
                    help="with --batch: also time the same steps with the instances stepped one after another")
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_2402_08404_amd", "tuning.json"))
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
        out = pmc_summary(a[0], a[1], a[2], a[3], float(a[4]), TRAFFIC_FILE)
        print(json.dumps({k: round(v["bytes"] / 1e6, 1) for k, v in out["kernels"].items()}, indent=1))
        return
    if args.trace_summary:
        print(json.dumps(trace_summary(args.trace_summary), indent=1))
        return
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

    if args.batch:
        return batch_main(args, log)
    if args.unet:
        return unet_main(args, log)

    cfg, counts, kT, region, np = workload(args.workload)
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
    sim = pic.Simulation(cfg, caps=caps, precision=pic.PIC_F32 if fp32 else pic.PIC_F64, solver=solver,
                         step_rtol=1e-8, step_maxit=20000, sort_every=args.sort_every, stencil_blocks=stencil_blocks,
                         step_guess=args.step_guess)
    log(f"[bench] init done ({time.perf_counter() - t_setup:.1f} s), generating {sum(counts)} particles")
    load = W.initial_load(cfg, counts=counts, kT_eV=kT, region=region,
                          dtype=np.float32 if fp32 else np.float64)
    sim.load(load)
    del load
    sim.step(1, pic.STEP_DEPOSIT)
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
    # iterations as captured graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps, pic.STEP_FULL)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m1 = sim.moments()
    log(f"[bench] timed {args.steps} steps in {wall:.3f} s")
    # profiled pass over the next steps: HIP events on the library stream
    # around each phase and each hot kernel (the same kernels, launched one
    # by one)
    pic.pic_profile(sim.ctx, True)
    pic.pic_timers(sim.ctx, reset=True)
    it_p0 = m1["cg_iters_total"]
    sim.step(args.prof_steps, pic.STEP_FULL)
    tm = pic.pic_timers(sim.ctx, reset=True)
    pic.pic_profile(sim.ctx, False)
    m2 = sim.moments()
    log(f"[bench] profiled {args.prof_steps} steps")

    n_avg = 0.5 * (m0["n_alive"].sum() + m1["n_alive"].sum())
    n_prof = 0.5 * (m1["n_alive"].sum() + m2["n_alive"].sum())
    ne_avg = 0.5 * (m1["n_alive"][0] + m2["n_alive"][0])
    ms_step = 1e3 * wall / args.steps
    value = n_avg * args.steps / wall

    def avg(name):
        ms, cnt = tm[name]
        return ms / cnt if cnt else float("nan")

    psteps = args.prof_steps
    particle_ms = tm["inject"][0] + tm["particles"][0] + tm["collide"][0]
    k_push_e = avg("push_e")
    pb = push_bytes(ne_avg, nn, fp32)
    kernels = {"push_electrons": {"avg_ms": k_push_e, "launches": tm["push_e"][1], "bytes": pb,
                                  "gbs": pb / (k_push_e * 1e-3) / 1e9}}
    # A solve launches its iterations in chunks, so some launches of the
    # solver kernels come after convergence and return at once: each kernel's
    # total event time is divided by the iterations that did work (the
    # returning launches' few microseconds stay in the total, so the average
    # errs high and the bandwidth low).
    iters_prof = int(m2["cg_iters_total"] - it_p0)
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
                   "particles": list(counts), "particle_state": "fp32" if fp32 else "fp64",
                   "poisson": f"{args.solver} fp64 rtol 1e-8, guess "
                              + ("extrapolated from the two previous steps" if args.step_guess else "previous step"),
                   "sort_every": args.sort_every,
                   "stencil_blocks": stencil_blocks or 1024},
        "roofline": roof,
        "profiled_pass_ms_per_step": {k2: tm[k2][0] / psteps for k2 in
                                      ("inject", "particles", "push", "collide", "mcc", "solve", "step")},
        "particle_phases": {"value": float(n_prof * psteps / (particle_ms * 1e-3)) if particle_ms else None,
                            "unit": "particle-steps/s", "what": "emission + push/deposit/binning + collisions, "
                                                                "HIP-event time on the library stream (profiled pass)"},
        "kernels": kernels,
        "cg": dict(cg_info, step_iters_avg=(m1["cg_iters_total"] - it0) / args.steps,
                   profiled_iters_avg=(m2["cg_iters_total"] - it_p0) / psteps),
        "alive": [int(x) for x in m1["n_alive"]],
        "events_total": [int(x) for x in m1["events"]],
    }
    if not args.no_learned:
        out["cg"]["learned"] = learned_leg(sim, pic, args, log)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_sample, args.cpu_steps, np)
    else:
        out["cpu_baseline"] = None
    sim.close()
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
    b = batch.Batch(items, tuning=tuning)
    log(f"[bench] batch of {len(items)} instances ready ({time.perf_counter() - t0:.1f} s), "
        f"{sum(sum(c) for _, c in items)} particles")
    b.step(args.warmup)
    n0 = b.alive()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(args.steps)
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


if __name__ == "__main__":
    main()
