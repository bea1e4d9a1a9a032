"""Batched local-field sweep: independent PIC-MCC instances stepped together.

Each instance is one context of the library on its own HIP stream (default
priority). A host thread per instance drives its steps (the library calls
release the interpreter lock), so the kernels of all instances are in flight
together and a small instance fills the gaps of a large one; each instance's
Poisson solver replays its own captured graphs. Instances share nothing, so
every instance's result equals that of the same instance run alone.

The autotuner times short runs of candidate launch settings (reorder period
of the particle arrays, block count of the z-marching solver kernels) per
grid shape and keeps the fastest; its choices are stored as JSON.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import pic
from . import workloads as W

SWEEP_FIELDS = tuple(6.0e9 + 0.5e9 * k for k in range(16))   # 6.0, 6.5, ..., 13.5 GV/m


def sweep_sizes(n_inst: int = 16, seed: int = 100, n_min: float = 1e6, n_max: float = 40e6, scale: float = 1.0):
    """Particle counts N_k = n_min (n_max/n_min)^u_k, u_k ~ U(0, 1) seeded: a
    power law p(N) ~ 1/N between n_min and n_max, randomly assigned to the
    fields. scale shrinks every count (for tests)."""
    rng = np.random.default_rng(seed)
    u = rng.random(n_inst)
    return [max(1000, int(round(scale * n_min * (n_max / n_min) ** x))) for x in u]


def grid_for(n: int, scale: float = 1.0):
    """Grid by particle count: < 4 M -> 64 x 64 x 256, < 15 M -> 96 x 96 x 384,
    else 128 x 128 x 512 (1 nm spacing, the r = 10 nm, H = 100 nm tip). With
    scale < 1 the thresholds shrink with the counts."""
    if n < 4e6 * scale:
        return 64, 64, 256
    if n < 15e6 * scale:
        return 96, 96, 384
    return 128, 128, 512


def sweep_configs(n_inst: int = 16, scale: float = 1.0, seed: int = 100):
    """(config, counts) per instance of the sweep: species split 80 / 5 / 15 %."""
    out = []
    for k, n in enumerate(sweep_sizes(n_inst, seed=seed, scale=scale)):
        nx, ny, nz = grid_for(n, scale)
        base = W.gpu_scale(seed=seed + k)
        cfg = dataclasses.replace(base, nx=nx, ny=ny, nz=nz, apex_field=SWEEP_FIELDS[k % len(SWEEP_FIELDS)])
        counts = (int(0.80 * n), int(0.05 * n), n - int(0.80 * n) - int(0.05 * n))
        out.append((cfg, counts))
    return out


class Batch:
    """Instances of a sweep, each a pic.Simulation on its own stream."""

    def __init__(self, items, kT_eV=(5.0, 1.0, 0.1), region="box", precision=pic.PIC_F32,
                 solver=pic.PIC_SOLVER_MGCG, tuning: dict | None = None, step_rtol=1e-8, load_seed=7, log=None):
        self.sims = []
        self.items = items
        tuning = tuning or {}
        dt = np.float32 if precision == pic.PIC_F32 else np.float64
        for k, (cfg, counts) in enumerate(items):
            t = tuning.get(shape_key(cfg), {})
            caps = (counts[0] + counts[2] + max(counts[0] // 8, 4096), counts[1] + counts[2] + max(counts[1] // 8, 4096),
                    counts[2] + 1024)
            st = torch.cuda.Stream()
            sim = pic.Simulation(cfg, caps=caps, precision=precision, solver=solver, stream=st, step_rtol=step_rtol,
                                 sort_every=t.get("sort_every", 16), stencil_blocks=t.get("stencil_blocks", 0))
            sim.load(W.initial_load(cfg, counts=counts, kT_eV=kT_eV, region=region, seed=load_seed + k, dtype=dt))
            sim.step(1, pic.STEP_DEPOSIT)
            sim.solve(solver=solver, guess=pic.PIC_GUESS_PREVIOUS, rtol=step_rtol, maxit=100000)
            self.sims.append(sim)
            if log:
                log(f"[batch] instance {k} ready: {shape_key(cfg)}, {sum(counts)} particles")
        torch.cuda.synchronize()
        self._pool = ThreadPoolExecutor(max_workers=max(1, len(self.sims)))

    def step(self, nsteps: int, flags: int = pic.STEP_FULL):
        """nsteps steps of every instance, concurrently; returns when all are done."""
        futs = [self._pool.submit(pic.pic_step, s.ctx, nsteps, flags) for s in self.sims]
        for f in futs:
            f.result()
        torch.cuda.synchronize()

    def alive(self) -> int:
        return int(sum(int(s.moments()["n_alive"].sum()) for s in self.sims))

    def close(self):
        self._pool.shutdown()
        for s in self.sims:
            s.close()
        self.sims = []


def shape_key(cfg) -> str:
    return f"{cfg.nx}x{cfg.ny}x{cfg.nz}"


def autotune(items, candidates_sort=(8, 16, 32), candidates_blocks=(1024, 2048, 4096), steps: int = 3,
             warmup: int = 2, log=None) -> dict:
    """For each grid shape of the sweep, time `steps` full steps of its
    smallest instance for each candidate setting (one parameter at a time,
    starting from the defaults) and keep the fastest. Returns
    {shape: {"sort_every": s, "stencil_blocks": b, "ms": {...}}}."""
    by_shape = {}
    for cfg, counts in items:
        k = shape_key(cfg)
        if k not in by_shape or sum(counts) < sum(by_shape[k][1]):
            by_shape[k] = (cfg, counts)
    result = {}
    for key, (cfg, counts) in by_shape.items():
        best = {"sort_every": 16, "stencil_blocks": 1024}
        timings = {}
        for param, cands in (("stencil_blocks", candidates_blocks), ("sort_every", candidates_sort)):
            times = {}
            for v in cands:
                t = dict(best, **{param: v})
                b = Batch([(cfg, counts)], tuning={key: t})
                b.step(warmup)
                t0 = time.perf_counter()
                b.step(steps)
                times[v] = 1e3 * (time.perf_counter() - t0) / steps
                b.close()
                if log:
                    log(f"[autotune] {key} {param}={v}: {times[v]:.2f} ms/step")
            best[param] = min(times, key=times.get)
            timings[param] = times
        result[key] = dict(best, ms=timings)
    return result


def save_tuning(t: dict, path: str):
    with open(path, "w") as f:
        json.dump(t, f, indent=1, sort_keys=True)


def load_tuning(path: str) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)
