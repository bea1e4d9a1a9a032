"""Ensemble parity over 1000 steps: the trajectories of two PIC-MCC runs part
at the first differing random draw, so beyond single steps the GPU path and
the oracle are compared as ensembles of independent realizations of the tiny
workload: 32 GPU runs (seeds 1 .. 32) against 32 FP64 oracle runs (seeds
101 .. 132, recorded in tests/golden/ensemble_tiny.json by
tests/golden/make_ensemble_tiny.py, which calls only the oracle). After 250,
500 and 1000 steps each observable's ensemble means are compared by
z = |mean_gpu - mean_oracle| / sqrt(s_gpu^2/R + s_oracle^2/R).

The test is a 3-sigma test of the whole family of m comparisons (m = 36
non-constant ones): the probability that a correct implementation fails it
is that of one 3-sigma test, 0.27 %. Applied to each comparison separately,
3 sigma would fail a correct implementation in 1 - 0.9973^m (about 9 %) of
seed choices, and the GPU runs are deterministic given their seeds, so such a
failure would be permanent. Two criteria, each at the family-wise 0.27 %
level: every z below the Bonferroni bound Phi^-1(1 - 0.0027 / (2 m)) (3.96
for m = 36), and sum z^2 below the 0.9973 quantile of chi-square with m
degrees of freedom (the quantile of independent comparisons; the observables
are correlated, which widens the spread of the sum)."""
import dataclasses
import json
import os

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ensemble_tiny.json")


def observables(m):
    return ([int(x) for x in m["n_alive"]] + [int(x) for x in m["events"][1:5]] + [int(m["injected"])] +
            [int(x) for x in np.asarray(m["absorbed"]).sum(axis=1)] + [float(m["i_sr"])] +
            [float(x) for x in m["ke"]])


def test_ensemble_means_agree_over_1000_steps():
    from paper_2402_08404_amd import pic
    from paper_2402_08404_amd import workloads as W
    gold = json.load(open(GOLDEN))
    names, steps = gold["names"], gold["steps"]
    R = len(gold["seeds"])
    orc = {s: np.array([gold["runs"][str(seed)][str(s)] for seed in gold["seeds"]], float) for s in steps}
    gpu = {s: [] for s in steps}
    for r in range(R):
        cfg = dataclasses.replace(W.tiny(), seed=1 + r)
        sim = pic.Simulation(cfg, caps=(60000, 8000, 4000), precision=pic.PIC_F64, solver=pic.PIC_SOLVER_MGCG,
                             step_rtol=1e-8)
        sim.load(W.initial_load(cfg, seed=1 + r))
        sim.step(1, pic.STEP_DEPOSIT)
        sim.solve(solver=pic.PIC_SOLVER_MGCG, rtol=1e-8)
        done = 0
        for s in steps:
            sim.step(s - done, pic.STEP_FULL)
            done = s
            gpu[s].append(observables(sim.moments()))
        print("seed", 1 + r, "done", flush=True)
        sim.close()
    from scipy import stats
    zs, const = [], []
    for s in steps:
        g, o = np.array(gpu[s], float), orc[s]
        mg, mo = g.mean(0), o.mean(0)
        se = np.sqrt(g.var(0, ddof=1) / R + o.var(0, ddof=1) / R)
        for k, name in enumerate(names):
            if se[k] == 0:
                const.append((s, name, mg[k], mo[k]))
                continue
            z = abs(mg[k] - mo[k]) / se[k]
            zs.append((s, name, z))
            print(f"step {s:4d} {name:16s} gpu {mg[k]:.6g} oracle {mo[k]:.6g} se {se[k]:.3g} z {z:.2f}", flush=True)
    # observables constant over both ensembles must be equal
    assert all(a == b for _, _, a, b in const), const
    m = len(zs)
    alpha = 2 * stats.norm.sf(3.0)                    # 0.0027, one 3-sigma test
    z_bound = stats.norm.isf(alpha / (2 * m))
    chi2 = sum(z * z for _, _, z in zs)
    chi2_bound = stats.chi2.isf(alpha, m)
    print(f"{m} comparisons: max z {max(z for _, _, z in zs):.2f} (bound {z_bound:.2f}), "
          f"sum z^2 {chi2:.1f} (bound {chi2_bound:.1f})", flush=True)
    bad = [(s, name, round(z, 2)) for s, name, z in zs if z > z_bound]
    assert not bad, bad
    assert chi2 <= chi2_bound
