"""Writes ensemble_tiny.json: observables of R independent FP64 oracle runs of
the tiny workload (32 x 32 x 64 nodes at 2 nm, tip r = 4 nm, H = 40 nm,
10 GV/m; 20 000 e, 200 Cu+, 2 000 Cu near the tip; constant cross sections;
dt = 5e-17 s), seeds 101 .. 100 + R, each run for 1000 whole steps
(emission, push, collisions, field ionization, deposit, Poisson solve to
1e-8), recorded after 250, 500 and 1000 steps.

Only the oracle runs here (test infrastructure); the GPU ensemble test
compares its own runs on seeds 1 .. R with these values.

    python tests/golden/make_ensemble_tiny.py [R] [processes]
"""
import dataclasses
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

CHECKPOINTS = (250, 500, 1000)
NAMES = ["n_e", "n_ion", "n_neutral", "ev_elastic", "ev_ionize", "ev_cx", "ev_field_ion", "injected",
         "absorbed_e", "absorbed_ion", "absorbed_neutral", "i_sr", "ke_e", "ke_ion", "ke_neutral"]


def observables(m):
    return ([int(x) for x in m["n"]] + [int(x) for x in m["events"][1:5]] + [int(m["injected"])] +
            [int(x) for x in m["absorbed"].sum(axis=1)] + [float(m["i_sr"])] + [float(x) for x in m["ke"]])


def run(seed):
    import oracle
    from paper_2402_08404_amd import workloads as W
    cfg = dataclasses.replace(W.tiny(), seed=seed)
    o = oracle.Oracle(cfg)
    o.load(W.initial_load(cfg, seed=seed))
    o.deposit()
    o.solve(rtol=1e-8)
    out = {}
    t0 = time.time()
    for s in range(1, CHECKPOINTS[-1] + 1):
        o.step(rtol=1e-8)
        if s in CHECKPOINTS:
            out[str(s)] = observables(o.moments())
            print(f"seed {seed} step {s} ({time.time() - t0:.0f} s)", flush=True)
    return seed, out


def main():
    R = int(sys.argv[1]) if len(sys.argv) > 1 else 32
    procs = int(sys.argv[2]) if len(sys.argv) > 2 else 8
    seeds = list(range(101, 101 + R))
    with Pool(procs) as p:
        res = dict(p.map(run, seeds))
    doc = {"workload": "tiny", "steps": list(CHECKPOINTS), "names": NAMES, "seeds": seeds,
           "runs": {str(s): res[s] for s in seeds}}
    with open(os.path.join(HERE, "ensemble_tiny.json"), "w") as f:
        json.dump(doc, f, indent=0)


if __name__ == "__main__":
    main()
