"""Pins of the oracle's superparticle weights (Sec. 2.3.2), each against a
closed form or a statistic written here from the passage:

- N_coll: a pair of superparticles with weights w_a < w_b collides in
  Binomial(w_a, P) sub-particle collisions, P = 1 - exp(-u n w_b sigma dt);
- elastic and charge-exchange events between weighted superparticles split
  off the collided units and conserve weight, momentum and energy exactly;
- impact ionization of N_coll units: the neutral loses N_coll, an ion and an
  electron of weight N_coll appear, the kinetic energy drops by N_coll xi;
- field ionization of a neutral superparticle of weight w: Binomial(w, P dt);
- the injection weight of evaporated neutrals, min(ceil(max(1,
  sqrt((n_cell / n_max) N_inj))), w_max), with the atoms conserved;
- the deposit and the moments count every unit of a superparticle.
"""
import math

import numpy as np
import pytest
import scipy.constants as sc

import oracle
from paper_2402_08404_amd import workloads as W


def _cells(cfg, n, rng):
    pool = [(i, j, k) for k in range(4, cfg.nz - 4) for j in range(1, cfg.ny - 2) for i in range(1, cfg.nx - 2)]
    pick = rng.choice(len(pool), size=n, replace=False)
    return [pool[p] for p in pick]


def _pair_load(cells, rng, a, wa, wb, speed):
    n = len(cells)
    c = np.array(cells, float)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    la = {"x": c[:, 0] + 0.3, "y": c[:, 1] + 0.5, "z": c[:, 2] + 0.5, "vx": d[:, 0] * speed,
          "vy": d[:, 1] * speed, "vz": d[:, 2] * speed, "w": np.full(n, wa)}
    lb = {"x": c[:, 0] + 0.6, "y": c[:, 1] + 0.5, "z": c[:, 2] + 0.5, "vx": np.zeros(n), "vy": np.zeros(n),
          "vz": np.zeros(n), "w": np.full(n, wb)}
    return {a: la, "neutral": lb}


def _mom_energy(st, masses, sv):
    p = np.zeros(3)
    e = 0.0
    for s in range(3):
        w = st[s]["w"].astype(float)
        v = np.column_stack([st[s]["vx"], st[s]["vy"], st[s]["vz"]]) * sv
        p += masses[s] * (w[:, None] * v).sum(0)
        e += 0.5 * masses[s] * float((w * (v * v).sum(1)).sum())
    return p, e


def pin_ncoll_binomial():
    cfg = W.small(nx=24, ny=24, nz=24, tip_r=1e-9, tip_h=2e-9, seed=61)
    cfg.xs_el, cfg.xs_iz, cfg.xs_cx = W.constant_tables(4e-19, 0.0, 0.0)
    rng = np.random.default_rng(61)
    ncell, wa, wb = 3000, 6, 9
    u = 1.2e7
    cells = _cells(cfg, ncell, rng)
    o = oracle.Oracle(cfg, laplace=False)
    o.load(_pair_load(cells, rng, "e", wa, wb, u * cfg.dt / cfg.h))
    before = o.state()
    o.collide(oracle.COLL_MCC1)
    after = o.state()
    P = 1 - math.exp(-u * (1 / cfg.h ** 3) * wb * 4e-19 * cfg.dt)
    ncoll = int(o.events_w[1])
    mean, var = ncell * wa * P, ncell * wa * P * (1 - P)
    assert abs(ncoll - mean) < 3.5 * math.sqrt(var), (ncoll, mean)
    # per event N_coll is the weight the split-off electron (or the whole one) carries
    assert len(o.last_events) == int(np.sum(np.array([e[0] for e in o.last_events]) == 1))
    # weights, momentum and energy conserved
    for s in (0, 2):
        assert before[s]["w"].sum() == after[s]["w"].sum()
    masses = (sc.m_e, cfg.m_ion, cfg.m_ion)
    sv = cfg.h / cfg.dt
    p0, e0 = _mom_energy(before, masses, sv)
    p1, e1 = _mom_energy(after, masses, sv)
    assert np.abs(p1 - p0).max() <= 1e-10 * np.abs(p0).max()
    assert e1 == pytest.approx(e0, rel=1e-12)
    # split-off superparticles: new ids, weights summing with their parents'
    nsplit = o.splits
    assert nsplit > 0 and len(after[0]["id"]) + len(after[2]["id"]) == 2 * ncell + nsplit


def test_ncoll_binomial_and_conservation():
    pin_ncoll_binomial()


def pin_weighted_ionization():
    cfg = W.small(nx=24, ny=24, nz=24, tip_r=1e-9, tip_h=2e-9, seed=62)
    cfg.xs_el, cfg.xs_iz, cfg.xs_cx = W.constant_tables(0.0, 3e-19, 0.0)
    rng = np.random.default_rng(62)
    ncell, wa, wb = 2000, 3, 5
    u = 1.5e7                                   # 640 eV, far above xi
    cells = _cells(cfg, ncell, rng)
    o = oracle.Oracle(cfg, laplace=False)
    o.load(_pair_load(cells, rng, "e", wa, wb, u * cfg.dt / cfg.h))
    before = o.state()
    o.collide(oracle.COLL_MCC1)
    after = o.state()
    c = int(o.events_w[2])
    P = 1 - math.exp(-u * (1 / cfg.h ** 3) * wb * 3e-19 * cfg.dt)
    assert abs(c - ncell * wa * P) < 3.5 * math.sqrt(ncell * wa * P * (1 - P)), (c, ncell * wa * P)
    assert after[0]["w"].sum() == before[0]["w"].sum() + c
    assert after[1]["w"].sum() == c
    assert after[2]["w"].sum() == before[2]["w"].sum() - c
    # every product pair carries the N_coll of its event
    ev = {int(e[2]): e for e in o.last_events}
    ion_w = dict(zip(after[1]["id"].tolist(), after[1]["w"].tolist()))
    e_w = dict(zip(after[0]["id"].tolist(), after[0]["w"].tolist()))
    assert all(ion_w[int(e[3])] == e_w[int(e[4])] for e in ev.values())
    masses = (sc.m_e, cfg.m_ion, cfg.m_ion)
    sv = cfg.h / cfg.dt
    _, e0 = _mom_energy(before, masses, sv)
    _, e1 = _mom_energy(after, masses, sv)
    assert e0 - e1 == pytest.approx(c * cfg.xi * sc.e, rel=1e-6)


def test_weighted_impact_ionization():
    pin_weighted_ionization()


def pin_weighted_field_ionization():
    cfg = W.small(nx=24, ny=24, nz=48, tip_r=1e-9, tip_h=2e-9, seed=63)
    o = oracle.Oracle(cfg, laplace=False)
    F = 12e9
    o.set_phi(np.repeat(np.arange(cfg.nz) * cfg.h * F, cfg.nx * cfg.ny))
    rng = np.random.default_rng(63)
    N, w = 4000, 7
    pos = np.column_stack([rng.uniform(1, cfg.nx - 2, N), rng.uniform(1, cfg.ny - 2, N), rng.uniform(10, 40, N)])
    z = np.zeros(N)
    o.load({"neutral": {"x": pos[:, 0], "y": pos[:, 1], "z": pos[:, 2], "vx": z, "vy": z, "vz": z,
                        "w": np.full(N, w)}})
    o.collide(oracle.COLL_FI)
    p = o.adk_rate(F * 1e-9) * cfg.dt * 1e15
    c = int(o.events_w[4])
    assert abs(c - N * w * p) < 3.5 * math.sqrt(N * w * p * (1 - p)), (c, N * w * p)
    st = o.state()
    assert st[1]["w"].sum() == c and st[0]["w"].sum() == c and st[2]["w"].sum() == N * w - c


def test_weighted_field_ionization():
    pin_weighted_field_ionization()


def pin_injection_weights():
    cfg = W.tiny()
    cfg.surface_T = 3200.0
    cfg.dt = 4e-10              # hundreds of atoms per patch and step; nothing moves here
    cfg.fn_rings, cfg.fn_az = 1, 1
    cfg.w_max, cfg.n_max = 40, 1e28     # weights between 1 and w_max for these counts
    o = oracle.Oracle(cfg, laplace=False)
    rng = np.random.default_rng(64)
    o.cell_count = rng.integers(0, 60, size=o.cell_count.size).astype(np.int64)
    o.step_no = 3
    o.evaporate()
    st = o.state()[2]
    R, H = cfg.tip_r / cfg.h, cfg.tip_h / cfg.h
    zc, xc = H - R, (cfg.nx - 1) / 2
    # patch of every atom: 0 = the cap, 1 + q = the side ring q <= z < q + 1
    patch = np.where(st["z"] > zc + 1e-9, 0, 1 + np.floor(st["z"]).astype(np.int64))
    P = o.fn_patches()
    seen = 0
    for p in np.unique(patch):
        m = patch == p
        ws = st["w"][m][np.argsort(st["id"][m])]
        atoms = int(ws.sum())
        g = P[p]
        cnt = o.cell_count[((int(g[2] + g[5]) * (cfg.ny - 1) + int(g[1] + g[4])) * (cfg.nx - 1)
                            + int(g[0] + g[3]))]
        r = math.sqrt(cnt / cfg.h ** 3 / cfg.n_max * atoms)
        want = 1 if atoms <= 1 else min(math.ceil(max(1.0, r)), cfg.w_max)
        k = -(-atoms // want)
        assert len(ws) == k, (p, atoms, want, len(ws))
        assert (ws[:-1] == want).all() and ws[-1] == atoms - (k - 1) * want
        seen += int(want > 1)
    assert seen >= 3
    assert int(st["w"].sum()) == o.evap_atoms and len(st["w"]) == o.evaporated


def test_injection_weight_rule():
    pin_injection_weights()


def test_weighted_deposit_and_moments():
    cfg = W.tiny()
    o = oracle.Oracle(cfg, laplace=False)
    rng = np.random.default_rng(65)
    n = 500
    load = {}
    for name in ("e", "ion"):
        load[name] = {"x": rng.uniform(2, 28, n), "y": rng.uniform(2, 28, n), "z": rng.uniform(30, 60, n),
                      "vx": rng.normal(0, 0.01, n), "vy": rng.normal(0, 0.01, n), "vz": rng.normal(0, 0.01, n),
                      "w": rng.integers(1, 50, n)}
    o.load(load)
    Q = o.deposit()
    assert int(Q.sum()) == 2 ** 40 * int(load["ion"]["w"].sum() - load["e"]["w"].sum())
    m = o.moments()
    sv = cfg.h / cfg.dt
    for s, name, mass in ((0, "e", sc.m_e), (1, "ion", cfg.m_ion)):
        d = load[name]
        ke = np.sum(d["w"] * 0.5 * mass * (d["vx"] ** 2 + d["vy"] ** 2 + d["vz"] ** 2) * sv * sv)
        assert m["ke"][s] == pytest.approx(ke, rel=1e-12)
        assert m["n_phys"][s] == d["w"].sum()
