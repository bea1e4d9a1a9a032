"""Pins of the oracle's same-species and Coulomb pairing (Table colls: Cu + Cu
elastic, Coulomb collisions of the charged particles), each computed here
from its definition rather than from the oracle's code:

- Cu-Cu elastic: pairs of neutrals with a known relative speed u collide at
  the rate P = 1 - exp(-u n sigma dt), n = N / h^3 (binomial statistics);
  every collision conserves momentum and energy exactly and scatters
  isotropically in the centre-of-mass frame (<cos> = 0, <cos^2> = 1/3);
- Coulomb (Takizuka-Abe): the scattering angle of a pair satisfies
  <tan^2(theta/2)> = q_a^2 q_b^2 n_L ln(Lambda) dt / (8 pi eps0^2 mu^2 u^3)
  at two speeds (the u^-3 law) and for e-e and e-Cu+ pairs (the reduced
  mass); momentum and energy are conserved;
- the pairing: ascending ids rotated by floor(U_c N) with U_c from Philox
  (cell, step, tag), consecutive pairs, the last one out for odd N (Cu-Cu),
  the first three in a triangle for odd N (Coulomb), every particle of the
  more numerous species in one e-Cu+ pair;
- recombination Cu+ + e -> Cu: pairs at a known relative speed recombine at
  the rate 1 - exp(-u n sigma dt); the atom appears at the ion's position
  with the pair's centre-of-mass velocity and a new id, in ascending order
  of the ion ids; the electron and the ion are gone.
"""
import math

import numpy as np
import pytest
import scipy.constants as sc

import oracle
from paper_2402_08404_amd import workloads as W

from test_oracle_readings import _draw

TAG_PAIR_NN, TAG_NN, TAG_PAIR_EE = 8, 9, 10


def _cfg(seed=31):
    cfg = W.small(nx=24, ny=24, nz=24, tip_r=1e-9, tip_h=2e-9, seed=seed)
    cfg.xs_el, cfg.xs_iz, cfg.xs_cx = W.constant_tables(0.0, 0.0, 0.0)
    return cfg


def _cells(cfg, n, rng):
    pool = [(i, j, k) for k in range(4, cfg.nz - 4) for j in range(1, cfg.ny - 2) for i in range(1, cfg.nx - 2)]
    return [pool[p] for p in rng.choice(len(pool), size=n, replace=False)]


def _two_per_cell(cells, rng, V):
    """Two particles per cell moving apart along a random axis at +-V (grid
    units per step): relative speed 2V for the pair whatever the pairing."""
    n = len(cells)
    c = np.repeat(np.array(cells, float), 2, axis=0)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    v = np.empty((2 * n, 3))
    v[0::2] = d * V
    v[1::2] = -d * V
    return {"x": c[:, 0] + rng.uniform(0.1, 0.9, 2 * n), "y": c[:, 1] + rng.uniform(0.1, 0.9, 2 * n),
            "z": c[:, 2] + rng.uniform(0.1, 0.9, 2 * n), "vx": v[:, 0], "vy": v[:, 1], "vz": v[:, 2]}


def _by_id(st):
    order = np.argsort(st["id"])
    return {k: v[order] for k, v in st.items()}


def pin_nn_rate_and_isotropy():
    cfg = _cfg()
    cfg.sigma_nn = 1e-14                          # P = 0.22 at these u, n, dt
    rng = np.random.default_rng(31)
    ncell, u = 6000, 2000.0                       # m/s relative speed
    V = 0.5 * u * cfg.dt / cfg.h
    cells = _cells(cfg, ncell, rng)
    o = oracle.Oracle(cfg, laplace=False)
    o.load({"neutral": _two_per_cell(cells, rng, V)})
    b = _by_id(o.state()[2])
    o.collide(oracle.COLL_NN)
    a = _by_id(o.state()[2])
    n = 2.0 / cfg.h ** 3
    P = 1.0 - math.exp(-u * n * cfg.sigma_nn * cfg.dt)
    vb = np.column_stack([b["vx"], b["vy"], b["vz"]])
    va = np.column_stack([a["vx"], a["vy"], a["vz"]])
    hit = np.abs(va - vb).max(axis=1)[0::2] > 1e-14 * V
    k = int(hit.sum())
    assert abs(k - ncell * P) < 3.5 * math.sqrt(ncell * P * (1 - P)), (k, ncell * P)
    # per pair: momentum and energy exactly, relative speed unchanged
    pb, pa = vb[0::2] + vb[1::2], va[0::2] + va[1::2]
    assert np.abs(pa - pb).max() < 1e-15 * 4 * V
    eb = (vb ** 2).sum(1)[0::2] + (vb ** 2).sum(1)[1::2]
    ea = (va ** 2).sum(1)[0::2] + (va ** 2).sum(1)[1::2]
    np.testing.assert_allclose(ea, eb, rtol=1e-13)
    # isotropic scattering: the angle between old and new relative velocity
    ub, ua = (vb[0::2] - vb[1::2])[hit], (va[0::2] - va[1::2])[hit]
    cos = (ub * ua).sum(1) / (np.linalg.norm(ub, axis=1) * np.linalg.norm(ua, axis=1))
    assert abs(cos.mean()) < 3.5 / math.sqrt(3 * k)
    assert abs((cos ** 2).mean() - 1 / 3) < 3.5 * math.sqrt(4 / 45 / k)


def test_nn_rate_conservation_isotropy():
    pin_nn_rate_and_isotropy()


def _ta_var(cfg, qa, qb, ma, mb, n_l, u, dts):
    mu = ma * mb / (ma + mb)
    return qa * qa * qb * qb * n_l * cfg.coulomb_log * dts / (8 * math.pi * sc.epsilon_0 ** 2 * mu * mu * u ** 3)


def pin_coulomb_angle():
    cfg = _cfg(seed=32)
    rng = np.random.default_rng(32)
    ncell = 4000
    n = 2.0 / cfg.h ** 3
    for species, mass, u in (("e", sc.m_e, 2e7), ("e", sc.m_e, 4e7), ("ion", cfg.m_ion, 2e5)):
        # ln(Lambda) chosen for a small mean square angle (0.01 at u = 2e7 m/s for electrons)
        cfg.coulomb_log = 10.0
        var10 = _ta_var(cfg, sc.e, sc.e, mass, mass, n, 2e7 if species == "e" else u, cfg.dt)
        cfg.coulomb_log = 10.0 * 0.01 / var10
        cells = _cells(cfg, ncell, rng)
        o = oracle.Oracle(cfg, laplace=False)
        V = 0.5 * u * cfg.dt / cfg.h
        o.load({species: _two_per_cell(cells, rng, V)})
        s = 0 if species == "e" else 1
        b = _by_id(o.state()[s])
        o.collide(oracle.COLL_COUL)
        a = _by_id(o.state()[s])
        vb = np.column_stack([b["vx"], b["vy"], b["vz"]])
        va = np.column_stack([a["vx"], a["vy"], a["vz"]])
        ub, ua = vb[0::2] - vb[1::2], va[0::2] - va[1::2]
        np.testing.assert_allclose(np.linalg.norm(ua, axis=1), np.linalg.norm(ub, axis=1), rtol=1e-12)
        assert np.abs((va[0::2] + va[1::2]) - (vb[0::2] + vb[1::2])).max() < 1e-14 * 2 * V
        cos = np.clip((ub * ua).sum(1) / (np.linalg.norm(ub, axis=1) * np.linalg.norm(ua, axis=1)), -1, 1)
        t2 = (1 - cos) / (1 + cos)                 # tan^2(theta / 2)
        want = _ta_var(cfg, sc.e, sc.e, mass, mass, n, u, cfg.dt)
        assert abs(t2.mean() - want) < 3.5 * want * math.sqrt(2.0 / ncell), (species, u, t2.mean(), want)


def test_coulomb_scattering_angle():
    pin_coulomb_angle()


def pin_coulomb_e_ion():
    """Cells of 5 electrons (one velocity per cell) and 2 resting ions: every
    electron scatters once (the ions twice or three times), each cell keeps
    its momentum and energy, and the mean square angle of the electrons
    follows the e-Cu+ variance with n_L = 2 / h^3 and the reduced mass."""
    cfg = _cfg(seed=33)
    rng = np.random.default_rng(33)
    ncell, u = 3000, 2e7
    n_l = 2.0 / cfg.h ** 3
    cfg.coulomb_log = 10.0
    v10 = _ta_var(cfg, sc.e, sc.e, sc.m_e, cfg.m_ion, n_l, u, cfg.dt)
    cfg.coulomb_log = 10.0 * 0.002 / v10
    cells = _cells(cfg, ncell, rng)
    c = np.array(cells, float)
    # the five electrons of a cell share one velocity, so that they do not
    # scatter off each other (u = 0) and only the e-Cu+ pairs act
    d = rng.standard_normal((ncell, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    ve = np.repeat(d, 5, axis=0) * u * cfg.dt / cfg.h
    ce = np.repeat(c, 5, axis=0)
    ci = np.repeat(c, 2, axis=0)
    z = np.zeros(ncell * 2)
    load = {"e": {"x": ce[:, 0] + 0.5, "y": ce[:, 1] + 0.5, "z": ce[:, 2] + 0.5, "vx": ve[:, 0], "vy": ve[:, 1],
                  "vz": ve[:, 2]},
            "ion": {"x": ci[:, 0] + 0.4, "y": ci[:, 1] + 0.4, "z": ci[:, 2] + 0.4, "vx": z, "vy": z, "vz": z}}
    o = oracle.Oracle(cfg, laplace=False)
    o.load(load)
    be, bi = _by_id(o.state()[0]), _by_id(o.state()[1])
    o.collide(oracle.COLL_COUL)
    ae, ai = _by_id(o.state()[0]), _by_id(o.state()[1])
    V = lambda d: np.column_stack([d["vx"], d["vy"], d["vz"]])
    pe = sc.m_e * (V(ae) - V(be)).reshape(ncell, 5, 3).sum(1)
    pi = cfg.m_ion * (V(ai) - V(bi)).reshape(ncell, 2, 3).sum(1)
    assert np.abs(pe + pi).max() < 1e-12 * sc.m_e * np.abs(ve).max()
    ke = lambda d, m, k: 0.5 * m * (V(d) ** 2).sum(1).reshape(ncell, k).sum(1)
    np.testing.assert_allclose(ke(ae, sc.m_e, 5) + ke(ai, cfg.m_ion, 2), ke(be, sc.m_e, 5) + ke(bi, cfg.m_ion, 2),
                               rtol=1e-10)
    assert (np.abs(V(ae) - V(be)).max(axis=1) > 0).all()
    # electrons scatter off nearly resting ions: the angle of each electron's
    # velocity change follows the e-Cu+ variance (ions move ~1e-4 u by then)
    ub, ua = V(be), V(ae)
    cos = np.clip((ub * ua).sum(1) / (np.linalg.norm(ub, axis=1) * np.linalg.norm(ua, axis=1)), -1, 1)
    t2 = (1 - cos) / (1 + cos)
    want = _ta_var(cfg, sc.e, sc.e, sc.m_e, cfg.m_ion, n_l, u, cfg.dt)
    assert abs(t2.mean() - want) < 3.5 * want * math.sqrt(2.0 / len(t2)) + 0.02 * want, (t2.mean(), want)


def test_coulomb_electron_ion():
    pin_coulomb_e_ion()


def pin_pairing_enumerated():
    """Neutral cells of N = 2 .. 9 with a cross section making P = 1: the
    pairs are (q0, q1), (q2, q3), .. of the ids rotated by floor(U_c N), and
    with N odd the last one keeps its velocity; e-e Coulomb cells of N = 3
    scatter all three."""
    cfg = _cfg(seed=34)
    cfg.sigma_nn = 1e-10
    rng = np.random.default_rng(34)
    counts = list(range(2, 10)) * 4
    cells = _cells(cfg, len(counts), rng)
    cols = {k: [] for k in ("x", "y", "z", "vx", "vy", "vz")}
    for (i, j, k), N in zip(cells, counts):
        cols["x"].append(i + rng.uniform(0.1, 0.9, N))
        cols["y"].append(j + rng.uniform(0.1, 0.9, N))
        cols["z"].append(k + rng.uniform(0.1, 0.9, N))
        for key in ("vx", "vy", "vz"):
            cols[key].append(rng.normal(0, 1e-3, N))
    load = {"neutral": {k: np.concatenate(v) for k, v in cols.items()}}
    o = oracle.Oracle(cfg, laplace=False)
    o.load(load)
    b = _by_id(o.state()[2])
    o.collide(oracle.COLL_NN)
    a = _by_id(o.state()[2])
    dv = np.column_stack([a[k] - b[k] for k in ("vx", "vy", "vz")])
    base = 0
    for (i, j, k), N in zip(cells, counts):
        ids = list(range(base, base + N))
        base += N
        cell = (k * (cfg.ny - 1) + j) * (cfg.nx - 1) + i
        uc, _ = _draw(cfg.seed, cell, 0, TAG_PAIR_NN, 0)
        sh = min(int(math.floor(uc * N)), N - 1)
        q = [ids[(sh + t) % N] for t in range(N)]
        for t in range(0, N - 1, 2):
            a_, b_ = q[t], q[t + 1]
            assert np.abs(dv[a_]).max() > 0 and np.allclose(dv[a_], -dv[b_], rtol=1e-12, atol=1e-18)
        if N % 2:
            assert np.abs(dv[q[-1]]).max() == 0.0


def test_pairing_enumerated():
    pin_pairing_enumerated()


def test_coulomb_triangle_for_odd_cells():
    cfg = _cfg(seed=35)
    rng = np.random.default_rng(35)
    cells = _cells(cfg, 200, rng)
    c = np.repeat(np.array(cells, float), 3, axis=0)
    v = rng.normal(0, 0.05, (600, 3))
    o = oracle.Oracle(cfg, laplace=False)
    o.load({"e": {"x": c[:, 0] + 0.5, "y": c[:, 1] + 0.5, "z": c[:, 2] + 0.5, "vx": v[:, 0], "vy": v[:, 1],
                  "vz": v[:, 2]}})
    b = _by_id(o.state()[0])
    o.collide(oracle.COLL_COUL)
    a = _by_id(o.state()[0])
    vb = np.column_stack([b["vx"], b["vy"], b["vz"]]).reshape(200, 3, 3)
    va = np.column_stack([a["vx"], a["vy"], a["vz"]]).reshape(200, 3, 3)
    assert (np.abs(va - vb).max(axis=2) > 0).all()
    np.testing.assert_allclose(va.sum(1), vb.sum(1), atol=1e-15)
    np.testing.assert_allclose((va ** 2).sum((1, 2)), (vb ** 2).sum((1, 2)), rtol=1e-12)


def test_weighted_particles_rejected():
    cfg = _cfg()
    o = oracle.Oracle(cfg, laplace=False)
    o.load({"e": {"x": [5.5, 5.6], "y": [5.5, 5.5], "z": [5.5, 5.5], "vx": [0.1, 0], "vy": [0, 0], "vz": [0, 0],
                  "w": [2, 1]}})
    with pytest.raises(ValueError):
        o.collide(oracle.COLL_COUL)


def pin_recombination():
    cfg = _cfg(seed=36)
    cfg.sigma_rec = 5e-18                         # P = 0.27 at u = 1e7 m/s
    rng = np.random.default_rng(36)
    ncell, u = 5000, 1e7
    cells = _cells(cfg, ncell, rng)
    c = np.array(cells, float)
    d = rng.standard_normal((ncell, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    ve = d * u * cfg.dt / cfg.h
    vi = rng.normal(0, 1e-4, (ncell, 3))
    load = {"e": {"x": c[:, 0] + 0.3, "y": c[:, 1] + 0.5, "z": c[:, 2] + 0.5, "vx": ve[:, 0], "vy": ve[:, 1],
                  "vz": ve[:, 2]},
            "ion": {"x": c[:, 0] + 0.6, "y": c[:, 1] + 0.4, "z": c[:, 2] + 0.7, "vx": vi[:, 0], "vy": vi[:, 1],
                    "vz": vi[:, 2]}}
    o = oracle.Oracle(cfg, laplace=False)
    o.load(load)
    next0 = o.next_id
    o.collide(oracle.COLL_REC)
    st = o.state()
    k = o.recombinations
    urel = np.linalg.norm(ve - vi, axis=1) * cfg.h / cfg.dt
    P = 1.0 - np.exp(-urel * (1.0 / cfg.h ** 3) * cfg.sigma_rec * cfg.dt)
    assert abs(k - P.sum()) < 3.5 * math.sqrt((P * (1 - P)).sum()), (k, P.sum())
    gone_e = sorted(set(range(ncell)) - set(int(i) for i in st[0]["id"]))
    gone_i = sorted(set(range(ncell, 2 * ncell)) - set(int(i) for i in st[1]["id"]))
    assert len(gone_e) == len(gone_i) == k > 500
    # one electron and one ion per cell: the pair of cell j is (j, ncell + j)
    assert [g - ncell for g in gone_i] == gone_e
    nn = st[2]
    assert list(nn["id"]) == list(range(next0, next0 + k))
    j = np.array(gone_e)
    mt = sc.m_e + cfg.m_ion
    for key, col in (("vx", 0), ("vy", 1), ("vz", 2)):
        want = (sc.m_e * ve[j, col] + cfg.m_ion * vi[j, col]) / mt
        np.testing.assert_allclose(nn[key], want, rtol=1e-12, atol=1e-18)
    for key in ("x", "y", "z"):
        np.testing.assert_array_equal(nn[key], load["ion"][key][j])


def test_recombination():
    pin_recombination()
