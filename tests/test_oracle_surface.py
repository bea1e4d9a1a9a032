"""Pins of the oracle's surface and circuit terms (Sec. 2.3.1, Sec. 2.3.3),
each against a closed form or a statistic written here from its definition:

- the Clausius-Clapeyron evaporation flux, at the boiling point (where the
  exponential is 1) and as a ratio between two temperatures;
- the expected number of evaporated atoms per step (flux x tip area x dt),
  the counts within their Poisson spread, the atoms on the surface, and their
  velocities: Rayleigh-distributed outward normal component and Gaussian
  tangential components of variance k_B T / m;
- the bombardment energy: ions reaching the cathode plane or the tip in a
  field-free box carry exactly sum m v^2 / 2;
- the RC circuit: with a constant gap current the gap voltage relaxes
  geometrically to V0 - R I;
- the Shockley-Ramo current of a push between parallel plates, I = sum q v.E0
  with E0 = -z/L.
"""
import math

import numpy as np
import pytest
import scipy.constants as sc
import scipy.stats as st

import oracle
from paper_2402_08404_amd import workloads as W

T_BOIL = 2835.0           # boiling point of Cu [K]
E_VAP = 3.43              # eV, the paper's value for Cu
P_ATM = sc.atm


def _flux(cfg, T):
    m = cfg.m_ion
    return P_ATM / math.sqrt(2 * math.pi * m * sc.k * T) * math.exp(E_VAP * sc.e / sc.k * (1 / T_BOIL - 1 / T))


def pin_evaporation_flux():
    cfg = W.tiny()
    o = oracle.Oracle(cfg, laplace=False)
    f_b = o.L.orc_evap_flux(o.c, T_BOIL)
    assert f_b == pytest.approx(P_ATM / math.sqrt(2 * math.pi * cfg.m_ion * sc.k * T_BOIL), rel=1e-12)
    for T in (1500.0, 2200.0, 3300.0):
        assert o.L.orc_evap_flux(o.c, T) == pytest.approx(_flux(cfg, T), rel=1e-12)
    assert o.L.orc_evap_flux(o.c, 0.0) == 0.0


def test_evaporation_flux_closed_form():
    pin_evaporation_flux()


def pin_evaporation_atoms():
    cfg = W.tiny()
    cfg.surface_T = 3000.0
    cfg.dt = 2e-11          # many atoms per step; nothing moves in this test
    cfg.fn_rings, cfg.fn_az = 8, 16
    o = oracle.Oracle(cfg, laplace=False)
    R, H = cfg.tip_r / cfg.h, cfg.tip_h / cfg.h
    area = (2 * math.pi * R * R + 2 * math.pi * R * (H - R)) * cfg.h ** 2
    per_step = _flux(cfg, cfg.surface_T) * area * cfg.dt
    steps = 30
    for s in range(steps):
        o.step_no = s
        o.evaporate()
    assert o.evap_expected == pytest.approx(steps * per_step, rel=1e-10)
    k = o.evaporated
    assert 200 < k and abs(k - o.evap_expected) < 3.5 * math.sqrt(o.evap_expected), (k, o.evap_expected)
    s = o.state()[2]
    assert len(s["id"]) == k and np.array_equal(s["id"], np.arange(k, dtype=np.uint32))
    xc = (cfg.nx - 1) / 2
    zc = H - R
    X, Y, Z = s["x"] - xc, s["y"] - xc, s["z"]
    # outward normal of the surface point each atom sits on (1e-3 outside)
    on_cap = Z > zc + 1e-9
    n = np.where(on_cap[:, None], np.column_stack([X, Y, Z - zc]), np.column_stack([X, Y, np.zeros_like(Z)]))
    d = np.linalg.norm(n, axis=1)
    np.testing.assert_allclose(d, R + 1e-3, rtol=1e-9)
    n /= d[:, None]
    sig = math.sqrt(sc.k * cfg.surface_T / cfg.m_ion) * cfg.dt / cfg.h
    v = np.column_stack([s["vx"], s["vy"], s["vz"]]) / sig
    vn = np.sum(v * n, axis=1)
    assert (vn > 0).all()
    # Rayleigh normal component (flux-weighted Maxwellian)
    assert st.kstest(vn, lambda x: 1 - np.exp(-x * x / 2)).pvalue > 1e-3
    vt = v - vn[:, None] * n
    t2 = np.sum(vt * vt, axis=1)     # sum of two unit Gaussians: exponential with mean 2
    assert st.kstest(t2, lambda x: 1 - np.exp(-x / 2)).pvalue > 1e-3


def test_evaporated_atoms_count_position_velocity():
    pin_evaporation_atoms()


def pin_bombardment_energy():
    cfg = W.tiny()
    o = oracle.Oracle(cfg, laplace=False)
    o.set_phi(np.zeros(cfg.nx * cfg.ny * cfg.nz))      # no field: velocities stay as loaded
    R, H = cfg.tip_r / cfg.h, cfg.tip_h / cfg.h
    xc = (cfg.nx - 1) / 2
    rng = np.random.default_rng(3)
    n = 40
    # ions moving into the cathode plane, ions moving into the tip side, ions
    # going elsewhere, electrons moving into the tip (not counted)
    zc0 = rng.uniform(0.05, 0.4, n)
    vz0 = -rng.uniform(0.5, 0.9, n)
    xt = xc + R + rng.uniform(0.05, 0.3, n)
    vxt = -rng.uniform(0.5, 0.9, n)
    load = {"ion": {"x": np.concatenate([rng.uniform(2, 8, n), xt, rng.uniform(2, 8, n)]),
                    "y": np.concatenate([rng.uniform(2, 8, n), np.full(n, xc), rng.uniform(2, 8, n)]),
                    "z": np.concatenate([zc0, rng.uniform(5, 15, n), rng.uniform(30, 40, n)]),
                    "vx": np.concatenate([rng.normal(0, 0.1, n), vxt, rng.normal(0, 0.1, n)]),
                    "vy": np.concatenate([rng.normal(0, 0.1, n), np.zeros(n), rng.normal(0, 0.1, n)]),
                    "vz": np.concatenate([vz0, np.zeros(n), rng.normal(0, 0.1, n)])},
            "e": {"x": xt, "y": np.full(n, xc), "z": rng.uniform(5, 15, n), "vx": vxt, "vy": np.zeros(n),
                  "vz": np.zeros(n)}}
    o.load(load)
    o.push()
    sv = cfg.h / cfg.dt
    vi = load["ion"]
    v2 = (vi["vx"] ** 2 + vi["vy"] ** 2 + vi["vz"] ** 2) * sv * sv
    e_cath = float(np.sum(0.5 * cfg.m_ion * v2[:n]))
    e_tip = float(np.sum(0.5 * cfg.m_ion * v2[n:2 * n]))
    assert o.absorbed[1, 1] == n and o.absorbed[1, 4] == n and o.absorbed[0, 4] == n
    assert o.bomb_energy[0] == pytest.approx(e_cath, rel=1e-12)
    assert o.bomb_energy[1] == pytest.approx(e_tip, rel=1e-12)


def test_bombardment_energy_tally():
    pin_bombardment_energy()


def pin_circuit_relaxation():
    cfg = W.tiny()
    cfg.circuit_R, cfg.circuit_C = 1e3, 1e-18
    o = oracle.Oracle(cfg, laplace=False)
    V0 = o.V0
    I = 2.5e-3
    a = cfg.dt / (cfg.circuit_R * cfg.circuit_C)
    vstar = V0 - cfg.circuit_R * I
    for n in range(1, 60):
        o.circuit_step(I)
        want = vstar + (V0 - vstar) * (1 - a) ** n
        assert o.V_gap == pytest.approx(want, rel=1e-12, abs=1e-12 * V0), n
    assert o.i_tot == pytest.approx((V0 - (vstar + (V0 - vstar) * (1 - a) ** 58)) / cfg.circuit_R, rel=1e-9)


def test_circuit_relaxation_closed_form():
    pin_circuit_relaxation()


def pin_shockley_ramo_push():
    h = 2e-9
    cfg = W.small(nx=16, ny=16, nz=32, h=h, tip_r=0.05 * h, tip_h=0.1 * h, field=1e3)  # two plates, weak field
    cfg.circuit_R, cfg.circuit_C = 1e3, 1e-18
    o = oracle.Oracle(cfg)
    L = (cfg.nz - 1) * h
    rng = np.random.default_rng(8)
    n = 50
    load = {}
    for name in ("e", "ion"):
        load[name] = {"x": rng.uniform(3, 12, n), "y": rng.uniform(3, 12, n), "z": rng.uniform(8, 22, n),
                      "vx": rng.normal(0, 0.01, n), "vy": rng.normal(0, 0.01, n), "vz": rng.normal(0, 0.02, n)}
    o.load(load)
    o.push()
    s = o.state()
    sv = h / cfg.dt
    want = (-sc.e) * np.sum(s[0]["vz"]) * sv * (-1 / L) + sc.e * np.sum(s[1]["vz"]) * sv * (-1 / L)
    assert len(s[0]["vz"]) == n and len(s[1]["vz"]) == n
    assert o.i_gap == pytest.approx(want, rel=1e-9)


def test_shockley_ramo_current_of_a_push():
    pin_shockley_ramo_push()
