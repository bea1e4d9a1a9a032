"""Pins of the oracle of the 2D axisymmetric (r, z) 2D3V variant
(oracle/rz.py; Sec. 2.2), each against a closed form:

- the finite-volume operator is exact for r^2 and z^2: A(r^2) = -4 times the
  axial coupling (the annulus area over pi), A(z^2) = -2 times it, on the
  axis too;
- without a tip the unit-anode potential is linear in z;
- a manufactured solution phi = sin(pi z / L) cos(pi r / r_max) (zero radial
  derivative on the axis and the side) converges at second order;
- the push without a field moves in a straight line in 3D: r_k =
  |(r0 + k v_r, k v_theta)|, and the angular momentum r v_theta is kept in a
  field (which has no azimuthal component);
- a particle crossing the axis with v_theta = 0 comes back mirrored;
- the deposit is exact: every particle adds 2^40 units, one on a node adds
  them all to that node.
"""
import math

import numpy as np
import pytest
import scipy.constants as sc

from oracle.rz import RZ, FREE


def _rz(nr=24, nz=48, tip_r=4e-9, tip_h=40e-9, h=2e-9):
    return RZ(nr, nz, h, tip_r, tip_h, 10e9, 5e-17, 63.546 * sc.atomic_mass)


def test_operator_exact_for_quadratics():
    o = _rz()
    nr, nz = o.nr, o.nz
    k, i = np.meshgrid(np.arange(nz), np.arange(nr), indexing="ij")
    for f, factor in (((i * i).astype(float), -4.0), ((k * k).astype(float), -2.0)):
        y = o.A @ f.reshape(-1)
        for kk in range(1, nz - 1):
            for ii in range(0, nr - 1):
                n = kk * nr + ii
                if o.type[n] != FREE:
                    continue
                _, _, cax = o.couplings(ii)
                assert y[n] == pytest.approx(factor * cax, abs=1e-9), (ii, kk)


def test_plates_without_tip_linear():
    o = RZ(16, 40, 2e-9, 0.0, 0.0, 10e9, 5e-17, 1e-25)
    z = np.repeat(np.arange(o.nz) / (o.nz - 1), o.nr)
    assert np.abs(o.phi1 - z).max() < 1e-12


def test_manufactured_second_order():
    errs = []
    for n in (16, 32, 64):
        o = RZ(n + 1, 2 * n + 1, 1.0 / n, 0.0, 0.0, 1.0, 1.0, 1.0)
        h = o.h
        rmax, L = n * h, 2 * n * h
        k, i = np.meshgrid(np.arange(o.nz), np.arange(o.nr), indexing="ij")
        r, z = i * h, k * h
        a, b = math.pi / rmax, math.pi / L
        exact = np.sin(b * z) * np.cos(a * r)
        # -laplacian in cylindrical coordinates; on the axis f'/r -> f''
        with np.errstate(divide="ignore", invalid="ignore"):
            frr = -a * a * np.cos(a * r)
            fr_r = np.where(r > 0, -a * np.sin(a * r) / np.where(r > 0, r, 1.0), -a * a)
        src = -(np.sin(b * z) * (frr + fr_r) - b * b * exact)
        # right-hand side: source times the control volume over pi h^2 (grid units)
        vol = np.array([o.couplings(ii)[2] for ii in range(o.nr)])[None, :] * np.ones((o.nz, 1))
        rhs = (src * vol * h * h).reshape(-1)
        held = o.type != FREE
        rhs[held] = exact.reshape(-1)[held]
        phi = o.solve_rhs(rhs)
        errs.append(np.abs(phi - exact.reshape(-1)).max())
    rates = [math.log2(errs[j] / errs[j + 1]) for j in range(2)]
    assert min(rates) > 1.8, (errs, rates)


def _single(o, s, r, z, vr, vt, vz):
    o.load(s, {"r": [r], "z": [z], "vr": [vr], "vt": [vt], "vz": [vz]}, [0])


def test_straight_line_in_3d():
    o = _rz()
    r0, vr, vt = 6.0, -0.31, 0.17
    _single(o, 2, r0, 30.0, vr, vt, 0.01)
    for k in range(1, 30):
        o.push()
        want = math.hypot(r0 + k * vr, k * vt)
        assert o.sp[2]["r"][0] == pytest.approx(want, rel=1e-12)
        speed = math.hypot(o.sp[2]["vr"][0], o.sp[2]["vt"][0])
        assert speed == pytest.approx(math.hypot(vr, vt), rel=1e-12)


def test_angular_momentum_kept_in_a_field():
    o = _rz()
    rng = np.random.default_rng(5)
    n = 200
    r = rng.uniform(3, 20, n)
    z = rng.uniform(25, 45, n)
    o.load(0, {"r": r, "z": z, "vr": rng.normal(0, 0.01, n), "vt": rng.normal(0, 0.01, n),
               "vz": rng.normal(0, 0.01, n)}, np.arange(n))
    L0 = dict(zip(o.sp[0]["id"].tolist(), (o.sp[0]["r"] * o.sp[0]["vt"]).tolist()))
    for _ in range(5):
        o.push()
    L1 = o.sp[0]["r"] * o.sp[0]["vt"]
    for i, l in zip(o.sp[0]["id"].tolist(), L1):
        assert l == pytest.approx(L0[i], rel=1e-12, abs=1e-15)


def test_axis_crossing_mirrors():
    o = _rz()
    _single(o, 2, 0.3, 30.0, -0.5, 0.0, 0.0)
    o.push()
    assert o.sp[2]["r"][0] == pytest.approx(0.2, abs=1e-15)
    assert o.sp[2]["vr"][0] == pytest.approx(0.5, abs=1e-15)


def test_deposit_exact():
    o = _rz()
    rng = np.random.default_rng(6)
    n = 500
    o.load(1, {"r": rng.uniform(0, 22, n), "z": rng.uniform(1, 46, n), "vr": np.zeros(n), "vt": np.zeros(n),
               "vz": np.zeros(n)}, np.arange(n))
    o.load(0, {"r": [5.0], "z": [30.0], "vr": [0.0], "vt": [0.0], "vz": [0.0]}, [n])
    Q = o.deposit()
    assert int(Q.sum()) == 2 ** 40 * (n - 1)
    o.load(1, {"r": [], "z": [], "vr": [], "vt": [], "vz": []}, [])
    Q = o.deposit()
    assert Q[30 * o.nr + 5] == -(2 ** 40) and np.count_nonzero(Q) == 1
