"""Pins of the collision, field-ionization and emission stages of the
axisymmetric oracle (oracle/rz.py; Sec. 2.2 with the processes of Table colls,
Eqs. colp, du, newv, dfi and the Fowler-Nordheim emission of Sec. 2.3.1),
each against a conservation law, an exact property of the process or the
statistics of a closed-form probability:

- elastic (e, Cu): momentum and kinetic energy of every pair are kept;
- charge exchange (Cu+, Cu): the two velocities are exchanged exactly;
- impact ionization: the ion keeps the neutral's position and velocity, the
  two electrons share E - xi in the neutral's frame, the ids continue in
  neutral-id order (ion, then electron);
- no particle takes part in two events of a step;
- the event count of a class over many cells with one relative speed
  follows P = 1 - exp(-u n sigma dt) with n = N_t over the annular cell
  volume pi (2 i + 1) h^3;
- field ionization: the count over many neutrals follows the ADK rate of
  their field times dt (in fs); none above the barrier-suppression field;
- emission: the ring patches tile the tip surface (areas add up to
  2 pi R^2 + 2 pi R (H - R)), their points lie on it with unit normals,
  electrons start 10^-3 spacings out, and the count per patch averages
  J A h^2 dt / e.
"""
import copy
import math

import numpy as np
import pytest
import scipy.constants as sc

from oracle.rz import RZ, XI2_CU, XI_CU

M_CU = 63.546 * sc.atomic_mass
EMIN, EMAX, NTAB = 1e-2, 1e4, 64


def _tables(el=0.0, iz=0.0, cx=0.0, iz2=None, izi=None):
    E = EMIN * (EMAX / EMIN) ** (np.arange(NTAB) / (NTAB - 1))
    t = (EMIN, EMAX, np.full(NTAB, el), np.where(E > XI_CU, iz, 0.0), np.full(NTAB, cx))
    if iz2 is not None:
        t = t + (np.where(E > XI_CU + XI2_CU, iz2, 0.0), np.where(E > XI2_CU, izi, 0.0))
    return t


def _rz(xs=None, apex=10e9, seed=7, nr=24, nz=48):
    cu2 = xs is not None and len(xs) > 5
    return RZ(nr, nz, 2e-9, 4e-9, 40e-9, apex, 5e-17, M_CU, seed=seed, xs=xs, cu2=cu2)


def _fill(o, rng, counts, cells, speed, rest_neutrals=False):
    """counts[s] particles of species s in each (i, k) cell of cells, with
    isotropic velocities of magnitude speed[s] (grid units per step)."""
    nid = 0
    for s in range(3):
        rr, zz = [], []
        for (i, k) in cells:
            rr.append(i + rng.uniform(0.05, 0.95, counts[s]))
            zz.append(k + rng.uniform(0.05, 0.95, counts[s]))
        r = np.concatenate(rr) if rr else np.zeros(0)
        z = np.concatenate(zz) if zz else np.zeros(0)
        m = len(r)
        ct = rng.uniform(-1, 1, m)
        ph = rng.uniform(0, 2 * math.pi, m)
        st = np.sqrt(1 - ct * ct)
        v = 0.0 if (s == 2 and rest_neutrals) else speed[s]
        o.load(s, {"r": r, "z": z, "vr": v * st * np.cos(ph), "vt": v * st * np.sin(ph), "vz": v * ct},
               np.arange(nid, nid + m))
        nid += m


def _by_id(d):
    return {int(i): p for p, i in enumerate(d["id"])}


def _vel(d, p):
    return np.array([d["vr"][p], d["vt"][p], d["vz"][p]])


_SP_A = {1: 0, 2: 0, 3: 1, 5: 0, 6: 0}
_SP_B = {1: 2, 2: 2, 3: 2, 4: 2, 5: 2, 6: 1}


def _participation(ev):
    seen = set()
    for kind, a, b in ev:
        xs = ((_SP_B[kind], b),) if kind == 4 else ((_SP_A[kind], a), (_SP_B[kind], b))
        for x in xs:
            assert x not in seen, ("twice", kind, x)
            seen.add(x)


def pin_elastic_conservation():
    o = _rz(_tables(el=3e-16))
    rng = np.random.default_rng(1)
    _fill(o, rng, (12, 0, 9), [(i, k) for i in (3, 8, 14) for k in (26, 30, 34)], (0.05, 0.0, 0.002))
    before = copy.deepcopy(o.sp)
    ev = o.collide()
    assert len(ev) > 20 and all(k == 1 for k, _, _ in ev)
    _participation(ev)
    ia, ib = _by_id(before[0]), _by_id(before[2])
    ja, jb = _by_id(o.sp[0]), _by_id(o.sp[2])
    for _, a, b in ev:
        va0, vb0 = _vel(before[0], ia[a]), _vel(before[2], ib[b])
        va1, vb1 = _vel(o.sp[0], ja[a]), _vel(o.sp[2], jb[b])
        p0, p1 = sc.m_e * va0 + M_CU * vb0, sc.m_e * va1 + M_CU * vb1
        assert np.abs(p1 - p0).max() <= 1e-12 * np.abs(M_CU * vb0).max() + 1e-12 * sc.m_e * np.abs(va0).max()
        e0 = sc.m_e * va0 @ va0 + M_CU * vb0 @ vb0
        e1 = sc.m_e * va1 @ va1 + M_CU * vb1 @ vb1
        assert e1 == pytest.approx(e0, rel=1e-11)
        assert np.abs(va1 - va0).max() > 0.0


def pin_cx_swap():
    o = _rz(_tables(cx=2e-15))
    rng = np.random.default_rng(2)
    _fill(o, rng, (0, 10, 14), [(i, k) for i in (2, 9) for k in (25, 33)], (0.0, 0.003, 0.001))
    before = copy.deepcopy(o.sp)
    ev = o.collide()
    assert len(ev) > 5 and all(k == 3 for k, _, _ in ev)
    _participation(ev)
    ia, ib = _by_id(before[1]), _by_id(before[2])
    ja, jb = _by_id(o.sp[1]), _by_id(o.sp[2])
    for _, a, b in ev:
        assert np.array_equal(_vel(o.sp[1], ja[a]), _vel(before[2], ib[b]))
        assert np.array_equal(_vel(o.sp[2], jb[b]), _vel(before[1], ia[a]))
    # the particles without an event keep their velocities
    hit = {b for _, _, b in ev}
    for i, p in ib.items():
        if i not in hit:
            assert np.array_equal(_vel(o.sp[2], jb[i]), _vel(before[2], p))


def pin_ionization():
    o = _rz(_tables(iz=1e-16))
    rng = np.random.default_rng(3)
    _fill(o, rng, (9, 0, 11), [(i, k) for i in (4, 12) for k in (27, 31, 35)], (0.1, 0.0, 0.002))
    before = copy.deepcopy(o.sp)
    nid0 = o.next_id
    ev = o.collide()
    assert len(ev) > 10 and all(k == 2 for k, _, _ in ev)
    _participation(ev)
    sv = o.h / o.dt
    ia, ib = _by_id(before[0]), _by_id(before[2])
    ja, jion, jel = _by_id(o.sp[0]), _by_id(o.sp[1]), _by_id(o.sp[0])
    neutral_order = sorted(b for _, _, b in ev)
    for _, a, b in ev:
        r = neutral_order.index(b)
        ion, el = nid0 + 2 * r, nid0 + 2 * r + 1
        assert b not in _by_id(o.sp[2])
        assert ion in jion and el in jel and el not in jion, (ion, el)
        pn = ib[b]
        vn = _vel(before[2], pn)
        assert np.array_equal(_vel(o.sp[1], jion[ion]), vn)
        for d, j in ((o.sp[1], jion[ion]), (o.sp[0], jel[el])):
            assert d["r"][j] == before[2]["r"][pn] and d["z"][j] == before[2]["z"][pn]
        u = (_vel(before[0], ia[a]) - vn) * sv
        E = 0.5 * sc.m_e * (u @ u) / sc.e
        w1 = (_vel(o.sp[0], ja[a]) - vn) * sv
        w2 = (_vel(o.sp[0], jel[el]) - vn) * sv
        E12 = 0.5 * sc.m_e * (w1 @ w1 + w2 @ w2) / sc.e
        assert E12 == pytest.approx(E - XI_CU, rel=1e-9, abs=1e-9)
    assert o.next_id == nid0 + 2 * len(ev)


def pin_collision_rate():
    """Electrons of one speed against neutrals at rest in cells of columns
    i = 0 .. 5: the elastic count over 30 steps against the sum of the pair
    probabilities with the annular cell volume."""
    sig = 1e-17
    o = _rz(_tables(el=sig), seed=11)
    rng = np.random.default_rng(4)
    cells = [(i, k) for i in range(6) for k in (26, 30, 34, 38)]
    nE, nN = 6, 10
    speed = 0.04
    _fill(o, rng, (nE, 0, nN), cells, (speed, 0.0, 0.0), rest_neutrals=True)
    u = speed * o.h / o.dt
    want = 0.0
    for (i, k) in cells:
        vol = math.pi * (2 * i + 1) * o.h ** 3
        want += nE * (1.0 - math.exp(-u * (nN / vol) * sig * o.dt))
    want *= 30
    state = copy.deepcopy(o.sp)
    got = 0
    for step in range(30):
        o.sp = copy.deepcopy(state)
        o.step_no = step
        got += sum(1 for k, _, _ in o.collide() if k == 1)
    sd = math.sqrt(want)
    assert abs(got - want) <= 5.0 * sd, (got, want)
    assert 0.05 * 30 * nE * len(cells) < want < 0.6 * 30 * nE * len(cells)


def pin_field_ionization():
    """Neutrals on a shell around the apex: the count against the sum of
    their ADK probabilities; none above the barrier-suppression field."""
    o = _rz(apex=25e9, seed=5)
    rng = np.random.default_rng(6)
    n = 4000
    th = rng.uniform(0, 0.5 * math.pi, n)
    rad = o.R + rng.uniform(0.3, 2.0, n)
    zc = o.H - o.R
    r, z = rad * np.sin(th), zc + rad * np.cos(th)
    o.load(2, {"r": r, "z": z, "vr": np.zeros(n), "vt": np.zeros(n), "vz": np.zeros(n)}, np.arange(n))
    want = 0.0
    for p in range(n):
        er, ez = o.gather(r[p], z[p])
        Eg = math.hypot(er, ez) * 1e-9
        assert Eg < 1.5 * XI_CU ** 1.5
        want += min(o.adk_rate(Eg) * o.dt * 1e15, 1.0)
    ev = o.collide()
    got = sum(1 for k, _, _ in ev if k == 4)
    assert want > 30, want
    assert abs(got - want) <= 5.0 * math.sqrt(want), (got, want)
    # above the barrier-suppression field nothing ionizes
    o2 = _rz(apex=60e9, seed=5)
    o2.load(2, {"r": r, "z": z, "vr": np.zeros(n), "vt": np.zeros(n), "vz": np.zeros(n)}, np.arange(n))
    strong = [p for p in range(n) if math.hypot(*o2.gather(r[p], z[p])) * 1e-9 > 1.5 * XI_CU ** 1.5]
    assert len(strong) > 100
    hit = {b for k, _, b in o2.collide() if k == 4}
    assert not hit & set(strong)


def pin_emission_geometry():
    o = _rz(apex=20e9)
    R, zc = o.R, o.H - o.R
    area = sum(o.patch_point(p, 0.5)[4] for p in range(o.patches()))
    assert area == pytest.approx(2 * math.pi * R * R + 2 * math.pi * R * zc, rel=1e-12)
    for p in range(o.patches()):
        for ua in (0.0, 0.37, 1.0):
            r, z, nr_, nz_, _ = o.patch_point(p, ua)
            assert nr_ * nr_ + nz_ * nz_ == pytest.approx(1.0, abs=1e-12)
            if z > zc:
                assert r * r + (z - zc) ** 2 == pytest.approx(R * R, rel=1e-12)
                assert (r / R, (z - zc) / R) == pytest.approx((nr_, nz_), abs=1e-12)
            else:
                assert r == pytest.approx(R) and (nr_, nz_) == (1.0, 0.0)
    added = o.emit()
    e = o.sp[0]
    assert added == len(e["id"]) > 0
    assert np.array_equal(e["id"], np.arange(added))
    for p in range(added):
        d = math.hypot(e["r"][p], max(e["z"][p] - zc, 0.0)) - R if e["z"][p] > zc else e["r"][p] - R
        assert d == pytest.approx(1e-3, abs=1e-9)
        assert e["vr"][p] == e["vt"][p] == e["vz"][p] == 0.0


def pin_emission_count():
    o = _rz(apex=15e9)
    want_step = 0.0
    for p in range(o.patches()):
        r, z, nr_, nz_, area = o.patch_point(p, 0.5)
        F = o.interp(o.phi, r + nr_, z + nz_) / o.h
        want_step += o.fn_current(F) * area * o.h ** 2 * o.dt / sc.e
    steps = 60
    got = 0
    for s in range(steps):
        o.step_no = s
        got += o.emit()
    want = want_step * steps
    assert want > 50, want
    assert abs(got - want) <= 5.0 * math.sqrt(want) + 1.0, (got, want)


def pin_double_ionization():
    """Cu + e -> Cu2+ + 3e: the ion at the neutral's place and velocity with
    charge state 2, three electrons sharing E - xi - xi2 in the neutral's
    frame, the ids in neutral-id order (ion, then two electrons)."""
    o = _rz(_tables(iz2=1e-16, izi=0.0))
    rng = np.random.default_rng(13)
    _fill(o, rng, (9, 0, 11), [(i, k) for i in (4, 12) for k in (27, 31, 35)], (0.12, 0.0, 0.002))
    before = copy.deepcopy(o.sp)
    nid0 = o.next_id
    ev = o.collide()
    assert len(ev) > 10 and all(k == 5 for k, _, _ in ev), ev[:3]
    _participation(ev)
    sv = o.h / o.dt
    ia, ib = _by_id(before[0]), _by_id(before[2])
    je, jion = _by_id(o.sp[0]), _by_id(o.sp[1])
    order = sorted(b for _, _, b in ev)
    for _, a, b in ev:
        r = order.index(b)
        ion, e1, e2 = nid0 + 3 * r, nid0 + 3 * r + 1, nid0 + 3 * r + 2
        assert ion in jion and e1 in je and e2 in je and e1 not in jion, (ion, e1, e2)
        pn = ib[b]
        vn = _vel(before[2], pn)
        assert o.sp[1]["q"][jion[ion]] == 2
        assert np.array_equal(_vel(o.sp[1], jion[ion]), vn)
        for j in (jion[ion],):
            assert o.sp[1]["r"][j] == before[2]["r"][pn] and o.sp[1]["z"][j] == before[2]["z"][pn]
        for e in (e1, e2):
            assert o.sp[0]["r"][je[e]] == before[2]["r"][pn] and o.sp[0]["z"][je[e]] == before[2]["z"][pn]
        u = (_vel(before[0], ia[a]) - vn) * sv
        E = 0.5 * sc.m_e * (u @ u) / sc.e
        w = [(_vel(o.sp[0], je[x]) - vn) * sv for x in (a, e1, e2)]
        E3 = 0.5 * sc.m_e * sum(x @ x for x in w) / sc.e
        assert E3 == pytest.approx(E - XI_CU - XI2_CU, rel=1e-9, abs=1e-9)
    assert o.next_id == nid0 + 3 * len(ev)


def pin_ion_ionization():
    """Cu+ + e -> Cu2+ + 2e: the ion keeps its place, id and velocity and
    takes charge state 2; the two electrons share E - xi2 in the ion's
    frame; ions already at charge state 2 are not ionized again."""
    o = _rz(_tables(iz2=0.0, izi=1e-16))
    rng = np.random.default_rng(14)
    cells = [(i, k) for i in (4, 12) for k in (27, 31, 35)]
    _fill(o, rng, (9, 11, 0), cells, (0.1, 0.002, 0.0))
    o.sp[1]["q"][::3] = 2
    before = copy.deepcopy(o.sp)
    nid0 = o.next_id
    ev = o.collide()
    assert len(ev) > 10 and all(k == 6 for k, _, _ in ev), ev[:3]
    _participation(ev)
    sv = o.h / o.dt
    ia, ii = _by_id(before[0]), _by_id(before[1])
    je, jion = _by_id(o.sp[0]), _by_id(o.sp[1])
    order = sorted(b for _, _, b in ev)
    for _, a, b in ev:
        assert before[1]["q"][ii[b]] == 1
        assert o.sp[1]["q"][jion[b]] == 2
        assert np.array_equal(_vel(o.sp[1], jion[b]), _vel(before[1], ii[b]))
        e = nid0 + order.index(b)
        assert e in je
        assert o.sp[0]["r"][je[e]] == before[1]["r"][ii[b]] and o.sp[0]["z"][je[e]] == before[1]["z"][ii[b]]
        vi = _vel(before[1], ii[b])
        u = (_vel(before[0], ia[a]) - vi) * sv
        E = 0.5 * sc.m_e * (u @ u) / sc.e
        w = [(_vel(o.sp[0], je[x]) - vi) * sv for x in (a, e)]
        E2 = 0.5 * sc.m_e * sum(x @ x for x in w) / sc.e
        assert E2 == pytest.approx(E - XI2_CU, rel=1e-9, abs=1e-9)
    assert o.next_id == nid0 + len(ev)
    assert int((o.sp[1]["q"] == 2).sum()) == int((before[1]["q"] == 2).sum()) + len(ev)


def pin_ion_ionization_rate():
    """Electrons of one speed against Cu+ at rest in cells of columns 0-5:
    the count over 30 steps against the sum of the pair probabilities with
    the annular cell volume."""
    sig = 1e-17
    o = _rz(_tables(iz2=0.0, izi=sig), seed=19)
    rng = np.random.default_rng(15)
    cells = [(i, k) for i in range(6) for k in (26, 30, 34, 38)]
    nE, nI = 6, 10
    speed = 0.1
    _fill(o, rng, (nE, nI, 0), cells, (speed, 0.0, 0.0))
    u = speed * o.h / o.dt
    want = 0.0
    for (i, k) in cells:
        vol = math.pi * (2 * i + 1) * o.h ** 3
        want += nE * (1.0 - math.exp(-u * (nI / vol) * sig * o.dt))
    want *= 30
    state = copy.deepcopy(o.sp)
    nid = o.next_id
    got = 0
    for step in range(30):
        o.sp = copy.deepcopy(state)
        o.next_id = nid
        o.step_no = step
        got += sum(1 for k, _, _ in o.collide() if k == 6)
    assert abs(got - want) <= 5.0 * math.sqrt(want), (got, want)
    assert want > 100, want


def pin_cu2_push_deposit():
    """A Cu2+ ion takes twice the kick of a Cu+ ion at the same place and
    deposits twice its charge."""
    o = _rz(_tables(iz2=0.0, izi=0.0), apex=12e9)
    r = np.array([6.3, 6.3, 9.1, 9.1])
    z = np.array([30.2, 30.2, 33.7, 33.7])
    zero = np.zeros(4)
    o.load(1, {"r": r, "z": z, "vr": zero, "vt": zero, "vz": zero, "q": [1, 2, 1, 2]}, np.arange(4))
    o.push()
    d = o.sp[1]
    for a, b in ((0, 1), (2, 3)):
        assert d["vz"][b] == 2.0 * d["vz"][a] and d["vr"][b] == 2.0 * d["vr"][a]
        assert d["vz"][a] != 0.0
    Q = o.deposit()
    assert int(Q.sum()) == (1 + 2 + 1 + 2) * 2 ** 40


def test_double_ionization():
    pin_double_ionization()


def test_ion_ionization():
    pin_ion_ionization()


def test_ion_ionization_rate():
    pin_ion_ionization_rate()


def test_cu2_push_deposit():
    pin_cu2_push_deposit()


def test_all_processes_one_event_each():
    """Every process at once: no particle in two events of a step."""
    o = _rz(_tables(el=3e-17, iz=3e-17, cx=5e-16, iz2=3e-17, izi=5e-17), apex=14e9)
    rng = np.random.default_rng(16)
    _fill(o, rng, (12, 10, 14), [(i, k) for i in (3, 7, 11) for k in range(24, 30)], (0.12, 0.003, 0.001))
    ev = o.collide()
    kinds = {k for k, _, _ in ev}
    assert {1, 2, 3, 5, 6} <= kinds, kinds
    _participation(ev)


def test_elastic_conservation():
    pin_elastic_conservation()


def test_cx_swap():
    pin_cx_swap()


def test_ionization():
    pin_ionization()


def test_collision_rate():
    pin_collision_rate()


def test_field_ionization():
    pin_field_ionization()


def test_emission_geometry():
    pin_emission_geometry()


def test_emission_count():
    pin_emission_count()


def test_whole_steps_with_all_stages():
    """Five steps with emission and collisions: ids stay unique, every
    particle is accounted for."""
    o = _rz(_tables(el=1e-17, iz=1e-17, cx=1e-16), apex=12e9)
    rng = np.random.default_rng(8)
    _fill(o, rng, (20, 10, 40), [(i, k) for i in (3, 6) for k in range(22, 30)], (0.05, 0.002, 0.001))
    n0 = sum(len(o.sp[s]["id"]) for s in range(3))
    for _ in range(5):
        o.step(emit=True, collide=True)
    ids = np.concatenate([o.sp[s]["id"] for s in range(3)])
    assert len(np.unique(ids)) == len(ids)
    n_iz = o.events[2] + o.events[4]
    alive = sum(len(o.sp[s]["id"]) for s in range(3))
    assert alive + o.absorbed.sum() == n0 + o.injected + n_iz
    for s in range(3):
        assert np.all(np.diff(o.sp[s]["id"].astype(np.int64)) > 0)
