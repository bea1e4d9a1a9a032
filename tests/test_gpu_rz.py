"""GPU parity of the axisymmetric (r, z) 2D3V variant (include/pic_rz.h,
Sec. 2.2) against the FP64 oracle of oracle/rz.py: node types bit-exact, the
unit-anode potential and V0, the node field, one push with the rotation
back into the r-z plane (positions and velocities per particle by id,
removals), the fixed-point deposit bit-exact, and whole steps of push,
deposit and solve."""
import math

import numpy as np
import pytest
import scipy.constants as sc

torch = pytest.importorskip("torch")

from oracle.rz import RZ

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2402_08404_amd import rz  # noqa: E402

M_CU = 63.546 * sc.atomic_mass
GEOM = dict(nr=32, nz=80, h=2e-9, tip_r=4e-9, tip_h=40e-9, apex_field=10e9, dt=5e-17, m_ion=M_CU)


def _load(o, rng, n=(3000, 1500, 1500)):
    out = {}
    for s, m in enumerate(n):
        r = rng.uniform(0.0, o.nr - 1.5, m)
        z = rng.uniform(0.5, o.nz - 1.5, m)
        ok = ~o.inside_tip(r, z)
        r, z = r[ok], z[ok]
        k = len(r)
        sv = (0.05, 0.002, 0.001)[s]
        out[s] = {"r": r, "z": z, "vr": rng.normal(0, sv, k), "vt": rng.normal(0, sv, k),
                  "vz": rng.normal(0, sv, k)}
    return out


def _pair(seed=1, n=(3000, 1500, 1500)):
    o = RZ(GEOM["nr"], GEOM["nz"], GEOM["h"], GEOM["tip_r"], GEOM["tip_h"], GEOM["apex_field"], GEOM["dt"],
           GEOM["m_ion"])
    load = _load(o, np.random.default_rng(seed), n)
    nid = 0
    for s in range(3):
        m = len(load[s]["r"])
        o.load(s, load[s], np.arange(nid, nid + m))
        nid += m
    g = rz.RZSimulation(**GEOM, load=load, laplace_rtol=1e-13, step_rtol=1e-14)
    return g, o


def _compare(g, o, tol):
    gs = g.state()
    for s in range(3):
        a, b = gs[s], o.sp[s]
        assert np.array_equal(np.sort(a["id"]), np.sort(b["id"])), s
        if len(b["id"]) == 0:
            continue
        ia, ib = np.argsort(a["id"]), np.argsort(b["id"])
        for k in ("r", "z", "vr", "vt", "vz"):
            d = np.abs(a[k][ia] - b[k][ib])
            scale = np.abs(b[k][ib]) + 1e-3 * np.abs(b[k]).max() + 1e-300
            assert (d <= tol * scale).all(), (s, k, (d / scale).max())


def test_rz_types_laplace_field():
    g, o = _pair()
    assert np.array_equal(g.grid("node_type"), o.type)
    m = g.moments()
    assert m["v0"] == pytest.approx(o.V0, rel=1e-10)
    phi1 = g.grid("phi1")
    assert np.abs(phi1 - o.phi1).max() <= 1e-10
    E = g.grid("field").reshape(-1, 2)
    assert np.abs(E - o.E).max() <= 1e-9 * np.abs(o.E).max()


def test_rz_push_and_deposit():
    g, o = _pair(seed=2)
    g.set_phi(o.phi)
    for _ in range(5):
        g.step(1, rz.PIC_RZ_PUSH | rz.PIC_RZ_DEPOSIT)
        o.push()
        o.deposit()
        _compare(g, o, 1e-12)
        assert np.array_equal(g.grid("rho"), o.Q)
    m = g.moments()
    assert np.array_equal(m["absorbed"], o.absorbed)
    assert m["q_total"] == int(o.Q.sum())


def test_rz_rotation_closed_form():
    """Neutrals with an azimuthal velocity move on straight lines in 3D:
    r_k = |(r0 + k v_r, k v_theta)| after k pushes (no field acts on them)."""
    o = RZ(GEOM["nr"], GEOM["nz"], GEOM["h"], GEOM["tip_r"], GEOM["tip_h"], GEOM["apex_field"], GEOM["dt"],
           GEOM["m_ion"])
    rng = np.random.default_rng(3)
    n = 500
    r0 = rng.uniform(6, 20, n)
    vr = rng.uniform(-0.4, 0.4, n)
    vt = rng.uniform(-0.3, 0.3, n)
    load = {2: {"r": r0, "z": np.full(n, 60.0), "vr": vr, "vt": vt, "vz": np.zeros(n)}}
    g = rz.RZSimulation(**GEOM, load=load)
    for k in range(1, 21):
        g.step(1, rz.PIC_RZ_PUSH)
        st = g.state()[2]
        idx = st["id"].astype(np.int64)
        want = np.hypot(r0[idx] + k * vr[idx], k * vt[idx])
        np.testing.assert_allclose(st["r"], want, rtol=1e-12)
        np.testing.assert_allclose(st["r"] * st["vt"], r0[idx] * vt[idx], rtol=1e-11)


def test_rz_whole_steps():
    """Ten steps of push, deposit and solve (to a relative residual of 1e-14,
    the oracle solving directly): charge bit-exact, particles to 1e-9."""
    g, o = _pair(seed=4, n=(20000, 2000, 0))
    g.set_phi(o.phi)
    g.step(1, rz.PIC_RZ_DEPOSIT | rz.PIC_RZ_SOLVE)
    o.deposit()
    o.solve()
    for s in range(10):
        g.step(1, rz.PIC_RZ_FULL)
        o.step()
        assert np.array_equal(g.grid("rho"), o.Q)
        _compare(g, o, 1e-9)
        phi = g.grid("phi")
        assert np.abs(phi - o.phi).max() <= 1e-9 * np.abs(o.phi).max()
    m = g.moments()
    print("alive", m["n_alive"], "absorbed", m["absorbed"].sum(axis=1), "CG", m["last_cg_iters"], flush=True)
    assert np.array_equal(m["absorbed"], o.absorbed)


# -- collisions, field ionization, emission -----------------------------------
from paper_2402_08404_amd import workloads as W  # noqa: E402


def _tables(scale=1e4):
    el, iz, cx = W.synthetic_tables()
    return (1e-2, 1e4, el * scale, iz * scale, cx * scale)


def _tables_cu2(scale=1e4):
    iz2, izi = W.synthetic_tables_cu2()
    return _tables(scale) + (iz2 * scale, izi * scale)


def _pair_all(seed=1, n=(3000, 1500, 6000), apex=10e9, xs=True, fn_rings=0, caps=None, load=None, cu2=False,
              sort_every=0):
    geom = dict(GEOM, apex_field=apex)
    tabs = (_tables_cu2() if cu2 else _tables()) if xs else None
    o = RZ(geom["nr"], geom["nz"], geom["h"], geom["tip_r"], geom["tip_h"], geom["apex_field"], geom["dt"],
           geom["m_ion"], seed=seed, xs=tabs, fn_rings=fn_rings or 16, cu2=cu2)
    if load is None:
        load = _load(o, np.random.default_rng(seed), n)
    nid = 0
    for s in range(3):
        m = len(load[s]["r"]) if s in load else 0
        if m:
            o.load(s, load[s], np.arange(nid, nid + m))
        nid += m
    if caps is None:
        cnt = [len(load[s]["r"]) if s in load else 0 for s in range(3)]
        caps = [cnt[0] + cnt[2] + 4096, cnt[1] + cnt[2] + 1, cnt[2] + 1]
    g = rz.RZSimulation(**geom, load=load, laplace_rtol=1e-13, step_rtol=1e-14, seed=seed, xs=tabs,
                        fn_rings=fn_rings, caps=caps, cu2=cu2, sort_every=sort_every)
    g.set_phi(o.phi)
    return g, o


def _compare_all(g, o, tol):
    gs = g.state()
    for s in range(3):
        b = o.sp[s]
        a = gs[s]
        if b is None:
            assert len(a["id"]) == 0
            continue
        assert np.array_equal(a["id"], b["id"]), (s, len(a["id"]), len(b["id"]))
        for k in ("r", "z", "vr", "vt", "vz"):
            d = np.abs(a[k] - b[k])
            scale = np.abs(b[k]) + 1e-3 * (np.abs(b[k]).max() if len(b[k]) else 0.0) + 1e-300
            assert (d <= tol * scale).all(), (s, k, (d / scale).max())
        if "q" in a:
            assert np.array_equal(a["q"], b["q"]), s


def test_rz_collide_parity():
    """Four collision stages (no push): the same pairs, events, velocities
    and products by id; ids in slot order."""
    print("case: rz collide, seed 21", flush=True)
    g, o = _pair_all(seed=21)
    for step in range(4):
        g.step(1, rz.PIC_RZ_COLLIDE | rz.PIC_RZ_ADVANCE)
        o.collide()
        o.step_no += 1
        _compare_all(g, o, 1e-12)
        m = g.moments()
        assert np.array_equal(m["events"], o.events), (m["events"], o.events)
        assert m["next_id"] == o.next_id
    assert o.events[1] > 50 and o.events[2] > 20 and o.events[3] > 20, o.events


def test_rz_field_ionization_parity():
    """Neutrals on a shell around the apex at 25 GV/m: the same neutrals
    ionize, with the same products."""
    print("case: rz field ionization", flush=True)
    rng = np.random.default_rng(5)
    o0 = RZ(GEOM["nr"], GEOM["nz"], GEOM["h"], GEOM["tip_r"], GEOM["tip_h"], 25e9, GEOM["dt"], GEOM["m_ion"])
    n = 6000
    th = rng.uniform(0, 0.5 * math.pi, n)
    rad = o0.R + rng.uniform(0.3, 3.0, n)
    zc = o0.H - o0.R
    load = {0: {k: np.zeros(0) for k in ("r", "z", "vr", "vt", "vz")},
            1: {k: np.zeros(0) for k in ("r", "z", "vr", "vt", "vz")},
            2: {"r": rad * np.sin(th), "z": zc + rad * np.cos(th), "vr": rng.normal(0, 1e-3, n),
                "vt": rng.normal(0, 1e-3, n), "vz": rng.normal(0, 1e-3, n)}}
    g, o = _pair_all(seed=9, apex=25e9, load=load, caps=[n, n, n])
    for step in range(3):
        g.step(1, rz.PIC_RZ_COLLIDE | rz.PIC_RZ_ADVANCE)
        o.collide()
        o.step_no += 1
        _compare_all(g, o, 1e-14)
    m = g.moments()
    assert np.array_equal(m["events"], o.events)
    assert o.events[4] > 40, o.events


def test_rz_many_products_parity():
    """About 11 000 impact ionizations in one stage (ionization cross
    section scaled up 10^6, electrons and neutrals in the same 200 cells):
    a product list longer than the in-LDS sort (4096 entries) and prefix sums
    over several chunks of the product list; states, events and products by
    id as the oracle's, twice."""
    print("case: rz many products", flush=True)
    el, iz, cx = W.synthetic_tables()
    tabs = (1e-2, 1e4, el, iz * 1e6, cx)
    geom = dict(GEOM)
    o = RZ(geom["nr"], geom["nz"], geom["h"], geom["tip_r"], geom["tip_h"], geom["apex_field"], geom["dt"],
           geom["m_ion"], seed=3, xs=tabs, fn_rings=16)
    rng = np.random.default_rng(3)
    n = 12000
    v = 0.1  # grid units a step: about 45 eV electrons
    load = {0: {"r": rng.uniform(10, 20, n), "z": rng.uniform(50, 70, n), "vr": rng.normal(0, v, n),
                "vt": rng.normal(0, v, n), "vz": rng.normal(0, v, n)},
            1: {k: np.zeros(0) for k in ("r", "z", "vr", "vt", "vz")},
            2: {"r": rng.uniform(10, 20, n), "z": rng.uniform(50, 70, n), "vr": np.zeros(n), "vt": np.zeros(n),
                "vz": np.zeros(n)}}
    o.load(0, load[0], np.arange(n))
    o.load(2, load[2], np.arange(n, 2 * n))
    g = rz.RZSimulation(**geom, load=load, laplace_rtol=1e-13, step_rtol=1e-14, seed=3, xs=tabs, fn_rings=0,
                        caps=[40000, 16000, n + 1])
    g.set_phi(o.phi)
    for step in range(2):
        g.step(1, rz.PIC_RZ_COLLIDE | rz.PIC_RZ_ADVANCE)
        o.collide()
        o.step_no += 1
        _compare_all(g, o, 1e-12)
        m = g.moments()
        assert np.array_equal(m["events"], o.events), (m["events"], o.events)
        assert m["next_id"] == o.next_id
    assert o.events[2] > 8000, o.events


def test_rz_emission_parity():
    print("case: rz emission", flush=True)
    load = {s: {k: np.zeros(0) for k in ("r", "z", "vr", "vt", "vz")} for s in range(3)}
    g, o = _pair_all(seed=3, apex=20e9, load=load, fn_rings=16, caps=[4096, 16, 16], xs=False)
    for step in range(20):
        g.step(1, rz.PIC_RZ_EMIT | rz.PIC_RZ_ADVANCE)
        o.emit()
        o.step_no += 1
    _compare_all(g, o, 1e-14)
    m = g.moments()
    assert m["injected"] == o.injected > 20, (m["injected"], o.injected)


def test_rz_all_stages_steps():
    """Ten whole steps with emission, push, collisions, deposit and solve:
    the charge bit-exact, particles and events as the oracle's."""
    print("case: rz all stages", flush=True)
    g, o = _pair_all(seed=31, n=(4000, 1500, 8000), apex=14e9, fn_rings=16, caps=[40000, 20000, 8000])
    g.step(1, rz.PIC_RZ_DEPOSIT | rz.PIC_RZ_SOLVE)
    o.deposit()
    o.solve()
    for s in range(10):
        g.step(1, rz.PIC_RZ_ALL)
        o.step(emit=True, collide=True)
        assert np.array_equal(g.grid("rho"), o.Q)
        _compare_all(g, o, 1e-9)
    m = g.moments()
    print("events", m["events"], "injected", m["injected"], "alive", m["n_alive"], flush=True)
    assert np.array_equal(m["events"], o.events)
    assert np.array_equal(m["absorbed"], o.absorbed)
    assert m["injected"] == o.injected


def test_rz_capacity_and_ids():
    print("case: rz capacity and ids", flush=True)
    load = {s: {k: np.zeros(0) for k in ("r", "z", "vr", "vt", "vz")} for s in range(3)}
    g, o = _pair_all(seed=3, apex=20e9, load=load, fn_rings=16, caps=[1, 1, 1], xs=False)
    with pytest.raises(rz.PicError) as e:
        g.step(5, rz.PIC_RZ_EMIT | rz.PIC_RZ_ADVANCE)
    assert e.value.code == -3
    assert g.moments()["n_slots"][0] <= 1
    # an initial id may not be the free-slot marker; any order is fine
    ld = {2: {"r": np.array([10.0, 11.0]), "z": np.array([50.0, 50.0]), "vr": np.zeros(2), "vt": np.zeros(2),
              "vz": np.zeros(2)}}
    with pytest.raises(rz.PicError):
        rz.RZSimulation(**GEOM, load=ld, ids={2: np.array([5, 0xFFFFFFFF], np.uint32)})
    g2 = rz.RZSimulation(**GEOM, load=ld, ids={2: np.array([5, 4], np.uint32)})
    assert g2.moments()["next_id"] == 6


def test_rz_collide_dense_cells():
    """Cells beyond the per-thread ranks (more than 64 particles of a species:
    the LDS sort) and beyond the LDS sort (more than 4096: rank counting),
    over a background load."""
    print("case: rz collide dense cells", flush=True)
    o0 = RZ(GEOM["nr"], GEOM["nz"], GEOM["h"], GEOM["tip_r"], GEOM["tip_h"], GEOM["apex_field"], GEOM["dt"],
            GEOM["m_ion"])
    rng = np.random.default_rng(12)
    base = _load(o0, rng, (2000, 800, 2000))
    dense = {0: [((5, 40), 150), ((10, 45), 300)], 1: [((5, 40), 200), ((12, 50), 90)],
             2: [((5, 40), 5000), ((10, 45), 100), ((12, 50), 700)]}
    load = {}
    for s in range(3):
        parts = [base[s]]
        for (i, k), m in dense[s]:
            sv = (0.05, 0.002, 0.001)[s]
            parts.append({"r": i + rng.uniform(0.01, 0.99, m), "z": k + rng.uniform(0.01, 0.99, m),
                          "vr": rng.normal(0, sv, m), "vt": rng.normal(0, sv, m), "vz": rng.normal(0, sv, m)})
        load[s] = {key: np.concatenate([p[key] for p in parts]) for key in ("r", "z", "vr", "vt", "vz")}
    g, o = _pair_all(seed=17, load=load)
    for step in range(3):
        g.step(1, rz.PIC_RZ_COLLIDE | rz.PIC_RZ_ADVANCE)
        o.collide()
        o.step_no += 1
        _compare_all(g, o, 1e-12)
    m = g.moments()
    assert np.array_equal(m["events"], o.events), (m["events"], o.events)
    assert o.events[1] > 100 and o.events[3] > 50, o.events


def test_rz_multigrid_levels_solve():
    """A grid whose cell counts halve (32 x 80 cells: four multigrid levels):
    the unit-anode potential and a solve with charge as the oracle's direct
    solution, in a few preconditioned iterations."""
    print("case: rz multigrid levels", flush=True)
    geom = dict(GEOM, nr=33, nz=81)
    o = RZ(geom["nr"], geom["nz"], geom["h"], geom["tip_r"], geom["tip_h"], geom["apex_field"], geom["dt"],
           geom["m_ion"])
    load = _load(o, np.random.default_rng(41), (20000, 8000, 0))
    nid = 0
    for s in range(3):
        m = len(load[s]["r"])
        o.load(s, load[s], np.arange(nid, nid + m))
        nid += m
    g = rz.RZSimulation(**geom, load=load, laplace_rtol=1e-13, step_rtol=1e-12)
    assert np.abs(g.grid("phi1") - o.phi1).max() <= 1e-10
    g.step(1, rz.PIC_RZ_DEPOSIT)
    o.deposit()
    info = g.solve(1e-12, 1000)
    o.solve()
    assert info["converged"] and info["iterations"] <= 20, info
    phi = g.grid("phi")
    assert np.abs(phi - o.phi).max() <= 1e-9 * np.abs(o.phi).max()


@pytest.mark.parametrize("shape", [(8, 1025, 4e-9, 40e-9), (1025, 8, 4e-9, 8e-9), (32, 161, 4e-9, 40e-9),
                                   (5, 12, 2e-9, 10e-9)])
def test_rz_multigrid_one_dimension_halved(shape):
    """Grids where only one dimension halves (7 x 1024, 1024 x 7 and 31 x 160
    cells): the multigrid levels above the LDS-resident ones coarsen along z
    only or along r only; on 31 x 160 cells the coarsest level (32 x 6 nodes)
    is too large for the exact solve and is swept instead; a grid of 60 nodes
    is its own coarsest level, solved exactly. The unit-anode potential and a
    solve with charge as the oracle's direct solution."""
    nr, nz, tip_r, tip_h = shape
    print(f"case: rz multigrid one dimension halved nr={nr} nz={nz}", flush=True)
    geom = dict(GEOM, nr=nr, nz=nz, tip_r=tip_r, tip_h=tip_h)
    o = RZ(geom["nr"], geom["nz"], geom["h"], geom["tip_r"], geom["tip_h"], geom["apex_field"], geom["dt"],
           geom["m_ion"])
    load = _load(o, np.random.default_rng(43), (8000, 4000, 0))
    nid = 0
    for s in range(3):
        m = len(load[s]["r"])
        o.load(s, load[s], np.arange(nid, nid + m))
        nid += m
    g = rz.RZSimulation(**geom, load=load, laplace_rtol=1e-13, step_rtol=1e-12)
    assert np.abs(g.grid("phi1") - o.phi1).max() <= 1e-10
    g.step(1, rz.PIC_RZ_DEPOSIT)
    o.deposit()
    info = g.solve(1e-12, 5000)
    o.solve()
    assert info["converged"], info
    phi = g.grid("phi")
    assert np.abs(phi - o.phi).max() <= 1e-9 * np.abs(o.phi).max()


def _load_cu2(seed, n=(3000, 1500, 6000)):
    o0 = RZ(GEOM["nr"], GEOM["nz"], GEOM["h"], GEOM["tip_r"], GEOM["tip_h"], GEOM["apex_field"], GEOM["dt"],
            GEOM["m_ion"])
    rng = np.random.default_rng(seed)
    load = _load(o0, rng, n)
    # electrons fast enough for both Cu2+ processes, a third of the ions Cu2+
    for k in ("vr", "vt", "vz"):
        load[0][k] = rng.normal(0, 0.08, len(load[0]["r"]))
    q = np.ones(len(load[1]["r"]), np.uint8)
    q[::3] = 2
    load[1]["q"] = q
    return load


def test_rz_cu2_collide_parity():
    """Cu2+ as an ion charge state: four collision stages with every process
    (double ionization of Cu, ionization of Cu+), states, charge states,
    events and products by id."""
    print("case: rz Cu2+ collide", flush=True)
    g, o = _pair_all(seed=23, load=_load_cu2(23), cu2=True)
    for step in range(4):
        g.step(1, rz.PIC_RZ_COLLIDE | rz.PIC_RZ_ADVANCE)
        o.collide()
        o.step_no += 1
        _compare_all(g, o, 1e-12)
        m = g.moments()
        assert np.array_equal(m["events"], o.events), (m["events"], o.events)
        assert m["next_id"] == o.next_id
        assert m["n_cu2"] == int((o.sp[1]["q"] == 2).sum())
    assert o.events[5] > 5 and o.events[6] > 20 and o.events[2] > 20, o.events


def test_rz_cu2_all_stages_steps():
    """Eight whole steps with Cu2+: the doubled kick and deposit of Cu2+,
    node charge bit-exact, particles and events as the oracle's."""
    print("case: rz Cu2+ all stages", flush=True)
    g, o = _pair_all(seed=29, load=_load_cu2(29, (4000, 1500, 8000)), apex=14e9, fn_rings=16, cu2=True,
                     caps=[40000, 20000, 8000])
    g.step(1, rz.PIC_RZ_DEPOSIT | rz.PIC_RZ_SOLVE)
    o.deposit()
    o.solve()
    assert np.array_equal(g.grid("rho"), o.Q)
    for s in range(8):
        g.step(1, rz.PIC_RZ_ALL)
        o.step(emit=True, collide=True)
        assert np.array_equal(g.grid("rho"), o.Q)
        _compare_all(g, o, 1e-9)
    m = g.moments()
    print("events", m["events"], "n_cu2", m["n_cu2"], flush=True)
    assert np.array_equal(m["events"], o.events)
    assert np.array_equal(m["absorbed"], o.absorbed)


def test_rz_reorder_all_stages():
    """Ten whole steps with every stage, Cu2+ and the particles reordered by
    cell every second step (slots change, ids stay): node charge bit-exact,
    particles, charge states and events as the oracle's; the slots in use
    shrink to the alive particles at a reorder."""
    print("case: rz reorder", flush=True)
    g, o = _pair_all(seed=37, load=_load_cu2(37, (4000, 1500, 8000)), apex=14e9, fn_rings=16, cu2=True,
                     caps=[40000, 20000, 8000], sort_every=2)
    g.step(1, rz.PIC_RZ_DEPOSIT | rz.PIC_RZ_SOLVE)
    o.deposit()
    o.solve()
    for s in range(10):
        g.step(1, rz.PIC_RZ_ALL)
        o.step(emit=True, collide=True)
        assert np.array_equal(g.grid("rho"), o.Q)
        _compare_all(g, o, 1e-9)
        m = g.moments()
        if s % 2 == 0:
            # reordered in this step after the push: no charged particle leaves
            # later in the step, so every electron and ion slot is alive
            assert m["n_slots"][0] == m["n_alive"][0] and m["n_slots"][1] == m["n_alive"][1], m
    m = g.moments()
    print("events", m["events"], "slots", m["n_slots"], "alive", m["n_alive"], flush=True)
    assert np.array_equal(m["events"], o.events)
    assert np.array_equal(m["absorbed"], o.absorbed)
    assert m["n_cu2"] == int((o.sp[1]["q"] == 2).sum())
