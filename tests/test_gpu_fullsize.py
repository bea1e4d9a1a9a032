"""GPU parity at the full workload size: 128 x 128 x 512 nodes at 1 nm and
20 M particles (16 M e, 1 M Cu+, 3 M Cu, FP32 particle state) in the launch
configuration the benchmark times (MG-preconditioned CG to 1e-8 with the
extrapolated step guess, the tuned solver block count and reorder period).

The oracle cannot run this size end to end; per stage it checks what it can
compute at this size or on a sample:
- the deposit, bit for bit over every particle (integer arithmetic);
- the potential: the true residual of the GPU solution, computed with the
  oracle's own operator and right-hand side, at the solver tolerance;
- the node field, node by node from the GPU potential (FP32 storage);
- one push of a sample of particles of every species from the same state;
- the collision and field-ionization events of every cell of a slab of
  planes through the tip apex, bit for bit (decisions are per cell).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2402_08404_amd import workloads as W

from gpu_common import compare_states, event_sets, kick_bounds

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2402_08404_amd import batch as B  # noqa: E402
from paper_2402_08404_amd import pic  # noqa: E402

COUNTS = (16_000_000, 1_000_000, 3_000_000)
KT = (5.0, 1.0, 0.1)


def oracle_with(cfg, st, phi):
    """An oracle instance holding the particles st (with their ids) in the
    potential phi (its field computed by the oracle)."""
    o = oracle.Oracle(cfg, laplace=False)
    o.load({name: {k: st[s][k] for k in ("x", "y", "z", "vx", "vy", "vz")} for s, name in enumerate(W.SPECIES)})
    for s in range(3):
        o.sp[s].id[:o.sp[s].n] = st[s]["id"]
    o.set_phi(phi)
    return o


def subset(st, keep):
    return [{k: v[keep[s]] for k, v in d.items()} for s, d in enumerate(st)]


@pytest.fixture(scope="module")
def full():
    cfg = W.gpu_scale()
    caps = (COUNTS[0] + COUNTS[2] + COUNTS[0] // 8, COUNTS[1] + COUNTS[2] + COUNTS[1] // 8, COUNTS[2] + 1024)
    tune = B.load_tuning(B.__file__.replace("batch.py", "tuning.json")).get(B.shape_key(cfg), {})
    print("full size: init", tune, flush=True)
    g = pic.Simulation(cfg, caps=caps, precision=pic.PIC_F32, solver=pic.PIC_SOLVER_MGCG, step_rtol=1e-8,
                       step_maxit=20000, sort_every=tune.get("sort_every", 16),
                       stencil_blocks=tune.get("stencil_blocks", 0), step_guess=1)
    load = W.initial_load(cfg, counts=COUNTS, kT_eV=KT, region="box", dtype=np.float32)
    g.load(load)
    del load
    g.step(1, pic.STEP_DEPOSIT)
    g.solve(solver=pic.PIC_SOLVER_MGCG, guess=pic.PIC_GUESS_PREVIOUS, rtol=1e-8, maxit=200000)
    print("full size: three full steps", flush=True)
    g.step(3, pic.STEP_FULL)
    yield cfg, g
    g.close()


def test_fullsize_deposit_and_poisson(full):
    cfg, g = full
    g.step(1, pic.STEP_DEPOSIT)
    rho = g.grid("rho")
    st = g.state()
    print("deposit of", [len(d["x"]) for d in st], "particles", flush=True)
    o = oracle_with(cfg, st, g.grid("phi"))
    assert np.array_equal(rho, o.deposit())
    # from a zero guess, so that the whole MG-preconditioned iteration runs
    info = g.solve(solver=pic.PIC_SOLVER_MGCG, guess=pic.PIC_GUESS_ZERO, rtol=1e-8, maxit=200000)
    print("solve", info, flush=True)
    assert info["converged"] and info["relres"] <= 1e-8 and 3 <= info["iterations"] <= 12
    phi = g.grid("phi")
    anode = o.type == 2
    V0 = float(phi[anode][0])
    assert np.all(phi[anode] == V0) and np.all(phi[o.type == 1] == 0.0)
    free = o.type == 0
    b = o.rhs(rho, V0)
    r = (b - o.apply_A(np.where(free, phi, 0.0)))[free]
    rel = np.linalg.norm(r) / np.linalg.norm(b[free])
    print("true relative residual", rel, flush=True)
    assert rel <= 2e-8


def test_fullsize_field(full):
    cfg, g = full
    phi = g.grid("phi")
    o = oracle.Oracle(cfg, laplace=False)
    o.set_phi(phi)
    E = g.grid("field").reshape(-1, 4)[:, :3].astype(np.float64)
    ref = o.E.reshape(-1, 3)
    err = np.abs(E - ref).max() / np.abs(ref).max()
    print("field max error / max |E|", err, flush=True)
    assert err <= 1e-6


def test_fullsize_push_sample(full):
    cfg, g = full
    phi = g.grid("phi")
    st0 = g.state()
    rng = np.random.default_rng(5)
    keep = [np.sort(rng.choice(len(d["x"]), size=min(len(d["x"]), 100_000), replace=False)) for d in st0]
    o = oracle_with(cfg, subset(st0, keep), phi)
    ids = [d["id"][k] for d, k in zip(st0, keep)]
    kick = kick_bounds(cfg, o.state(), o.E)
    g.step(1, pic.STEP_PUSH)
    o.push()
    st1 = g.state()
    mine = [np.isin(d["id"], ids[s]) for s, d in enumerate(st1)]
    n = compare_states(cfg, subset(st1, mine), o.state(), 1e-6, None, margin_tol=1e-4, kick=kick)
    print("pushed and compared", n, flush=True)
    assert n > 250_000


def _fi_expected_by_plane(cfg, st, field):
    """Expected field-ionization events per cell plane of the neutrals in
    st (Eq. dfi at the field of the nearest node, zero above the
    barrier-suppression limit): used only to choose a slab where field
    ionization occurs."""
    xi = cfg.xi
    n = 3.69 / np.sqrt(xi)
    E = field.reshape(cfg.nz, cfg.ny, cfg.nx, 4)[..., :3].astype(np.float64)
    d = st[2]
    i = np.clip(np.rint(d["x"]).astype(np.int64), 0, cfg.nx - 1)
    j = np.clip(np.rint(d["y"]).astype(np.int64), 0, cfg.ny - 1)
    k = np.clip(np.rint(d["z"]).astype(np.int64), 0, cfg.nz - 1)
    F = np.linalg.norm(E[k, j, i], axis=1) * 1e-9
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        rate = (1.52 * 4 ** n * xi / (n * math.gamma(2 * n)) * (20.5 * xi ** 1.5 / F) ** (2 * n - 1)
                * np.exp(-6.83 * xi ** 1.5 / F))
    p = np.where((F > 1.0) & (F <= 1.5 * xi ** 1.5), rate * cfg.dt * 1e15, 0.0)
    return np.bincount(np.clip(np.floor(d["z"]).astype(np.int64), 0, cfg.nz - 2), weights=p,
                       minlength=cfg.nz - 1)


def test_fullsize_collisions_slab(full):
    cfg, g = full
    g.step(1, pic.STEP_DEPOSIT)
    st = g.state()
    phi = g.grid("phi")
    step_no = int(g.moments()["step"])
    # every cell of 12 planes: the window with the most expected field
    # ionizations (the field is strongest near the tip and in the space
    # charge of the electron cloud)
    per_plane = _fi_expected_by_plane(cfg, st, g.grid("field"))
    win = np.convolve(per_plane, np.ones(12), mode="valid")
    k0 = int(np.argmax(win))
    print("slab planes", k0, "to", k0 + 12, "expected field ionizations", float(win[k0]), flush=True)
    keep = [(np.floor(d["z"]) >= k0) & (np.floor(d["z"]) < k0 + 12) for d in st]
    sub = subset(st, keep)
    o = oracle_with(cfg, sub, phi)
    o.step_no = step_no
    ids = np.concatenate([d["id"] for d in sub])
    g.step(1, pic.STEP_DEPOSIT | pic.STEP_COLLIDE | pic.STEP_EVENTS)
    o.collide()
    ge_all = g.events()
    assert len(ge_all) < g.caps[2]  # the device event buffer (capacity caps[2]) did not fill
    # field-ionization events carry no charged particle (id_a is 0xFFFFFFFF):
    # an event belongs to the slab when either of its particles does
    ida = np.array([int(e[1]) for e in ge_all], np.uint32)
    idb = np.array([int(e[2]) for e in ge_all], np.uint32)
    ge = [e for e, m in zip(ge_all, np.isin(ida, ids) | np.isin(idb, ids)) if m]
    ev_g = event_sets(ge, o.last_fragile)
    ev_o = event_sets(o.last_events, o.last_fragile)
    kinds = sorted({k for k, _, _ in ev_o})
    print("slab particles", [len(d["x"]) for d in sub], "events", len(ev_o), "kinds", kinds, "fragile",
          len(o.last_fragile), "field ionizations", sum(1 for k, _, _ in ev_o if k == 4), flush=True)
    assert len(ev_o) > 100 and 4 in kinds
    assert ev_g == ev_o
