"""Seeded synthetic inputs for the PIC-MCC step: configurations, cross-section
tables and initial particle loads.

This module is the one place both the GPU library's users and the CPU oracle's
tests take their inputs from. It holds no arithmetic of the method itself (no
push, deposit, collision or solver step): only the numbers and random draws
that define a workload.

The paper's own runs (Sec. 3.2) need a coupled FEM model, GETELEC and measured
cross sections that are not available; these synthetic workloads stand in for
them with the shapes, sizes and velocity distributions listed in each preset.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Physical constants needed to draw thermal velocities and to state the Cu
# mass (CODATA 2022).
_KB = 1.380649e-23
_QE = 1.602176634e-19
_ME = 9.1093837139e-31
_AMU = 1.66053906892e-27

CU_MASS_U = 63.546       # standard atomic weight of Cu
CU_XI_EV = 7.726380      # first ionization energy of Cu [eV] (NIST ASD)

SPECIES = ("e", "ion", "neutral")


@dataclasses.dataclass
class Config:
    """Scalar parameters of one PIC-MCC instance (SI units unless noted)."""

    nx: int
    ny: int
    nz: int
    h: float                 # node spacing [m]
    tip_r: float             # tip radius [m]
    tip_h: float             # total tip height to the apex [m]
    apex_field: float        # requested local field at the apex [V/m]
    phi_w: float = 4.5       # work function [eV]
    temperature: float = 300.0
    dt: float = 5e-17        # time step [s]
    seed: int = 1            # Philox key
    xi: float = CU_XI_EV
    m_ion: float = CU_MASS_U * _AMU
    xs_emin: float = 1e-2    # first cross-section table node [eV]
    xs_emax: float = 1e4     # last cross-section table node [eV]
    xs_el: np.ndarray = None
    xs_iz: np.ndarray = None
    xs_cx: np.ndarray = None
    fn_rings: int = 16
    fn_az: int = 64
    surface_T: float = 0.0   # prescribed tip surface temperature for neutral evaporation [K] (0: none)
    circuit_R: float = 0.0   # series resistance of the external RC circuit [ohm] (0: fixed anode potential)
    circuit_C: float = 0.0   # gap capacitance of the RC circuit [F]
    w_max: int = 1           # largest superparticle weight that injection and merging create
    n_max: float = 1e24      # SP number density above which evaporated neutrals get heavier [1/m^3] (1e-6 per A^3)
    merge_every: int = 0     # merging of superparticles every this many steps (0: never)
    merge_max: int = 0       # superparticles of one species per cell above which pairs of them merge
    same_species: int = 0    # bit 1: Cu-Cu elastic, bit 2: Coulomb (Takizuka-Abe), bit 4: Cu+ + e -> Cu recombination
    sigma_nn: float = 0.0    # Cu-Cu elastic (hard-sphere) cross section [m^2]
    coulomb_log: float = 10.0  # Coulomb logarithm ln(Lambda)
    sigma_rec: float = 0.0   # recombination cross section [m^2]

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_cells(self) -> int:
        return (self.nx - 1) * (self.ny - 1) * (self.nz - 1)


def constant_tables(sigma_el: float, sigma_iz: float, sigma_cx: float, n: int = 256):
    """Energy-independent cross sections as flat tables [m^2]."""
    return (np.full(n, sigma_el), np.full(n, sigma_iz), np.full(n, sigma_cx))


def synthetic_tables(n: int = 256, emin: float = 1e-2, emax: float = 1e4, xi: float = CU_XI_EV):
    """Smooth positive stand-ins for the measured cross sections the paper
    cites but does not print (Table colls), sampled on n log-spaced energies:
    elastic ~ 5e-20 (1 + E/20 eV)^-1/2, ionization in Lotz form
    4.5e-18 ln(E/xi) / (E xi) above xi, charge exchange in Rapp-Francis form
    (7.0e-10 - 0.5e-10 ln E)^2, all in m^2 with E in eV."""
    E = emin * (emax / emin) ** (np.arange(n) / (n - 1))
    el = 5e-20 / np.sqrt(1.0 + E / 20.0)
    iz = np.where(E > xi, 4.5e-18 * np.log(np.maximum(E, xi) / xi) / (E * xi), 0.0)
    cx = (7.0e-10 - 0.5e-10 * np.log(E)) ** 2
    return el, iz, cx


CU_XI2_EV = 20.29239     # second ionization energy of Cu [eV] (NIST ASD)


def synthetic_tables_cu2(n: int = 256, emin: float = 1e-2, emax: float = 1e4, xi: float = CU_XI_EV,
                         xi2: float = CU_XI2_EV):
    """The two Cu2+ processes in the same Lotz form as the single ionization
    (their measured cross sections are cited, not given): Cu + e -> Cu2+ +
    3e above xi + xi2 at a tenth of that form's height, and Cu+ + e -> Cu2+ +
    2e above xi2, in m^2 on n log-spaced energies."""
    E = emin * (emax / emin) ** (np.arange(n) / (n - 1))
    x2 = xi + xi2
    iz2 = np.where(E > x2, 0.45e-18 * np.log(np.maximum(E, x2) / x2) / (E * x2), 0.0)
    izi = np.where(E > xi2, 4.5e-18 * np.log(np.maximum(E, xi2) / xi2) / (E * xi2), 0.0)
    return iz2, izi


def _with_tables(cfg: Config, tabs) -> Config:
    cfg.xs_el, cfg.xs_iz, cfg.xs_cx = (np.ascontiguousarray(t, dtype=np.float64) for t in tabs)
    return cfg


def tiny(seed: int = 1) -> Config:
    """32x32x64 nodes at 2 nm, tip r = 4 nm, H = 40 nm, 10 GV/m at the apex,
    constant cross sections (elastic 5e-20, ionization 1e-20, charge exchange
    5e-20 m^2), dt = 5e-17 s."""
    cfg = Config(nx=32, ny=32, nz=64, h=2e-9, tip_r=4e-9, tip_h=40e-9, apex_field=10e9, seed=seed)
    return _with_tables(cfg, constant_tables(5e-20, 1e-20, 5e-20))


def gpu_scale(seed: int = 2) -> Config:
    """128x128x512 nodes at 1 nm, tip r = 10 nm, H = 100 nm, 10 GV/m at the
    apex, synthetic energy-dependent tables of 256 log-spaced nodes."""
    cfg = Config(nx=128, ny=128, nz=512, h=1e-9, tip_r=10e-9, tip_h=100e-9, apex_field=10e9, seed=seed)
    return _with_tables(cfg, synthetic_tables())


def small(nx=16, ny=16, nz=32, h=2e-9, tip_r=4e-9, tip_h=24e-9, field=10e9, seed=7,
          tables="constant") -> Config:
    """Reduced instances for fast tests (same physics, fewer nodes)."""
    cfg = Config(nx=nx, ny=ny, nz=nz, h=h, tip_r=tip_r, tip_h=tip_h, apex_field=field, seed=seed)
    tabs = constant_tables(5e-20, 1e-20, 5e-20) if tables == "constant" else synthetic_tables()
    return _with_tables(cfg, tabs)


def _outside_tip_with_margin(cfg: Config, X, Y, Z, margin: float):
    """True where a point (grid units) is at least `margin` spacings away from
    the tip body (a conservative exclusion zone used only to place inputs)."""
    R = cfg.tip_r / cfg.h + margin
    zc = cfg.tip_h / cfg.h - cfg.tip_r / cfg.h
    xc, yc = 0.5 * (cfg.nx - 1), 0.5 * (cfg.ny - 1)
    rho2 = (X - xc) ** 2 + (Y - yc) ** 2
    in_cyl = (Z <= zc) & (rho2 <= R * R)
    in_cap = (Z > zc) & (rho2 + (Z - zc) ** 2 <= R * R)
    return ~(in_cyl | in_cap)


def sample_positions(cfg: Config, n: int, rng: np.random.Generator, region: str = "near_tip"):
    """n positions in grid units, uniform in the region and clear of the tip.

    region "near_tip": the cylinder rho <= 3 r around the tip axis with
    0 < z < H + 2 r; region "box": the whole vacuum box."""
    xc, yc = 0.5 * (cfg.nx - 1), 0.5 * (cfg.ny - 1)
    R = cfg.tip_r / cfg.h
    H = cfg.tip_h / cfg.h
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = max(1024, int(1.6 * (n - out.shape[0])))
        if region == "near_tip":
            rr = 3.0 * R * np.sqrt(rng.random(m))
            th = 2.0 * math.pi * rng.random(m)
            X = xc + rr * np.cos(th)
            Y = yc + rr * np.sin(th)
            Z = (H + 2.0 * R) * rng.random(m)
        elif region == "box":
            X = (cfg.nx - 1) * rng.random(m)
            Y = (cfg.ny - 1) * rng.random(m)
            Z = (cfg.nz - 1) * rng.random(m)
        else:
            raise ValueError(region)
        keep = _outside_tip_with_margin(cfg, X, Y, Z, 0.25)
        keep &= (Z > 0.05) & (Z < cfg.nz - 1.05) & (X > 0.0) & (X < cfg.nx - 1.0) & (Y > 0.0) & (Y < cfg.ny - 1.0)
        pts = np.stack([X[keep], Y[keep], Z[keep]], axis=1)
        out = np.concatenate([out, pts])
    return out[:n]


def maxwellian(cfg: Config, n: int, kT_eV: float, mass: float, rng: np.random.Generator):
    """Thermal velocities (each component normal with variance kT/m) in grid
    units per step, v dt / h."""
    s = math.sqrt(kT_eV * _QE / mass)
    return rng.standard_normal((n, 3)) * s * cfg.dt / cfg.h


def initial_load(cfg: Config, counts=(20000, 200, 2000), kT_eV=None, region="near_tip", seed=None,
                 dtype=np.float64):
    """A seeded initial particle load: dict species -> dict of SoA arrays
    x, y, z, vx, vy, vz in grid units. Ids are not part of the load: the
    library and the oracle both number particles in load order (electrons,
    then ions, then neutrals)."""
    if kT_eV is None:
        kT = _KB * cfg.temperature / _QE
        kT_eV = (kT, kT, kT)
    rng = np.random.default_rng(np.random.Philox(key=(cfg.seed if seed is None else seed) + 1000))
    masses = (_ME, cfg.m_ion, cfg.m_ion)
    load = {}
    for s, n, kt, m in zip(SPECIES, counts, kT_eV, masses):
        pos = sample_positions(cfg, n, rng, region)
        vel = maxwellian(cfg, n, kt, m, rng)
        arr = np.concatenate([pos, vel], axis=1).astype(dtype)
        load[s] = {k: np.ascontiguousarray(arr[:, i]) for i, k in enumerate(("x", "y", "z", "vx", "vy", "vz"))}
    return load


def synthetic_potential(cfg: Config, V0: float, amp: float = 0.05, seed: int = 3):
    """A smooth potential on the nodes [V]: a linear ramp 0..V0 along z plus
    a few random low-order Fourier modes of relative amplitude `amp`. Used as
    a common, solver-independent field for single-stage tests."""
    rng = np.random.default_rng(seed)
    z = np.arange(cfg.nz) / (cfg.nz - 1)
    y = np.arange(cfg.ny) / (cfg.ny - 1)
    x = np.arange(cfg.nx) / (cfg.nx - 1)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    phi = V0 * Z
    for _ in range(4):
        kx, ky, kz = rng.integers(1, 4, size=3)
        a = amp * V0 * rng.standard_normal()
        phi = phi + a * np.sin(math.pi * kz * Z) * np.cos(math.pi * kx * X) * np.cos(math.pi * ky * Y)
    return np.ascontiguousarray(phi.reshape(-1))


def rz_context(seed: int = 3) -> dict:
    """The axisymmetric variant on the paper's own geometry (Sec. 2.2 and the
    runs of Sec. 3): tip radius 50 nm, height 2.5 um (50 r), anode 7.68 um
    above the cathode (about 150 r), radial extent 1.28 um, 5 nm spacing
    (257 x 1537 nodes: 256 and 1536 cells, which halve down to a few nodes
    for the multigrid preconditioner), 10 GV/m at the apex, dt = 2.5e-16 s
    (an electron at 10^6 m/s moves 0.05 spacings a step), the synthetic
    tables with the two Cu2+ processes (all four species of the paper), 64
    emission rings."""
    el, iz, cx = synthetic_tables()
    iz2, izi = synthetic_tables_cu2()
    return dict(nr=257, nz=1537, h=5e-9, tip_r=50e-9, tip_h=2.5e-6, apex_field=10e9, dt=2.5e-16,
                m_ion=CU_MASS_U * _AMU, seed=seed, xs=(1e-2, 1e4, el, iz, cx, iz2, izi), fn_rings=64, cu2=True)


def rz_load(geo: dict, counts=(4_000_000, 4_000_000, 4_000_000), r_max: float = 200.0, z_max: float = 1000.0,
            rng: np.random.Generator | None = None) -> dict:
    """Particles of each species uniform in volume over r < r_max, 1 < z <
    z_max (grid units), clear of the tip by a spacing: electrons with
    normal velocity components of 0.02 spacings a step, ions and neutrals
    2e-4 (grid units per step). Returns species -> dict r, z, vr, vt, vz."""
    rng = rng or np.random.default_rng(geo.get("seed", 3))
    R, H = geo["tip_r"] / geo["h"] + 1.0, geo["tip_h"] / geo["h"] + 1.0
    zc = H - R
    out = {}
    for s, n in enumerate(counts):
        r = np.zeros(0)
        z = np.zeros(0)
        while len(r) < n:
            m = int(1.2 * (n - len(r))) + 16
            rr = r_max * np.sqrt(rng.uniform(0.0, 1.0, m))
            zz = rng.uniform(1.0, z_max, m)
            inside = ((zz <= zc) & (rr <= R)) | ((zz > zc) & (rr * rr + (zz - zc) ** 2 <= R * R))
            r = np.concatenate([r, rr[~inside]])
            z = np.concatenate([z, zz[~inside]])
        sv = 0.02 if s == 0 else 2e-4
        out[s] = {"r": r[:n], "z": z[:n], "vr": rng.normal(0, sv, n), "vt": rng.normal(0, sv, n),
                  "vz": rng.normal(0, sv, n)}
    return out
