"""FP64 CPU oracle of the 2D axisymmetric (r, z) 2D3V variant of the
particle-mesh step (Sec. 2.2: the axisymmetric vacuum mesh, the 2D3V method,
particles rotated back into the r-z plane every step, reflection at the
axis, removal at the cathode, the anode and the open side; leapfrog).

TEST INFRASTRUCTURE ONLY: imported by tests/ only. Plain numpy and scipy;
it shares no code with the GPU library.

Readings (the paper leaves the discretization to its references):
- nodes at (r, z) = (i h, k h), i < nr, k < nz; the tip is the body of
  revolution of the 3D variant (a cylinder of radius R up to H - R, a
  hemisphere on top) on the axis; nodes of the plane k = 0 and inside the tip
  are held at 0 V, k = nz - 1 at V0; the side r = (nr - 1) h has zero normal
  field;
- Poisson's equation in finite-volume form on annular node control volumes
  r in [r_i - h/2, r_i + h/2] (clipped to [0, (nr - 1) h]), z in
  [z_k - h/2, z_k + h/2]: sum_j c_ij (phi_i - phi_j) = Q_i / (pi eps0 h) with
  the face areas over pi h as couplings: radial faces 2 (i +- 1/2), axial
  faces (r_hi^2 - r_lo^2) / h^2;
- node field by central differences, E_r = 0 on the axis and on the side,
  one-sided E_z on the two z planes; bilinear gather in (r, z);
- the push: kick of (v_r, v_z) by the gathered field, drift in Cartesian
  coordinates of the particle's r-z half plane, x = r + v_r, y = v_theta,
  then rotation back into the r-z plane: r' = sqrt(x^2 + y^2),
  (v_r', v_theta') = (c v_r + s v_theta, -s v_r + c v_theta), c = x / r',
  s = y / r' (a particle crossing the axis comes back mirrored, the
  reflection at the axis); removal: z <= 0 cathode, z >= nz - 1 anode,
  r >= nr - 1 side, inside the tip;
- the deposit: bilinear weights in (r, z) quantized per axis to 2^-20, so a
  particle deposits exactly 2^40 units of 2^-40 e onto its four nodes.
Positions are in grid units (r / h, z / h), velocities in grid units per
step (v dt / h), with the azimuthal velocity v_theta as a third component.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.constants as sc
import scipy.sparse as sp
import scipy.sparse.linalg as spla

FREE, DIR0, DIRV = 0, 1, 2
ALIVE, CATHODE, ANODE, SIDE, TIP = 0, 1, 2, 3, 4


class RZ:
    """The state of one axisymmetric instance: grid, potential, particles."""

    def __init__(self, nr, nz, h, tip_r, tip_h, apex_field, dt, m_ion):
        self.nr, self.nz, self.h, self.dt, self.m_ion = nr, nz, h, dt, m_ion
        self.R, self.H = tip_r / h, tip_h / h
        self.type = self.node_types()
        self.A = self.operator()
        self.free = np.flatnonzero(self.type == FREE)
        # unit-anode Laplace solution and the anode potential for the apex field
        self.phi1 = self.solve_dirichlet(np.zeros(nr * nz, np.int64), 1.0)
        self.F1 = self.interp(self.phi1, 0.0, self.H + 1.0) / h
        self.V0 = apex_field / self.F1
        self.phi = self.phi1 * self.V0
        self.E = self.field(self.phi)
        self.sp = [None, None, None]
        self.charges = (-sc.e, sc.e, 0.0)
        self.masses = (sc.m_e, m_ion, m_ion)
        self.absorbed = np.zeros((3, 5), np.int64)

    # -- geometry and operator -------------------------------------------------
    def inside_tip(self, r, z):
        zc = self.H - self.R
        r = np.asarray(r, float)
        z = np.asarray(z, float)
        cyl = (z >= 0) & (z <= zc) & (r <= self.R)
        cap = (z > zc) & (r * r + (z - zc) ** 2 <= self.R * self.R)
        return cyl | cap

    def node_types(self):
        k, i = np.meshgrid(np.arange(self.nz), np.arange(self.nr), indexing="ij")
        t = np.zeros((self.nz, self.nr), np.uint8)
        t[self.inside_tip(i, k)] = DIR0
        t[0, :] = DIR0
        t[-1, :] = DIRV
        return t.reshape(-1)

    def couplings(self, i):
        """(radial inner, radial outer, axial) couplings of column i, over pi h."""
        nr = self.nr
        cin = 2.0 * (i - 0.5) if i > 0 else 0.0
        cout = 2.0 * (i + 0.5) if i < nr - 1 else 0.0
        r_hi = min(i + 0.5, nr - 1.0)
        r_lo = max(i - 0.5, 0.0)
        return cin, cout, r_hi * r_hi - r_lo * r_lo

    def operator(self):
        """The matrix of the finite-volume equations over all nodes (rows of
        held nodes are identity rows)."""
        nr, nz = self.nr, self.nz
        rows, cols, vals = [], [], []
        for k in range(nz):
            for i in range(nr):
                n = k * nr + i
                if self.type[n] != FREE:
                    rows.append(n); cols.append(n); vals.append(1.0)
                    continue
                cin, cout, cax = self.couplings(i)
                diag = 0.0
                for m, c in ((n - 1, cin), (n + 1, cout), (n - nr, cax), (n + nr, cax)):
                    if c == 0.0:
                        continue
                    diag += c
                    rows.append(n); cols.append(m); vals.append(-c)
                rows.append(n); cols.append(n); vals.append(diag)
        return sp.csr_matrix((vals, (rows, cols)), shape=(nr * nz, nr * nz))

    def rhs(self, Q, V0):
        """Right-hand side: Q / (pi eps0 h) on free nodes (Q in 2^-40 e), the
        held values on held nodes."""
        b = np.asarray(Q, np.float64) * (2.0 ** -40 * sc.e / (math.pi * sc.epsilon_0 * self.h))
        b[self.type == DIR0] = 0.0
        b[self.type == DIRV] = V0
        return b

    def solve_dirichlet(self, Q, V0):
        return spla.spsolve(self.A.tocsc(), self.rhs(Q, V0))

    def solve_rhs(self, b):
        return spla.spsolve(self.A.tocsc(), b)

    def field(self, phi):
        nr, nz, h = self.nr, self.nz, self.h
        p = phi.reshape(nz, nr)
        Er = np.zeros((nz, nr))
        Er[:, 1:-1] = -(p[:, 2:] - p[:, :-2]) / (2.0 * h)
        Ez = np.zeros((nz, nr))
        Ez[1:-1] = -(p[2:] - p[:-2]) / (2.0 * h)
        Ez[0] = -(p[1] - p[0]) / h
        Ez[-1] = -(p[-1] - p[-2]) / h
        return np.stack([Er.reshape(-1), Ez.reshape(-1)], axis=1)

    # -- interpolation ---------------------------------------------------------
    def _cell(self, r, z):
        i = min(max(int(math.floor(r)), 0), self.nr - 2)
        k = min(max(int(math.floor(z)), 0), self.nz - 2)
        return i, k, r - i, z - k

    def interp(self, f, r, z):
        i, k, fr, fz = self._cell(r, z)
        n = k * self.nr + i
        return ((1 - fr) * (1 - fz) * f[n] + fr * (1 - fz) * f[n + 1] + (1 - fr) * fz * f[n + self.nr]
                + fr * fz * f[n + self.nr + 1])

    def gather(self, r, z):
        return self.interp(self.E[:, 0], r, z), self.interp(self.E[:, 1], r, z)

    # -- particles -------------------------------------------------------------
    def load(self, s, arrays, ids):
        self.sp[s] = {k: np.asarray(v, np.float64).copy() for k, v in arrays.items()}
        self.sp[s]["id"] = np.asarray(ids, np.uint32).copy()

    def push(self):
        """One leapfrog step of every particle with rotation back into the r-z
        plane; removed particles leave the arrays (order kept)."""
        for s in range(3):
            d = self.sp[s]
            if d is None or len(d["r"]) == 0:
                continue
            kq = self.charges[s] / self.masses[s] * self.dt ** 2 / self.h
            keep = np.ones(len(d["r"]), bool)
            for p in range(len(d["r"])):
                r, z = d["r"][p], d["z"][p]
                vr, vt, vz = d["vr"][p], d["vt"][p], d["vz"][p]
                if kq != 0.0:
                    er, ez = self.gather(r, z)
                    vr += kq * er
                    vz += kq * ez
                x, y = r + vr, vt
                z = z + vz
                rn = math.sqrt(x * x + y * y)
                c, s_ = (x / rn, y / rn) if rn > 0.0 else (1.0, 0.0)
                vr, vt = c * vr + s_ * vt, -s_ * vr + c * vt
                d["r"][p], d["z"][p], d["vr"][p], d["vt"][p], d["vz"][p] = rn, z, vr, vt, vz
                code = ALIVE
                if z <= 0.0:
                    code = CATHODE
                elif z >= self.nz - 1:
                    code = ANODE
                elif rn >= self.nr - 1:
                    code = SIDE
                elif self.inside_tip(rn, z):
                    code = TIP
                if code != ALIVE:
                    keep[p] = False
                    self.absorbed[s, code] += 1
            for k in d:
                d[k] = d[k][keep]

    @staticmethod
    def _q(f, bits):
        t = math.ldexp(f, bits)
        q = math.floor(t)
        return int(q) + (1 if t - q >= 0.5 else 0)

    def deposit(self):
        """Node charge in units of 2^-40 e (exact integers)."""
        Q = np.zeros(self.nr * self.nz, np.int64)
        for s, sign in ((0, -1), (1, 1)):
            d = self.sp[s]
            if d is None:
                continue
            for r, z in zip(d["r"], d["z"]):
                i, k, fr, fz = self._cell(r, z)
                qr, qz = self._q(fr, 20), self._q(fz, 20)
                n = k * self.nr + i
                w = ((n, (2 ** 20 - qr) * (2 ** 20 - qz)), (n + 1, qr * (2 ** 20 - qz)),
                     (n + self.nr, (2 ** 20 - qr) * qz), (n + self.nr + 1, qr * qz))
                for m, v in w:
                    Q[m] += sign * v
        self.Q = Q
        return Q

    def solve(self):
        self.phi = self.solve_dirichlet(self.Q, self.V0)
        self.E = self.field(self.phi)
        return self.phi

    def step(self):
        self.push()
        self.deposit()
        self.solve()
