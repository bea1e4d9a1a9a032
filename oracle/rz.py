"""FP64 CPU oracle of the 2D axisymmetric (r, z) 2D3V variant of the
particle-mesh step (Sec. 2.2: the axisymmetric vacuum mesh, the 2D3V method,
particles rotated back into the r-z plane every step, reflection at the
axis, removal at the cathode, the anode and the open side; leapfrog).

TEST INFRASTRUCTURE ONLY: imported by tests/ only. Plain numpy and scipy,
with the 3D oracle's Philox draws and rate routines; it shares no code with
the GPU library.

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
  particle deposits exactly 2^40 units of 2^-40 e onto its four nodes;
- collisions, field ionization and emission: see RZ.
Positions are in grid units (r / h, z / h), velocities in grid units per
step (v dt / h), with the azimuthal velocity v_theta as a third component.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import scipy.constants as sc
import scipy.sparse as sp
import scipy.sparse.linalg as spla

FREE, DIR0, DIRV = 0, 1, 2
ALIVE, CATHODE, ANODE, SIDE, TIP = 0, 1, 2, 3, 4
TAG_MCC1, TAG_MCC2, TAG_PAIR1, TAG_PAIR2, TAG_FI, TAG_INJ = 1, 2, 3, 4, 5, 6
TAG_PAIR3, TAG_MCC3 = 36, 37
XI_CU = 7.726380            # first ionization energy of Cu [eV]
XI2_CU = 20.29239           # second ionization energy of Cu [eV]


class RZ:
    """The state of one axisymmetric instance: grid, potential, particles.

    Collisions, field ionization and emission (collide, emit) follow the
    readings of the 3D oracle (its Philox draws, cross-section tables, ADK
    and Murphy-Good routines), with these for the axisymmetric mesh: the
    particles of a cell (i, k) (between the nodes i, i + 1 and k, k + 1) are
    paired as in a 3D cell, their (v_r, v_theta, v_z) taken as Cartesian
    components (the azimuthal positions of a pair are not tracked, so the
    local frames of the two are taken as one); the per-cell draw is keyed by
    k (nr - 1) + i; the density is N_t over the annular cell volume
    pi (2 i + 1) h^3; the emission patches are rings: fn_rings equal-area rings of the cap, then
    rings one spacing high on the side, each with the Murphy-Good current at
    phi(s + h n) / h and N = J A dt / e electrons, floor(N) plus one with
    probability frac(N), placed uniformly on the ring 10^-3 spacings out
    with zero velocity."""

    def __init__(self, nr, nz, h, tip_r, tip_h, apex_field, dt, m_ion, seed=1, xs=None, xi=XI_CU,
                 phi_w=4.5, fn_rings=16, cu2=False, xi2=XI2_CU):
        self.nr, self.nz, self.h, self.dt, self.m_ion = nr, nz, h, dt, m_ion
        self.seed, self.xi, self.phi_w, self.fn_rings = seed, xi, phi_w, fn_rings
        # cross-section tables (emin, emax, el, iz, cx[, iz2, izi]) on
        # log-spaced energies; with cu2 also Cu + e -> Cu2+ + 3e (iz2) and
        # Cu+ + e -> Cu2+ + 2e (izi), the ions carrying a charge state q
        self.xs = xs
        self.cu2, self.xi2 = cu2, xi2
        self.next_id = 0
        self.step_no = 0
        self.events = np.zeros(7, np.int64)
        self.injected = 0
        self.last_events = []
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
        self.sp[s] = {k: np.asarray(arrays[k], np.float64).copy() for k in ("r", "z", "vr", "vt", "vz")}
        self.sp[s]["id"] = np.asarray(ids, np.uint32).copy()
        if s == 1:
            q = arrays.get("q")
            self.sp[s]["q"] = (np.asarray(q, np.uint8).copy() if q is not None
                               else np.ones(len(ids), np.uint8))
        if len(ids):
            self.next_id = max(self.next_id, int(np.max(ids)) + 1)

    # -- random numbers, rates (the 3D oracle's routines) ----------------------
    def _c(self):
        import oracle
        if getattr(self, "_cfg", None) is None:
            self._cfg = oracle._Config(phi_w=self.phi_w, xi=self.xi, h=self.h, dt=self.dt, seed=self.seed)
            if self.xs is not None:
                emin, emax = self.xs[0], self.xs[1]
                self._tabs = [np.ascontiguousarray(t, np.float64) for t in self.xs[2:]]
                self._cfg.xs_n, self._cfg.xs_emin, self._cfg.xs_emax = len(self._tabs[0]), emin, emax
            self._L = oracle.lib()
        return self._L, self._cfg

    def xs_at(self, k, E):
        """Cross section k (0 elastic, 1 ionization, 2 charge exchange, 3
        double ionization of Cu, 4 ionization of Cu+) at E [eV]: the 3D
        oracle's table interpolation."""
        L, c = self._c()
        return L.orc_xs(C.byref(c), self._tabs[k], E)

    def draw2(self, a, step, tag, sub):
        import oracle
        w = oracle.philox([a & 0xFFFFFFFF, step, tag, sub], [self.seed & 0xFFFFFFFF, self.seed >> 32])
        return oracle.uniform(int(w[0]), int(w[1])), oracle.uniform(int(w[2]), int(w[3]))

    def adk_rate(self, E_GVm):
        """Eq. dfi: field-ionization rate per fs at E in GV/m."""
        L, c = self._c()
        return L.orc_adk_rate(C.byref(c), E_GVm)

    def fn_current(self, F):
        """Murphy-Good current density [A/m^2] at F [V/m] (f clamped at 1)."""
        L, c = self._c()
        cl = C.c_int(0)
        return L.orc_fn_current(C.byref(c), F, C.byref(cl))

    # -- emission ------------------------------------------------------------------
    def patches(self):
        zc = self.H - self.R
        return self.fn_rings + max(int(math.ceil(zc)), 0)

    def patch_point(self, p, ua):
        """(r, z, n_r, n_z, area) of patch p at the uniform ua (grid units)."""
        R, zc = self.R, self.H - self.R
        if p < self.fn_rings:
            ct = 1.0 - (p + ua) / self.fn_rings
            st = math.sqrt(1.0 - ct * ct)
            return R * st, zc + R * ct, st, ct, 2.0 * math.pi * R * R / self.fn_rings
        q = p - self.fn_rings
        zlo, zhi = float(q), min(q + 1.0, zc)
        return R, zlo + ua * (zhi - zlo), 1.0, 0.0, 2.0 * math.pi * R * (zhi - zlo)

    def emit(self):
        """Fowler-Nordheim emission of one step; returns the number of
        electrons added (ids in patch order)."""
        new = {k: [] for k in ("r", "z", "vr", "vt", "vz", "id")}
        for p in range(self.patches()):
            r, z, nr_, nz_, area = self.patch_point(p, 0.5)
            F = self.interp(self.phi, r + nr_, z + nz_) / self.h
            N = self.fn_current(F) * area * self.h * self.h * self.dt / sc.e
            u0, _ = self.draw2(p, self.step_no, TAG_INJ, 0)
            k = int(math.floor(N)) + (1 if u0 < N - math.floor(N) else 0)
            for j in range(k):
                ua, _ = self.draw2(p, self.step_no, TAG_INJ, 1 + j)
                r, z, nr_, nz_, _ = self.patch_point(p, ua)
                new["r"].append(r + 1e-3 * nr_)
                new["z"].append(z + 1e-3 * nz_)
                for key in ("vr", "vt", "vz"):
                    new[key].append(0.0)
                new["id"].append(self.next_id)
                self.next_id += 1
        self._append(0, new)
        self.injected += len(new["id"])
        return len(new["id"])

    def _append(self, s, new):
        if self.sp[s] is None:
            self.sp[s] = {k: np.zeros(0) for k in ("r", "z", "vr", "vt", "vz")}
            self.sp[s]["id"] = np.zeros(0, np.uint32)
            if s == 1:
                self.sp[s]["q"] = np.zeros(0, np.uint8)
        for k in ("r", "z", "vr", "vt", "vz"):
            self.sp[s][k] = np.concatenate([self.sp[s][k], np.asarray(new[k], np.float64)])
        self.sp[s]["id"] = np.concatenate([self.sp[s]["id"], np.asarray(new["id"], np.uint32)])
        if s == 1:
            q = new.get("q", [1] * len(new["id"]))
            self.sp[s]["q"] = np.concatenate([self.sp[s]["q"], np.asarray(q, np.uint8)])

    # -- collisions -------------------------------------------------------------------
    @staticmethod
    def _du(u, ct2, ph2):
        """Eq. du: R^-1(theta, phi) [R^-1(theta', phi') - I] (0, 0, |u|)."""
        um = math.sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2])
        up = math.sqrt(u[0] * u[0] + u[1] * u[1])
        ct, st = u[2] / um, up / um
        cp, sp_ = (u[0] / up, u[1] / up) if up > 0.0 else (1.0, 0.0)
        st2 = math.sqrt(1.0 - ct2 * ct2)
        w0, w1, w2 = um * st2 * math.cos(ph2), um * st2 * math.sin(ph2), um * (ct2 - 1.0)
        return (ct * cp * w0 - sp_ * w1 + st * cp * w2, ct * sp_ * w0 + cp * w1 + st * sp_ * w2, -st * w0 + ct * w2)

    @staticmethod
    def _iso(ct, ph):
        st = math.sqrt(1.0 - ct * ct)
        return st * math.cos(ph), st * math.sin(ph), ct

    def cell_of(self, s):
        d = self.sp[s]
        i = np.clip(np.floor(d["r"]).astype(np.int64), 0, self.nr - 2)
        k = np.clip(np.floor(d["z"]).astype(np.int64), 0, self.nz - 2)
        return k * (self.nr - 1) + i

    def collide(self):
        """(e, Cu) pairs (elastic, impact ionization; with cu2 also double
        ionization), (Cu+, Cu) pairs (charge exchange), with cu2 (e, Cu+)
        pairs (ionization of Cu+ to Cu2+), then field ionization of the
        neutrals without an event, then the products: impact ionizations,
        then field ionizations, each in ascending neutral id, then the
        ionized ions in ascending ion id; a product's ion (if new) takes the
        next id, its new electrons the following ones. Returns the events as
        (kind, id_a, id_b): 1 elastic, 2 impact ionization, 3 charge
        exchange, 4 field ionization, 5 double ionization of Cu, 6
        ionization of Cu+."""
        h, dt = self.h, self.dt
        V = ("vr", "vt", "vz")
        for s in range(3):
            if self.sp[s] is None:
                self._append(s, {k: [] for k in ("r", "z", "vr", "vt", "vz", "id")})
        cells = [self.cell_of(s) for s in range(3)]
        used = [np.zeros(len(self.sp[s]["id"]), bool) for s in range(3)]
        prods = []            # (kind, key id, index, charge state of the new ion, new electron velocities)
        events = []
        N = self.sp[2]
        I = self.sp[1]
        for cls in ((1, 2, 3) if self.cu2 else (1, 2)):
            sa = 1 if cls == 2 else 0
            sb = 1 if cls == 3 else 2
            A, B = self.sp[sa], self.sp[sb]
            ma, mb = (self.m_ion if cls == 2 else sc.m_e), self.m_ion
            mu = ma * mb / (ma + mb)
            tag_pair, tag = {1: (TAG_PAIR1, TAG_MCC1), 2: (TAG_PAIR2, TAG_MCC2), 3: (TAG_PAIR3, TAG_MCC3)}[cls]
            for c in np.unique(cells[sa]):
                ia = np.flatnonzero(cells[sa] == c)
                ib = np.flatnonzero(cells[sb] == c)
                if len(ib) == 0:
                    continue
                ia = ia[np.argsort(A["id"][ia])]
                ib = ib[np.argsort(B["id"][ib])]
                a_proj = len(ia) <= len(ib)
                P_, T_ = (ia, ib) if a_proj else (ib, ia)
                NT = len(T_)
                uc, _ = self.draw2(int(c), self.step_no, tag_pair, 0)
                shift = min(int(math.floor(uc * NT)), NT - 1)
                vol = math.pi * (2 * int(c % (self.nr - 1)) + 1) * h * h * h
                n = NT / vol
                for q, pp in enumerate(P_):
                    tt = T_[(shift + q) % NT]
                    xa, xb = (pp, tt) if a_proj else (tt, pp)
                    if cls == 2 and used[2][xb]:
                        continue
                    if cls == 3 and (used[0][xa] or used[1][xb] or B["q"][xb] != 1):
                        continue
                    pid = int((A if a_proj else B)["id"][pp])
                    u = [(A[k][xa] - B[k][xb]) * h / dt for k in V]
                    um = math.sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2])
                    E = 0.5 * ma * um * um / sc.e
                    if cls == 1:
                        sig = [self.xs_at(0, E), self.xs_at(1, E) if E > self.xi else 0.0]
                        if self.cu2:
                            sig.append(self.xs_at(3, E) if E > self.xi + self.xi2 else 0.0)
                    elif cls == 2:
                        sig = [self.xs_at(2, E)]
                    else:
                        sig = [self.xs_at(4, E) if E > self.xi2 else 0.0]
                    stot = sum(sig)
                    P = -math.expm1(-um * n * stot * dt)
                    U1, U2 = self.draw2(pid, self.step_no, tag, 0)
                    if not U1 < P:
                        continue
                    proc, cum = len(sig) - 1, 0.0
                    for kk, sg in enumerate(sig):
                        cum += sg
                        if U2 * stot < cum:
                            proc = kk
                            break
                    used[sa][xa] = True
                    used[sb][xb] = True
                    if cls == 2:
                        for k in V:
                            A[k][xa], N[k][xb] = N[k][xb], A[k][xa]
                        events.append((3, int(A["id"][xa]), int(N["id"][xb])))
                    elif cls == 1 and proc == 0:
                        u3, u4 = self.draw2(pid, self.step_no, TAG_MCC1, 1)
                        du = self._du(u, 2.0 * u3 - 1.0, 2.0 * math.pi * u4)
                        ka, kb = mu / ma * dt / h, mu / mb * dt / h
                        for k, d in zip(V, du):
                            A[k][xa] = A[k][xa] + ka * d
                            N[k][xb] = N[k][xb] - kb * d
                        events.append((1, int(A["id"][xa]), int(N["id"][xb])))
                    elif cls == 1 and proc == 1:
                        c1, p1 = self.draw2(pid, self.step_no, TAG_MCC1, 1)
                        c2, p2 = self.draw2(pid, self.step_no, TAG_MCC1, 2)
                        u5, _ = self.draw2(pid, self.step_no, TAG_MCC1, 3)
                        s1 = self._iso(2.0 * c1 - 1.0, 2.0 * math.pi * p1)
                        s2 = self._iso(2.0 * c2 - 1.0, 2.0 * math.pi * p2)
                        erem = E - self.xi
                        e1 = u5 * erem
                        e2 = erem - e1
                        w1 = math.sqrt(2.0 * e1 * sc.e / sc.m_e)
                        w2 = math.sqrt(2.0 * e2 * sc.e / sc.m_e)
                        vn = [N[k][xb] * h / dt for k in V]
                        for j, k in enumerate(V):
                            A[k][xa] = (vn[j] + w1 * s1[j]) * dt / h
                        prods.append((0, int(N["id"][xb]), xb, 1, [[(vn[j] + w2 * s2[j]) * dt / h for j in range(3)]]))
                        events.append((2, int(A["id"][xa]), int(N["id"][xb])))
                    elif cls == 1:
                        # Cu + e -> Cu2+ + 3e: in the neutral's frame the
                        # energy above xi + xi2 is shared as U5, U6 (1 - U5),
                        # the rest by the three electrons, each isotropic
                        c1, p1 = self.draw2(pid, self.step_no, TAG_MCC1, 1)
                        c2, p2 = self.draw2(pid, self.step_no, TAG_MCC1, 2)
                        u5, u6 = self.draw2(pid, self.step_no, TAG_MCC1, 3)
                        c3, p3 = self.draw2(pid, self.step_no, TAG_MCC1, 4)
                        dirs = [self._iso(2.0 * cc - 1.0, 2.0 * math.pi * pp_) for cc, pp_ in
                                ((c1, p1), (c2, p2), (c3, p3))]
                        rest = E - self.xi - self.xi2
                        f1 = u5 * rest
                        f2 = u6 * (rest - f1)
                        f3 = rest - f1 - f2
                        ws = [math.sqrt(2.0 * f * sc.e / sc.m_e) for f in (f1, f2, f3)]
                        vn = [N[k][xb] * h / dt for k in V]
                        for j, k in enumerate(V):
                            A[k][xa] = (vn[j] + ws[0] * dirs[0][j]) * dt / h
                        new_e = [[(vn[j] + ws[m] * dirs[m][j]) * dt / h for j in range(3)] for m in (1, 2)]
                        prods.append((0, int(N["id"][xb]), xb, 2, new_e))
                        events.append((5, int(A["id"][xa]), int(N["id"][xb])))
                    else:
                        # Cu+ + e -> Cu2+ + 2e: as the impact ionization of a
                        # neutral, in the ion's frame, above xi2; the ion keeps
                        # its place, id and velocity and takes charge state 2
                        c1, p1 = self.draw2(pid, self.step_no, TAG_MCC3, 1)
                        c2, p2 = self.draw2(pid, self.step_no, TAG_MCC3, 2)
                        u5, _ = self.draw2(pid, self.step_no, TAG_MCC3, 3)
                        s1 = self._iso(2.0 * c1 - 1.0, 2.0 * math.pi * p1)
                        s2 = self._iso(2.0 * c2 - 1.0, 2.0 * math.pi * p2)
                        rest3 = E - self.xi2
                        g1 = u5 * rest3
                        g2 = rest3 - g1
                        v1 = math.sqrt(2.0 * g1 * sc.e / sc.m_e)
                        v2 = math.sqrt(2.0 * g2 * sc.e / sc.m_e)
                        vi = [I[k][xb] * h / dt for k in V]
                        for j, k in enumerate(V):
                            A[k][xa] = (vi[j] + v1 * s1[j]) * dt / h
                        I["q"][xb] = 2
                        prods.append((2, int(I["id"][xb]), xb, 0, [[(vi[j] + v2 * s2[j]) * dt / h for j in range(3)]]))
                        events.append((6, int(A["id"][xa]), int(I["id"][xb])))
        # field ionization (Eq. dfi), none above the barrier-suppression field
        ebsi = 1.5 * self.xi ** 1.5
        for p in range(len(N["id"])):
            if used[2][p]:
                continue
            er, ez = self.gather(N["r"][p], N["z"][p])
            Eg = math.sqrt(er * er + ez * ez) * 1e-9
            if Eg > ebsi:
                continue
            pdt = self.adk_rate(Eg) * (dt * 1e15)
            U, _ = self.draw2(int(N["id"][p]), self.step_no, TAG_FI, 0)
            if pdt > U:
                used[2][p] = True
                prods.append((1, int(N["id"][p]), p, 1, [[N[k][p] for k in V]]))
                events.append((4, 0xFFFFFFFF, int(N["id"][p])))
        prods.sort(key=lambda t: (t[0], t[1]))
        ions = {k: [] for k in ("r", "z", "vr", "vt", "vz", "id", "q")}
        els = {k: [] for k in ("r", "z", "vr", "vt", "vz", "id")}
        gone = np.zeros(len(N["id"]), bool)
        for kind, key, x, qnew, ves in prods:
            src = I if kind == 2 else N
            if kind != 2:
                ions["r"].append(N["r"][x])
                ions["z"].append(N["z"][x])
                for k in V:
                    ions[k].append(N[k][x])
                ions["id"].append(self.next_id)
                ions["q"].append(qnew)
                self.next_id += 1
                gone[x] = True
            for ve in ves:
                els["r"].append(src["r"][x])
                els["z"].append(src["z"][x])
                for k, v in zip(V, ve):
                    els[k].append(v)
                els["id"].append(self.next_id)
                self.next_id += 1
        self._append(1, ions)
        self._append(0, els)
        for k in N:
            N[k] = N[k][~gone]
        for kind, _, _ in events:
            self.events[kind] += 1
        self.last_events = events
        return events

    def push(self):
        """One leapfrog step of every particle with rotation back into the r-z
        plane; removed particles leave the arrays (order kept)."""
        for s in range(3):
            d = self.sp[s]
            if d is None or len(d["r"]) == 0:
                continue
            kq0 = self.charges[s] / self.masses[s] * self.dt ** 2 / self.h
            keep = np.ones(len(d["r"]), bool)
            for p in range(len(d["r"])):
                r, z = d["r"][p], d["z"][p]
                vr, vt, vz = d["vr"][p], d["vt"][p], d["vz"][p]
                # a Cu2+ ion (charge state 2) feels twice the force of Cu+
                kq = kq0 * float(d["q"][p]) if s == 1 else kq0
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
        for s, sign0 in ((0, -1), (1, 1)):
            d = self.sp[s]
            if d is None:
                continue
            for p, (r, z) in enumerate(zip(d["r"], d["z"])):
                sign = sign0 * (int(d["q"][p]) if s == 1 else 1)
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

    def step(self, emit=False, collide=False):
        """One step in the order of the 3D oracle: emission, push,
        collisions and field ionization, deposit, solve."""
        if emit:
            self.emit()
        self.push()
        if collide:
            self.collide()
        self.deposit()
        self.solve()
        self.step_no += 1
