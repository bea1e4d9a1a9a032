"""Thin Python binding of the axisymmetric (r, z) 2D3V variant of libpic
(include/pic_rz.h): the ``pic_rz_*`` functions have the names and arguments
of the C entry points and only marshal them; :class:`RZSimulation` owns the
torch tensors of the buffers. Every step runs in the HIP kernels of libpic.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from .pic import DEAD, PIC_OK, PicError, lib as _pic_lib, pic_solve_info

PIC_RZ_PUSH, PIC_RZ_DEPOSIT, PIC_RZ_SOLVE, PIC_RZ_ADVANCE, PIC_RZ_FIELD = 1, 2, 4, 8, 16
PIC_RZ_EMIT, PIC_RZ_COLLIDE = 32, 64
PIC_RZ_FULL = 15
PIC_RZ_ALL = 111


class pic_rz_config(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nz", C.c_int32), ("h", C.c_double), ("tip_r", C.c_double),
                ("tip_h", C.c_double), ("apex_field", C.c_double), ("dt", C.c_double), ("m_ion", C.c_double),
                ("laplace_rtol", C.c_double), ("maxit", C.c_int32), ("sort_every", C.c_int32),
                ("step_rtol", C.c_double), ("seed", C.c_uint64), ("xi", C.c_double), ("phi_w", C.c_double),
                ("xs_emin", C.c_double), ("xs_emax", C.c_double), ("xs_n", C.c_int32), ("fn_rings", C.c_int32),
                ("cu2", C.c_int32), ("reserved3", C.c_int32), ("xi2", C.c_double)]


class pic_rz_buffers(C.Structure):
    _fields_ = [(k, C.c_void_p * 3) for k in ("r", "z", "vr", "vt", "vz", "id")] + \
               [("cap", C.c_int64 * 3), ("n", C.c_int64 * 3), ("phi", C.c_void_p), ("phi1", C.c_void_p),
                ("rho", C.c_void_p), ("field", C.c_void_p), ("node_type", C.c_void_p), ("scratch", C.c_void_p),
                ("scratch_bytes", C.c_size_t), ("xs", C.c_void_p), ("charge", C.c_void_p)]


class pic_rz_moments_t(C.Structure):
    _fields_ = [("n_alive", C.c_int64 * 3), ("absorbed", (C.c_int64 * 5) * 3), ("q_total", C.c_int64),
                ("step", C.c_int64), ("v0", C.c_double), ("apex_field1", C.c_double),
                ("last_cg_iters", C.c_int32), ("error", C.c_int32), ("n_slots", C.c_int64 * 3),
                ("events", C.c_int64 * 5), ("injected", C.c_int64), ("next_id", C.c_int64),
                ("double_ionizations", C.c_int64), ("ion_ionizations", C.c_int64), ("n_cu2", C.c_int64)]


_bound = False


def lib():
    global _bound
    L = _pic_lib()
    if not _bound:
        vp = C.c_void_p
        L.pic_rz_scratch_size.argtypes = [C.POINTER(pic_rz_config), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]
        L.pic_rz_init.argtypes = [C.POINTER(pic_rz_config), C.POINTER(pic_rz_buffers), vp, C.POINTER(vp)]
        L.pic_rz_step.argtypes = [vp, C.c_int32, C.c_uint32]
        L.pic_rz_solve.argtypes = [vp, C.c_double, C.c_int32, C.POINTER(pic_solve_info)]
        L.pic_rz_moments.argtypes = [vp, C.POINTER(pic_rz_moments_t)]
        L.pic_rz_last_error.argtypes = [vp]
        L.pic_rz_last_error.restype = C.c_char_p
        L.pic_rz_destroy.argtypes = [vp]
        for f in ("pic_rz_scratch_size", "pic_rz_init", "pic_rz_step", "pic_rz_solve", "pic_rz_moments"):
            getattr(L, f).restype = C.c_int
        _bound = True
    return L


def _check(code, ctx=None):
    if code != PIC_OK:
        msg = lib().pic_rz_last_error(ctx) if ctx else b""
        raise PicError(code, msg.decode() if msg else "")


def pic_rz_scratch_size(cfg, cap) -> int:
    n = C.c_size_t()
    _check(lib().pic_rz_scratch_size(C.byref(cfg), (C.c_int64 * 3)(*cap), C.byref(n)))
    return n.value


def pic_rz_init(cfg, bufs, stream_ptr):
    ctx = C.c_void_p()
    code = lib().pic_rz_init(C.byref(cfg), C.byref(bufs), C.c_void_p(stream_ptr), C.byref(ctx))
    _check(code)
    return ctx


def pic_rz_step(ctx, nsteps, flags):
    _check(lib().pic_rz_step(ctx, nsteps, flags), ctx)


def pic_rz_solve(ctx, rtol, maxit) -> dict:
    info = pic_solve_info()
    _check(lib().pic_rz_solve(ctx, rtol, maxit, C.byref(info)), ctx)
    return {"iterations": info.iterations, "converged": bool(info.converged)}


def pic_rz_moments(ctx) -> dict:
    m = pic_rz_moments_t()
    _check(lib().pic_rz_moments(ctx, C.byref(m)), ctx)
    return {"n_alive": np.array(m.n_alive[:]), "absorbed": np.array([list(r) for r in m.absorbed]),
            "q_total": m.q_total, "step": m.step, "v0": m.v0, "apex_field1": m.apex_field1,
            "last_cg_iters": m.last_cg_iters, "error": m.error, "n_slots": np.array(m.n_slots[:]),
            "events": np.array(list(m.events[:]) + [m.double_ionizations, m.ion_ionizations]),
            "injected": m.injected, "next_id": m.next_id, "n_cu2": m.n_cu2}


class RZSimulation:
    """One axisymmetric instance on a GPU. load: dict species index ->
    dict r, z, vr, vt, vz (grid units, FP64); particles are numbered in load
    order (species 0, 1, 2) unless ids (species -> uint32 array) is given.
    xs: (emin, emax, elastic, ionization, charge exchange[, double
    ionization, ionization of Cu+]) cross-section tables for the collisions;
    fn_rings > 0 enables the emission; cu2 adds Cu2+ as an ion charge state
    (load[1]["q"] gives the initial states)."""

    def __init__(self, nr, nz, h, tip_r, tip_h, apex_field, dt, m_ion, load, caps=None, laplace_rtol=1e-13,
                 step_rtol=1e-10, maxit=100000, device="cuda", seed=1, xs=None, xi=7.726380, phi_w=4.5,
                 fn_rings=0, ids=None, cu2=False, xi2=20.29239, sort_every=0):
        self.device = torch.device(device)
        self.cfg = pic_rz_config(nr=nr, nz=nz, h=h, tip_r=tip_r, tip_h=tip_h, apex_field=apex_field, dt=dt,
                                 m_ion=m_ion, laplace_rtol=laplace_rtol, maxit=maxit, step_rtol=step_rtol,
                                 seed=seed, xi=xi, phi_w=phi_w, fn_rings=fn_rings, cu2=1 if cu2 else 0, xi2=xi2,
                                 sort_every=sort_every)
        self.xs = None
        if xs is not None:
            self.cfg.xs_emin, self.cfg.xs_emax = xs[0], xs[1]
            self.cfg.xs_n = len(xs[2])
            ntab = 5 if cu2 else 3
            self.xs = torch.as_tensor(np.concatenate([np.asarray(t, np.float64) for t in xs[2:2 + ntab]])).to(
                self.device)
        n = [len(load[s]["r"]) if s in load else 0 for s in range(3)]
        caps = caps or [max(k, 1) for k in n]
        self.sp = []
        b = pic_rz_buffers()
        nid = 0
        ids_given = ids
        for s in range(3):
            d = {}
            for k in ("r", "z", "vr", "vt", "vz"):
                t = torch.zeros(caps[s], dtype=torch.float64, device=self.device)
                if n[s]:
                    t[: n[s]] = torch.as_tensor(np.asarray(load[s][k], np.float64))
                d[k] = t
                getattr(b, k)[s] = t.data_ptr()
            ids = torch.full((caps[s],), -1, dtype=torch.int32, device=self.device)
            if n[s] and ids_given is not None:
                ids[: n[s]] = torch.as_tensor(np.asarray(ids_given[s], np.uint32).view(np.int32))
            elif n[s]:
                ids[: n[s]] = torch.arange(nid, nid + n[s], dtype=torch.int32)
            nid += n[s]
            d["id"] = ids
            b.id[s] = ids.data_ptr()
            b.cap[s] = caps[s]
            b.n[s] = n[s]
            self.sp.append(d)
        nn = nr * nz
        self.phi = torch.zeros(nn, dtype=torch.float64, device=self.device)
        self.phi1 = torch.zeros(nn, dtype=torch.float64, device=self.device)
        self.rho = torch.zeros(nn, dtype=torch.int64, device=self.device)
        self.field = torch.zeros(2 * nn, dtype=torch.float64, device=self.device)
        self.node_type = torch.zeros(nn, dtype=torch.uint8, device=self.device)
        sb = pic_rz_scratch_size(self.cfg, caps)
        self.scratch = torch.zeros(sb + 256, dtype=torch.uint8, device=self.device)
        for k in ("phi", "phi1", "rho", "field", "node_type", "scratch"):
            setattr(b, k, getattr(self, k).data_ptr())
        b.scratch_bytes = sb + 256
        b.xs = self.xs.data_ptr() if self.xs is not None else None
        self.charge = None
        if cu2:
            self.charge = torch.ones(max(caps[1], 1), dtype=torch.uint8, device=self.device)
            if n[1] and "q" in load[1]:
                self.charge[: n[1]] = torch.as_tensor(np.asarray(load[1]["q"], np.uint8))
            b.charge = self.charge.data_ptr()
        self.bufs = b
        self.n = n
        torch.cuda.synchronize(self.device)
        self.ctx = pic_rz_init(self.cfg, b, torch.cuda.current_stream(self.device).cuda_stream)

    def step(self, nsteps=1, flags=PIC_RZ_FULL):
        pic_rz_step(self.ctx, nsteps, flags)

    def solve(self, rtol=1e-10, maxit=100000):
        return pic_rz_solve(self.ctx, rtol, maxit)

    def moments(self):
        return pic_rz_moments(self.ctx)

    def state(self):
        """Alive particles of each species in ascending id order."""
        n = self.moments()["n_slots"]
        out = []
        for s in range(3):
            ids = self.sp[s]["id"][: n[s]].cpu().numpy().view(np.uint32)
            alive = np.flatnonzero(ids != DEAD)
            alive = alive[np.argsort(ids[alive], kind="stable")]
            d = {k: self.sp[s][k][: n[s]].cpu().numpy()[alive] for k in ("r", "z", "vr", "vt", "vz")}
            d["id"] = ids[alive]
            if s == 1 and self.charge is not None:
                d["q"] = self.charge[: n[s]].cpu().numpy()[alive]
            out.append(d)
        return out

    def set_phi(self, phi):
        self.phi.copy_(torch.as_tensor(np.asarray(phi, np.float64)).to(self.device))
        torch.cuda.synchronize(self.device)
        pic_rz_step(self.ctx, 1, PIC_RZ_FIELD)

    def grid(self, name):
        torch.cuda.synchronize(self.device)
        return getattr(self, name).cpu().numpy()

    def close(self):
        if self.ctx:
            lib().pic_rz_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
