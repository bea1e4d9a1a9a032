"""Thin Python binding of libpic (include/pic.h).

The functions ``pic_*`` below have the names and arguments of the C entry
points and only marshal arguments; every step of the computation runs in the
HIP kernels of libpic. PyTorch is used for device memory (all buffers are
torch tensors owned by :class:`Simulation`) and for the HIP stream.

libpic must be built (``paper_2402_08404_amd.build.build()``); importing this
module on a machine without it raises, there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime libpic links against)

from . import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK = 0
ERRORS = {-1: "INVALID_ARG", -2: "HIP", -3: "CAPACITY", -4: "OVERFLOW", -5: "NOT_CONVERGED", -6: "STATE"}
PIC_F64, PIC_F32 = 0, 1
PIC_SOLVER_CG, PIC_SOLVER_MGCG, PIC_SOLVER_MIXED = 0, 1, 2
PIC_GUESS_ZERO, PIC_GUESS_PREVIOUS, PIC_GUESS_LAPLACE, PIC_GUESS_LEARNED = 0, 1, 2, 3
STEP_INJECT, STEP_PUSH, STEP_DEPOSIT, STEP_COLLIDE = 0x01, 0x02, 0x04, 0x08
STEP_SOLVE, STEP_FIELD, STEP_ADVANCE, STEP_EVENTS = 0x10, 0x20, 0x40, 0x80
STEP_FULL = STEP_INJECT | STEP_PUSH | STEP_COLLIDE | STEP_SOLVE | STEP_ADVANCE
DEAD = 0xFFFFFFFF


class PicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libpic error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class pic_config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("precision", C.c_int32),
                ("h", C.c_double), ("tip_r", C.c_double), ("tip_h", C.c_double), ("apex_field", C.c_double),
                ("phi_w", C.c_double), ("dt", C.c_double), ("xi", C.c_double), ("m_ion", C.c_double),
                ("seed", C.c_uint64), ("xs_n", C.c_int32), ("solver", C.c_int32),
                ("xs_emin", C.c_double), ("xs_emax", C.c_double),
                ("xs_el", C.POINTER(C.c_double)), ("xs_iz", C.POINTER(C.c_double)), ("xs_cx", C.POINTER(C.c_double)),
                ("fn_rings", C.c_int32), ("fn_az", C.c_int32), ("laplace_rtol", C.c_double),
                ("step_rtol", C.c_double), ("step_maxit", C.c_int32), ("sort_every", C.c_int32),
                ("id_capacity", C.c_int64), ("stencil_blocks", C.c_int32), ("step_guess", C.c_int32),
                ("surface_T", C.c_double), ("circuit_R", C.c_double), ("circuit_C", C.c_double),
                ("weighted", C.c_int32), ("w_max", C.c_int32), ("n_max", C.c_double),
                ("merge_every", C.c_int32), ("merge_max", C.c_int32), ("same_species", C.c_int32),
                ("reserved2", C.c_int32), ("sigma_nn", C.c_double), ("coulomb_log", C.c_double),
                ("sigma_rec", C.c_double)]


class pic_buffers(C.Structure):
    _fields_ = [(k, C.c_void_p * 3) for k in ("x", "y", "z", "vx", "vy", "vz")] + \
               [("id", C.c_void_p * 3), ("cap", C.c_int64 * 3), ("phi", C.c_void_p), ("phi1", C.c_void_p),
                ("rho", C.c_void_p), ("field", C.c_void_p), ("field0", C.c_void_p), ("node_type", C.c_void_p),
                ("scratch", C.c_void_p), ("scratch_bytes", C.c_size_t), ("w", C.c_void_p * 3)]


class pic_particles(C.Structure):
    _fields_ = [("species", C.c_int32), ("pad", C.c_int32), ("n", C.c_int64)] + \
               [(k, C.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz")] + [("w", C.c_void_p)]


class pic_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("relres", C.c_double), ("relres0", C.c_double),
                ("fell_back", C.c_int32), ("reserved", C.c_int32)]


class pic_moments_t(C.Structure):
    _fields_ = [("n_alive", C.c_int64 * 3), ("n_slots", C.c_int64 * 3), ("absorbed", (C.c_int64 * 5) * 3),
                ("events", C.c_int64 * 5), ("injected", C.c_int64), ("fn_clamped", C.c_int64),
                ("bsi_count", C.c_int64), ("q_total", C.c_int64), ("next_id", C.c_int64), ("step", C.c_int64),
                ("ke", C.c_double * 3), ("i_sr", C.c_double), ("fn_expected", C.c_double), ("v0", C.c_double),
                ("apex_field1", C.c_double), ("error", C.c_int32), ("last_cg_iters", C.c_int32),
                ("last_cg_relres", C.c_double), ("cg_iters_total", C.c_int64),
                ("evaporated", C.c_int64), ("evap_expected", C.c_double), ("bomb_energy", C.c_double * 2),
                ("v_gap", C.c_double), ("i_gap", C.c_double), ("i_tot", C.c_double),
                ("n_phys", C.c_int64 * 3), ("events_w", C.c_int64 * 5), ("splits", C.c_int64),
                ("evap_atoms", C.c_int64), ("merges", C.c_int64 * 3), ("nn_events", C.c_int64),
                ("coulomb_pairs", C.c_int64), ("recombinations", C.c_int64)]


class pic_unet_config(C.Structure):
    _fields_ = [("base_channels", C.c_int32), ("reserved", C.c_int32 * 7)]


class pic_event(C.Structure):
    _fields_ = [("kind", C.c_int32), ("id_a", C.c_uint32), ("id_b", C.c_uint32), ("new_ion", C.c_uint32),
                ("new_e", C.c_uint32)]


_lib = None


def lib():
    """Load libpic.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run paper_2402_08404_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.pic_scratch_size.argtypes = [C.POINTER(pic_config), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]
        L.pic_init.argtypes = [C.POINTER(pic_config), C.POINTER(pic_buffers), vp, C.POINTER(vp)]
        L.pic_inject.argtypes = [vp, C.POINTER(pic_particles), C.POINTER(C.c_int64)]
        L.pic_inject_noalloc.argtypes = [vp, C.POINTER(C.c_int64)]
        L.pic_step.argtypes = [vp, C.c_int32, C.c_uint32]
        L.pic_solve_poisson.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, C.c_int32, C.POINTER(pic_solve_info)]
        L.pic_moments.argtypes = [vp, C.POINTER(pic_moments_t)]
        L.pic_events.argtypes = [vp, C.POINTER(pic_event), C.c_int64, C.POINTER(C.c_int64)]
        L.pic_profile.argtypes = [vp, C.c_int32]
        L.pic_timers.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]
        L.pic_profile.restype = C.c_int32
        L.pic_timers.restype = C.c_int32
        L.pic_last_error.argtypes = [vp]
        L.pic_last_error.restype = C.c_char_p
        L.pic_destroy.argtypes = [vp]
        L.pic_destroy.restype = None
        up = C.POINTER(pic_unet_config)
        L.unet_param_count.argtypes = [up, C.POINTER(C.c_int64)]
        L.unet_workspace_size.argtypes = [up, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
        L.unet_create.argtypes = [up, vp, vp, vp, C.c_size_t, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp,
                                  C.POINTER(vp)]
        L.unet_forward.argtypes = [vp, vp, vp]
        L.unet_backward.argtypes = [vp, vp, C.POINTER(C.c_double)]
        L.unet_adam_step.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float]
        L.unet_sync_params.argtypes = [vp]
        L.unet_destroy.argtypes = [vp]
        L.unet_destroy.restype = None
        L.pic_set_learned_guess.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_int32]
        L.pic_training_sample.argtypes = [vp, vp, vp, C.POINTER(C.c_double)]
        for f in ("pic_scratch_size", "pic_init", "pic_inject", "pic_inject_noalloc", "pic_step", "pic_solve_poisson", "pic_moments",
                  "pic_events", "unet_param_count", "unet_workspace_size", "unet_create", "unet_forward",
                  "unet_backward", "unet_adam_step", "unet_sync_params", "pic_set_learned_guess",
                  "pic_training_sample"):
            getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


def _check(code: int, ctx=None):
    if code != PIC_OK:
        msg = lib().pic_last_error(ctx)
        raise PicError(code, msg.decode() if msg else "")


# --------------------------------------------------------------------------
# Entry points (same names as the C ABI)


def pic_scratch_size(cfg: pic_config, cap) -> int:
    n = C.c_size_t()
    _check(lib().pic_scratch_size(C.byref(cfg), (C.c_int64 * 3)(*cap), C.byref(n)))
    return n.value


def pic_init(cfg: pic_config, bufs: pic_buffers, stream: int):
    ctx = C.c_void_p()
    _check(lib().pic_init(C.byref(cfg), C.byref(bufs), C.c_void_p(stream), C.byref(ctx)))
    return ctx


def pic_inject(ctx, src: pic_particles | None) -> int:
    n = C.c_int64()
    _check(lib().pic_inject(ctx, C.byref(src) if src is not None else None, C.byref(n)), ctx)
    return n.value


def pic_inject_noalloc(ctx) -> int:
    n = C.c_int64()
    _check(lib().pic_inject_noalloc(ctx, C.byref(n)), ctx)
    return n.value


def pic_step(ctx, nsteps: int, flags: int) -> int:
    code = lib().pic_step(ctx, nsteps, flags)
    if code not in (PIC_OK, -5):
        _check(code, ctx)
    return code


def pic_solve_poisson(ctx, solver: int, guess: int, rtol: float, maxit: int, allow_unconverged: bool = False) -> dict:
    info = pic_solve_info()
    code = lib().pic_solve_poisson(ctx, solver, guess, rtol, maxit, C.byref(info))
    if code != PIC_OK and not (allow_unconverged and code == -5):
        _check(code, ctx)
    return {"iterations": info.iterations, "converged": bool(info.converged), "relres": info.relres,
            "relres0": info.relres0, "fell_back": bool(info.fell_back)}


def pic_moments(ctx) -> dict:
    m = pic_moments_t()
    _check(lib().pic_moments(ctx, C.byref(m)), ctx)
    return {"n_alive": np.array(m.n_alive[:]), "n_slots": np.array(m.n_slots[:]),
            "absorbed": np.array([list(r) for r in m.absorbed]), "events": np.array(m.events[:]),
            "injected": m.injected, "fn_clamped": m.fn_clamped, "bsi_count": m.bsi_count, "q_total": m.q_total,
            "next_id": m.next_id, "step": m.step, "ke": np.array(m.ke[:]), "i_sr": m.i_sr,
            "fn_expected": m.fn_expected, "v0": m.v0, "apex_field1": m.apex_field1, "error": m.error,
            "last_cg_iters": m.last_cg_iters, "last_cg_relres": m.last_cg_relres, "cg_iters_total": m.cg_iters_total,
            "evaporated": m.evaporated, "evap_expected": m.evap_expected, "bomb_energy": np.array(m.bomb_energy[:]),
            "v_gap": m.v_gap, "i_gap": m.i_gap, "i_tot": m.i_tot, "n_phys": np.array(m.n_phys[:]),
            "events_w": np.array(m.events_w[:]), "splits": m.splits, "evap_atoms": m.evap_atoms,
            "merges": np.array(m.merges[:]), "nn_events": m.nn_events, "coulomb_pairs": m.coulomb_pairs,
            "recombinations": m.recombinations}


def pic_events(ctx, cap: int) -> list:
    buf = (pic_event * max(cap, 1))()
    n = C.c_int64()
    _check(lib().pic_events(ctx, buf, cap, C.byref(n)), ctx)
    m = min(n.value, cap)
    return [(buf[i].kind, buf[i].id_a, buf[i].id_b, buf[i].new_ion, buf[i].new_e) for i in range(m)]


TIMERS = ("inject", "push_e", "push", "particles", "collide", "mcc", "solve", "cg_a", "cg_b", "step", "mg", "deposit",
          "bin", "mg_first", "mg_restrict", "mg_corr", "mg_last")


def pic_profile(ctx, enable: bool):
    _check(lib().pic_profile(ctx, 1 if enable else 0), ctx)


def pic_timers(ctx, reset: bool = True) -> dict:
    ms = (C.c_double * len(TIMERS))()
    cnt = (C.c_int64 * len(TIMERS))()
    _check(lib().pic_timers(ctx, ms, cnt, 1 if reset else 0), ctx)
    return {name: (ms[i], cnt[i]) for i, name in enumerate(TIMERS)}


def pic_last_error(ctx) -> str:
    s = lib().pic_last_error(ctx)
    return s.decode() if s else ""


def pic_destroy(ctx):
    lib().pic_destroy(ctx)


# --------------------------------------------------------------------------
# Memory plumbing: one instance with torch-owned device buffers


def unet_param_count(cfg: pic_unet_config) -> int:
    n = C.c_int64()
    _check(lib().unet_param_count(C.byref(cfg), C.byref(n)))
    return n.value


def unet_workspace_size(cfg: pic_unet_config, batch: int, d: int, h: int, w: int) -> int:
    n = C.c_size_t()
    _check(lib().unet_workspace_size(C.byref(cfg), batch, d, h, w, C.byref(n)))
    return n.value


def unet_create(cfg, params: int, grads: int, workspace: int, ws_bytes: int, batch, d, h, w, stream: int):
    out = C.c_void_p()
    _check(lib().unet_create(C.byref(cfg), params, grads, workspace, ws_bytes, batch, d, h, w, stream,
                             C.byref(out)))
    return out.value


def unet_forward(net, x: int, y: int | None):
    _check(lib().unet_forward(net, x, y))


def unet_backward(net, target: int, want_loss: bool = True) -> float | None:
    loss = C.c_double()
    _check(lib().unet_backward(net, target, C.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def unet_adam_step(net, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().unet_adam_step(net, lr, beta1, beta2, eps))


def unet_sync_params(net):
    _check(lib().unet_sync_params(net))


def unet_destroy(net):
    lib().unet_destroy(net)


def pic_set_learned_guess(ctx, net, smooth_passes: int = 0, project: bool = True, fallback: bool = True):
    """Attach a network for PIC_GUESS_LEARNED (None detaches); with project
    the network output is weighted by the energy-norm projection, with
    fallback plain CG judges the guess against V0 phi1 before each solve (see
    include/pic.h)."""
    _check(lib().pic_set_learned_guess(ctx, net, smooth_passes, 1 if project else 0, 1 if fallback else 0), ctx)


def pic_training_sample(ctx, x: int, y: int) -> float:
    s = C.c_double()
    _check(lib().pic_training_sample(ctx, x, y, C.byref(s)), ctx)
    return s.value


def make_config(cfg: workloads.Config, precision=PIC_F64, solver=PIC_SOLVER_CG, laplace_rtol=1e-13,
                step_rtol=1e-8, step_maxit=20000, sort_every=16, id_capacity=0, stencil_blocks=0, step_guess=0,
                weighted=False):
    keep = [np.ascontiguousarray(t, dtype=np.float64) for t in (cfg.xs_el, cfg.xs_iz, cfg.xs_cx)]
    dp = C.POINTER(C.c_double)
    c = pic_config(nx=cfg.nx, ny=cfg.ny, nz=cfg.nz, precision=precision, h=cfg.h, tip_r=cfg.tip_r,
                   tip_h=cfg.tip_h, apex_field=cfg.apex_field, phi_w=cfg.phi_w, dt=cfg.dt, xi=cfg.xi,
                   m_ion=cfg.m_ion, seed=cfg.seed, xs_n=len(keep[0]), solver=solver, xs_emin=cfg.xs_emin,
                   xs_emax=cfg.xs_emax, xs_el=keep[0].ctypes.data_as(dp), xs_iz=keep[1].ctypes.data_as(dp),
                   xs_cx=keep[2].ctypes.data_as(dp), fn_rings=cfg.fn_rings, fn_az=cfg.fn_az,
                   laplace_rtol=laplace_rtol, step_rtol=step_rtol, step_maxit=step_maxit, sort_every=sort_every,
                   id_capacity=id_capacity, stencil_blocks=stencil_blocks, step_guess=step_guess,
                   surface_T=getattr(cfg, "surface_T", 0.0), circuit_R=getattr(cfg, "circuit_R", 0.0),
                   circuit_C=getattr(cfg, "circuit_C", 0.0), weighted=1 if weighted else 0,
                   w_max=int(getattr(cfg, "w_max", 1)), n_max=float(getattr(cfg, "n_max", 1e24)),
                   merge_every=int(getattr(cfg, "merge_every", 0)), merge_max=int(getattr(cfg, "merge_max", 0)),
                   same_species=int(getattr(cfg, "same_species", 0)), sigma_nn=float(getattr(cfg, "sigma_nn", 0.0)),
                   coulomb_log=float(getattr(cfg, "coulomb_log", 10.0)), sigma_rec=float(getattr(cfg, "sigma_rec", 0.0)))
    return c, keep


class Simulation:
    """One PIC-MCC instance on a GPU: torch tensors for every buffer of
    pic_buffers, and the context."""

    def __init__(self, cfg: workloads.Config, caps=(1 << 16, 1 << 14, 1 << 14), precision=PIC_F64,
                 solver=PIC_SOLVER_CG, device="cuda", stream: torch.cuda.Stream | None = None, weighted=False, **kw):
        """weighted: every superparticle carries a weight (Sec. 2.3.2)."""
        self.cfg = cfg
        self.weighted = bool(weighted)
        kw["weighted"] = self.weighted
        self.device = torch.device(device)
        self.dtype = torch.float32 if precision == PIC_F32 else torch.float64
        self.precision = precision
        self.c, self._keep = make_config(cfg, precision=precision, solver=solver, **kw)
        self.caps = tuple(int(x) for x in caps)
        nn = cfg.nx * cfg.ny * cfg.nz
        dev = self.device
        self.sp = []
        for s in range(3):
            cap = max(self.caps[s], 1)
            arrs = {k: torch.zeros(cap, dtype=self.dtype, device=dev) for k in ("x", "y", "z", "vx", "vy", "vz")}
            arrs["id"] = torch.full((cap,), -1, dtype=torch.int32, device=dev)
            if self.weighted:
                arrs["w"] = torch.ones(cap, dtype=torch.int32, device=dev)
            self.sp.append(arrs)
        self.phi = torch.zeros(nn, dtype=torch.float64, device=dev)
        self.phi1 = torch.zeros(nn, dtype=torch.float64, device=dev)
        self.rho = torch.zeros(nn, dtype=torch.int64, device=dev)
        self.field = torch.zeros(4 * nn, dtype=self.dtype, device=dev)
        self.field0 = torch.zeros(4 * nn, dtype=self.dtype, device=dev)
        self.node_type = torch.zeros(nn, dtype=torch.uint8, device=dev)
        nbytes = pic_scratch_size(self.c, self.caps)
        self._scratch_raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self._scratch_raw.data_ptr()
        self._scratch_off = (-base) % 256
        b = pic_buffers()
        for s in range(3):
            for k in ("x", "y", "z", "vx", "vy", "vz"):
                getattr(b, k)[s] = self.sp[s][k].data_ptr()
            b.id[s] = self.sp[s]["id"].data_ptr()
            b.cap[s] = self.caps[s]
            if self.weighted:
                b.w[s] = self.sp[s]["w"].data_ptr()
        b.phi, b.phi1, b.rho = self.phi.data_ptr(), self.phi1.data_ptr(), self.rho.data_ptr()
        b.field, b.field0, b.node_type = self.field.data_ptr(), self.field0.data_ptr(), self.node_type.data_ptr()
        b.scratch = base + self._scratch_off
        b.scratch_bytes = nbytes
        self.bufs = b
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        torch.cuda.synchronize(dev)
        self.ctx = pic_init(self.c, b, self.stream.cuda_stream)

    def close(self):
        if self.ctx is not None:
            pic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- convenience wrappers ------------------------------------------------
    def load(self, load: dict):
        """Append a particle load (dict species name -> x..vz arrays), in the
        order electrons, ions, neutrals."""
        for s, name in enumerate(workloads.SPECIES):
            if name not in load:
                continue
            a = load[name]
            n = len(a["x"])
            if n == 0:
                continue
            t = {k: torch.as_tensor(np.asarray(a[k]), dtype=self.dtype).to(self.device) for k in
                 ("x", "y", "z", "vx", "vy", "vz")}
            src = pic_particles(species=s, n=n, **{k: v.data_ptr() for k, v in t.items()})
            if self.weighted and "w" in a:
                tw = torch.as_tensor(np.asarray(a["w"], np.int64).astype(np.int32)).to(self.device)
                t["w"] = tw
                src.w = tw.data_ptr()
            torch.cuda.synchronize(self.device)
            pic_inject(self.ctx, src)

    def inject(self) -> int:
        return pic_inject(self.ctx, None)

    def step(self, nsteps=1, flags=STEP_FULL) -> int:
        return pic_step(self.ctx, nsteps, flags)

    def solve(self, solver=PIC_SOLVER_CG, guess=PIC_GUESS_PREVIOUS, rtol=1e-8, maxit=100000, **kw) -> dict:
        return pic_solve_poisson(self.ctx, solver, guess, rtol, maxit, **kw)

    def moments(self) -> dict:
        return pic_moments(self.ctx)

    def events(self, cap=None) -> list:
        if cap is None:
            cap = self.caps[2] + 16
        return pic_events(self.ctx, cap)

    def set_phi(self, phi: np.ndarray):
        self.phi.copy_(torch.as_tensor(np.asarray(phi, np.float64)).to(self.device))
        torch.cuda.synchronize(self.device)
        pic_step(self.ctx, 1, STEP_FIELD)

    def state(self) -> list:
        """Alive particles per species as numpy arrays (ids as uint32)."""
        m = self.moments()
        out = []
        for s in range(3):
            n = int(m["n_slots"][s])
            d = {k: self.sp[s][k][:n].cpu().numpy().astype(np.float64) for k in ("x", "y", "z", "vx", "vy", "vz")}
            ids = self.sp[s]["id"][:n].cpu().numpy().view(np.uint32)
            alive = ids != DEAD
            d = {k: v[alive] for k, v in d.items()}
            d["id"] = ids[alive]
            d["w"] = (self.sp[s]["w"][:n].cpu().numpy().view(np.uint32)[alive] if self.weighted
                      else np.ones(int(alive.sum()), np.uint32))
            out.append(d)
        return out

    def grid(self, name: str) -> np.ndarray:
        t = getattr(self, name)
        torch.cuda.synchronize(self.device)
        return t.cpu().numpy()


class UNet:
    """The warm-start network of include/pic.h on torch-owned device memory:
    fp32 parameters and gradients, and the work memory."""

    def __init__(self, batch: int, d: int, h: int, w: int, base_channels: int = 16, seed: int = 0,
                 params: torch.Tensor | None = None, device="cuda"):
        self.cfg = pic_unet_config(base_channels=base_channels)
        self.shape = (batch, d, h, w)
        self.device = torch.device(device)
        self.n_params = unet_param_count(self.cfg)
        if params is None:
            params = init_unet_params(self.layers(), self.n_params, seed)
        self.params = torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous()
        self.grads = torch.zeros_like(self.params)
        nb = unet_workspace_size(self.cfg, batch, d, h, w)
        self._ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws.data_ptr()) % 256
        self.stream = torch.cuda.current_stream(self.device)
        torch.cuda.synchronize(self.device)
        self.net = unet_create(self.cfg, self.params.data_ptr(), self.grads.data_ptr(), self._ws.data_ptr() + off, nb,
                               batch, d, h, w, self.stream.cuda_stream)

    def layers(self):
        return unet_layers(self.cfg.base_channels)

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        x = x.to(self.device, torch.float32).contiguous()
        assert tuple(x.shape) == self.shape
        y = torch.empty_like(x)
        unet_forward(self.net, x.data_ptr(), y.data_ptr())
        return y

    def train_step(self, x: torch.Tensor, target: torch.Tensor, lr: float, want_loss=True):
        x = x.to(self.device, torch.float32).contiguous()
        target = target.to(self.device, torch.float32).contiguous()
        assert tuple(x.shape) == self.shape and tuple(target.shape) == self.shape
        unet_forward(self.net, x.data_ptr(), None)
        loss = unet_backward(self.net, target.data_ptr(), want_loss)
        unet_adam_step(self.net, lr)
        return loss

    def gradients(self, x: torch.Tensor, target: torch.Tensor) -> tuple[float, torch.Tensor]:
        x = x.to(self.device, torch.float32).contiguous()
        target = target.to(self.device, torch.float32).contiguous()
        unet_forward(self.net, x.data_ptr(), None)
        loss = unet_backward(self.net, target.data_ptr(), True)
        return loss, self.grads.clone()

    def sync(self):
        torch.cuda.synchronize(self.device)
        unet_sync_params(self.net)

    def close(self):
        if self.net is not None:
            torch.cuda.synchronize(self.device)
            unet_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def unet_layers(base: int = 16):
    """(kind, cin, cout) of every layer in parameter order, then the head;
    kind is "conv3" (3x3x3), "down" (2x2x2 stride 2) or "up" (2x2x2 stride-2
    transposed). This is the layout of the parameter vector in include/pic.h."""
    c = [base, 2 * base, 4 * base, 8 * base]
    L = [("conv3", 8, c[0]), ("conv3", c[0], c[0])]
    for lv in range(1, 4):
        L += [("down", c[lv - 1], c[lv]), ("conv3", c[lv], c[lv]), ("conv3", c[lv], c[lv])]
    for lv in (2, 1, 0):
        L += [("up", c[lv + 1], c[lv]), ("conv3", 2 * c[lv], c[lv]), ("conv3", c[lv], c[lv])]
    return L


def init_unet_params(layers, n_params: int, seed: int) -> np.ndarray:
    """He-normal weights (fan-in = taps x cin), zero biases, head weights of
    scale 1/sqrt(cin). The first layer's fan-in counts its one live channel."""
    rng = np.random.default_rng(seed)
    out = []
    for i, (kind, cin, cout) in enumerate(layers):
        taps = 27 if kind == "conv3" else 8
        fan = taps * (1 if i == 0 else cin) if kind != "up" else cin
        out.append(rng.standard_normal(taps * cin * cout) * np.sqrt(2.0 / fan))
        out.append(np.zeros(cout))
    base = layers[-1][2]
    out.append(rng.standard_normal(base) / np.sqrt(base))
    out.append(np.zeros(1))
    p = np.concatenate(out).astype(np.float32)
    assert p.size == n_params, (p.size, n_params)
    return p
