"""ctypes binding of the C ABI in ``include/lbm.h``.

Argument marshalling only: every step of the lattice Boltzmann update runs in
the HIP kernels of ``liblbm.so``.  PyTorch supplies device memory (the
workspace and field buffers) and the stream.  If the shared library is
missing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

OK, ERR_INVALID_ARG, ERR_EOS_DOMAIN, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_HIP, ERR_NO_CONVERGENCE = (
    0, -1, -2, -3, -4, -5, -6)
MODEL_P, MODEL_FE = 0, 1
EOS_VDW, EOS_CS = 0, 1
FP64, FP32_SHIFTED = 0, 1
BOUNDARY_PERIODIC, BOUNDARY_WALLS = 0, 1
FLAG_NONFINITE, FLAG_PSI_CLAMP, FLAG_EOS_DOMAIN = 1, 2, 4

BATCH_ACTIVE, BATCH_CONVERGED, BATCH_UNSTABLE, BATCH_MAXSTEPS, BATCH_DROPPED = 0, 1, 2, 3, 4
BATCH_STALLED, BATCH_STALL_CHECKS = 5, 100
KF_SET, KF_NT_STORE, KF_REGCAP, KF_PIPELINE, KF_NO_XCD_REMAP, KF_TWO_STEP, KF_STRIP128 = (
    0x80000000, 1, 2, 4, 8, 16, 32)
KF_STRIP192 = 64

EXPORTED_SYMBOLS = [
    "lbm_status_string", "lbm_workspace_bytes", "lbm_init", "lbm_step", "lbm_observe",
    "lbm_get_populations", "lbm_set_populations", "lbm_destroy", "lbm_launch_info",
    "lbm_autotune",
    "lbm_eos_eval", "lbm_eos_critical", "lbm_maxwell", "lbm_sigma_li_theory", "lbm_fe_planar_theory",
    "lbm_match_p_to_fe",
    "lbm_batch_workspace_bytes", "lbm_batch_create", "lbm_batch_run", "lbm_batch_state",
    "lbm_batch_observe", "lbm_batch_destroy", "lbm_batch_set_limit", "lbm_batch_set_partner",
    "lbm_batch_stats", "lbm_batch_launch_info",
    "lbm_mlp_forward", "lbm_mlp_workspace_bytes", "lbm_mlp_grad", "lbm_mlp_adam",
    "lbm_mlp_train_step", "lbm_mlp_grad_noalloc",
]

MLP_NPARAMS = 34180
MLP_BF16 = 1


class LbmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("model", ctypes.c_int32), ("eos", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("boundary", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("R", ctypes.c_double), ("T", ctypes.c_double),
                ("tau", ctypes.c_double * 9),
                ("sigma_li", ctypes.c_double), ("kappa_li", ctypes.c_double),
                ("kappa_p", ctypes.c_double), ("kappa", ctypes.c_double),
                ("A", ctypes.c_double), ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("rho_ref", ctypes.c_double),
                ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("kernel_flags", ctypes.c_uint32), ("tile_rounds", ctypes.c_int32),
                ("x_split", ctypes.c_int32),
                ("ax", ctypes.c_double), ("rho_ave", ctypes.c_double),
                ("ax_from_step", ctypes.c_int64), ("g", ctypes.c_double),
                ("grav_rho0", ctypes.c_double), ("grav_y0", ctypes.c_double)]


class MlpNorm(ctypes.Structure):
    _fields_ = [("x_shift", ctypes.c_float * 4), ("x_scale", ctypes.c_float * 4),
                ("y_shift", ctypes.c_float * 4), ("y_scale", ctypes.c_float * 4)]

    @classmethod
    def make(cls, x_shift, x_scale, y_shift, y_scale) -> "MlpNorm":
        n = cls()
        for name, v in (("x_shift", x_shift), ("x_scale", x_scale), ("y_shift", y_shift),
                        ("y_scale", y_scale)):
            arr = getattr(n, name)
            for i in range(4):
                arr[i] = float(v[i])
        return n

    def as_dict(self) -> dict:
        import numpy as np
        return {k: np.array(list(getattr(self, k)), dtype=np.float64)
                for k, _ in self._fields_}


class Obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("mass", ctypes.c_double),
                ("max_u", ctypes.c_double), ("rho_min", ctypes.c_double),
                ("rho_max", ctypes.c_double), ("rho_in", ctypes.c_double),
                ("rho_out", ctypes.c_double), ("dp", ctypes.c_double),
                ("r_equimolar", ctypes.c_double), ("du_max", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Launch(ctypes.Structure):
    _fields_ = [("steps_per_launch", ctypes.c_int32), ("strip", ctypes.c_int32),
                ("segment", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None


def lib():
    """Load liblbm.so (built by ``paper_2403_11167_amd.build``); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        D = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(Params)
        L.lbm_status_string.argtypes = [ctypes.c_int]
        L.lbm_status_string.restype = ctypes.c_char_p
        L.lbm_workspace_bytes.argtypes = [P, ctypes.POINTER(sz)]
        L.lbm_init.argtypes = [P, vp, sz, vp, vp, ctypes.POINTER(vp)]
        L.lbm_step.argtypes = [vp, ctypes.c_int64]
        L.lbm_observe.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Obs),
                                  vp, vp, vp]
        L.lbm_get_populations.argtypes = [vp, vp]
        L.lbm_set_populations.argtypes = [vp, vp]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_eos_eval.argtypes = [ctypes.c_int32] + [ctypes.c_double] * 5 + [D] * 2
        L.lbm_eos_critical.argtypes = [ctypes.c_int32] + [ctypes.c_double] * 3 + [D] * 3
        L.lbm_maxwell.argtypes = [ctypes.c_int32] + [ctypes.c_double] * 4 + [D] * 3
        L.lbm_sigma_li_theory.argtypes = [ctypes.c_int32] + [ctypes.c_double] * 4 + [D] * 2
        L.lbm_fe_planar_theory.argtypes = [ctypes.c_int32] + [ctypes.c_double] * 5 + [D] * 2
        L.lbm_match_p_to_fe.argtypes = [ctypes.c_int32] + [ctypes.c_double] * 6 + [D] * 3
        L.lbm_autotune.argtypes = [P, vp, sz, vp, vp, ctypes.c_int32, P, D]
        L.lbm_batch_workspace_bytes.argtypes = [ctypes.c_int32, P, ctypes.POINTER(sz)]
        L.lbm_batch_create.argtypes = [ctypes.c_int32, P, ctypes.POINTER(vp), vp, sz, vp,
                                       ctypes.POINTER(vp)]
        L.lbm_batch_run.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_int64)]
        L.lbm_batch_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.lbm_batch_launch_info.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(Launch)]
        L.lbm_batch_state.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int64), D,
                                      ctypes.POINTER(ctypes.c_uint32)]
        L.lbm_batch_observe.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(Obs), vp, vp, vp]
        L.lbm_batch_destroy.argtypes = [vp]
        L.lbm_batch_set_limit.argtypes = [vp, ctypes.c_int32, ctypes.c_int64]
        L.lbm_batch_set_partner.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
        NP = ctypes.POINTER(MlpNorm)
        i32, f32 = ctypes.c_int32, ctypes.c_float
        L.lbm_mlp_forward.argtypes = [vp, NP, vp, i32, vp, i32, vp]
        L.lbm_launch_info.argtypes = [vp, ctypes.POINTER(Launch)]
        L.lbm_mlp_workspace_bytes.argtypes = [i32, ctypes.POINTER(sz)]
        L.lbm_mlp_grad.argtypes = [vp, NP, vp, vp, i32, vp, i32, vp, vp, i32, vp, sz, vp]
        L.lbm_mlp_grad_noalloc.argtypes = [vp, NP, vp, vp, i32, vp, i32, vp, vp, i32, vp]
        L.lbm_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_int64, f32, f32, f32, f32, vp]
        L.lbm_mlp_train_step.argtypes = [vp, vp, vp, ctypes.c_int64, f32, NP, vp, vp, i32, vp,
                                         i32, vp, vp, i32, vp, sz, vp]
        for name in EXPORTED_SYMBOLS:
            if name != "lbm_status_string":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(st: int) -> str:
    return lib().lbm_status_string(int(st)).decode()


def _check(st: int, what: str):
    if st != OK:
        raise LbmError(st, what)


# ---- host thermodynamics ---------------------------------------------------
def _outs(n):
    return [ctypes.c_double() for _ in range(n)]


def eos_eval(eos: int, a: float, b: float, R: float, T: float, rho: float):
    """(p, dp/drho) of the EOS at rho."""
    o = _outs(2)
    _check(lib().lbm_eos_eval(eos, a, b, R, T, rho, *[ctypes.byref(v) for v in o]),
           "lbm_eos_eval")
    return tuple(v.value for v in o)


def eos_critical(eos: int, a: float, b: float, R: float):
    o = _outs(3)
    _check(lib().lbm_eos_critical(eos, a, b, R, *[ctypes.byref(v) for v in o]), "lbm_eos_critical")
    return tuple(v.value for v in o)


def maxwell(eos: int, a: float, b: float, R: float, T: float):
    o = _outs(3)
    _check(lib().lbm_maxwell(eos, a, b, R, T, *[ctypes.byref(v) for v in o]), "lbm_maxwell")
    return tuple(v.value for v in o)  # rho_l, rho_v, p0


def sigma_li_theory(eos: int, a: float, b: float, R: float, T: float):
    o = _outs(2)
    _check(lib().lbm_sigma_li_theory(eos, a, b, R, T, *[ctypes.byref(v) for v in o]),
           "lbm_sigma_li_theory")
    return tuple(v.value for v in o)  # eps, sigma_li


def fe_planar_theory(eos: int, a: float, b: float, R: float, T: float, kappa: float):
    o = _outs(2)
    _check(lib().lbm_fe_planar_theory(eos, a, b, R, T, kappa, *[ctypes.byref(v) for v in o]),
           "lbm_fe_planar_theory")
    return tuple(v.value for v in o)  # width, gamma


def match_p_to_fe(eos: int, a: float, b: float, R: float, T: float, kappa_fe: float,
                  target_width: float = 0.0):
    o = _outs(3)
    _check(lib().lbm_match_p_to_fe(eos, a, b, R, T, kappa_fe, target_width,
                                   *[ctypes.byref(v) for v in o]), "lbm_match_p_to_fe")
    return tuple(v.value for v in o)  # sigma_li, kappa_p, kappa_li


# ---- simulation --------------------------------------------------------------
@dataclass
class Config:
    """Python mirror of ``lbm_params``."""
    nx: int
    ny: int
    model: int
    eos: int
    a: float
    b: float
    R: float
    T: float
    tau: list = field(default_factory=lambda: [1.0] * 9)
    sigma_li: float = 0.0
    kappa_li: float = 0.0
    kappa_p: float = 1.0
    kappa: float = 0.0
    A: float = 0.0
    fx: float = 0.0
    fy: float = 0.0
    precision: int = FP64
    rho_ref: float = 0.0
    tile_x: int = 0
    tile_y: int = 0
    kernel_flags: int = 0
    tile_rounds: int = 0
    walls: bool = False  # Zou-He no-slip walls on the rows y = 0 and ny - 1
    # droplet-collision drive a(x) |rho - rho_ave| (Sec. 5.4)
    ax: float = 0.0
    x_split: int = 0
    rho_ave: float = 0.0
    ax_from_step: int = 0
    # free-energy gravity (Sec. 2.2): p_g = grav_rho0 g (y - grav_y0), walls only
    g: float = 0.0
    grav_rho0: float = 0.0
    grav_y0: float = 0.0

    def c_params(self) -> Params:
        p = Params()
        p.nx, p.ny, p.model, p.eos = self.nx, self.ny, self.model, self.eos
        p.precision, p.boundary = self.precision, BOUNDARY_WALLS if self.walls else 0
        p.a, p.b, p.R, p.T = self.a, self.b, self.R, self.T
        for i, t in enumerate(self.tau):
            p.tau[i] = float(t)
        p.sigma_li, p.kappa_li, p.kappa_p = self.sigma_li, self.kappa_li, self.kappa_p
        p.kappa, p.A, p.fx, p.fy, p.rho_ref = self.kappa, self.A, self.fx, self.fy, self.rho_ref
        p.tile_x, p.tile_y, p.kernel_flags = self.tile_x, self.tile_y, self.kernel_flags
        p.tile_rounds = int(self.tile_rounds)
        p.x_split, p.ax, p.rho_ave = int(self.x_split), float(self.ax), float(self.rho_ave)
        p.ax_from_step = int(self.ax_from_step)
        p.g, p.grav_rho0, p.grav_y0 = float(self.g), float(self.grav_rho0), float(self.grav_y0)
        return p

    def with_launch(self, tile_x: int, tile_y: int, kernel_flags: int) -> "Config":
        import dataclasses
        return dataclasses.replace(self, tile_x=tile_x, tile_y=tile_y, kernel_flags=kernel_flags)


def workspace_bytes(cfg: Config) -> int:
    n = ctypes.c_size_t()
    p = cfg.c_params()
    _check(lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)), "lbm_workspace_bytes")
    return n.value


class Simulation:
    """One lattice on one stream.  ``rho0`` is a torch float64 tensor of shape
    (ny, nx) on the GPU (or anything with ``data_ptr()``)."""

    def __init__(self, cfg: Config, rho0, stream=None, device=None):
        import torch
        self.cfg = cfg
        self._p = cfg.c_params()
        if device is None:
            device = rho0.device
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        nbytes = workspace_bytes(cfg)
        # torch's allocator returns 256-byte aligned blocks (at least 512 B)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        assert rho0.dtype == torch.float64 and rho0.is_contiguous()
        assert tuple(rho0.shape) == (cfg.ny, cfg.nx)
        self._rho0 = rho0
        ctx = ctypes.c_void_p()
        st = lib().lbm_init(ctypes.byref(self._p), ctypes.c_void_p(self.workspace.data_ptr()),
                            nbytes, ctypes.c_void_p(rho0.data_ptr()),
                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        _check(st, "lbm_init")
        self._ctx = ctx

    def step(self, n: int = 1):
        _check(lib().lbm_step(self._ctx, int(n)), "lbm_step")

    def observe(self, cx: int = 0, cy: int = 0, fields: bool = False):
        """Observables (dict); with fields=True also (rho, ux, uy) tensors."""
        import torch
        o = Obs()
        rho = ux = uy = None
        if fields:
            shp = (self.cfg.ny, self.cfg.nx)
            rho = torch.empty(shp, dtype=torch.float64, device=self.device)
            ux = torch.empty_like(rho)
            uy = torch.empty_like(rho)
        ptr = (lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None)
        _check(lib().lbm_observe(self._ctx, int(cx), int(cy), ctypes.byref(o),
                                 ptr(rho), ptr(ux), ptr(uy)), "lbm_observe")
        d = o.as_dict()
        if fields:
            return d, (rho, ux, uy)
        return d

    def launch_info(self) -> dict:
        """The launch shape carrying the run (see lbm_launch_info)."""
        out = Launch()
        _check(lib().lbm_launch_info(self._ctx, ctypes.byref(out)), "lbm_launch_info")
        return out.as_dict()

    def populations(self):
        import torch
        f = torch.empty((9, self.cfg.ny, self.cfg.nx), dtype=torch.float64, device=self.device)
        _check(lib().lbm_get_populations(self._ctx, ctypes.c_void_p(f.data_ptr())),
               "lbm_get_populations")
        return f

    def set_populations(self, f):
        assert f.dtype.is_floating_point and f.is_contiguous()
        _check(lib().lbm_set_populations(self._ctx, ctypes.c_void_p(f.data_ptr())),
               "lbm_set_populations")

    def close(self):
        if getattr(self, "_ctx", None) is not None:
            lib().lbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(cfg: Config, rho0, steps: int = 20, stream=None):
    """Fastest launch shape for cfg (see lbm_autotune): (Config, ms/step)."""
    import torch
    stream = stream if stream is not None else torch.cuda.current_stream(rho0.device)
    nbytes = workspace_bytes(cfg)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=rho0.device)
    p = cfg.c_params()
    best = Params()
    ms = ctypes.c_double()
    _check(lib().lbm_autotune(ctypes.byref(p), ctypes.c_void_p(ws.data_ptr()), nbytes,
                              ctypes.c_void_p(rho0.data_ptr()), ctypes.c_void_p(stream.cuda_stream),
                              int(steps), ctypes.byref(best), ctypes.byref(ms)), "lbm_autotune")
    return cfg.with_launch(best.tile_x, best.tile_y, best.kernel_flags), ms.value


class Batch:
    """Independent lattices advanced in lockstep until each converges or
    turns unstable (see lbm_batch_run).  rho0s: list of float64 (ny, nx)
    device tensors, one per Config."""

    def __init__(self, cfgs, rho0s, stream=None):
        import torch
        assert len(cfgs) == len(rho0s) and len(cfgs) > 0
        self.cfgs = list(cfgs)
        self.n = len(cfgs)
        dev = rho0s[0].device
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._p = (Params * self.n)(*[c.c_params() for c in cfgs])
        nbytes = ctypes.c_size_t()
        _check(lib().lbm_batch_workspace_bytes(self.n, self._p, ctypes.byref(nbytes)),
               "lbm_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
        for c, r in zip(cfgs, rho0s):
            assert r.dtype == torch.float64 and r.is_contiguous() and tuple(r.shape) == (c.ny, c.nx)
        self._rho0 = list(rho0s)
        ptrs = (ctypes.c_void_p * self.n)(*[r.data_ptr() for r in rho0s])
        h = ctypes.c_void_p()
        _check(lib().lbm_batch_create(self.n, self._p, ptrs,
                                      ctypes.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "lbm_batch_create")
        self._h = h

    def run(self, check_every: int = 100, du_tol: float = 1e-9, max_steps: int = 200000) -> int:
        done = ctypes.c_int64()
        _check(lib().lbm_batch_run(self._h, int(check_every), float(du_tol), int(max_steps),
                                   ctypes.byref(done)), "lbm_batch_run")
        return done.value

    def set_limit(self, i: int, max_steps: int):
        """Step limit of problem i (see lbm_batch_set_limit)."""
        _check(lib().lbm_batch_set_limit(self._h, int(i), int(max_steps)), "lbm_batch_set_limit")

    def set_partner(self, i: int, j: int):
        """Problems i and j form one unit (see lbm_batch_set_partner)."""
        _check(lib().lbm_batch_set_partner(self._h, int(i), int(j)), "lbm_batch_set_partner")

    def stats(self) -> dict:
        """Node updates issued, GPU milliseconds of the chunks and chunk count
        of all runs so far (see lbm_batch_stats)."""
        nu, ms, ch = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
        _check(lib().lbm_batch_stats(self._h, ctypes.byref(nu), ctypes.byref(ms),
                                     ctypes.byref(ch)), "lbm_batch_stats")
        return dict(node_updates=nu.value, gpu_ms=ms.value, chunks=ch.value)

    def launch_info(self, i: int) -> dict:
        """Problem i's launch shape in the batch (see lbm_batch_launch_info)."""
        out = Launch()
        _check(lib().lbm_batch_launch_info(self._h, int(i), ctypes.byref(out)),
               "lbm_batch_launch_info")
        return out.as_dict()

    def state(self):
        """(state, steps, du, flags) lists."""
        n = self.n
        st = (ctypes.c_int32 * n)()
        steps = (ctypes.c_int64 * n)()
        du = (ctypes.c_double * n)()
        fl = (ctypes.c_uint32 * n)()
        _check(lib().lbm_batch_state(self._h, st, steps, du, fl), "lbm_batch_state")
        return list(st), list(steps), list(du), list(fl)

    def observe(self, i: int, cx: int = 0, cy: int = 0, fields: bool = False):
        import torch
        o = Obs()
        rho = ux = uy = None
        if fields:
            c = self.cfgs[i]
            rho = torch.empty((c.ny, c.nx), dtype=torch.float64, device=self.device)
            ux = torch.empty_like(rho)
            uy = torch.empty_like(rho)
        ptr = (lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None)
        _check(lib().lbm_batch_observe(self._h, int(i), int(cx), int(cy), ctypes.byref(o),
                                       ptr(rho), ptr(ux), ptr(uy)), "lbm_batch_observe")
        d = o.as_dict()
        return (d, (rho, ux, uy)) if fields else d

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlups(nodes: int, steps: int, seconds: float) -> float:
    return nodes * steps / seconds / 1e6 if seconds > 0 else math.nan


# ---- calibration surrogate ------------------------------------------------------
def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_ptr(stream):
    return ctypes.c_void_p(stream.cuda_stream) if stream is not None else None


def mlp_forward(params, norm: MlpNorm, x, bf16: bool = True, stream=None):
    """Predictions (n, 4) float32 device tensor for features x (n, 4)."""
    import torch
    assert params.dtype == torch.float32 and params.numel() == MLP_NPARAMS
    assert x.dtype == torch.float32 and x.is_contiguous() and x.dim() == 2 and x.shape[1] == 4
    y = torch.empty_like(x)
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    _check(lib().lbm_mlp_forward(_ptr(params), ctypes.byref(norm), _ptr(x), int(x.shape[0]),
                                 _ptr(y), MLP_BF16 if bf16 else 0, _stream_ptr(st)),
           "lbm_mlp_forward")
    return y


def mlp_workspace(n: int, device):
    import torch
    nbytes = ctypes.c_size_t()
    _check(lib().lbm_mlp_workspace_bytes(int(n), ctypes.byref(nbytes)), "lbm_mlp_workspace_bytes")
    return torch.empty(nbytes.value, dtype=torch.uint8, device=device)


def mlp_grad(params, norm: MlpNorm, x, y, idx=None, n=None, bf16: bool = True, stream=None,
             workspace=None):
    """(loss tensor (1,), gradient tensor (MLP_NPARAMS,)) over the rows idx
    (int32 device tensor) of (x, y), or over the first n rows."""
    import torch
    dev = x.device
    nrows = int(x.shape[0])
    if n is None:
        n = int(idx.numel()) if idx is not None else nrows
    ws = workspace if workspace is not None else mlp_workspace(n, dev)
    grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(lib().lbm_mlp_grad(_ptr(params), ctypes.byref(norm), _ptr(x), _ptr(y), nrows,
                              _ptr(idx), int(n), _ptr(grad), _ptr(loss),
                              MLP_BF16 if bf16 else 0, _ptr(ws), ws.numel(), _stream_ptr(st)),
           "lbm_mlp_grad")
    return loss, grad


MLP_NOALLOC_MAX_N = 1024


def mlp_grad_noalloc(params, norm: MlpNorm, x, y, idx=None, n=None, bf16: bool = True,
                     stream=None, out=None):
    """mlp_grad through lbm_mlp_grad_noalloc (partials in the library's fixed
    device array, n <= MLP_NOALLOC_MAX_N).  `out` = (loss, grad) tensors to
    write into (allocated here when None)."""
    import torch
    dev = x.device
    nrows = int(x.shape[0])
    if n is None:
        n = int(idx.numel()) if idx is not None else nrows
    if out is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
        grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=dev)
    else:
        loss, grad = out
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(lib().lbm_mlp_grad_noalloc(_ptr(params), ctypes.byref(norm), _ptr(x), _ptr(y), nrows,
                                      _ptr(idx), int(n), _ptr(grad), _ptr(loss),
                                      MLP_BF16 if bf16 else 0, _stream_ptr(st)),
           "lbm_mlp_grad_noalloc")
    return loss, grad


def mlp_adam(params, m, v, grad, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
             stream=None):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(params.device)
    _check(lib().lbm_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(t), float(lr),
                              float(beta1), float(beta2), float(eps), _stream_ptr(st)),
           "lbm_mlp_adam")


class Surrogate:
    """The calibration surrogate's parameters, Adam state and normalisation,
    trained and evaluated by the library's kernels.  Inputs are tuples
    (model, Tr, w, kappa); outputs (rho_l, rho_v, sigma, W)."""

    # fixed input map: model in {0, 1}, Tr in [0.5, 0.95], w in [2, 8],
    # kappa in [0.5, 2] all sent to [-1, 1]
    X_LO = (0.0, 0.5, 2.0, 0.5)
    X_HI = (1.0, 0.95, 8.0, 2.0)

    def __init__(self, params0, device=None, bf16: bool = True):
        import numpy as np
        import torch
        dev = device if device is not None else torch.device("cuda:0")
        self.device = dev
        self.bf16 = bf16
        p0 = np.asarray(params0, dtype=np.float32)
        assert p0.size == MLP_NPARAMS
        self.params = torch.from_numpy(p0.copy()).to(dev)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        lo, hi = np.array(self.X_LO), np.array(self.X_HI)
        self.x_shift = 0.5 * (lo + hi)
        self.x_scale = 2.0 / (hi - lo)
        self.norm = MlpNorm.make(self.x_shift, self.x_scale, [0.0] * 4, [1.0] * 4)

    def set_target_scaling(self, y):
        """Output normalisation from training targets: mean and standard
        deviation of log y per output."""
        import numpy as np
        ly = np.log(np.asarray(y, dtype=np.float64))
        sd = ly.std(axis=0)
        sd[sd == 0] = 1.0
        self.norm = MlpNorm.make(self.x_shift, self.x_scale, ly.mean(axis=0), sd)

    def fit(self, x, y, epochs: int, batch: int = 256, lr: float = 2e-3, seed: int = 0,
            lr_final: float | None = None):
        """Adam on mini-batches drawn without replacement each epoch
        (numpy default_rng(seed) permutations); returns per-epoch mean
        loss (host list)."""
        import numpy as np
        import torch
        xs = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(self.device)
        ys = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(self.device)
        n = xs.shape[0]
        rng = np.random.default_rng(seed)
        ws = mlp_workspace(min(batch, n), self.device)
        grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=self.device)
        nb = (n + batch - 1) // batch
        # one loss slot per step, written by the kernels, read once at the end
        lbuf = torch.empty(epochs * nb, dtype=torch.float32, device=self.device)
        st = torch.cuda.current_stream(self.device)
        flags = MLP_BF16 if self.bf16 else 0
        L = lib()
        perms = torch.from_numpy(
            np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)).to(self.device)
        for e in range(epochs):
            if lr_final is not None and epochs > 1:
                lr_e = lr * (lr_final / lr) ** (e / (epochs - 1))
            else:
                lr_e = lr
            for b in range(nb):
                idx = perms[e, b * batch:(b + 1) * batch]
                self.t += 1
                _check(L.lbm_mlp_train_step(_ptr(self.params), _ptr(self.m), _ptr(self.v),
                                            self.t, float(lr_e), ctypes.byref(self.norm),
                                            _ptr(xs), _ptr(ys), int(n), _ptr(idx),
                                            int(idx.numel()), _ptr(grad), _ptr(lbuf[e * nb + b:]),
                                            flags, _ptr(ws), ws.numel(), _stream_ptr(st)),
                       "lbm_mlp_train_step")
        per_step = lbuf.cpu().numpy().reshape(epochs, nb)
        sizes = np.array([min(batch, n - b * batch) for b in range(nb)], dtype=np.float64)
        return list(per_step @ sizes / n)

    def predict(self, x):
        """Host (n, 4) float64 predictions."""
        import numpy as np
        import torch
        xs = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(self.device)
        return mlp_forward(self.params, self.norm, xs, self.bf16).cpu().numpy().astype(np.float64)

