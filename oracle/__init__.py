"""FP64 CPU oracle for the D2Q9 multiphase lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  The oracle exists to check the GPU library against
a slow, plainly written implementation of Czelusniak et al. (arXiv 2403.11167).
Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  The product package never imports it, and it
imports nothing from the product package.

Contents
  * ``liboracle.so`` (built from ``lbm_oracle.c`` by :func:`build`) -- the
    time step, in velocity space with explicit M / M^-1 products;
  * :mod:`oracle.theory` -- thermodynamics and planar-interface theory in
    numpy/scipy (Maxwell rule, App. B epsilon, Eq. 26 / 44 / 46 profiles,
    App. D / E discrete planar relations).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

MODEL_P, MODEL_FE = 0, 1
EOS_VDW, EOS_CS = 0, 1
FLAG_NONFINITE, FLAG_PSI_CLAMP, FLAG_EOS_DOMAIN = 1, 2, 4


def build() -> str:
    """Compile the oracle with gcc: FP64, no contraction, OpenMP over rows."""
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-shared", "-fPIC", "-Wall", "-o", _LIB_PATH, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("model", ctypes.c_int32), ("eos", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("R", ctypes.c_double), ("T", ctypes.c_double),
                ("tau", ctypes.c_double * 9),
                ("sigma_li", ctypes.c_double), ("kappa_li", ctypes.c_double),
                ("kappa_p", ctypes.c_double), ("kappa", ctypes.c_double),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("walls", ctypes.c_int32), ("x_split", ctypes.c_int32),
                ("ax", ctypes.c_double), ("rho_ave", ctypes.c_double),
                ("A", ctypes.c_double), ("g", ctypes.c_double),
                ("rho0_g", ctypes.c_double), ("y_g", ctypes.c_double)]


@dataclass
class OracleParams:
    """Problem statement of Sec. 2 / Sec. 5: periodic grid, model, EOS,
    MRT relaxation times (Eq. 3), model coefficients, body force; walls = 1
    puts Zou-He no-slip walls on the rows y = 0 and y = ny - 1 (Sec. 5.3).
    ax != 0 adds the droplet-collision drive of Sec. 5.4, an x force
    a(x) |rho - rho_ave| with a = +ax for x <= x_split and -ax beyond, in the
    steps that start at t >= ax_from_step; rho_ave <= 0 takes the mean of
    the initial density.  Free energy only: A is the viscosity-tuning
    parameter of Eq. 20, and g, rho0_g, y_g its gravity (walls only):
    p_g = rho0_g g (y - y_g) in Eq. 20, buoyancy -(rho - rho0_g) g in y,
    d_y p_g in Eq. 21; g > 0 pulls toward -y."""
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
    fx: float = 0.0
    fy: float = 0.0
    walls: int = 0
    ax: float = 0.0
    x_split: int = 0
    rho_ave: float = 0.0
    ax_from_step: int = 0
    A: float = 0.0
    g: float = 0.0
    rho0_g: float = 0.0
    y_g: float = 0.0

    def _c(self) -> _Params:
        p = _Params()
        p.nx, p.ny, p.model, p.eos = self.nx, self.ny, self.model, self.eos
        p.a, p.b, p.R, p.T = self.a, self.b, self.R, self.T
        for i, t in enumerate(self.tau):
            p.tau[i] = t
        p.sigma_li, p.kappa_li, p.kappa_p = self.sigma_li, self.kappa_li, self.kappa_p
        p.kappa, p.fx, p.fy = self.kappa, self.fx, self.fy
        p.walls = int(self.walls)
        p.x_split, p.ax, p.rho_ave = int(self.x_split), float(self.ax), float(self.rho_ave)
        p.A = float(self.A)
        p.g, p.rho0_g, p.y_g = float(self.g), float(self.rho0_g), float(self.y_g)
        return p


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_Params)
        L.orc_pressure.argtypes = [P, ctypes.c_double]
        L.orc_pressure.restype = ctypes.c_double
        L.orc_mu_b.argtypes = [P, ctypes.c_double]
        L.orc_mu_b.restype = ctypes.c_double
        L.orc_psi.argtypes = [P, ctypes.c_double]
        L.orc_psi.restype = ctypes.c_double
        L.orc_matrices.argtypes = [_D, _D, _D]
        L.orc_feq.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, _D]
        L.orc_forcing_fe.argtypes = [ctypes.c_double] * 6 + [_D]
        L.orc_feq_fe_full.argtypes = [ctypes.c_double] * 5 + [_D, _D]
        L.orc_forcing_fe_full.argtypes = [ctypes.c_double] * 7 + [_D]
        L.orc_sc_sum.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D]
        L.orc_q_tensor.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_double,
                                   ctypes.c_double, _D, _D, _D]
        L.orc_gradient.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D]
        L.orc_laplacian.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D]
        L.orc_init.argtypes = [P, _D, _D, _D, _D]
        L.orc_step.argtypes = [P, _D, ctypes.c_int64]
        L.orc_step.restype = ctypes.c_uint32
        L.orc_fields.argtypes = [P, _D, _D, _D, _D]
        L.orc_fields.restype = ctypes.c_uint32
        L.orc_num_threads.restype = ctypes.c_int32
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def matrices():
    """(M of Eq. 48, M^-1 as printed in Eq. 49, 36 M^-1 as applied)."""
    m = np.zeros((9, 9))
    mi = np.zeros((9, 9))
    mi36 = np.zeros((9, 9))
    lib().orc_matrices(_ptr(m), _ptr(mi), _ptr(mi36))
    return m, mi, mi36


def feq(model: int, rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_feq(model, rho, ux, uy, _ptr(out))
    return out


def forcing_fe(ux, uy, Fx, Fy, gx, gy) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_forcing_fe(ux, uy, Fx, Fy, gx, gy, _ptr(out))
    return out


def feq_fe_full(rho, ux, uy, pg, A, du) -> np.ndarray:
    """Eq. 20 in full; du = (d_x u_x, d_y u_x, d_x u_y, d_y u_y)."""
    out = np.zeros(9)
    lib().orc_feq_fe_full(rho, ux, uy, pg, A, _ptr(np.ascontiguousarray(du, dtype=np.float64)),
                          _ptr(out))
    return out


def forcing_fe_full(ux, uy, Fx, Fy, gx, gy, dpgy) -> np.ndarray:
    """Eq. 21 in full, with d_y p_g = dpgy."""
    out = np.zeros(9)
    lib().orc_forcing_fe_full(ux, uy, Fx, Fy, gx, gy, dpgy, _ptr(out))
    return out


def pressure(p: OracleParams, rho: float) -> float:
    c = p._c()
    return lib().orc_pressure(ctypes.byref(c), rho)


def mu_b(p: OracleParams, rho: float) -> float:
    c = p._c()
    return lib().orc_mu_b(ctypes.byref(c), rho)


def psi(p: OracleParams, rho: float) -> float:
    c = p._c()
    return lib().orc_psi(ctypes.byref(c), rho)


def sc_sum(phi: np.ndarray):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    sx, sy = np.zeros_like(phi), np.zeros_like(phi)
    lib().orc_sc_sum(nx, ny, _ptr(phi), _ptr(sx), _ptr(sy))
    return sx, sy


def q_tensor(psi_field: np.ndarray, kappa_p: float, kappa_li: float):
    psi_field = np.ascontiguousarray(psi_field, dtype=np.float64)
    ny, nx = psi_field.shape
    qxx, qyy, qxy = (np.zeros_like(psi_field) for _ in range(3))
    lib().orc_q_tensor(nx, ny, _ptr(psi_field), kappa_p, kappa_li,
                       _ptr(qxx), _ptr(qyy), _ptr(qxy))
    return qxx, qyy, qxy


def gradient(phi: np.ndarray):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    gx, gy = np.zeros_like(phi), np.zeros_like(phi)
    lib().orc_gradient(nx, ny, _ptr(phi), _ptr(gx), _ptr(gy))
    return gx, gy


def laplacian(phi: np.ndarray):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    out = np.zeros_like(phi)
    lib().orc_laplacian(nx, ny, _ptr(phi), _ptr(out))
    return out


class Simulation:
    """Populations f[9, ny, nx] (post-streaming) advanced by the oracle."""

    def __init__(self, params: OracleParams, rho0: np.ndarray,
                 ux0: np.ndarray | None = None, uy0: np.ndarray | None = None):
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        assert rho0.shape == (params.ny, params.nx)
        if params.ax != 0.0 and params.rho_ave <= 0.0:
            import dataclasses
            params = dataclasses.replace(params, rho_ave=math.fsum(rho0.ravel().tolist()) / rho0.size)
        self.p = params
        self._cp = params._c()  # the drive on
        self._cp_off = params._c()
        self._cp_off.ax = 0.0
        self.f = np.zeros((9, params.ny, params.nx))
        ux0 = None if ux0 is None else np.ascontiguousarray(ux0, dtype=np.float64)
        uy0 = None if uy0 is None else np.ascontiguousarray(uy0, dtype=np.float64)
        lib().orc_init(ctypes.byref(self._cp), _ptr(rho0), _ptr(ux0), _ptr(uy0),
                       _ptr(self.f))
        self.flags = 0
        self.t = 0

    def _cparams(self):
        return self._cp if self.t >= self.p.ax_from_step else self._cp_off

    def step(self, n: int) -> int:
        n = int(n)
        while n > 0:
            k = n
            if self.t < self.p.ax_from_step:
                k = min(n, self.p.ax_from_step - self.t)
            fl = lib().orc_step(ctypes.byref(self._cparams()), _ptr(self.f), k)
            self.flags |= int(fl)
            self.t += k
            n -= k
        return self.flags

    def fields(self):
        """(rho, ux, uy) of Eq. 6a-b for the current populations."""
        shp = (self.p.ny, self.p.nx)
        rho, ux, uy = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        fl = lib().orc_fields(ctypes.byref(self._cparams()), _ptr(self.f), _ptr(rho),
                              _ptr(ux), _ptr(uy))
        self.flags |= int(fl)
        return rho, ux, uy

    def observe(self, cx: int, cy: int) -> dict:
        """Observables of a run: mass (compensated sum), max |u|, rho extrema,
        centre / far-corner densities, the pressure jump between them and the
        equimolar radius (Sec. 5.2)."""
        rho, ux, uy = self.fields()
        ny, nx = rho.shape
        rin = rho[cy % ny, cx % nx]
        rout = rho[(cy + ny // 2) % ny, (cx + nx // 2) % nx]
        mass = math.fsum(rho.ravel().tolist())
        dp = pressure(self.p, rin) - pressure(self.p, rout)
        excess = mass - rho.size * rout
        denom = math.pi * (rin - rout)
        r_eq = math.sqrt(excess / denom) if denom != 0 and excess / denom > 0 else float("nan")
        return dict(mass=mass, max_u=float(np.sqrt(ux ** 2 + uy ** 2).max()),
                    rho_min=float(rho.min()), rho_max=float(rho.max()),
                    rho_in=float(rin), rho_out=float(rout), dp=dp,
                    r_equimolar=r_eq, flags=self.flags)
