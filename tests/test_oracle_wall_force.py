"""Pins of the oracle's Zou-He walls under a force normal to them (Sec. 5.3).

A wall row is a fluid row held at u = 0 (Eq. 6b) by rebuilding the three
populations that enter it from outside.  With a normal body force f_y the
rebuilt node must carry sum_i f_i c_iy = -f_y / 2, and its density is the sum
of the rebuilt populations (Eq. 6a).  These tests check the oracle against
an independent solve of that closure, and against what the scheme must reach
at rest: zero velocity, a constant mass, and (free energy, all tau = 1) the
stationarity condition of the step at u = 0.
"""
import numpy as np
import pytest

import oracle
from oracle import theory as th
from paper_2403_11167_amd import inputs

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def _cs(a, Tr):
    T = Tr * th.critical(th.CS, a, 4.0, 1.0)[0]
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    return T, rl, rv


def _model_kw(model, a, T):
    tau = [1.0] * 9
    if model == oracle.MODEL_FE:
        return tau, dict(kappa=0.5)
    m = th.match_p_to_fe(th.CS, a, 4.0, 1.0, T, 0.5)
    tau[4] = tau[6] = 1 / 1.99
    return tau, dict(sigma_li=m["sigma_li"], kappa_p=m["kappa_p"], kappa_li=m["kappa_li"])


def _closed(fn, side, jx, jy):
    """Zou and He's closure solved as a 3x3 linear system: the normal unknown
    equals its opposite, and the three unknowns (c_y = side) make the node's
    momentum (jx, jy)."""
    unk = [i for i in range(1, 9) if CY[i] == side]
    nrm = [i for i in unk if CX[i] == 0][0]
    opp = [i for i in range(1, 9) if CY[i] == -side and CX[i] == 0][0]
    known = [i for i in range(9) if i not in unk]
    A = np.zeros((3, 3))
    rhs = np.zeros(3)
    A[0, unk.index(nrm)] = 1.0
    rhs[0] = fn[opp]
    for r, c in ((1, CX), (2, CY)):
        A[r] = [c[i] for i in unk]
        rhs[r] = (jx if r == 1 else jy) - sum(fn[i] * c[i] for i in known)
    out = fn.copy()
    out[unk] = np.linalg.solve(A, rhs)
    return out


@pytest.mark.parametrize("model", [oracle.MODEL_FE, oracle.MODEL_P])
def test_wall_density_is_the_sum_of_the_closed_populations(model):
    """Eq. 6a at every wall node of a layered channel under f_x and a normal
    f_y, during a transient: the density the step uses equals the sum of the
    populations closed so that the node carries -F/2 (u = 0), solved here
    independently.  The layered state is x-uniform, so the interaction force
    has no x part and F = (f_x, f_y) on a wall row (the mirrored rows cancel
    its y part).  Both walls: a closure that moved the density by +j_y on the
    top wall, where the unknown diagonals have c_y = -1, is off by f_y."""
    a = 0.25
    T, rl, rv = _cs(a, 0.8)
    tau, kw = _model_kw(model, a, T)
    nx, ny, fx, fy = 4, 16, 1e-6, -2e-5
    p = oracle.OracleParams(nx, ny, model, oracle.EOS_CS, a, 4.0, 1.0, T, tau=tau, fx=fx,
                            fy=fy, walls=1, **kw)
    s = oracle.Simulation(p, inputs.layered(nx, ny, rl, rv, width=4.0, y_i=7.3))
    s.step(40)
    rho, ux, uy = s.fields()
    for y, side in ((0, 1), (ny - 1, -1)):
        for x in range(nx):
            fc = _closed(s.f[:, y, x].copy(), side, -0.5 * fx, -0.5 * fy)
            assert abs(rho[y, x] - fc.sum()) < 1e-14 * rho[y, x], (y, x, rho[y, x] - fc.sum())
            assert abs(ux[y, x]) < 1e-15 and abs(uy[y, x]) < 1e-15
    assert s.flags == 0


@pytest.mark.parametrize("model", [oracle.MODEL_FE, oracle.MODEL_P])
def test_liquid_column_under_normal_force_comes_to_rest(model):
    """A liquid column between the walls under a constant normal force
    f_y = -1e-5 rho_l (Sec. 5.3 walls) settles: after the start-up transient
    the velocity decays and the mass stops changing.  The pseudopotential
    column comes to rest exactly (|u| < 1e-12, mass constant to 1e-13).  The
    free-energy column keeps a residual flow of ~1e-9 through the wall rows
    and loses ~6e-12 of its mass per step, a rate that scales as f_y^2 (the
    Zou-He closure meets the force-form pressure of Eq. 20-21 only to second
    order in f_y); the bars leave a factor of ten.  With the top wall's
    density moved by +j_y instead of -j_y both columns keep a velocity of
    ~5e-6 and gain ~5e-4 of their mass in these 4000 steps."""
    a = 0.25
    T, rl, _ = _cs(a, 0.8)
    tau, kw = _model_kw(model, a, T)
    nx, ny = 3, 32
    p = oracle.OracleParams(nx, ny, model, oracle.EOS_CS, a, 4.0, 1.0, T, tau=tau,
                            fy=-1e-5 * rl, walls=1, **kw)
    s = oracle.Simulation(p, inputs.uniform(nx, ny, rl))
    m0 = s.observe(0, 0)["mass"]
    s.step(12000)
    m1 = s.observe(0, 0)["mass"]
    s.step(4000)
    o = s.observe(0, 0)
    if model == oracle.MODEL_P:
        assert o["max_u"] < 1e-12, o["max_u"]
        assert abs(o["mass"] - m1) < 1e-13 * m1
    else:
        assert o["max_u"] < 1e-8, o["max_u"]
        assert abs(o["mass"] - m1) < 4000 * 6e-11 * m1, (o["mass"] - m1) / m1
    assert abs(m1 - m0) < 2e-6 * m0
    assert s.flags == 0


def test_free_energy_column_at_rest_is_stationary():
    """With every tau = 1 the free-energy step at u = 0 stores
    f*_i = f^eq_i(rho, 0) + w_i c_i . F / (2 c_s^2) (Eq. 1, 20 and 21 at
    u = 0), so a state at rest after streaming needs
    (1/2) sum_i w_i c_i c_i . F(x - c_i) / c_s^2 + F(x) = 0 (Eq. 6b), which on
    an x-uniform column reads F(y-1) + 2 F(y) + F(y+1) = 0 for the total force
    F_y = -rho d_y mu + f_y.  The settled column must satisfy it at every
    interior row, with mu and its gradient recomputed here from the density
    field with the Eq. 24 stencils (their 1-D forms).  The condition allows
    F = (-1)^y (A + B y), the odd-even null mode: the wall rows carry
    F_y = f_y, so the settled column is hydrostatic only on average."""
    a = 0.25
    T, rl, _ = _cs(a, 0.8)
    nx, ny, fy, kappa = 3, 32, -1e-5 * rl, 0.5
    p = oracle.OracleParams(nx, ny, oracle.MODEL_FE, oracle.EOS_CS, a, 4.0, 1.0, T,
                            kappa=kappa, fy=fy, walls=1)
    s = oracle.Simulation(p, inputs.uniform(nx, ny, rl))
    s.step(12000)
    rho, _, uy = s.fields()
    rho, umax = rho[:, 0], np.abs(uy).max()
    assert umax < 1e-8
    ext = np.concatenate([[rho[1]], rho, [rho[-2]]])  # mirrored rows past the walls
    mu = th.mu_b(th.CS, ext[1:-1], a, 4.0, 1.0, T) - kappa * (ext[2:] - 2 * ext[1:-1] + ext[:-2])
    F = -rho[1:-1] * 0.5 * (mu[2:] - mu[:-2]) + fy  # rows 1 .. ny-2
    resid = F[:-2] + 2 * F[1:-1] + F[2:]            # rows 2 .. ny-3
    # at rest the residual vanishes; the column still carries |u| ~ 1e-9
    # (above), which leaves a residual of at most a few rho |u|
    assert np.abs(resid).max() < 8 * rl * umax + 1e-12 * abs(fy), np.abs(resid).max() / abs(fy)
    assert s.flags == 0
