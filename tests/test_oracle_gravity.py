"""Pins of the oracle's free-energy gravity (Sec. 2.2: p_g in Eq. 20, the
buoyancy F_g = -(rho - rho_0) g j in the total force, d p_g in Eq. 21).

p_g = rho_0 g (y - y_g) is not periodic, so gravity runs between the Zou-He
walls of Sec. 5.3.  With g > 0 gravity pulls toward -y: the momentum gains
-d_y p_g + F_g = -rho g, so a fluid at rest has d_y mu = -g.
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


def test_fe_forcing_moments_with_gravity():
    """Eq. 21 in full, through its lattice sums: zeroth moment 0, first
    moment F, second moment u_a B_b + u_b B_a + c_s^2 delta_ab u . grad(rho)
    with B = F - grad(p_g) + c_s^2 grad(rho) (the D2Q9 isotropy sums
    sum w c_a c_b c_g c_d = c_s^4 (3 delta terms) and
    sum w c_a c_b |c|^2 = 4 c_s^4 delta_ab).  A dropped or sign-flipped
    d_y p_g changes the second moment by 2 u_y d_y p_g in yy."""
    rng = np.random.default_rng(12)
    for _ in range(20):
        ux, uy, Fx, Fy, gx, gy = rng.uniform(-0.1, 0.1, 6)
        dpgy = rng.uniform(-0.05, 0.05)
        Fi = oracle.forcing_fe_full(ux, uy, Fx, Fy, gx, gy, dpgy)
        u = np.array([ux, uy])
        B = np.array([Fx, Fy - dpgy]) + np.array([gx, gy]) / 3
        assert abs(Fi.sum()) < 1e-16
        assert np.allclose([(Fi * CX).sum(), (Fi * CY).sum()], [Fx, Fy], atol=1e-16, rtol=0)
        P = np.array([[(Fi * CX * CX).sum(), (Fi * CX * CY).sum()],
                      [(Fi * CY * CX).sum(), (Fi * CY * CY).sum()]])
        want = np.outer(u, B) + np.outer(B, u) + np.eye(2) * (u @ np.array([gx, gy])) / 3
        assert np.allclose(P, want, atol=2e-16, rtol=0)


def _column(Tr=0.9, ny=64, g=2e-6, y_g=0.0, steps=20000):
    """A two-phase free-energy column between the walls, liquid below and
    vapour above (C-S a = 0.25, kappa = 0.5, all tau = 1, rho_0 = rho_l)."""
    a = 0.25
    T, rl, rv = _cs(a, Tr)
    W = th.fe_planar(th.CS, a, 4.0, 1.0, T, 0.5)["width"]
    rho0 = np.ascontiguousarray(inputs.layered(3, ny, rl, rv, width=W)[::-1])
    p = oracle.OracleParams(3, ny, oracle.MODEL_FE, oracle.EOS_CS, a, 4.0, 1.0, T, kappa=0.5,
                            walls=1, g=g, rho0_g=rl, y_g=y_g)
    s = oracle.Simulation(p, rho0)
    s.step(steps)
    return s, (a, T, rl, rv)


def test_gravity_reference_row_is_neutral():
    """Only the gradient of p_g carries physics: moving the row where p_g = 0
    adds the same rest-state vector w_i dp / c_s^2 (i > 0),
    -(1 - w_0) dp / c_s^2 (i = 0) to the equilibrium at every node, which
    streaming, the collision (linear in it, no mass, no momentum) and the
    wall closure carry along unchanged.  Two runs with y_g = 0 and 17.3 give
    the same density and velocity fields to rounding."""
    s0, _ = _column(steps=3000)
    s1, _ = _column(y_g=17.3, steps=3000)
    r0, ux0, uy0 = s0.fields()
    r1, ux1, uy1 = s1.fields()
    assert np.abs(r1 - r0).max() < 1e-13 * r0.max()
    assert np.abs(uy1 - uy0).max() < 1e-14  # rounding of sum f c (populations ~ rho)
    assert s0.flags == s1.flags == 0


def test_gravity_column_is_hydrostatic():
    """At rest the free-energy step with every tau = 1 stores
    f*_i = f^eq_i(rho, 0; p_g) + w_i c_i . F / (2 c_s^2) (Eq. 1, 20, 21 at
    u = 0).  Streaming the p_g part of Eq. 20 gives the momentum
    (p_g(y-1) - p_g(y+1))/2 = -rho_0 g exactly (p_g is linear), so u = 0 after
    streaming (Eq. 6b) needs F(y-1) + 2 F(y) + F(y+1) = 4 rho_0 g for the
    total force F_y = -rho d_y mu - (rho - rho_0) g of an x-uniform column:
    smoothly, d_y mu = -g, the well-balanced hydrostatic state across the
    interface.  Checked on the settled two-phase column (Tr = 0.9, g = 2e-6)
    with mu recomputed here from the density field (Eq. 24 in 1-D); the
    column still carries a residual flow |u| ~ 3e-9 (the free-energy walls'
    flux under a normal force), which bounds the residual.  A flipped
    buoyancy or a p_g missing from the equilibrium leaves a residual of
    order rho g.  The liquid is compressed at the bottom.  The walls (whose
    rows carry F_y = F_g) leave the odd-even null mode F = (-1)^y (A + B y) of
    that condition in the column, visible as a 1e-4 checkerboard in rho."""
    g = 2e-6
    s, (a, T, rl, rv) = _column(g=g)
    rho, _, uy = s.fields()
    r, umax = rho[:, 0], np.abs(uy).max()
    assert umax < 1e-8 and s.flags == 0
    ext = np.concatenate([[r[1]], r, [r[-2]]])  # mirrored rows past the walls
    mu = th.mu_b(th.CS, ext[1:-1], a, 4.0, 1.0, T) - 0.5 * (ext[2:] - 2 * ext[1:-1] + ext[:-2])
    F = -r[1:-1] * 0.5 * (mu[2:] - mu[:-2]) - (r[1:-1] - rl) * g   # rows 1 .. ny-2
    resid = F[:-2] + 2 * F[1:-1] + F[2:] - 4 * rl * g                # rows 2 .. ny-3
    assert np.abs(resid).max() < 8 * rl * umax + 1e-9 * rl * g, np.abs(resid).max() / (rl * g)
    # four-row means (an even count cancels the odd-even mode of the column)
    m4 = [r[k:k + 4].mean() for k in (2, 8, 14)]
    assert m4[0] > m4[1] > m4[2]


def test_gravity_channel_flow_matches_eq89():
    """Flow along the walls (F_x = 1e-7) of a liquid compressed by gravity
    (g = 2e-5, 1.2 % density change across the channel): the steady
    velocity follows App. F Eq. 89 for the lattice's own density profile,
    mu(y) = rho(y) c_s^2 (tau_nu - 1/2), to 1e-3 of its peak (measured
    3.0e-4; without gravity the profile is exact to 4e-9)."""
    a = 0.25
    T, rl, _ = _cs(a, 0.8)
    ny, fx, g = 33, 1e-7, 2e-5
    tau = [1.0] * 9
    tau[7] = tau[8] = 0.8
    p = oracle.OracleParams(3, ny, oracle.MODEL_FE, oracle.EOS_CS, a, 4.0, 1.0, T, tau=tau,
                            kappa=0.5, walls=1, fx=fx, g=g, rho0_g=rl, y_g=(ny - 1) / 2)
    s = oracle.Simulation(p, inputs.uniform(3, ny, rl))
    s.step(30000)
    rho, ux, _ = s.fields()
    assert 0.01 < np.ptp(rho) / rl < 0.015 and s.flags == 0
    ud = th.plates_diffuse(fx, np.arange(ny), rho[:, 0] * 0.3 / 3)
    assert np.abs(ux[:, 0] - ud).max() < 1e-3 * ud.max()
