"""FP64 thermodynamics and planar-interface theory for the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Plain numpy/scipy
implementations of the host-side theory of Czelusniak et al. (arXiv
2403.11167), written independently of the product library's C++ versions so
that the two can be compared:

  * equations of state: Carnahan-Starling (Eq. 28) with mu_b of Eq. 29, and
    van der Waals with mu_b as the antiderivative of (1/rho) dp/drho;
  * critical points (p' = p'' = 0);
  * Maxwell equal-area coexistence (the rule of Eq. 27 / App. B);
  * epsilon and sigma^Li from the mechanical-stability condition (Eq. 18) by
    Newton iteration on Simpson integrals (App. B, Eq. 13-14);
  * free-energy planar profile and surface tension (Eq. 26, App. B Eq. 15);
  * pseudopotential planar profile and surface tension (App. C Eq. 44, 46);
  * kappa^P / kappa^Li matching to a free-energy interface (Sec. 3-4);
  * the discrete planar relations of App. D (Eq. 60) and App. E (Eq. 76),
    solved as nonlinear systems on a periodic 1-D lattice.

Readings adopted where the paper is ambiguous:
  * App. B Eq. 14 is printed without the minus sign that d(psi^-eps)/d(eps)
    produces; the derivative used here is -int (p - p0) psi' ln(psi)/psi^(1+eps).
  * Interface width is the max-slope width (rho_l - rho_v) / max |d rho/dx|.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

G = -1.0
CS2 = 1.0 / 3.0
VDW, CS = 0, 1


# --------------------------------------------------------------------------
# equations of state
def pressure(eos, rho, a, b, R, T):
    rho = np.asarray(rho, dtype=np.float64)
    if eos == CS:
        e = b * rho / 4.0
        return rho * R * T * (1 + e + e ** 2 - e ** 3) / (1 - e) ** 3 - a * rho ** 2
    return rho * R * T / (1 - b * rho) - a * rho ** 2


def dpressure(eos, rho, a, b, R, T):
    """d p_EOS / d rho in closed form."""
    rho = np.asarray(rho, dtype=np.float64)
    if eos == CS:
        e = b * rho / 4.0
        # d/d rho [rho RT g(e)] = RT (g + e g'), g = (1+e+e^2-e^3)/(1-e)^3
        g = (1 + e + e ** 2 - e ** 3) / (1 - e) ** 3
        gp = ((1 + 2 * e - 3 * e ** 2) * (1 - e) + 3 * (1 + e + e ** 2 - e ** 3)) / (1 - e) ** 4
        return R * T * (g + e * gp) - 2 * a * rho
    return R * T / (1 - b * rho) ** 2 - 2 * a * rho


def mu_b(eos, rho, a, b, R, T):
    rho = np.asarray(rho, dtype=np.float64)
    RT = R * T
    if eos == CS:
        e = b * rho / 4.0
        return RT * (3 - e) / (1 - e) ** 3 + RT * np.log(rho) + RT - 2 * a * rho
    return RT * np.log(rho / (1 - b * rho)) + RT * b * rho / (1 - b * rho) - 2 * a * rho


def psi(eos, rho, a, b, R, T):
    """Eq. 11 with G = -1: sqrt(2 (rho c_s^2 - p_EOS)); nan where imaginary."""
    arg = 2.0 * (pressure(eos, rho, a, b, R, T) - np.asarray(rho) * CS2) / G
    with np.errstate(invalid="ignore"):
        return np.where(arg >= 0, np.sqrt(np.maximum(arg, 0.0)), np.nan)


def dpsi(eos, rho, a, b, R, T):
    """d psi / d rho = (c_s^2 - p') / psi for G = -1."""
    return (CS2 - dpressure(eos, rho, a, b, R, T)) / psi(eos, rho, a, b, R, T)


# --------------------------------------------------------------------------
# critical point
def critical(eos, a, b, R):
    """(T_c, rho_c, p_c).  Van der Waals in closed form; Carnahan-Starling
    by solving p' = p'' = 0 numerically."""
    if eos == VDW:
        return 8 * a / (27 * b * R), 1 / (3 * b), a / (27 * b * b)
    # p'(rho) = 0 and p''(rho) = 0 in terms of eta = b rho / 4:
    # RT h(eta) = 2 a rho with h = g + eta g'; RT h'(eta) (b/4) = 2 a.
    def h(e):
        g = (1 + e + e ** 2 - e ** 3) / (1 - e) ** 3
        gp = ((1 + 2 * e - 3 * e ** 2) * (1 - e) + 3 * (1 + e + e ** 2 - e ** 3)) / (1 - e) ** 4
        return g + e * gp

    # eliminate RT: h(e) / (hp(e) b/4) = rho = 4 e / b  ->  h(e) = e hp(e)
    def resid(e):
        return h(e) - e * _hp_exact(e)

    e_c = optimize.brentq(resid, 0.05, 0.5, xtol=1e-15)
    rho_c = 4 * e_c / b
    T_c = 2 * a * rho_c / (R * h(e_c))
    p_c = float(pressure(CS, rho_c, a, b, R, T_c))
    return T_c, rho_c, p_c


def _hp_exact(e):
    """Derivative of h(e) = g + e g' for the CS g, by symbolic-free complex
    step (analytic function, exact to rounding)."""
    d = 1e-30
    z = complex(e, d)
    g = (1 + z + z ** 2 - z ** 3) / (1 - z) ** 3
    gp = ((1 + 2 * z - 3 * z ** 2) * (1 - z) + 3 * (1 + z + z ** 2 - z ** 3)) / (1 - z) ** 4
    # h'(e) needs g'' too: differentiate h = g + e g' via complex step of h
    hz = g + z * gp
    return hz.imag / d


# --------------------------------------------------------------------------
# Maxwell rule
def spinodals(eos, a, b, R, T):
    """Densities where p' = 0 (vapour-side max and liquid-side min)."""
    if eos == VDW:
        hi = 1.0 / b * (1 - 1e-12)
    else:
        hi = 4.0 / b * (1 - 1e-12)
    grid = np.linspace(hi * 1e-6, hi * 0.999, 200001)
    dp = dpressure(eos, grid, a, b, R, T)
    idx = np.nonzero(np.diff(np.sign(dp)))[0]
    if len(idx) < 2:
        raise ValueError("no two-phase region at this temperature")
    f = lambda r: float(dpressure(eos, r, a, b, R, T))
    r1 = optimize.brentq(f, grid[idx[0]], grid[idx[0] + 1], xtol=1e-15)
    r2 = optimize.brentq(f, grid[idx[1]], grid[idx[1] + 1], xtol=1e-15)
    return r1, r2


def maxwell(eos, a, b, R, T, tol=1e-14):
    """(rho_l, rho_v, p0) with p(rho_v) = p(rho_l) = p0 and
    mu_b(rho_v) = mu_b(rho_l) (equivalent to the integral of (p - p0)/rho^2
    vanishing, App. B)."""
    s1, s2 = spinodals(eos, a, b, R, T)
    # Parametrise by p0 between the spinodal pressures; for each p0 the two
    # outer roots are unique.  Solve mu equality by bracketing in p0.
    pmin = max(float(pressure(eos, s2, a, b, R, T)), 1e-300)
    pmax = float(pressure(eos, s1, a, b, R, T))
    hi = (1.0 / b if eos == VDW else 4.0 / b) * (1 - 1e-15)

    def roots(p0):
        fv = lambda r: float(pressure(eos, r, a, b, R, T)) - p0
        rv = optimize.brentq(fv, 1e-300 if fv(1e-300) < 0 else 0.0, s1, xtol=1e-300, rtol=1e-15)
        rl = optimize.brentq(fv, s2, hi, xtol=1e-300, rtol=1e-15)
        return rl, rv

    def g(p0):
        rl, rv = roots(p0)
        return float(mu_b(eos, rl, a, b, R, T) - mu_b(eos, rv, a, b, R, T))

    lo_p = pmin + 1e-12 * (pmax - pmin)
    hi_p = pmax - 1e-12 * (pmax - pmin)
    p0 = optimize.brentq(g, lo_p, hi_p, xtol=1e-300, rtol=1e-15, maxiter=500)
    rl, rv = roots(p0)
    # polish with 2-D Newton on (p(rl) - p(rv), mu(rl) - mu(rv))
    for _ in range(5):
        F = np.array([float(pressure(eos, rl, a, b, R, T) - pressure(eos, rv, a, b, R, T)),
                      float(mu_b(eos, rl, a, b, R, T) - mu_b(eos, rv, a, b, R, T))])
        dl, dv = float(dpressure(eos, rl, a, b, R, T)), float(dpressure(eos, rv, a, b, R, T))
        J = np.array([[dl, -dv], [dl / rl, -dv / rv]])
        step = np.linalg.solve(J, -F)
        rl, rv = rl + step[0], rv + step[1]
        if np.abs(step).max() < tol * rl:
            break
    p0 = float(pressure(eos, rl, a, b, R, T))
    return float(rl), float(rv), p0


# --------------------------------------------------------------------------
# App. B: epsilon and sigma^Li
def _simpson(fvals, h):
    n = len(fvals) - 1
    assert n % 2 == 0
    return h / 3 * (fvals[0] + fvals[-1] + 4 * fvals[1:-1:2].sum() + 2 * fvals[2:-1:2].sum())


def epsilon_li(eos, a, b, R, T, n_intervals=40000, eps0=2.0, tol=1e-13, max_iter=60):
    """Newton on F(eps) = int_{rho_v}^{rho_l} (p - p0) psi' / psi^(1+eps) drho
    (App. B Eq. 13) with dF/deps = -int (p - p0) psi' ln(psi) / psi^(1+eps)
    (Eq. 14 with the sign of the derivative restored); Simpson's rule with
    n_intervals, starting from eps = 2.  Returns (eps, sigma_li = -eps/(16G))."""
    rl, rv, p0 = maxwell(eos, a, b, R, T)
    rho = np.linspace(rv, rl, n_intervals + 1)
    ps = psi(eos, rho, a, b, R, T)
    if not np.all(np.isfinite(ps)) or np.any(ps <= 0):
        raise ValueError("psi is not real on [rho_v, rho_l]; epsilon undefined")
    dps = dpsi(eos, rho, a, b, R, T)
    dpp = pressure(eos, rho, a, b, R, T) - p0
    h = (rl - rv) / n_intervals
    lnps = np.log(ps)
    eps = eps0
    for _ in range(max_iter):
        w = dpp * dps / ps ** (1 + eps)
        F = _simpson(w, h)
        dF = -_simpson(w * lnps, h)
        step = -F / dF
        eps += step
        if abs(step) < tol:
            break
    return eps, -eps / (16 * G)


# --------------------------------------------------------------------------
# planar-interface theory (profiles on a fine density grid)
_NGRID = 40000  # Simpson intervals over [rho_v, rho_l]


def _cumulative(fvals, x):
    """Cumulative integral from x[0] (composite Simpson on pairs of panels,
    trapezoid-corrected on odd points)."""
    return integrate.cumulative_simpson(fvals, x=x, initial=0.0)


def _max_on_grid(x, y):
    """Maximum of a sampled smooth function, refined by a parabola through
    the three samples around the largest one."""
    k = int(np.argmax(y))
    k = min(max(k, 1), len(y) - 2)
    y0, y1, y2 = y[k - 1], y[k], y[k + 1]
    den = y0 - 2 * y1 + y2
    if den == 0:
        return y1
    t = 0.5 * (y0 - y2) / den
    return y1 - 0.25 * (y0 - y2) * t


def fe_planar(eos, a, b, R, T, kappa, n=_NGRID):
    """FE planar theory: dict(rho_l, rho_v, p0, width, gamma).
    Profile from Eq. 26, (d rho/dx)^2 = (2 rho/kappa) int_{rho_v}^{rho}
    (p - p0)/s^2 ds; max-slope width; gamma = int (p_xx - p_yy) dx
    (App. B Eq. 15) = kappa int (d rho/dx) d rho with the FE tensor (Eq. 25)."""
    rl, rv, p0 = maxwell(eos, a, b, R, T)
    r = np.linspace(rv, rl, n + 1)
    integrand = (pressure(eos, r, a, b, R, T) - p0) / r ** 2
    cum = _cumulative(integrand, r)
    slope2 = np.maximum(2 * r / kappa * cum, 0.0)
    slope = np.sqrt(slope2)
    smax = math.sqrt(_max_on_grid(r, slope2))
    gamma = kappa * _simpson(slope, r[1] - r[0])
    return dict(rho_l=rl, rho_v=rv, p0=p0, width=(rl - rv) / smax, gamma=gamma)


def p_planar(eos, a, b, R, T, kappa_p, kappa_li, eps=None, n=_NGRID):
    """Pseudopotential planar theory: dict(rho_l, rho_v, p0, eps, width,
    gamma, I).  Profile from App. C Eq. 44 with G = -1,
    (d psi/dx)^2 = (8 psi^eps/(G kappa^P)) int_{rho_v}^{rho} (p0 - p)
    psi'/psi^(1+eps) ds; d rho/dx = (d psi/dx)/psi'; surface tension from
    Eq. 46, gamma = -(G/6)(kappa^P - kappa^Li) int psi' (d psi/dx) d rho."""
    rl, rv, p0 = maxwell(eos, a, b, R, T)
    if eps is None:
        eps, _ = epsilon_li(eos, a, b, R, T)
    r = np.linspace(rv, rl, n + 1)
    ps = psi(eos, r, a, b, R, T)
    dps = dpsi(eos, r, a, b, R, T)
    integrand = (p0 - pressure(eos, r, a, b, R, T)) * dps / ps ** (1 + eps)
    cum = _cumulative(integrand, r)
    z2 = np.maximum(8 * ps ** eps / (G * kappa_p) * cum, 0.0)
    slope2 = z2 / dps ** 2
    smax = math.sqrt(_max_on_grid(r, slope2))
    I = _simpson(np.abs(dps) * np.sqrt(z2), r[1] - r[0])
    gamma = -G / 6.0 * (kappa_p - kappa_li) * I
    return dict(rho_l=rl, rho_v=rv, p0=p0, eps=eps, width=(rl - rv) / smax,
                gamma=gamma, I=I)


def match_p_to_fe(eos, a, b, R, T, kappa_fe, target_width=None):
    """kappa^P so that the Eq. 44 max-slope width equals the FE width (or a
    given width), then kappa^Li so that the Eq. 46 surface tension equals the
    FE one (Sec. 3 and Sec. 4).  The width scales as sqrt(kappa^P) and
    int psi' (d psi/dx) d rho as 1/sqrt(kappa^P) (Eq. 44)."""
    fe = fe_planar(eos, a, b, R, T, kappa_fe)
    w_target = fe["width"] if target_width is None else target_width
    p1 = p_planar(eos, a, b, R, T, 1.0, 0.0)
    kp = (w_target / p1["width"]) ** 2
    I_kp = p1["I"] / math.sqrt(kp)
    kli = kp - 6.0 * fe["gamma"] / (-G * I_kp)
    return dict(kappa_p=kp, kappa_li=kli, sigma_li=-p1["eps"] / (16 * G), eps=p1["eps"],
                fe=fe)


# --------------------------------------------------------------------------
# discrete planar relations (App. D, App. E) on a periodic 1-D lattice
def _newton(F, J, x0, tol=1e-14, max_iter=200, valid=None):
    """Newton's method with step halving: a step is shortened until the
    residual norm decreases and ``valid(x)`` (if given) holds."""
    x = x0.copy()
    r = F(x)
    for _ in range(max_iter):
        dx = np.linalg.solve(J(x), -r)
        lam = 1.0
        while True:
            xn = x + lam * dx
            if valid is None or valid(xn):
                rn = F(xn)
                if np.all(np.isfinite(rn)) and (np.linalg.norm(rn) <= np.linalg.norm(r) or lam < 1e-3):
                    break
            lam *= 0.5
            if lam < 1e-12:
                return x, False
        x, r = xn, rn
        if np.abs(lam * dx).max() < tol * max(1.0, np.abs(x).max()):
            return x, True
    return x, False


def discrete_planar_fe(eos, a, b, R, T, kappa, rho_init):
    """Solve App. D Eq. 60 on a periodic lattice: mu_b(rho_n) -
    kappa (rho_{n+1} - 2 rho_n + rho_{n-1}) = mu_0 for all n, with the total
    mass of rho_init.  Unknowns (rho_0..rho_{N-1}, mu_0)."""
    rho_init = np.asarray(rho_init, dtype=np.float64)
    N = rho_init.size
    mass = rho_init.sum()

    def F(x):
        r, m0 = x[:N], x[N]
        lap = np.roll(r, -1) - 2 * r + np.roll(r, 1)
        return np.concatenate([mu_b(eos, r, a, b, R, T) - kappa * lap - m0, [r.sum() - mass]])

    def J(x):
        r = x[:N]
        Jm = np.zeros((N + 1, N + 1))
        dmu = dpressure(eos, r, a, b, R, T) / r
        for n in range(N):
            Jm[n, n] = dmu[n] + 2 * kappa
            Jm[n, (n + 1) % N] -= kappa
            Jm[n, (n - 1) % N] -= kappa
            Jm[n, N] = -1.0
        Jm[N, :N] = 1.0
        return Jm

    x0 = np.concatenate([rho_init, [float(np.mean(mu_b(eos, rho_init, a, b, R, T)))]])
    hi = 1.0 / b if eos == VDW else 4.0 / b
    x, ok = _newton(F, J, x0, valid=lambda x: bool(np.all(x[:N] > 0) and np.all(x[:N] < hi)))
    if not ok:
        raise RuntimeError("discrete FE planar solve did not converge")
    return x[:N], x[N]


def planar_p_invariant(eos, a, b, R, T, kappa_p, sigma_li, rho):
    """Per-node quantity of App. E Eq. 76 for a periodic planar profile:
    p_EOS(rho_n) + (G/4) kappa^P psi_n (psi_{n+1} - 2 psi_n + psi_{n-1})
    + 2 G^2 kappa^P sigma^Li ((psi_{n+1} - psi_{n-1})/2)^2  (c = dt = dx = 1)."""
    rho = np.asarray(rho, dtype=np.float64)
    ps = psi(eos, rho, a, b, R, T)
    pp, pm = np.roll(ps, -1), np.roll(ps, 1)
    return (pressure(eos, rho, a, b, R, T) + G / 4 * kappa_p * ps * (pp - 2 * ps + pm)
            + 2 * G * G * kappa_p * sigma_li * ((pp - pm) / 2) ** 2)


def discrete_planar_p(eos, a, b, R, T, kappa_p, sigma_li, rho_init):
    """Solve App. E Eq. 76 = p_0 for all n with the total mass of rho_init.
    Unknowns (rho_0..rho_{N-1}, p_0).  Jacobian by complex-free central
    differences of the banded residual."""
    rho_init = np.asarray(rho_init, dtype=np.float64)
    N = rho_init.size
    mass = rho_init.sum()

    def F(x):
        r, p0 = x[:N], x[N]
        return np.concatenate([planar_p_invariant(eos, a, b, R, T, kappa_p, sigma_li, r) - p0,
                               [r.sum() - mass]])

    def J(x):
        Jm = np.zeros((N + 1, N + 1))
        r = x[:N]
        for k in range(N):
            h = 1e-7 * max(abs(r[k]), 1e-3)
            rp, rm = r.copy(), r.copy()
            rp[k] += h
            rm[k] -= h
            col = (planar_p_invariant(eos, a, b, R, T, kappa_p, sigma_li, rp)
                   - planar_p_invariant(eos, a, b, R, T, kappa_p, sigma_li, rm)) / (2 * h)
            Jm[:N, k] = col
        Jm[:N, N] = -1.0
        Jm[N, :N] = 1.0
        return Jm

    x0 = np.concatenate([rho_init, [float(np.mean(
        planar_p_invariant(eos, a, b, R, T, kappa_p, sigma_li, rho_init)))]])
    hi = 1.0 / b if eos == VDW else 4.0 / b
    x, ok = _newton(F, J, x0, tol=1e-13,
                    valid=lambda x: bool(np.all(x[:N] > 0) and np.all(x[:N] < hi)
                                         and np.all(np.isfinite(psi(eos, x[:N], a, b, R, T)))))
    if not ok:
        raise RuntimeError("discrete P planar solve did not converge")
    return x[:N], x[N]


# --------------------------------------------------------------------------
# two-phase flow between parallel plates (Sec. 5.3, App. F)
def plates_sharp(Fx, H, mu1, mu2, y):
    """App. F Eq. 88: steady velocity between no-slip plates at y = 0 and
    y = H, fluid 1 (dynamic viscosity mu1) below H/2 and fluid 2 (mu2) above,
    driven by the body force Fx, with velocity and shear stress continuous at
    the sharp interface y = H/2.  C_1 as printed; C_2 is the value that
    u_1(0) = 0 requires, F_x H^2 / (8 mu1) - C_1 H / 2 (the printed C_2 has
    H for H^2 and the opposite sign of its first term, which violates the
    no-slip condition it is meant to satisfy)."""
    y = np.asarray(y, dtype=np.float64)
    C1 = Fx * H / 4 * (mu2 - mu1) / (mu1 * (mu1 + mu2))
    C2 = Fx * H * H / (8 * mu1) - C1 * H / 2
    u1 = -Fx / (2 * mu1) * (H / 2 - y) ** 2 + C1 * (H / 2 - y) + C2
    u2 = -Fx / (2 * mu2) * (y - H / 2) ** 2 - mu1 * C1 / mu2 * (y - H / 2) + C2
    return np.where(y <= H / 2, u1, u2)


def plates_diffuse(Fx, y_nodes, mu_nodes, refine=64):
    """App. F Eq. 89: steady velocity between no-slip plates at y_nodes[0]
    and y_nodes[-1] for a viscosity mu(y) that varies continuously,
    u(y) = -Fx int_0^y y'/mu dy' + mu(0) u'(0) int_0^y dy'/mu, with the
    constant mu(0) u'(0) fixed by u = 0 on the upper plate.  mu(y) is the
    cubic spline through the nodal values (mu = rho c_s^2 (tau_nu - 1/2) of a
    density profile); the integrals use composite Simpson on a grid refined
    refine times.  Returns u at y_nodes."""
    from scipy.interpolate import CubicSpline
    y_nodes = np.asarray(y_nodes, dtype=np.float64)
    y0 = y_nodes[0]
    spl = CubicSpline(y_nodes - y0, np.asarray(mu_nodes, dtype=np.float64))
    n = (len(y_nodes) - 1) * refine + 1
    yf = np.linspace(0.0, y_nodes[-1] - y0, n)
    mu = spl(yf)
    i1 = _cumulative(yf / mu, yf)
    i0 = _cumulative(1.0 / mu, yf)
    c = Fx * i1[-1] / i0[-1]
    u = -Fx * i1 + c * i0
    return u[::refine]
