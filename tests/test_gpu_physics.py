"""Physics of the GPU path at the paper's geometries (no oracle in the loop:
these compare the library's equilibria with the theory the paper states)."""
import math

import numpy as np
import pytest

from oracle import theory as th
from paper_2403_11167_amd import inputs, lbm

pytestmark = pytest.mark.gpu


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def droplet_batch(Tr, radii, precision=lbm.FP64, a=0.25):
    """256^2 droplets of both models (C-S a = 0.25; FE kappa = 0.5,
    tau_e = 0.75; P with App. B sigma^Li, kappa^P and kappa^Li matched to the
    FE width and surface tension, tau_q = 1/1.99), run to equilibrium."""
    T = Tr * th.critical(th.CS, a, 4.0, 1.0)[0]
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    m = th.match_p_to_fe(th.CS, a, 4.0, 1.0, T, 0.5)
    cfgs, r0s, meta = [], [], []
    for model in (lbm.MODEL_FE, lbm.MODEL_P):
        tau = [1.0] * 9
        if model == lbm.MODEL_FE:
            tau[1] = 0.75
            kw = dict(kappa=0.5)
        else:
            tau[4] = tau[6] = 1 / 1.99
            kw = dict(sigma_li=m["sigma_li"], kappa_p=m["kappa_p"], kappa_li=m["kappa_li"])
        for R in radii:
            cfgs.append(lbm.Config(256, 256, model, lbm.EOS_CS, a, 4.0, 1.0, T, tau=tau,
                                   precision=precision, **kw))
            r0s.append(inputs.droplet(256, 256, rl, rv, radius=R))
            meta.append((model, R))
    b = lbm.Batch(cfgs, [to_dev(r) for r in r0s])
    b.run(check_every=500, du_tol=1e-11, max_steps=60000)
    st, steps, du, fl = b.state()
    obs = [b.observe(i, 128, 128) for i in range(len(cfgs))]
    b.close()
    return meta, obs, st, m["fe"]["gamma"], T


# per-temperature bars on dp R_e / gamma (each radius), on the fitted slope
# and on its intercept (relative to the largest dp)
LAPLACE_BARS = {0.9: (0.02, 0.03, 0.02), 0.8: (0.03, 0.04, 0.02), 0.7: (0.03, 0.04, 0.02),
                0.6: (0.05, 0.06, 0.04)}


@pytest.mark.parametrize("Tr", [0.9, 0.8, 0.7, 0.6])
def test_laplace_law_on_256_droplets(Tr):
    """Sec. 5.2 / Fig. 3: dp against 1/R for R in {20, 30, 40, 60} on 256^2
    lattices is a line through the origin whose slope is the planar theory's
    surface tension (App. B Eq. 15 with Eq. 26 for FE; Eq. 46 for P, whose
    kappa^Li is matched to that value), at every temperature of the grid.
    Curvature corrections of order W / R reach ~2-3 % at Tr = 0.8, where
    the smallest droplet evaporates to R_e ~ 16 against a width W ~ 6; at
    Tr = 0.9 (W ~ 8.8) the R = 20 droplet is below the critical radius of
    the box and evaporates completely (checked: no droplet left), and the
    others are within 0.5 %.  At Tr = 0.6 (W ~ 4.2) the free-energy droplets
    sit 2-4 % below the planar theory and still approach it slowly (R = 30:
    0.961, 0.972, 0.979 after 6e4, 1.5e5, 3e5 steps), the pseudopotential
    ones within 1.5 %."""
    radii = (20.0, 30.0, 40.0, 60.0)
    bar_r, bar_slope, bar_icpt = LAPLACE_BARS[Tr]
    meta, obs, st, gamma, _ = droplet_batch(Tr, radii)
    for model in (lbm.MODEL_FE, lbm.MODEL_P):
        idx = [i for i, (m, _) in enumerate(meta) if m == model]
        assert all(st[i] in (lbm.BATCH_CONVERGED, lbm.BATCH_MAXSTEPS) for i in idx)
        for i in idx:
            assert obs[i]["flags"] == 0
        if Tr == 0.9:
            small = [i for i in idx if meta[i][1] == 20.0]
            for i in small:  # evaporated: uniform vapour, no pressure jump
                assert abs(obs[i]["dp"]) < 0.01 * gamma / 20.0
            idx = [i for i in idx if i not in small]
        x = np.array([1.0 / obs[i]["r_equimolar"] for i in idx])
        y = np.array([obs[i]["dp"] for i in idx])
        for i in idx:
            assert abs(obs[i]["dp"] * obs[i]["r_equimolar"] / gamma - 1) < bar_r, (model, meta[i])
        slope, icpt = np.polyfit(x, y, 1)
        assert abs(slope / gamma - 1) < bar_slope, model
        assert abs(icpt) < bar_icpt * y.max()


def test_free_energy_droplet_is_thermodynamically_consistent():
    """The well-balanced free-energy model reaches a uniform chemical
    potential, so inside and outside a droplet mu_b(rho_in) = mu_b(rho_out)
    (Sec. 2.2, Eq. 29) while the pressures differ by the Laplace jump: the
    vapour is the Laplace-shifted coexistence density, not the planar
    Maxwell one (Sec. 5.2).  96^2 box (chemical equilibrium needs mass to
    diffuse through the vapour, slow on large boxes), C-S a = 0.25,
    Tr = 0.7, R = 16 and 24.  The scale of an inconsistency is
    dp / (rho_l - rho_v) (what mu_out - mu_in would be with the vapour at
    its planar density); the bar is 1 % of it, and the vapour density within
    10 % of the first-order Laplace shift of the planar Maxwell value."""
    a = 0.25
    T = 0.7 * th.critical(th.CS, a, 4.0, 1.0)[0]
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    tau = [1.0] * 9
    tau[1] = 0.75
    cfgs = [lbm.Config(96, 96, lbm.MODEL_FE, lbm.EOS_CS, a, 4.0, 1.0, T, tau=tau, kappa=0.5)
            for _ in (16.0, 24.0)]
    r0s = [inputs.droplet(96, 96, rl, rv, radius=R) for R in (16.0, 24.0)]
    b = lbm.Batch(cfgs, [to_dev(r) for r in r0s])
    b.run(check_every=1000, du_tol=1e-13, max_steps=400000)
    st, steps, du, fl = b.state()
    for i in range(2):
        o = b.observe(i, 48, 48)
        assert o["flags"] == 0
        mu_in = th.mu_b(th.CS, o["rho_in"], a, 4.0, 1.0, T)
        mu_out = th.mu_b(th.CS, o["rho_out"], a, 4.0, 1.0, T)
        scale = o["dp"] / (rl - rv)
        assert abs(mu_in - mu_out) < 0.01 * scale, (i, st[i], steps[i], mu_in - mu_out, scale)
        dpv = o["dp"] * rv / (rl - rv)
        drv = dpv / th.dpressure(th.CS, rv, a, 4.0, 1.0, T)
        assert abs(o["rho_out"] - (rv + drv)) < 0.1 * drv, (i, o["rho_out"], rv, drv)
    b.close()


@pytest.mark.parametrize("tau_v", [0.55, 0.75, 1.0, 1.2])
def test_table1_fe_vapor_error_independent_of_tau(tau_v):
    """Table 1 (Sec. 5.1): for the free-energy model the coexistence error is
    the same for every tau_v (C-S a = 0.5, Tr = 0.65, kappa = 0.5, L_x = 100,
    all other tau = 1): the GPU flat interface reaches the App. D discrete
    relation's 0.0536 % (Table 1 prints 0.0605 %)."""
    a = 0.5
    T = 0.65 * th.critical(th.CS, a, 4.0, 1.0)[0]
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    tau = [1.0] * 9
    tau[7] = tau[8] = tau_v
    cfg = lbm.Config(100, 1, lbm.MODEL_FE, lbm.EOS_CS, a, 4.0, 1.0, T, tau=tau, kappa=0.5)
    sim = lbm.Simulation(cfg, to_dev(inputs.planar_slab(100, 1, rl, rv, width=5.0)))
    sim.step(60000)
    obs, (rho, _, _) = sim.observe(fields=True)
    sim.close()
    err = 100 * abs(float(rho.min()) - rv) / rv
    assert abs(err - 0.0536) < 0.001
    assert obs["flags"] == 0


def test_table1_pseudopotential_rows():
    """Table 1 (Sec. 5.1), pseudopotential rows: C-S a = 0.5, Tr = 0.65,
    L_x = 100, kappa^Li = 0, kappa^P matched to the FE width (kappa = 0.5),
    tau_v in {0.55, 0.75, 1, 1.2}, tau_q = 1 and 1/1.99, every other tau = 1;
    60000 steps from a tanh slab.  Each GPU state equals the oracle's
    (field-relative 1e-10), and the rows show what Table 1 shows: with
    tau_q = 1 the vapour error falls with tau_v, with tau_q = 1/1.99 it stays
    put, and at tau_v = tau_e = 1 both rows are the same state (App. E: the
    q rows drop out of the planar relation).  Measured here 5.54, 4.22, 2.70,
    1.57 % and 2.714, 2.708, 2.699, 2.692 %; Table 1 prints 50.6, 40.0, 27.6,
    18.4 and 27.7, 27.7, 27.6, 27.6: the same pattern (ratios to the
    tau_v = 1 entry 2.05 / 1.56 / 0.58 against 1.83 / 1.45 / 0.67, flat rows
    within 0.6 % and 0.4 %), ten times smaller, as the App. E relation
    solved independently also gives at tau_v = 1 (2.71 %)."""
    from test_gpu_parity import field_rel_err, oracle_run
    a = 0.5
    T = 0.65 * th.critical(th.CS, a, 4.0, 1.0)[0]
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    m = th.match_p_to_fe(th.CS, a, 4.0, 1.0, T, 0.5)
    rho0 = inputs.planar_slab(100, 1, rl, rv, width=5.0)
    err, states = {}, {}
    for tq in (1.0, 1 / 1.99):
        for tv in (0.55, 0.75, 1.0, 1.2):
            tau = [1.0] * 9
            tau[7] = tau[8] = tv
            tau[4] = tau[6] = tq
            cfg = lbm.Config(100, 1, lbm.MODEL_P, lbm.EOS_CS, a, 4.0, 1.0, T, tau=tau,
                             sigma_li=m["sigma_li"], kappa_p=m["kappa_p"], kappa_li=0.0)
            sim = lbm.Simulation(cfg, to_dev(rho0))
            sim.step(60000)
            obs, (rho, _, _) = sim.observe(fields=True)
            sim.close()
            rho = rho.cpu().numpy()
            assert obs["flags"] == 0
            ref = oracle_run(cfg, rho0, 60000).fields()[0]
            assert field_rel_err(rho, ref) < 1e-10
            err[tq, tv] = 100 * abs(rho.min() - rv) / rv
            states[tq, tv] = rho
    r1 = [err[1.0, tv] for tv in (0.55, 0.75, 1.0, 1.2)]
    r2 = [err[1 / 1.99, tv] for tv in (0.55, 0.75, 1.0, 1.2)]
    assert r1[0] > r1[1] > r1[2] > r1[3]
    paper = [50.6 / 27.6, 40.0 / 27.6, 18.4 / 27.6]
    for got, want in zip((r1[0] / r1[2], r1[1] / r1[2], r1[3] / r1[2]), paper):
        assert abs(got / want - 1) < 0.2, (got, want)
    assert (max(r2) - min(r2)) / r2[2] < 0.01
    assert np.abs(states[1.0, 1.0] - states[1 / 1.99, 1.0]).max() < 1e-10 * rl
    assert 2.5 < r1[2] < 2.9


def _planar_invariant(model, a, T, sig, rho):
    """Per-node left-hand side of App. D Eq. 60 (FE, kappa = 0.5) or App. E
    Eq. 76 (P, kappa^P = 1) on a periodic row, and the size of its largest
    bulk term across the profile (the scale a residual is measured against)."""
    if model == lbm.MODEL_FE:
        mu = th.mu_b(th.CS, rho, a, 4.0, 1.0, T)
        inv = mu - 0.5 * (np.roll(rho, -1) - 2 * rho + np.roll(rho, 1))
        return inv, np.abs(mu - inv.mean()).max()
    inv = th.planar_p_invariant(th.CS, a, 4.0, 1.0, T, 1.0, sig, rho)
    return inv, np.abs(th.pressure(th.CS, rho, a, 4.0, 1.0, T) - inv.mean()).max()


def test_coexistence_curves_match_discrete_theory():
    """Fig. 2 (Sec. 5.1): coexistence densities of flat interfaces over the
    reduced temperature, for both models and two EOS scalings (C-S
    a = 0.25, 0.5; L_x = 100; all tau = 1 except tau_q = 1/1.99 for P;
    FE kappa = 0.5; P with the App. B sigma^Li, kappa^P = 1, kappa^Li = 0).
    Every GPU steady state satisfies the model's discrete planar relation --
    App. D Eq. 60 (FE) or App. E Eq. 76 (P) -- at every node to 1e-8 of its
    bulk terms (the batch retires a problem once its velocity change stalls;
    the slowest FE transient, a = 0.25 Tr = 0.65, is then at ~2e-9), with
    the initial mass; FE reaches Maxwell to 0.1 % while P
    sits at its O(dx^2) distance from it (Sec. 5.1).  The relation is checked
    through its per-node residual, not by solving it: at high Tr a shift of
    the wide interface along the lattice is nearly free, so the solution is
    fixed only to ~1e-7 there while the residual stays well conditioned.
    a = 0.5, Tr = 0.7 FE leaves the smooth state (see the odd-even test
    below), so that point is run there."""
    L = 100
    cases, cfgs, r0s = [], [], []
    for a, trs in ((0.25, (0.9, 0.8, 0.7, 0.65)), (0.5, (0.9, 0.8, 0.65))):
        for Tr in trs:
            T = Tr * th.critical(th.CS, a, 4.0, 1.0)[0]
            rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
            _, sig = th.epsilon_li(th.CS, a, 4.0, 1.0, T)
            for model in (lbm.MODEL_FE, lbm.MODEL_P):
                tau = [1.0] * 9
                if model == lbm.MODEL_FE:
                    cfg = lbm.Config(L, 1, model, lbm.EOS_CS, a, 4.0, 1.0, T, tau=tau, kappa=0.5)
                else:
                    tau[4] = tau[6] = 1 / 1.99
                    cfg = lbm.Config(L, 1, model, lbm.EOS_CS, a, 4.0, 1.0, T, tau=tau,
                                     sigma_li=sig, kappa_p=1.0, kappa_li=0.0)
                cases.append((a, Tr, model, T, rl, rv, sig))
                cfgs.append(cfg)
                r0s.append(inputs.planar_slab(L, 1, rl, rv, width=5.0))
    b = lbm.Batch(cfgs, [to_dev(r) for r in r0s])
    b.run(check_every=1000, du_tol=0.0, max_steps=100000)
    st, nsteps, _, fl = b.state()
    for i, (a, Tr, model, T, rl, rv, sig) in enumerate(cases):
        assert fl[i] == 0 and st[i] in (lbm.BATCH_CONVERGED, lbm.BATCH_MAXSTEPS)
        _, (rho, _, _) = b.observe(i, fields=True)
        rho = rho.cpu().numpy()[0]
        assert abs(rho.sum() / r0s[i].sum() - 1) < 1e-12
        inv, scale = _planar_invariant(model, a, T, sig, rho)
        assert np.ptp(inv) < 1e-8 * scale, (a, Tr, model, nsteps[i], np.ptp(inv) / scale)
        if model == lbm.MODEL_FE:
            assert abs(rho.min() / rv - 1) < 1e-3, (a, Tr)
        assert abs(rho.max() / rl - 1) < 0.05 and abs(rho.min() / rv - 1) < 0.10
    b.close()


def test_free_energy_odd_even_planar_state():
    """A property of the FE scheme that App. D's derivation of Eq. 60 passes
    over: at rest, F = -rho grad(mu) with the central (1-D reduction of the
    9-point) gradient vanishes when mu is constant on each parity
    sublattice, not only when it is uniform.  For sharp interfaces the
    smooth planar state is unstable to that odd-even mode: for C-S a = 0.5,
    Tr = 0.7, kappa = 0.5, L_x = 100, all tau = 1 it grows from rounding
    after ~60k steps and saturates by ~100k in a stationary state whose
    liquid alternates between two densities and whose vapour sits 0.2 %
    below Maxwell.  The oracle takes the same path; the GPU must reach the
    same state: Eq. 60's residual constant on each sublattice to 1e-9 of its
    bulk terms, the two sublattice values apart, and the vapour density and
    the sublattice split equal to the oracle's to 1e-6 (the state is an
    attractor, so rounding differences along the way do not matter; which
    sublattice is higher can differ, so the split is compared unsigned)."""
    import oracle
    a, L, steps = 0.5, 100, 200000
    T = 0.7 * th.critical(th.CS, a, 4.0, 1.0)[0]
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    rho0 = inputs.planar_slab(L, 1, rl, rv, width=5.0)
    cfg = lbm.Config(L, 1, lbm.MODEL_FE, lbm.EOS_CS, a, 4.0, 1.0, T, tau=[1.0] * 9, kappa=0.5)
    sim = lbm.Simulation(cfg, to_dev(rho0))
    sim.step(steps)
    obs, (rho, _, _) = sim.observe(fields=True)
    sim.close()
    rho = rho.cpu().numpy()[0]
    ref = oracle.Simulation(oracle.OracleParams(L, 1, 1, 1, a, 4.0, 1.0, T, tau=[1.0] * 9,
                                                kappa=0.5), rho0)
    ref.step(steps)
    rho_o = ref.fields()[0][0]
    assert obs["flags"] == 0
    for r in (rho, rho_o):
        inv, scale = _planar_invariant(lbm.MODEL_FE, a, T, 0.0, r)
        assert np.ptp(inv[0::2]) < 1e-9 * scale and np.ptp(inv[1::2]) < 1e-9 * scale
        assert np.ptp(inv) > 1e-3 * scale
    split = lambda r: abs(r[0::2].max() - r[1::2].max())
    assert abs(rho.min() - rho_o.min()) < 1e-6 * rv
    assert abs(split(rho) - split(rho_o)) < 1e-6 * rl
    assert -0.3e-2 < rho.min() / rv - 1 < -0.1e-2
