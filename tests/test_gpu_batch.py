"""Batched lattices and the autotuner, through the C ABI, against the oracle."""
import math

import numpy as np
import pytest

import oracle
from oracle import theory as th
from paper_2403_11167_amd import inputs, lbm

pytestmark = pytest.mark.gpu

FP64_RTOL = 1e-10


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def cs_T(a, Tr):
    return Tr * th.critical(th.CS, a, 4.0, 1.0)[0]


def oparams(c: lbm.Config):
    return oracle.OracleParams(c.nx, c.ny, c.model, c.eos, c.a, c.b, c.R, c.T, tau=list(c.tau),
                               sigma_li=c.sigma_li, kappa_li=c.kappa_li, kappa_p=c.kappa_p,
                               kappa=c.kappa, fx=c.fx, fy=c.fy)


def oracle_rho(c, rho0, steps):
    s = oracle.Simulation(oparams(c), rho0)
    s.step(steps)
    return s.fields()[0], s.flags


def rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def mixed_cases(precision=lbm.FP64):
    """Problems of different sizes, models and EOS (all stable for a while)."""
    cases = []
    a = 0.25
    T = cs_T(a, 0.8)
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    tauP = [1.0] * 9
    tauP[4] = tauP[6] = 1 / 1.99
    tauF = [1.0] * 9
    tauF[1] = 0.75
    for (nx, ny, model, geo) in [(64, 64, 0, "drop"), (100, 70, 1, "drop"), (257, 33, 0, "flat"),
                                 (128, 128, 1, "flat"), (300, 90, 0, "drop"), (64, 64, 1, "drop")]:
        if model == 0:
            c = lbm.Config(nx, ny, 0, lbm.EOS_CS, a, 4.0, 1.0, T, tau=tauP, sigma_li=0.11,
                           kappa_p=0.9, kappa_li=-0.5, precision=precision)
        else:
            c = lbm.Config(nx, ny, 1, lbm.EOS_CS, a, 4.0, 1.0, T, tau=tauF, kappa=0.5,
                           precision=precision)
        r0 = (inputs.droplet(nx, ny, rl, rv, radius=min(nx, ny) / 4) if geo == "drop"
              else inputs.planar_slab(nx, ny, rl, rv))
        cases.append((c, r0))
    # a van der Waals pseudopotential problem (psi real at Tr = 0.9)
    Tv = 0.9 * 4 / 7
    rlv, rvv, _ = th.maxwell(th.VDW, 9 / 49, 2 / 21, 1.0, Tv)
    c = lbm.Config(96, 40, 0, lbm.EOS_VDW, 9 / 49, 2 / 21, 1.0, Tv, precision=precision)
    cases.append((c, inputs.planar_slab(96, 40, rlv, rvv)))
    return cases


def test_batch_lockstep_matches_oracle():
    cases = mixed_cases()
    b = lbm.Batch([c for c, _ in cases], [to_dev(r) for _, r in cases])
    steps = 120
    done = b.run(check_every=40, du_tol=0.0, max_steps=steps)
    assert done == steps
    st, nsteps, du, fl = b.state()
    assert all(s == lbm.BATCH_MAXSTEPS for s in st)
    assert all(n == steps for n in nsteps)
    for i, (c, r0) in enumerate(cases):
        obs, (rho, _, _) = b.observe(i, fields=True)
        rref, fref = oracle_rho(c, r0, steps)
        assert rel(rho.cpu().numpy(), rref) < FP64_RTOL, i
        assert obs["flags"] == fref
        assert obs["step"] == steps
    b.close()


def test_batch_fp32_lockstep_within_fp32_bound():
    cases = mixed_cases(lbm.FP32_SHIFTED)[:4]
    b = lbm.Batch([c for c, _ in cases], [to_dev(r) for _, r in cases])
    steps = 100
    b.run(check_every=50, du_tol=0.0, max_steps=steps)
    for i, (c, r0) in enumerate(cases):
        _, (rho, _, _) = b.observe(i, fields=True)
        rref, _ = oracle_rho(c, r0, steps)
        bound = 4.0 * math.sqrt(steps) * 2.0 ** -24 * float(rref.max() / rref.min())
        assert rel(rho.cpu().numpy(), rref) < bound, i
    b.close()


def test_batch_convergence_and_retirement():
    """Planar problems converge (max |du| over a check interval below the
    tolerance) and retire; an unstable free-energy van der Waals problem
    retires as unstable without disturbing the others.  Each retired
    problem's state equals the oracle after the same number of steps."""
    a = 0.5
    T = cs_T(a, 0.7)
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    _, sig = th.epsilon_li(th.CS, a, 4.0, 1.0, T)
    tauP = [1.0] * 9
    tauP[4] = tauP[6] = 1 / 1.99
    cfgs = [lbm.Config(100, 4, 1, lbm.EOS_CS, a, 4.0, 1.0, T, kappa=0.5),
            lbm.Config(64, 8, 0, lbm.EOS_CS, a, 4.0, 1.0, T, tau=tauP, sigma_li=sig),
            lbm.Config(80, 6, 0, lbm.EOS_CS, a, 4.0, 1.0, T, tau=tauP, sigma_li=sig, kappa_p=0.7)]
    r0s = [inputs.planar_slab(c.nx, c.ny, rl, rv) for c in cfgs]
    Tv = 0.7 * 4 / 7
    rlv, rvv, _ = th.maxwell(th.VDW, 9 / 49, 2 / 21, 1.0, Tv)
    cfgs.append(lbm.Config(64, 64, 1, lbm.EOS_VDW, 9 / 49, 2 / 21, 1.0, Tv, kappa=0.5))
    r0s.append(inputs.spinodal(64, 64, 0.5 * (rlv + rvv), 0.01, seed=3))
    b = lbm.Batch(cfgs, [to_dev(r) for r in r0s])
    b.run(check_every=200, du_tol=1e-12, max_steps=60000)
    st, nsteps, du, fl = b.state()
    assert st[:3] == [lbm.BATCH_CONVERGED] * 3, (st, du)
    assert st[3] == lbm.BATCH_UNSTABLE and fl[3] & (lbm.FLAG_NONFINITE | lbm.FLAG_EOS_DOMAIN)
    for i in range(3):
        assert du[i] < 1e-12
        _, (rho, _, _) = b.observe(i, fields=True)
        rref, _ = oracle_rho(cfgs[i], r0s[i], nsteps[i])
        rho = rho.cpu().numpy()
        assert np.max(np.abs(rho - rref)) / rref.max() < FP64_RTOL
    b.close()


def test_partner_of_an_unstable_problem_retires_with_it():
    """Two problems paired as one unit: when the unstable free-energy van
    der Waals spinodal retires as unstable, its partner retires as dropped
    at the same step count and keeps its state (equal to the oracle's); a
    later step limit does not resume it; an unpaired copy of the partner
    runs on past that step."""
    a = 0.5
    T = cs_T(a, 0.7)
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    Tv = 0.7 * 4 / 7
    rlv, rvv, _ = th.maxwell(th.VDW, 9 / 49, 2 / 21, 1.0, Tv)
    cfgs = [lbm.Config(100, 4, 1, lbm.EOS_CS, a, 4.0, 1.0, T, kappa=0.5),
            lbm.Config(64, 64, 1, lbm.EOS_VDW, 9 / 49, 2 / 21, 1.0, Tv, kappa=0.5),
            lbm.Config(100, 4, 1, lbm.EOS_CS, a, 4.0, 1.0, T, kappa=0.5)]
    r0s = [inputs.planar_slab(100, 4, rl, rv),
           inputs.spinodal(64, 64, 0.5 * (rlv + rvv), 0.01, seed=3),
           inputs.planar_slab(100, 4, rl, rv)]
    b = lbm.Batch(cfgs, [to_dev(r) for r in r0s])
    for i, j in ((0, 0), (0, 3), (-1, 1)):
        with pytest.raises(lbm.LbmError):
            b.set_partner(i, j)
    b.set_partner(0, 1)
    b.set_partner(1, 0)  # the same pair again
    with pytest.raises(lbm.LbmError):
        b.set_partner(0, 2)  # 0 already has a partner
    steps = 30000
    b.run(check_every=200, du_tol=0.0, max_steps=steps)
    st, nsteps, _, fl = b.state()
    assert st[1] == lbm.BATCH_UNSTABLE and fl[1] & (lbm.FLAG_NONFINITE | lbm.FLAG_EOS_DOMAIN)
    assert nsteps[1] < steps
    assert st[0] == lbm.BATCH_DROPPED and nsteps[0] == nsteps[1], (st, nsteps)
    # the copy evolved identically, so it was active at that check too
    assert st[2] in (lbm.BATCH_CONVERGED, lbm.BATCH_MAXSTEPS) and nsteps[2] > nsteps[0]
    _, (rho, _, _) = b.observe(0, fields=True)
    rref, _ = oracle_rho(cfgs[0], r0s[0], nsteps[0])
    assert rel(rho.cpu().numpy(), rref) < FP64_RTOL
    b.set_limit(0, 10 ** 9)
    b.run(check_every=200, du_tol=0.0, max_steps=1000)
    st2, nsteps2, _, _ = b.state()
    assert st2[0] == lbm.BATCH_DROPPED and nsteps2[0] == nsteps[0]
    b.close()


@pytest.mark.parametrize("model", [0, 1])
def test_autotuned_launch_keeps_parity(model):
    a = 0.25
    T = cs_T(a, 0.8)
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    if model == 0:
        cfg = lbm.Config(320, 200, 0, lbm.EOS_CS, a, 4.0, 1.0, T, sigma_li=0.1, kappa_p=0.8)
    else:
        tau = [1.0] * 9
        tau[1] = 0.75
        cfg = lbm.Config(320, 200, 1, lbm.EOS_CS, a, 4.0, 1.0, T, tau=tau, kappa=0.5)
    r0 = inputs.droplet(320, 200, rl, rv, radius=40.0)
    tuned, ms = lbm.autotune(cfg, to_dev(r0), steps=5)
    assert tuned.tile_x in (64, 256) and tuned.tile_y >= 1 and ms > 0
    sim = lbm.Simulation(tuned, to_dev(r0))
    sim.step(60)
    _, (rho, _, _) = sim.observe(fields=True)
    rref, _ = oracle_rho(cfg, r0, 60)
    assert rel(rho.cpu().numpy(), rref) < FP64_RTOL


def test_step_limit_retires_and_resumes():
    """A per-problem step limit retires that problem at a check; raising the
    limit resumes it from its state; both histories equal the oracle."""
    cases = mixed_cases()[:3]
    b = lbm.Batch([c for c, _ in cases], [to_dev(r) for _, r in cases])
    b.set_limit(1, 80)
    b.set_limit(2, 0)  # retires before its first step
    b.run(check_every=40, du_tol=0.0, max_steps=160)
    st, nsteps, _, _ = b.state()
    assert st == [lbm.BATCH_MAXSTEPS] * 3 and nsteps == [160, 80, 0]
    b.set_limit(1, 120)
    b.set_limit(2, 40)
    b.run(check_every=40, du_tol=0.0, max_steps=200)
    st, nsteps, _, _ = b.state()
    assert nsteps == [160, 120, 40], nsteps
    for i, (c, r0) in enumerate(cases):
        _, (rho, _, _) = b.observe(i, fields=True)
        rref, _ = oracle_rho(c, r0, nsteps[i])
        assert rel(rho.cpu().numpy(), rref) < FP64_RTOL, i
    b.close()


def test_persistent_tile_loop_and_stats():
    """More tiles than resident workgroups (1024^2 lattices in 8-row
    segments: 512 tiles each, 2048 in all), so the persistent launch walks
    its table in several rounds: the batch equals the same lattices run one
    by one, bit for bit, and its statistics count every node update."""
    a = 0.25
    T = cs_T(a, 0.8)
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    tauF = [1.0] * 9
    tauF[1] = 0.75
    cfgs, r0s = [], []
    for k, model in enumerate((0, 1, 0, 1)):
        if model == 0:
            c = lbm.Config(1024, 1024, 0, lbm.EOS_CS, a, 4.0, 1.0, T, sigma_li=0.1, kappa_p=0.9)
        else:
            c = lbm.Config(1024, 1024, 1, lbm.EOS_CS, a, 4.0, 1.0, T, tau=tauF, kappa=0.5)
        cfgs.append(c.with_launch(256, 8, lbm.KF_SET | lbm.KF_NT_STORE))
        r0s.append(inputs.spinodal(1024, 1024, 0.5 * (rl + rv), 0.01, seed=10 + k))
    steps = 40
    b = lbm.Batch(cfgs, [to_dev(r) for r in r0s])
    b.run(check_every=20, du_tol=0.0, max_steps=steps)
    st = b.stats()
    assert st["node_updates"] == 4 * 1024 * 1024 * steps
    assert st["chunks"] == 2 and st["gpu_ms"] > 0
    for i, (c, r0) in enumerate(zip(cfgs, r0s)):
        _, (rb, _, _) = b.observe(i, fields=True)
        sim = lbm.Simulation(c, to_dev(r0))
        sim.step(steps)
        _, (rs, _, _) = sim.observe(fields=True)
        sim.close()
        assert np.array_equal(rb.cpu().numpy(), rs.cpu().numpy()), i
    b.close()


def test_stalled_problem_retires():
    """A uniform lattice under a constant body force accelerates for ever:
    its max |u(t) - u(t - K)| stays at about F K / rho (above the FP32 floor
    rule's 1e-6) and only rounding decides whether a check sets a new lowest
    value, so a run of LBM_BATCH_STALL_CHECKS checks without one soon comes
    and the problem retires as stalled; a problem at rest beside it
    converges."""
    a = 0.25
    T = cs_T(a, 0.8)
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    c0 = lbm.Config(32, 16, 1, lbm.EOS_CS, a, 4.0, 1.0, T, kappa=0.5, fx=1e-5)
    c1 = lbm.Config(32, 16, 1, lbm.EOS_CS, a, 4.0, 1.0, T, kappa=0.5)
    r0 = np.full((16, 32), rl)
    b = lbm.Batch([c0, c1], [to_dev(r0), to_dev(r0)])
    K = 2
    b.run(check_every=K, du_tol=1e-12, max_steps=K * 20 * lbm.BATCH_STALL_CHECKS)
    st, nsteps, du, fl = b.state()
    assert st == [lbm.BATCH_STALLED, lbm.BATCH_CONVERGED], (st, du, nsteps)
    assert nsteps[0] >= K * (lbm.BATCH_STALL_CHECKS + 2)
    assert du[0] > 1e-6 and fl[0] == 0
    b.close()


@pytest.mark.parametrize("precision", [lbm.FP64, lbm.FP32_SHIFTED])
def test_two_step_groups_equal_single_runs(precision):
    """Problems on 256-column tiles take two steps per launch in a batch
    (k_batch_step2), beside problems that take one: ragged strips and
    segments, both models, both equations of state, and chunks whose pair
    count is rounded down to even (8 steps: two pairs and four single steps;
    12 steps: four pairs and four) or not (10 steps: four pairs and two).
    A free-energy problem that asks for single steps on the same strip width
    forms its own group.  Every lattice equals the same lattice run alone,
    bit for bit, after runs resumed across three chunk lengths."""
    a = 0.25
    T = cs_T(a, 0.8)
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    Tv = 0.9 * 4 / 7
    rlv, rvv, _ = th.maxwell(th.VDW, 9 / 49, 2 / 21, 1.0, Tv)
    tauF = [1.0] * 9
    tauF[1] = 0.75
    single = lbm.KF_SET | lbm.KF_NT_STORE
    cases = [
        (lbm.Config(256, 40, 0, lbm.EOS_CS, a, 4.0, 1.0, T, sigma_li=0.1, kappa_p=0.9,
                    precision=precision).with_launch(256, 8, 0), 0.5 * (rl + rv), 21),
        (lbm.Config(320, 24, 1, lbm.EOS_CS, a, 4.0, 1.0, T, tau=tauF, kappa=0.5,
                    precision=precision).with_launch(256, 16, 0), 0.5 * (rl + rv), 22),
        (lbm.Config(300, 20, 0, lbm.EOS_VDW, 9 / 49, 2 / 21, 1.0, Tv,
                    precision=precision).with_launch(256, 8, 0), 0.5 * (rlv + rvv), 23),
        (lbm.Config(256, 32, 1, lbm.EOS_CS, a, 4.0, 1.0, T, kappa=0.5,
                    precision=precision).with_launch(256, 8, single), 0.5 * (rl + rv), 24),
        (lbm.Config(64, 48, 0, lbm.EOS_CS, a, 4.0, 1.0, T, sigma_li=0.1, kappa_p=0.9,
                    precision=precision).with_launch(64, 8, 0), 0.5 * (rl + rv), 25),
    ]
    cfgs = [c for c, _, _ in cases]
    r0s = [inputs.spinodal(c.nx, c.ny, m, 0.01, seed=s) for c, m, s in cases]
    b = lbm.Batch(cfgs, [to_dev(r) for r in r0s])
    # (steps per launch, strip, threads, workgroups) of each problem's kernel
    shapes = [(2, 256, 320, 5), (2, 128, 192, 3 * 2), (2, 256, 320, 2 * 3), (1, 256, 256, 4),
              (1, 64, 64, 6)]
    for i, want in enumerate(shapes):
        li = b.launch_info(i)
        assert (li["steps_per_launch"], li["strip"], li["threads"], li["workgroups"]) == want, i
    total = 0
    for k, (every, steps) in enumerate(((8, 16), (12, 12), (10, 10))):
        if k:
            for i in range(len(cfgs)):
                b.set_limit(i, 1 << 40)  # resume the problems the last run stopped
        assert b.run(check_every=every, du_tol=0.0, max_steps=steps) == steps
        total += steps
    states, nsteps, _, flags = b.state()
    assert all(n == total for n in nsteps)
    assert not any(f & (lbm.FLAG_NONFINITE | lbm.FLAG_EOS_DOMAIN) for f in flags)
    assert b.stats()["node_updates"] == sum(c.nx * c.ny for c in cfgs) * total
    for i, (c, r0) in enumerate(zip(cfgs, r0s)):
        _, (rb, ub, vb) = b.observe(i, fields=True)
        sim = lbm.Simulation(c, to_dev(r0))
        sim.step(total)
        os_, (rs, us, vs) = sim.observe(fields=True)
        sim.close()
        assert flags[i] == os_["flags"], i
        for f, g in ((rb, rs), (ub, us), (vb, vs)):
            assert np.array_equal(f.cpu().numpy(), g.cpu().numpy()), i
    b.close()


def test_automatic_segment_heights_follow_active_lattices():
    """Problems with tile_y = 0 (FP64 pseudopotential, two steps per launch):
    while sixteen 512^2 lattices are active their segments are taller than
    the lowest height (their tiles fill a round of resident workgroups with
    room to spare); once one is left it runs 4-row segments.  The heights
    change the tiling only: the survivor and a retired lattice equal the same
    lattices run alone, bit for bit."""
    a = 0.25
    T = cs_T(a, 0.8)
    rl, rv, _ = th.maxwell(th.CS, a, 4.0, 1.0, T)
    c = lbm.Config(512, 512, 0, lbm.EOS_CS, a, 4.0, 1.0, T, sigma_li=0.1,
                   kappa_p=0.9).with_launch(256, 0, 0)
    n = 16
    r0s = [inputs.spinodal(512, 512, 0.5 * (rl + rv), 0.01, seed=40 + k) for k in range(n)]
    b = lbm.Batch([c] * n, [to_dev(r) for r in r0s])
    assert b.run(check_every=10, du_tol=0.0, max_steps=20) == 20
    start = [b.launch_info(i) for i in range(n)]
    assert all(s["steps_per_launch"] == 2 and s["strip"] == 256 for s in start)
    seg0 = start[0]["segment"]
    assert seg0 in (8, 16, 32, 64, 128) and all(s["segment"] == seg0 for s in start)
    assert start[0]["workgroups"] == 2 * (512 // seg0)
    b.set_limit(0, 1 << 40)  # only problem 0 goes on
    assert b.run(check_every=10, du_tol=0.0, max_steps=20) == 20
    assert b.launch_info(0)["segment"] == 4 and b.launch_info(1)["segment"] == seg0
    _, nsteps, _, _ = b.state()
    assert nsteps[0] == 40 and all(k == 20 for k in nsteps[1:])
    for i, steps in ((0, 40), (7, 20)):
        _, (rb, ub, _) = b.observe(i, fields=True)
        sim = lbm.Simulation(c, to_dev(r0s[i]))
        sim.step(steps)
        _, (rs, us, _) = sim.observe(fields=True)
        sim.close()
        assert np.array_equal(rb.cpu().numpy(), rs.cpu().numpy()), i
        assert np.array_equal(ub.cpu().numpy(), us.cpu().numpy()), i
    b.close()
