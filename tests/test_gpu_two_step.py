"""Two steps per launch (temporal blocking, LBM_KF_TWO_STEP), both models.

The two-step kernels keep the first step's populations on chip and do
every node's arithmetic in the single-step kernel's order, so its fields
must equal those of two single steps bit for bit (and therefore the
oracle's to its bar): ragged strips and segments, segments of one row,
lattices narrower than the strip (columns wrap onto themselves), an odd
step count (the last step single), both equations of state (the van der
Waals case raises the psi clamp flag on both paths), FP64 and FP32-shifted
storage, and the 4096^2 throughput lattice in its launch configuration.
"""
import numpy as np
import pytest

from oracle import theory as th
from paper_2403_11167_amd import inputs, lbm
from test_gpu_parity import FP64_RTOL, cs_T, fe_cfg, oracle_run, p_cfg, rel_err, torch_dev

pytestmark = pytest.mark.gpu

ONE = lbm.KF_SET | lbm.KF_NT_STORE
TWO = lbm.KF_SET | lbm.KF_NT_STORE | lbm.KF_TWO_STEP


def run(cfg, rho0, steps):
    import torch
    sim = lbm.Simulation(cfg, torch.from_numpy(np.ascontiguousarray(rho0)).to(torch_dev()))
    sim.step(steps)
    obs, (rho, ux, uy) = sim.observe(fields=True)
    f = sim.populations()
    sim.close()
    return obs, rho.cpu().numpy(), f.cpu().numpy()


def noisy(cfg, amp=0.03, seed=4):
    rl, rv, _ = th.maxwell(cfg.eos, cfg.a, cfg.b, cfg.R, cfg.T)
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:cfg.ny, 0:cfg.nx]
    r = rv + (rl - rv) * (0.5 + 0.3 * np.sin(2 * np.pi * x / max(cfg.nx, 2) + 0.2)
                          * np.cos(2 * np.pi * y / max(cfg.ny, 2)))
    return r * (1 + amp * rng.uniform(-1, 1, size=r.shape))


CASES = [
    # (nx, ny, tile_y, steps)
    (300, 130, 0, 40), (300, 130, 7, 41), (257, 9, 1, 20), (512, 64, 64, 30),
    (70, 66, 16, 24), (5, 7, 3, 12), (256, 1, 0, 10),
]


@pytest.mark.parametrize("prec", [lbm.FP64, lbm.FP32_SHIFTED])
@pytest.mark.parametrize("nx,ny,ty,steps", CASES)
def test_two_step_equals_two_single_steps(nx, ny, ty, steps, prec):
    cfg = p_cfg(nx, ny, a=0.25, Tr=0.75, tau=[1.0, 0.8, 1.3, 1.0, 0.7, 1.0, 0.7, 1.1, 1.1],
                sigma_li=0.12, kappa_p=0.7, kappa_li=0.3, precision=prec)
    rho0 = noisy(cfg)
    o1, r1, f1 = run(cfg.with_launch(256, ty, ONE), rho0, steps)
    o2, r2, f2 = run(cfg.with_launch(256, ty, TWO), rho0, steps)
    assert o1["flags"] == o2["flags"] == 0
    assert np.array_equal(f1, f2), float(np.abs(f1 - f2).max())
    assert np.array_equal(r1, r2)
    if prec == lbm.FP64 and nx * ny <= 40000:
        ref = oracle_run(cfg, rho0, steps).fields()[0]
        assert rel_err(r2, ref) < FP64_RTOL


def test_two_step_vdw_clamp_flag():
    """van der Waals Tr = 0.8 flat interface (psi clamped in the vapour):
    the same flags and fields on both paths."""
    a, b, R, T = 9 / 49, 2 / 21, 1.0, 0.8 * 4 / 7
    rl, rv, _ = th.maxwell(th.VDW, a, b, R, T)
    rho0 = inputs.planar_slab(256, 4, rl, rv, width=5.0, noise=1e-6, seed=1)
    cfg = lbm.Config(256, 4, lbm.MODEL_P, lbm.EOS_VDW, a, b, R, T)
    o1, r1, f1 = run(cfg.with_launch(256, 0, ONE), rho0, 200)
    o2, r2, f2 = run(cfg.with_launch(256, 0, TWO), rho0, 200)
    assert o1["flags"] == o2["flags"] == lbm.FLAG_PSI_CLAMP
    assert np.array_equal(f1, f2)


@pytest.mark.parametrize("prec", [lbm.FP64, lbm.FP32_SHIFTED])
def test_two_step_throughput_lattice(prec):
    """4096^2 spinodal (C-S a = 0.25, Tr = 0.85), the benchmark's workload:
    the two-step path equals the single-step one after 6 steps."""
    E, a, b, R = lbm.EOS_CS, 0.25, 4.0, 1.0
    T = cs_T(a, 0.85)
    rl, rv, _ = th.maxwell(E, a, b, R, T)
    rho0 = inputs.spinodal(4096, 4096, 0.5 * (rl + rv), 0.01, seed=3)
    cfg = lbm.Config(4096, 4096, lbm.MODEL_P, E, a, b, R, T, precision=prec)
    o1, r1, f1 = run(cfg.with_launch(256, 0, ONE | lbm.KF_PIPELINE), rho0, 6)
    o2, r2, f2 = run(cfg.with_launch(256, 0, TWO), rho0, 6)
    assert o1["flags"] == o2["flags"]
    assert np.array_equal(r1, r2)
    assert np.array_equal(f1, f2)


# ---------------------------------------------------------------- free energy
FE_TAU = [1.0, 0.75, 1.2, 1.0, 0.8, 1.0, 0.8, 0.9, 0.9]


# two-step kernel variants: strip width (FP64 pulls the first step's row
# again for its collision, FP32 keeps it in registers)
FE_VARIANTS = {"256": TWO, "128": TWO | lbm.KF_STRIP128, "192": TWO | lbm.KF_STRIP192}


@pytest.mark.parametrize("variant", list(FE_VARIANTS))
@pytest.mark.parametrize("prec", [lbm.FP64, lbm.FP32_SHIFTED])
@pytest.mark.parametrize("nx,ny,ty,steps", CASES)
def test_fe_two_step_equals_two_single_steps(nx, ny, ty, steps, prec, variant):
    """Free energy (C-S a = 0.25, Tr = 0.75, kappa = 0.5, every tau
    different), every variant of the two-step kernel: ragged strips and
    segments, one-row segments, lattices narrower than the strip (the first
    step's five halo columns wrap onto the strip itself), odd step counts."""
    cfg = fe_cfg(nx, ny, a=0.25, Tr=0.75, tau=FE_TAU, precision=prec)
    rho0 = noisy(cfg)
    two = FE_VARIANTS[variant]
    o1, r1, f1 = run(cfg.with_launch(256, ty, ONE), rho0, steps)
    o2, r2, f2 = run(cfg.with_launch(256, ty, two), rho0, steps)
    assert o1["flags"] == o2["flags"] == 0
    assert np.array_equal(f1, f2), float(np.abs(f1 - f2).max())
    assert np.array_equal(r1, r2)
    if prec == lbm.FP64 and nx * ny <= 40000:
        ref = oracle_run(cfg, rho0, steps).fields()[0]
        assert rel_err(r2, ref) < FP64_RTOL


def test_fe_two_step_vdw_and_body_force():
    """van der Waals EOS with a constant body force (both enter the
    periodic kernel): the same fields and flags on both paths."""
    cfg = fe_cfg(300, 40, a=9 / 49, Tr=0.85, eos=lbm.EOS_VDW, kappa=0.02, fx=1e-6, fy=-2e-6,
                 tau=FE_TAU)
    rho0 = noisy(cfg, amp=0.01)
    o1, r1, f1 = run(cfg.with_launch(256, 0, ONE), rho0, 30)
    o2, r2, f2 = run(cfg.with_launch(256, 0, TWO), rho0, 30)
    assert o1["flags"] == o2["flags"]
    assert np.array_equal(f1, f2, equal_nan=True)


def test_fe_two_step_domain_flags():
    """A density past the EOS domain (C-S b rho / 4 >= 1, put into the
    populations after the start) and a NaN elsewhere are flagged by both
    paths, with the same flags."""
    import torch
    cfg = fe_cfg(260, 20, a=0.25, Tr=0.75, tau=FE_TAU)
    rho0 = noisy(cfg)
    flags = []
    for kf in (ONE, TWO):
        sim = lbm.Simulation(cfg.with_launch(256, 0, kf), torch.from_numpy(rho0).to(torch_dev()))
        f = sim.populations()
        f[0, 7, 100] += 1.2  # b rho / 4 > 1 at (100, 7)
        f[0, 15, 250] = float("nan")
        sim.set_populations(f.contiguous())
        sim.step(2)
        flags.append(sim.observe()["flags"])
        sim.close()
    assert flags[0] & lbm.FLAG_EOS_DOMAIN and flags[0] & lbm.FLAG_NONFINITE
    assert flags[0] == flags[1]


@pytest.mark.parametrize("variant", list(FE_VARIANTS))
@pytest.mark.parametrize("prec", [lbm.FP64, lbm.FP32_SHIFTED])
def test_fe_two_step_throughput_lattice(prec, variant):
    """4096^2 spinodal (C-S a = 0.25, Tr = 0.85, kappa = 0.5, tau_e = 0.75),
    the benchmark's free-energy workload: equal to the single-step path."""
    E, a, b, R = lbm.EOS_CS, 0.25, 4.0, 1.0
    T = cs_T(a, 0.85)
    rl, rv, _ = th.maxwell(E, a, b, R, T)
    rho0 = inputs.spinodal(4096, 4096, 0.5 * (rl + rv), 0.01, seed=3)
    tau = [1.0] * 9
    tau[1] = 0.75
    cfg = lbm.Config(4096, 4096, lbm.MODEL_FE, E, a, b, R, T, tau=tau, kappa=0.5, precision=prec)
    two = FE_VARIANTS[variant]
    o1, r1, f1 = run(cfg.with_launch(256, 0, ONE), rho0, 6)
    o2, r2, f2 = run(cfg.with_launch(256, 0, two), rho0, 6)
    assert o1["flags"] == o2["flags"]
    assert np.array_equal(r1, r2)
    assert np.array_equal(f1, f2)
