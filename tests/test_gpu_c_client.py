"""The C ABI from plain C: a client linked only against liblbm.so and the
HIP runtime (no Python in the process) runs a droplet, and its observables
equal the oracle's."""
import json
import math
import os
import subprocess

import pytest

import oracle
from oracle import theory as th
from paper_2403_11167_amd import inputs, lbm
from paper_2403_11167_amd import build as pkg_build

pytestmark = pytest.mark.gpu


def check_against_oracle(got, model, nx, ny, steps):
    a, b, R = 0.25, 4.0, 1.0
    T = 0.8 * th.critical(th.CS, a, b, R)[0]
    rl, rv, _ = th.maxwell(th.CS, a, b, R, T)
    tau = [1.0] * 9
    if model == lbm.MODEL_FE:
        tau[1] = 0.75
        op = oracle.OracleParams(nx, ny, oracle.MODEL_FE, oracle.EOS_CS, a, b, R, T, tau=tau,
                                 kappa=0.5)
    else:
        tau[4] = tau[6] = 1 / 1.99
        sig, kp, kli = lbm.match_p_to_fe(lbm.EOS_CS, a, b, R, T, 0.5, 0.0)
        op = oracle.OracleParams(nx, ny, oracle.MODEL_P, oracle.EOS_CS, a, b, R, T, tau=tau,
                                 sigma_li=sig, kappa_p=kp, kappa_li=kli)
    rho0 = inputs.droplet(nx, ny, rl, rv, radius=0.25 * min(nx, ny), width=5.0)
    s = oracle.Simulation(op, rho0)
    s.step(steps)
    ref = s.observe(nx // 2, ny // 2)
    assert got["steps"] == steps and got["flags"] == 0 == ref["flags"]
    assert math.isclose(got["mass"], ref["mass"], rel_tol=1e-12)
    assert math.isclose(got["mass0"], float(rho0.sum()), rel_tol=1e-12)
    assert math.isclose(got["rho_in"], ref["rho_in"], rel_tol=1e-10)
    assert math.isclose(got["rho_out"], ref["rho_out"], rel_tol=1e-10)
    assert math.isclose(got["dp"], ref["dp"], rel_tol=1e-7)
    assert math.isclose(got["r_equimolar"], ref["r_equimolar"], rel_tol=1e-9)


@pytest.mark.parametrize("model", [lbm.MODEL_P, lbm.MODEL_FE])
def test_c_client_matches_oracle(model):
    assert os.path.exists(pkg_build.DEMO), "build the library first (it builds the C client)"
    nx, ny, steps = 130, 98, 150
    res = subprocess.run([pkg_build.DEMO, str(model), str(nx), str(ny), str(steps)],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    got = json.loads(res.stdout.strip().splitlines()[-1])
    check_against_oracle(got, model, nx, ny, steps)


def test_c_client_batch_matches_oracle():
    """The batch entry points from plain C: both models' droplets in one
    paired batch, each equal to its own oracle run."""
    assert os.path.exists(pkg_build.DEMO), "build the library first (it builds the C client)"
    nx, ny, steps = 130, 98, 150
    res = subprocess.run([pkg_build.DEMO, "batch", str(nx), str(ny), str(steps)],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    lines = [json.loads(l) for l in res.stdout.strip().splitlines() if l.startswith("{")]
    assert [g["model"] for g in lines] == [lbm.MODEL_P, lbm.MODEL_FE]
    for got in lines:
        check_against_oracle(got, got["model"], nx, ny, steps)
