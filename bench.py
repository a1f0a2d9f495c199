#!/usr/bin/env python3
"""Throughput benchmark of the fused D2Q9 multiphase step on one MI355X.

Workload (default): 4096 x 4096 periodic lattice, spinodal decomposition
from the mean density (rho_l + rho_v)/2 with a seeded uniform +-1 %
perturbation, Carnahan-Starling EOS (a = 0.25, b = 4, R = 1, the paper's
EOS and droplet parameters) at Tr = 0.85; both models (pseudopotential and
well-balanced free energy), FP64 storage for the headline number,
FP32-shifted storage reported beside it.  ``--workload vdw-spinodal`` runs
the van der Waals (a = 9/49, b = 2/21, R = 1) Tr = 0.7 variant, which
leaves the EOS domain within ~50 steps on both models; its lines carry the
non-finite flags and its free-energy timing is inflated by the special-value
paths of log on non-finite data.  One
step = one update of each model's lattice.  Inputs are resident in HBM
before the timed region; the timed region is K back-to-back steps per model
(two per launch where the two-step kernels apply: periodic lattices at
least 256 wide, both models) bracketed by events recorded on the library's
stream.

Prints one JSON line (metric, value in MLUPS, roofline of the dominant
kernel, CPU oracle baseline on the host cores).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VDW = dict(a=9 / 49, b=2 / 21, R=1.0)
CS = dict(a=0.25, b=4.0, R=1.0)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("lbm_kernels.hip", "lbm_math.h"):
        with open(os.path.join(ROOT, "paper_2403_11167_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def workload(name: str, n: int):
    """(Config factory, rho0 numpy array, description)."""
    from paper_2403_11167_amd import inputs, lbm
    if name == "vdw-spinodal":
        e, eos, Tr = VDW, lbm.EOS_VDW, 0.7
    elif name == "cs-spinodal":
        e, eos, Tr = CS, lbm.EOS_CS, 0.85
    else:
        raise SystemExit(f"unknown workload {name}")
    Tc, _, _ = lbm.eos_critical(eos, e["a"], e["b"], e["R"])
    T = Tr * Tc
    rl, rv, _ = lbm.maxwell(eos, e["a"], e["b"], e["R"], T)
    rho0 = inputs.spinodal(n, n, 0.5 * (rl + rv), 0.01, seed=3)

    def cfg(model: int, precision: int) -> "lbm.Config":
        tau = [1.0] * 9
        if model == lbm.MODEL_FE:
            tau[1] = 0.75  # nu = c_s^2/2, nu_B = c_s^2/3 (Sec. 5.1)
            return lbm.Config(n, n, model, eos, e["a"], e["b"], e["R"], T, tau=tau, kappa=0.5,
                              precision=precision)
        return lbm.Config(n, n, model, eos, e["a"], e["b"], e["R"], T, tau=tau,
                          precision=precision)

    desc = (f"{n}x{n} periodic spinodal decomposition, {'vdW a=9/49 b=2/21' if eos == lbm.EOS_VDW else 'C-S a=0.25 b=4'}"
            f" R=1, Tr={Tr}, rho0=(rho_l+rho_v)/2*(1+0.01*U(-1,1)) seed 3")
    return cfg, rho0, desc


def time_variant(cfg, rho0_dev, steps: int, warmup: int):
    """(seconds for `steps` steps on the library's stream, final obs, the
    launch shape that carried them)."""
    import torch
    from paper_2403_11167_amd import lbm
    sim = lbm.Simulation(cfg, rho0_dev)
    sim.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(sim.stream)
    sim.step(steps)
    stop.record(sim.stream)
    torch.cuda.synchronize()
    seconds = start.elapsed_time(stop) / 1e3
    obs = sim.observe(cfg.nx // 2, cfg.ny // 2)
    info = sim.launch_info()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return seconds, obs, info


def cpu_baseline(cfg_factory, rho0, target_seconds: float):
    """The FP64 oracle, as it stands, on the host cores: both models on the
    same 4096^2 initial state, k steps each with k chosen so that the sample
    takes about `target_seconds`."""
    import oracle
    from paper_2403_11167_amd import lbm

    def oparams(c):
        return oracle.OracleParams(c.nx, c.ny, c.model, c.eos, c.a, c.b, c.R, c.T, tau=list(c.tau),
                                   sigma_li=c.sigma_li, kappa_li=c.kappa_li, kappa_p=c.kappa_p,
                                   kappa=c.kappa)

    N = rho0.size
    total_nodes, total_t, steps_done = 0, 0.0, {}
    for model in (lbm.MODEL_P, lbm.MODEL_FE):
        s = oracle.Simulation(oparams(cfg_factory(model, lbm.FP64)), rho0)
        t0 = time.perf_counter()
        s.step(1)
        t1 = time.perf_counter() - t0
        k = max(1, int(target_seconds / 2 / max(t1, 1e-9)) - 1)
        t0 = time.perf_counter()
        s.step(k)
        dt = time.perf_counter() - t0
        total_nodes += N * (k + 1)
        total_t += dt + t1
        steps_done["P" if model == lbm.MODEL_P else "FE"] = k + 1
        del s
    return dict(value=total_nodes / total_t / 1e6, unit="MLUPS", cores=oracle.num_threads(),
                kind="oracle",
                sample=f"{int(math.sqrt(N))}^2 lattice of the same workload, FP64, "
                       f"{steps_done['P']} P steps and {steps_done['FE']} FE steps from the "
                       f"initial state ({total_t:.1f} s)")


def load_traffic(variant: str):
    """(HBM bytes per launch from the committed counter runs, kernel name);
    bytes are None unless the counters were taken on the current kernel
    source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None, None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None, None
    k = d.get("kernels", {}).get(variant)
    if k is None:
        return None, None
    name = k.get("name")
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None, name
    return k.get("bytes_per_launch"), name


def batch_roofline(dev, L=512, n=64, steps=200):
    """The batch kernels on the calibration's largest class: n flat-interface
    lattices of L x L per model (as many nodes as the 4096^2 lattice),
    FP32-shifted, 256-column strips, automatic segment heights, one check
    interval of `steps` lockstep steps after one of warm-up (which also fixes
    the heights), timed by the batch's own GPU clock.  Algorithmic bytes: 72
    per node update."""
    import torch
    from paper_2403_11167_amd import calibration as cal, lbm
    out = []
    for model in (lbm.MODEL_P, lbm.MODEL_FE):
        t = cal.Tuple4(model, 0.75, 5.0, 1.25)
        rl, rv, W = cal.initial_guess(t)
        rho = torch.from_numpy(cal.flat_rho0(L, L, rl, rv, W)).to(dev)
        cfg = cal.model_config(t, L, L, lbm.FP32_SHIFTED).with_launch(256, 0, 0)
        b = lbm.Batch([cfg] * n, [rho] * n)
        b.run(check_every=steps, du_tol=0.0, max_steps=steps)
        for i in range(n):
            b.set_limit(i, 1 << 40)  # resume after the warm-up interval
        s0 = b.stats()
        b.run(check_every=steps, du_tol=0.0, max_steps=steps)
        s1 = b.stats()
        li = b.launch_info(0)
        b.close()
        nu = s1["node_updates"] - s0["node_updates"]
        sec = (s1["gpu_ms"] - s0["gpu_ms"]) * 1e-3
        gbs = 72 * nu / sec / 1e9
        out.append(dict(model="P" if model == lbm.MODEL_P else "FE", lattices=n, L=L,
                        steps=steps, node_updates=nu, gpu_s=sec, ns_per_node_update=sec * 1e9 / nu,
                        hbm_gbs_algorithmic=gbs, frac_of_8tbs=gbs / 8000.0, launch=li))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--workload", default="cs-spinodal", choices=["cs-spinodal", "vdw-spinodal"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-vdw", action="store_true",
                    help="skip the van der Waals Tr = 0.7 variant lines")
    ap.add_argument("--no-calibration", action="store_true",
                    help="skip the surrogate-seeded vs plain batched calibration leg")
    ap.add_argument("--no-options", action="store_true",
                    help="skip the general-kernel lines (walls, collision drive, A != 0)")
    ap.add_argument("--calib-train", type=int, default=2000)
    ap.add_argument("--calib-held", type=int, default=256)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    ap.add_argument("--batch-roofline", action="store_true",
                    help="only time the batch kernels: 64 lattices of 512^2 per model")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for {args.gpus}); "
              "the lattice would shard by 2-D domain decomposition, not implemented here.",
              file=sys.stderr)
        raise SystemExit(2)

    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    from paper_2403_11167_amd import lbm
    lbm.lib()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")

    if args.copy_calibration:
        nbytes = 1 << 31
        a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": nbytes, "launches": 3}))
        return

    if args.batch_roofline:
        for line in batch_roofline(dev):
            print(json.dumps(line))
        return

    cfg_factory, rho0, desc = workload(args.workload, args.n)
    rho0_dev = torch.from_numpy(rho0).to(dev)
    N = args.n * args.n
    K, W = args.steps, args.warmup

    variants = {}
    precs = [("fp64", lbm.FP64)] + ([] if args.no_fp32 else [("fp32_shifted", lbm.FP32_SHIFTED)])
    for pname, prec in precs:
        for mname, model in (("P", lbm.MODEL_P), ("FE", lbm.MODEL_FE)):
            secs, obs, info = time_variant(cfg_factory(model, prec), rho0_dev, K, W)
            es = 8 if prec == lbm.FP64 else 4
            ms = secs * 1e3 / K
            variants[f"{mname}_{pname}"] = dict(
                mlups=N * K / secs / 1e6, ms_per_step=ms,
                hbm_gbs_algorithmic=18 * es * N / (ms * 1e-3) / 1e9,
                steps_per_launch=info["steps_per_launch"], strip=info["strip"],
                segment=info["segment"],
                flags=int(obs["flags"]), finite=bool(math.isfinite(obs["mass"])))
            print(f"# {mname} {pname}: {ms:.4f} ms/step, {N * K / secs / 1e6:.0f} MLUPS, "
                  f"flags {obs['flags']}", file=sys.stderr, flush=True)

    variants_vdw = None
    if not args.no_vdw and args.workload != "vdw-spinodal":
        vf, vrho0, vdesc = workload("vdw-spinodal", args.n)
        vr = torch.from_numpy(vrho0).to(dev)
        variants_vdw = {
            "workload": vdesc,
            "valid_run": False,
            "reason": ("not runnable as configured: the van der Waals spinodal at Tr = 0.7 "
                       "(p'(rho_m) = -0.43, against c_s^2 = 1/3) drives velocities to ~0.1 "
                       "within 20 steps; on the oracle (64^2) the free-energy lattice turns "
                       "non-finite by step 10-40 for every kappa in [0.02, 1] with tau_e "
                       "0.75 or 1, and the pseudopotential one clamps psi (imaginary at low "
                       "and at high density, so the EOS loses its repulsion) and leaves the "
                       "EOS domain.  The timings below are of those runs, for per-step cost "
                       "only; 'first_flag_step' is the first of the checks at 5, 10, 20, ... "
                       "steps that showed a flag."),
        }
        for mname, model in (("P", lbm.MODEL_P), ("FE", lbm.MODEL_FE)):
            sim = lbm.Simulation(vf(model, lbm.FP64), vr)
            first, done = None, 0
            for t in (5, 10, 20, 40, 80, 160, 320, 640):
                sim.step(t - done)
                done = t
                if sim.observe()["flags"]:
                    first = t
                    break
            sim.close()
            variants_vdw[f"{mname}_first_flag_step"] = first
        for pname, prec in precs:
            for mname, model in (("P", lbm.MODEL_P), ("FE", lbm.MODEL_FE)):
                secs, obs, _ = time_variant(vf(model, prec), vr, K, W)
                ms = secs * 1e3 / K
                variants_vdw[f"{mname}_{pname}"] = dict(
                    mlups=N * K / secs / 1e6, ms_per_step=ms, flags=int(obs["flags"]),
                    finite=bool(math.isfinite(obs["mass"])))
                print(f"# vdW {mname} {pname}: {ms:.4f} ms/step, flags {obs['flags']}",
                      file=sys.stderr, flush=True)
        del vr
        torch.cuda.empty_cache()

    # The options of the general step kernel on the same lattice, FP64: Zou-He
    # walls (Sec. 5.3) with a tangential and a normal force, the
    # droplet-collision drive (Sec. 5.4), A != 0 (Eq. 20; a velocity pass of
    # the same kernel runs before each step) and free-energy gravity
    # (Sec. 2.2, between walls).  Algorithmic bytes as for the periodic step.
    options = None
    if not args.no_options:
        import dataclasses
        ko = min(K, 500)
        options = {"steps": ko, "precision": "fp64"}
        cases = []
        for mname, model in (("P", lbm.MODEL_P), ("FE", lbm.MODEL_FE)):
            base = cfg_factory(model, lbm.FP64)
            cases.append((f"{mname}_walls", dataclasses.replace(base, walls=True, fx=1e-7,
                                                                fy=-1e-7)))
            cases.append((f"{mname}_drive", dataclasses.replace(base, ax=5e-6, x_split=args.n // 2)))
        cases.append(("FE_A", dataclasses.replace(cfg_factory(lbm.MODEL_FE, lbm.FP64), A=0.1)))
        fe = cfg_factory(lbm.MODEL_FE, lbm.FP64)
        cases.append(("FE_gravity", dataclasses.replace(fe, walls=True, g=1e-6,
                                                        grav_rho0=float(rho0.mean()),
                                                        grav_y0=(args.n - 1) / 2)))
        for name, cfg in cases:
            secs, obs, _ = time_variant(cfg, rho0_dev, ko, min(W, 20))
            ms = secs * 1e3 / ko
            gbs = 18 * 8 * N / (ms * 1e-3) / 1e9
            options[name] = dict(mlups=N * ko / secs / 1e6, ms_per_step=ms,
                                 hbm_gbs_algorithmic=gbs, frac=gbs / HBM_PEAK_GBS,
                                 flags=int(obs["flags"]), finite=bool(math.isfinite(obs["mass"])))
            print(f"# option {name}: {ms:.4f} ms/step, {gbs / HBM_PEAK_GBS:.3f} of HBM peak",
                  file=sys.stderr, flush=True)

    calib = None
    if not args.no_calibration:
        from paper_2403_11167_amd import calibration
        try:
            calib = calibration.benchmark(
                n_train=args.calib_train, n_held=args.calib_held,
                log=lambda m: print(f"# calibration: {m}", file=sys.stderr, flush=True))
        except Exception as e:  # report, do not lose the step measurement
            calib = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()

    t_p = variants["P_fp64"]["ms_per_step"]
    t_fe = variants["FE_fp64"]["ms_per_step"]
    ms_per_step = t_p + t_fe
    value = 2 * N / (ms_per_step * 1e-3) / 1e6

    # the dominant kernel: the slower model's FP64 step kernel.  One launch
    # advances steps_per_launch time steps; its algorithmic bytes are those
    # of that many node-updates (9 population reads + 9 writes each, FP64),
    # its duration that many times the measured time per step
    dom = "P_fp64" if t_p >= t_fe else "FE_fp64"
    spl = variants[dom]["steps_per_launch"]
    launch_ms = spl * max(t_p, t_fe)
    algo_bytes = spl * 18 * 8 * N
    achieved = algo_bytes / (launch_ms * 1e-3) / 1e9
    traffic, kname = load_traffic(dom)
    roofline = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                    kernel=kname or dom, variant=dom, steps_per_launch=spl,
                    algorithmic_bytes_per_launch=algo_bytes, launch_ms=launch_ms)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg_factory, rho0, args.cpu_seconds)

    line = {
        "metric": "MLUPS + HBM GB/s % peak (4096\u00b2 D2Q9); calibration runs/sec, surrogate vs plain",
        "value": value,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "lattice": f"{args.n}x{args.n}",
                   "methods": ["pseudopotential (P)", "well-balanced free energy (FE)"],
                   "step": "one update of each model's lattice",
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
        "variants_vdw_spinodal": variants_vdw,
        "variants_options": options,
        "calibration": calib,
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
