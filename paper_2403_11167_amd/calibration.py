"""Calibration runs: equilibrium properties of the two models as functions of
(model, Tr, width parameter w, kappa), computed by batches of lattices.

The paper sets the pseudopotential parameters by theory (Sec. 3, App. B:
sigma^Li from the mechanical-stability condition; Sec. 4 / App. C: kappa^P
for the interface width, kappa^Li for the surface tension) and notes that
at low Tr they must instead be found by preliminary simulations (Sec. 5.1,
5.2).  A calibration unit here is one flat-interface and one droplet
lattice per tuple, run to equilibrium in a batch; the labels are

  rho_l, rho_v  bulk densities of the flat interface (Sec. 5.1),
  W             its max-slope width (rho_l - rho_v) / max |d_x rho|,
  sigma         surface tension from Laplace's law, dp * R (Sec. 5.2).

Tuple meaning (both models share the EOS: Carnahan-Starling, a = 0.25,
b = 4, R = 1, the EOS of the paper's Sec. 5.1 runs):
  kappa is the reduced gradient coefficient kappa_FE / a.  At fixed Tr the
      pressure scales with a, so the planar free-energy profile (Eq. 26)
      depends on kappa_FE / a only; kappa = 2 is the paper's a = 0.25,
      kappa_FE = 0.5 pair.  (Taking kappa_FE = kappa directly puts most of
      the range beyond the free-energy model's short-wave stability limit,
      which a uniform liquid at rest already shows near kappa_FE rho_l = 1/3.)
  P   sigma^Li from App. B at Tr; kappa^P so that the Eq. 44 max-slope width
      equals w; kappa^Li so that the Eq. 46 surface tension equals the FE
      one (Eq. 26) at kappa_FE.  tau = 1 except tau_q = 1/1.99 (Sec. 5.2).
  FE  kappa_FE = a kappa; tau = 1 except tau_e = 0.75 (Sec. 5.1).
Plain initial profiles are tanh profiles between the Maxwell densities with
width w (FE: width w as well; its equilibrium width is set by kappa).
Seeded initial profiles use predicted (rho_l, rho_v, W) instead.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

from . import inputs, lbm

EOS = lbm.EOS_CS
A, B, RGAS = 0.25, 4.0, 1.0
TR_RANGE = (0.5, 0.95)
W_RANGE = (2.0, 8.0)
KAPPA_RANGE = (0.5, 2.0)
SIZES = (64, 128, 256, 512)


@dataclass
class Tuple4:
    model: int
    Tr: float
    w: float
    kappa: float


def sample_tuples(n: int, seed: int):
    """n tuples with model uniform in {P, FE}, Tr ~ U[0.5, 0.95],
    w ~ U[2, 8], kappa ~ U[0.5, 2] (numpy default_rng(seed))."""
    rng = np.random.default_rng(seed)
    return [Tuple4(int(rng.integers(0, 2)), float(rng.uniform(*TR_RANGE)),
                   float(rng.uniform(*W_RANGE)), float(rng.uniform(*KAPPA_RANGE)))
            for _ in range(n)]


def sample_sizes(n: int, seed: int):
    rng = np.random.default_rng(seed + 1000)
    return [int(SIZES[rng.integers(0, len(SIZES))]) for _ in range(n)]


_TC = None


def critical_T():
    global _TC
    if _TC is None:
        _TC = lbm.eos_critical(EOS, A, B, RGAS)[0]
    return _TC


def kappa_fe(t: Tuple4) -> float:
    return A * t.kappa


_P_MATCH: dict = {}


def p_match(Tr: float, kfe: float, w: float):
    """(sigma^Li, kappa^P, kappa^Li) of a pseudopotential tuple (lbm.match_p_to_fe,
    kept per tuple: its planar-theory tabulations take milliseconds, and a
    tuple's flat and droplet lattices share the result)."""
    key = (Tr, kfe, w)
    if key not in _P_MATCH:
        _P_MATCH[key] = lbm.match_p_to_fe(EOS, A, B, RGAS, Tr * critical_T(), kfe, w)
    return _P_MATCH[key]


def prefill_p_match(tuples, workers: int = 16):
    """Compute p_match for the pseudopotential tuples not computed yet on a
    thread pool: the library call runs without the interpreter lock and
    has no shared state, and each result depends on its tuple alone."""
    from concurrent.futures import ThreadPoolExecutor
    keys = sorted({(t.Tr, kappa_fe(t), t.w) for t in tuples if t.model == lbm.MODEL_P}
                  - set(_P_MATCH))
    if len(keys) < 2:
        return
    lib = lbm.lib()  # load the library before the threads call it
    assert lib is not None
    Tc = critical_T()
    with ThreadPoolExecutor(max_workers=max(1, min(workers, os.cpu_count() or 1))) as ex:
        res = list(ex.map(lambda k: lbm.match_p_to_fe(EOS, A, B, RGAS, k[0] * Tc, k[1], k[2]),
                          keys))
    _P_MATCH.update(zip(keys, res))


def model_config(t: Tuple4, nx: int, ny: int, precision: int) -> lbm.Config:
    T = t.Tr * critical_T()
    tau = [1.0] * 9
    if t.model == lbm.MODEL_P:
        sig, kp, kli = p_match(t.Tr, kappa_fe(t), t.w)
        tau[4] = tau[6] = 1.0 / 1.99
        return lbm.Config(nx, ny, lbm.MODEL_P, EOS, A, B, RGAS, T, tau=tau, sigma_li=sig,
                          kappa_p=kp, kappa_li=kli, precision=precision)
    tau[1] = 0.75
    return lbm.Config(nx, ny, lbm.MODEL_FE, EOS, A, B, RGAS, T, tau=tau, kappa=kappa_fe(t),
                      precision=precision)


def initial_guess(t: Tuple4):
    """Plain initial profile parameters: Maxwell densities and width w."""
    T = t.Tr * critical_T()
    rl, rv, _ = lbm.maxwell(EOS, A, B, RGAS, T)
    return rl, rv, t.w


def flat_rho0(L: int, ny: int, rl: float, rv: float, W: float):
    return inputs.planar_slab(L, ny, rl, rv, width=max(W, 1.0))


def droplet_rho0(L: int, rl: float, rv: float, W: float):
    return inputs.droplet(L, L, rl, rv, radius=L / 5.0, width=max(W, 1.0))


def laplace_densities(cfg: lbm.Config, rl: float, rv: float, sigma: float, R: float):
    """Bulk densities (inside, outside) of a droplet of radius R in
    equilibrium, to first order about the planar coexistence densities: the
    bulk pressures differ by sigma / R (Laplace's law, Sec. 5.2) and the
    chemical potential (mu_b, Eq. 29, d mu = dp / rho) is equal on both
    sides, so dp_in / rho_l = dp_out / rho_v.  Exact to first order for the
    thermodynamically consistent free-energy model; for the pseudopotential
    model it is the estimate of its Maxwell-close coexistence."""
    _, dpl = lbm.eos_eval(cfg.eos, cfg.a, cfg.b, cfg.R, cfg.T, rl)
    _, dpv = lbm.eos_eval(cfg.eos, cfg.a, cfg.b, cfg.R, cfg.T, rv)
    if not (dpl > 0 and dpv > 0):
        raise ValueError("densities on an unstable branch")
    dp_v = (sigma / R) * rv / (rl - rv)
    dp_l = (sigma / R) * rl / (rl - rv)
    return rl + dp_l / dpl, rv + dp_v / dpv


def flat_labels(rho: np.ndarray):
    """(rho_l, rho_v, W) of a flat-interface equilibrium (rows identical).
    The bulk densities are the extremes of the profile averaged over
    neighbouring columns, which removes the free-energy model's odd-even
    mode (a density alternating between the two parity sublattices, which
    its stationary states admit); the central-difference slope compares
    nodes of one parity and does not see it."""
    prof = rho.mean(axis=0)
    pair = 0.5 * (prof + np.roll(prof, 1))
    rl, rv = float(pair.max()), float(pair.min())
    slope = np.abs(np.roll(prof, -1) - np.roll(prof, 1)).max() / 2
    return rl, rv, (rl - rv) / slope if slope > 0 else float("nan")


def droplet_sigma(obs: dict) -> float:
    """Laplace's law in 2-D: sigma = dp R with the equimolar radius, from the
    probe densities of lbm_observe (single nodes)."""
    return float(obs["dp"] * obs["r_equimolar"])


def droplet_sigma_field(rho: np.ndarray, cfg: lbm.Config):
    """(sigma, contrast) of a droplet centred at (nx/2, ny/2) from its
    density field: Laplace's law sigma = dp R_e (Sec. 5.2), with the inside
    and outside densities averaged over the 2 x 2 blocks at the centre and
    at the diagonally opposite corner, so that the odd-even mode of the
    free-energy model (one parity sublattice above the other) cancels; the
    single-node probes read it, and two runs of the same droplet from
    different starts, which settle with different amplitudes of that mode,
    then disagree by a few percent in sigma.  R_e is the equimolar radius
    from the total mass and the same block densities."""
    ny, nx = rho.shape
    cy, cx = ny // 2, nx // 2
    rin = float(rho[cy - 1:cy + 1, cx - 1:cx + 1].mean())
    rout = float(rho[np.ix_([ny - 1, 0], [nx - 1, 0])].mean())
    contrast = rin - rout
    if not (contrast > 0 and math.isfinite(contrast)):
        return math.nan, contrast
    Re = math.sqrt(max(float(rho.sum()) - rho.size * rout, 0.0) / (math.pi * contrast))
    try:
        pin = lbm.eos_eval(cfg.eos, cfg.a, cfg.b, cfg.R, cfg.T, rin)[0]
        pout = lbm.eos_eval(cfg.eos, cfg.a, cfg.b, cfg.R, cfg.T, rout)[0]
    except lbm.LbmError:  # a lattice that left the EOS domain has no label
        return math.nan, contrast
    return float((pin - pout) * Re), contrast


def _shape(size):
    """(flat nx, flat ny, droplet L) from an int L (both L x L) or a triple."""
    if isinstance(size, (tuple, list)):
        return tuple(int(v) for v in size)
    return int(size), int(size), int(size)


def with_tile(cfg: lbm.Config, tiles) -> lbm.Config:
    """cfg with the batch tile shape of its size class (model, nx, ny) from
    `tiles` (autotune_batch_tiles), if listed there."""
    if not tiles:
        return cfg
    tx_ty = tiles.get((cfg.model, cfg.nx, cfg.ny))
    if tx_ty is None:
        return cfg
    return cfg.with_launch(int(tx_ty[0]), int(tx_ty[1]), 0)


def build_problems(tuples, sizes, precision, guesses=None, tiles=None):
    """Configs and initial fields for one flat and one droplet lattice per
    tuple.  sizes: per tuple an int L (flat and droplet L x L) or a triple
    (flat nx, flat ny, droplet L).  guesses: per-tuple (rho_l, rho_v, W)
    (None: plain guesses).  tiles: batch tile shape per size class (see
    autotune_batch_tiles)."""
    prefill_p_match(tuples)
    cfgs, rho0s, meta = [], [], []
    for k, (t, size) in enumerate(zip(tuples, sizes)):
        g = guesses[k] if guesses is not None else initial_guess(t)
        rl, rv, W = g[:3]
        fx, fy, L = _shape(size)
        cfgs.append(with_tile(model_config(t, fx, fy, precision), tiles))
        rho0s.append(flat_rho0(fx, fy, rl, rv, W))
        meta.append((k, "flat"))
        cd = model_config(t, L, L, precision)
        dl, dv = rl, rv
        if len(g) > 3 and g[3] > 0:
            try:
                dl, dv = laplace_densities(cd, rl, rv, g[3], L / 5.0)
            except (ValueError, lbm.LbmError):
                dl, dv = rl, rv
            if not (0 < dv < dl):
                dl, dv = rl, rv
        cfgs.append(with_tile(cd, tiles))
        rho0s.append(droplet_rho0(L, dl, dv, W))
        meta.append((k, "droplet"))
    return cfgs, rho0s, meta


# (strip width, segment height); height 0: chosen by the batch for each
# group from its active lattices at every retirement.  Fixed heights are
# not candidates: timed on a full class, the best of them beats the
# automatic height by a few per cent, but it stays when the class has
# retired down to a few lattices, where it is several times slower.
TILE_CANDIDATES = ((64, 0), (256, 0))


def class_counts(tuples, sizes):
    """Lattices per size class (model, L): each tuple has a flat and a
    droplet lattice of its model."""
    out = {}
    for t, size in zip(tuples, sizes):
        fx, fy, L = _shape(size)
        for key in ((t.model, fx, fy), (t.model, L, L)):
            out[key] = out.get(key, 0) + 1
    return out


def autotune_batch_tiles(precision=lbm.FP32_SHIFTED, sizes=SIZES, steps=100, nodes=1 << 20,
                         counts=None, log=None):
    """The batch tile shape (tile_x, tile_y) of each size class (model, nx, ny)
    of a calibration: for every class, a batch of flat-interface lattices of
    that class (counts[class] of them when given, the class's share of the
    batch to be run; else the classes (model, L, L) for L in sizes, about
    `nodes` nodes each; mid-range tuple Tr = 0.75, w = 5, kappa = 1.25) runs
    `steps` lockstep steps per candidate shape in one check interval (as in
    a run, the last steps of an interval are single steps), timed by the
    batch's own GPU clock (lbm_batch_stats).  Strips of 256 columns (two
    steps per launch) are tried where nx >= 128; the least GPU time per node
    update wins.  Returns {(model, nx, ny): (tile_x, tile_y)} and the
    timings."""
    import torch
    say = log or (lambda *a: None)
    dev = torch.device("cuda:0")
    if counts:
        classes = sorted(counts)
    else:
        classes = [(m, L, L) for m in (lbm.MODEL_P, lbm.MODEL_FE) for L in sizes]
    best, table = {}, []
    for model, nx, ny in classes:
        t = Tuple4(model, 0.75, 5.0, 1.25)
        rl, rv, W = initial_guess(t)
        n = (counts or {}).get((model, nx, ny), 0) or max(2, nodes // (nx * ny))
        rho = torch.from_numpy(flat_rho0(nx, ny, rl, rv, W)).to(dev)
        timings = []
        for tx, ty in TILE_CANDIDATES:
            if (tx == 256 and nx < 128) or ty > ny:
                continue
            cfg = model_config(t, nx, ny, precision).with_launch(tx, ty, 0)
            b = lbm.Batch([cfg] * n, [rho] * n)
            b.run(check_every=steps, du_tol=0.0, max_steps=steps)
            st = b.stats()
            b.close()
            timings.append((st["gpu_ms"] * 1e6 / max(st["node_updates"], 1), tx, ty))
        ns, tx, ty = min(timings)
        best[(model, nx, ny)] = (tx, ty)
        name = "P" if model == lbm.MODEL_P else "FE"
        table.append(dict(model=name, nx=nx, ny=ny, lattices=n, tile_x=tx, tile_y=ty,
                          ns_per_node_update=ns,
                          candidates={f"{a}x{c}": v for v, a, c in timings}))
        say(f"batch tiles: {name} {nx}x{ny} ({n} lattices): {tx}x{ty or 'auto'}, "
            f"{ns:.4f} ns per node update")
    return best, table


def pair_units(batch, meta):
    """The flat and the droplet lattice of each tuple form one unit: a tuple
    whose lattice goes unstable has no labels, so its other lattice retires
    (lbm_batch_set_partner) instead of running on to the step limit."""
    first = {}
    for i, (k, _) in enumerate(meta):
        if k in first:
            batch.set_partner(first[k], i)
        else:
            first[k] = i


def batch_measurement(batch, run_seconds: float, precision: int) -> dict:
    """GPU share and algorithmic bandwidth of a batch's runs: node updates
    times the 9 population reads and 9 writes of one update, over the GPU
    time of its chunks (events around each graph launch); gpu_busy is that
    GPU time over the wall time of the run calls."""
    st = batch.stats()
    es = 8 if precision == lbm.FP64 else 4
    sec = st["gpu_ms"] * 1e-3
    gbs = 18 * es * st["node_updates"] / sec / 1e9 if sec > 0 else math.nan
    return dict(node_updates=st["node_updates"], gpu_s=sec, chunks=st["chunks"],
                run_s=run_seconds, gpu_busy=sec / run_seconds if run_seconds > 0 else math.nan,
                hbm_gbs_algorithmic=gbs, frac_of_8tbs=gbs / 8000.0,
                bytes_per_node_update=18 * es)


def run_calibration(tuples, sizes, precision=lbm.FP32_SHIFTED, guesses=None,
                    check_every=200, du_tol=1e-9, max_steps=200000, tiles=None):
    """Run the flat + droplet pair of every tuple to equilibrium in one batch.
    Returns (labels, info): labels[k] = dict(rho_l, rho_v, W, sigma, ok) and
    info = dict(seconds, steps, states, steps_per_problem, ...).  The timed
    region covers everything from the tuples to the labels, as in
    run_seeded_calibration: the configs and initial fields, the batch
    (initial populations on the device), the run to retirement and the
    measurement of the labels."""
    import time

    import torch
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    cfgs, rho0s, meta = build_problems(tuples, sizes, precision, guesses, tiles)
    batch = lbm.Batch(cfgs, [torch.from_numpy(r).to(dev) for r in rho0s])
    pair_units(batch, meta)
    tr = time.perf_counter()
    steps = batch.run(check_every=check_every, du_tol=du_tol, max_steps=max_steps)
    run_s = time.perf_counter() - tr
    labels = measure(batch, cfgs, meta, len(tuples))
    seconds = time.perf_counter() - t0
    states, nsteps, du, flags = batch.state()
    meas = batch_measurement(batch, run_s, precision)
    batch.close()
    units = sum(1 for lab in labels if lab["ok"])
    info = dict(seconds=seconds, steps=steps, states=states, steps_per_problem=nsteps,
                problems=len(cfgs), converged_units=units,
                units_per_second=units / seconds if seconds > 0 else math.nan, batch=meas)
    return labels, info


def measure(batch, cfgs, meta, ntuples, which=None, labels=None,
            accept=(lbm.BATCH_CONVERGED,)):
    """Labels of every tuple (or of the tuple indices in `which`, updating
    `labels`) from the batch's current state.  A tuple is ok when both of its
    lattices are in an accepted state, finite, and its droplet is still a
    droplet."""
    states = batch.state()[0]
    if labels is None:
        labels = [dict(rho_l=math.nan, rho_v=math.nan, W=math.nan, sigma=math.nan, ok=True)
                  for _ in range(ntuples)]
    sel = set(range(ntuples)) if which is None else set(which)
    for k in sel:
        labels[k]["ok"] = True
    for i, (k, kind) in enumerate(meta):
        if k not in sel:
            continue
        labels[k]["ok"] = labels[k]["ok"] and states[i] in accept
        if kind == "flat":
            _, (rho, _, _) = batch.observe(i, fields=True)
            rl, rv, W = flat_labels(rho.cpu().numpy())
            labels[k].update(rho_l=rl, rho_v=rv, W=W)
        else:
            _, (rho, _, _) = batch.observe(i, fields=True)
            sig, contrast = droplet_sigma_field(rho.cpu().numpy(), cfgs[i])
            labels[k]["sigma"] = sig
            labels[k]["drop_contrast"] = contrast
    for k in sel:
        lab = labels[k]
        # a droplet that dissolved (or a vapour bubble) measures no surface tension
        if not (lab.get("drop_contrast", 0.0) > 0.5 * (lab["rho_l"] - lab["rho_v"])):
            lab["ok"] = False
    return labels


CS_LATTICE = 1.0 / math.sqrt(3.0)


def lattice_labels(batch, cfgs, i, kind):
    """Labels one lattice measures: (rho_l, rho_v, W) of a flat interface or
    (sigma, drop_contrast) of a droplet, from the batch's current state."""
    if kind == "flat":
        _, (rho, _, _) = batch.observe(i, fields=True)
        rl, rv, W = flat_labels(rho.cpu().numpy())
        return dict(rho_l=rl, rho_v=rv, W=W)
    _, (rho, _, _) = batch.observe(i, fields=True)
    sig, contrast = droplet_sigma_field(rho.cpu().numpy(), cfgs[i])
    return dict(sigma=sig, drop_contrast=contrast)


def lattice_agrees(kind, m, p, rtol_rho=0.01, rtol_sigma=0.03, rtol_w=0.05) -> bool:
    """Verification of one lattice against the prediction p = (rho_l, rho_v,
    sigma, W): a flat lattice's measured densities within rtol_rho and width
    within rtol_w; a droplet's sigma within rtol_sigma, with the droplet
    still a droplet (core-to-far-field contrast above half the predicted
    density gap).  A NaN measurement never agrees."""
    if kind == "flat":
        return bool(abs(m["rho_l"] / p[0] - 1) <= rtol_rho and abs(m["rho_v"] / p[1] - 1) <= rtol_rho
                    and abs(m["W"] / p[3] - 1) <= rtol_w)
    return bool(m["drop_contrast"] > 0.5 * (p[0] - p[1])
                and abs(m["sigma"] / p[2] - 1) <= rtol_sigma)


def run_seeded_calibration(tuples, sizes, surrogate, precision=lbm.FP32_SHIFTED,
                           check_every=200, du_tol=1e-9, max_steps=200000,
                           crossings=8.0, rtol_rho=0.01, rtol_sigma=0.03, rtol_w=0.05,
                           tiles=None):
    """Calibration with the surrogate in front of the method.

    1. The surrogate predicts (rho_l, rho_v, sigma, W) for every tuple and
       seeds both lattices with tanh profiles of the predicted densities and
       width (free-energy tuples: Maxwell densities, see seeded_guesses).
    2. Verification: each lattice runs at most `crossings` sound crossings
       of its box (max(nx, ny) / c_s steps each), retiring earlier if it
       converges.
    3. Each lattice is judged on the labels it measures: a flat lattice
       whose densities agree with the prediction within rtol_rho and width
       within rtol_w, or a droplet whose sigma agrees within rtol_sigma (and
       that is still a droplet), is done with its measured labels, as is a
       lattice that met the convergence rule; every other lattice keeps
       running from its current state to the plain method's convergence
       rule (the fallback), within the plain run's step budget: max_steps
       per lattice, the verification steps included.
    A tuple is valid when both its lattices are done (accepted or
    converged) and its droplet is still a droplet.  Returns (labels, info)
    like run_calibration; info counts the tuples with both lattices
    accepted after verification ("accepted"), the accepted lattices, and
    holds the prediction array."""
    import time

    import torch
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    pred = surrogate.predict(features(tuples))
    cfgs, rho0s, meta = build_problems(tuples, sizes, precision,
                                       seeded_guesses(pred, tuples=tuples), tiles)
    batch = lbm.Batch(cfgs, [torch.from_numpy(r).to(dev) for r in rho0s])
    pair_units(batch, meta)
    for i, c in enumerate(cfgs):
        v = crossings * max(c.nx, c.ny) / CS_LATTICE
        batch.set_limit(i, int(math.ceil(v / check_every)) * check_every)
    tr = time.perf_counter()
    steps = batch.run(check_every=check_every, du_tol=du_tol, max_steps=max_steps)
    run_s = time.perf_counter() - tr
    states = batch.state()[0]
    lat = [None] * len(cfgs)
    accepted = [False] * len(cfgs)
    resume = []
    for i, (k, kind) in enumerate(meta):
        if states[i] == lbm.BATCH_CONVERGED:
            lat[i] = lattice_labels(batch, cfgs, i, kind)
            continue
        if states[i] != lbm.BATCH_MAXSTEPS:
            continue  # unstable, or dropped with its partner
        m = lattice_labels(batch, cfgs, i, kind)
        if lattice_agrees(kind, m, pred[k], rtol_rho, rtol_sigma, rtol_w):
            lat[i], accepted[i] = m, True
        else:
            resume.append(i)
    # the same per-lattice budget as the plain run: max_steps in total,
    # verification steps included
    for i in resume:
        batch.set_limit(i, max_steps)
    tr = time.perf_counter()
    steps2 = batch.run(check_every=check_every, du_tol=du_tol, max_steps=max_steps) if resume else 0
    run_s += time.perf_counter() - tr
    states, nsteps, du, flags = batch.state()
    for i in resume:
        if states[i] == lbm.BATCH_CONVERGED:
            lat[i] = lattice_labels(batch, cfgs, i, meta[i][1])
    labels = [dict(rho_l=math.nan, rho_v=math.nan, W=math.nan, sigma=math.nan, ok=True)
              for _ in tuples]
    both = [0] * len(tuples)
    for i, (k, kind) in enumerate(meta):
        if lat[i] is None:
            labels[k]["ok"] = False
        else:
            labels[k].update(lat[i])
        both[k] += accepted[i]
    for lab in labels:
        if not (lab.get("drop_contrast", 0.0) > 0.5 * (lab["rho_l"] - lab["rho_v"])):
            lab["ok"] = False
    seconds = time.perf_counter() - t0
    meas = batch_measurement(batch, run_s, precision)
    batch.close()
    units = sum(1 for lab in labels if lab["ok"])
    n_acc = sum(1 for v in both if v == 2)
    info = dict(seconds=seconds, steps=steps + steps2, states=states, steps_per_problem=nsteps,
                problems=len(cfgs), converged_units=units,
                units_per_second=units / seconds if seconds > 0 else math.nan,
                accepted=n_acc, accepted_lattices=int(sum(accepted)),
                fallback=len(tuples) - n_acc, prediction=pred, batch=meas)
    return labels, info


def features(tuples) -> np.ndarray:
    """Surrogate inputs (model, Tr, w, kappa)."""
    return np.array([[t.model, t.Tr, t.w, t.kappa] for t in tuples], dtype=np.float64)


def targets(labels) -> np.ndarray:
    """Surrogate outputs (rho_l, rho_v, sigma, W)."""
    return np.array([[l["rho_l"], l["rho_v"], l["sigma"], l["W"]] for l in labels],
                    dtype=np.float64)


def valid(labels):
    """Mask of tuples whose flat and droplet lattices both converged to a
    two-phase state with finite labels."""
    y = targets(labels)
    return np.array([lab["ok"] for lab in labels]) & np.all(np.isfinite(y), axis=1) & \
        np.all(y > 0, axis=1)


def training_set(n_tuples: int, seed: int, size=(64, 8, 128), **kw):
    """Calibration labels for n_tuples sampled tuples on small lattices
    (flat 64 x 8, droplet 128 x 128 by default): (features, targets, info)
    with only valid tuples kept.  Keyword arguments go to run_calibration
    (tiles: from autotune_batch_tiles on class_counts of the same tuples)."""
    tuples = sample_tuples(n_tuples, seed)
    labels, info = run_calibration(tuples, [size] * n_tuples, **kw)
    m = valid(labels)
    return features(tuples)[m], targets(labels)[m], info


def seeded_guesses(pred, laplace: bool = True, tuples=None):
    """Initial-profile parameters (rho_l, rho_v, W[, sigma]) from surrogate
    predictions (n x 4: rho_l, rho_v, sigma, W); with sigma, droplets start
    from the Laplace-shifted bulk densities (laplace_densities).

    With tuples given, a free-energy tuple takes its bulk densities from the
    Maxwell construction instead: that model is thermodynamically
    consistent, its flat-interface densities meet the Maxwell rule to its
    discretisation error (Sec. 5.1, Table 1: 0.06 % in rho_v), closer than
    the surrogate predicts them (about 0.5 %), and near Tc an error of that
    size in the seed makes the interfaces travel to conserve mass, which
    relaxes slowly.  Its width and sigma still come from the surrogate.  The
    pseudopotential model's coexistence departs from the Maxwell rule, so
    its seed takes all four predictions."""
    out = []
    for k, p in enumerate(pred):
        rl, rv = float(p[0]), float(p[1])
        if tuples is not None and tuples[k].model == lbm.MODEL_FE:
            rl, rv, _ = initial_guess(tuples[k])
        out.append((rl, rv, float(p[3]), float(p[2])) if laplace else (rl, rv, float(p[3])))
    return out


def compare(labels_a, labels_b):
    """Relative differences of b against a on tuples valid in both:
    dict(rho_l, rho_v, sigma, W) of arrays, plus the mask."""
    m = valid(labels_a) & valid(labels_b)
    ya, yb = targets(labels_a)[m], targets(labels_b)[m]
    rel = np.abs(yb / ya - 1)
    return {k: rel[:, i] for i, k in enumerate(("rho_l", "rho_v", "sigma", "W"))}, m


def by_size(rel, m, sizes):
    """Agreement of the labels compared by `compare` (rel, m) per lattice size
    L of the tuple, and over L >= 128: the 64^2 droplets (R = L/5 = 12.8)
    are only a few interface widths across."""
    L = np.array([_shape(v)[2] for v in sizes])[m]

    def part(sel):
        return dict(tuples=int(sel.sum()),
                    **{f"{k}_within_{int(100 * t)}pct": (float(np.mean(rel[k][sel] <= t))
                                                         if sel.any() else None)
                       for k, t in (("rho_l", 0.01), ("rho_v", 0.01), ("sigma", 0.03),
                                    ("sigma", 0.01), ("W", 0.03))})
    out = {str(v): part(L == v) for v in sorted(set(L.tolist()))}
    out["128_and_up"] = part(L >= 128)
    return out


def _stats(rel, tol):
    if len(rel) == 0:
        return dict(median=None, p95=None, max=None, frac_within=None, tol=tol)
    return dict(median=float(np.median(rel)), p95=float(np.percentile(rel, 95)),
                max=float(np.max(rel)), frac_within=float(np.mean(rel <= tol)), tol=tol)


def steps_by_class(tuples, sizes, info):
    """Median and maximum steps and the number of lattices that reached the
    step cap, per (model, kind, L) class of a calibration run."""
    out = {}
    for i, n in enumerate(info["steps_per_problem"]):
        k, kind = divmod(i, 2)
        t = tuples[k]
        key = f"{'P' if t.model == lbm.MODEL_P else 'FE'} {('flat', 'droplet')[kind]} L={_shape(sizes[k])[0]}"
        out.setdefault(key, []).append((n, info["states"][i]))
    return {key: dict(lattices=len(v), median_steps=int(np.median([a for a, _ in v])),
                      max_steps=int(max(a for a, _ in v)),
                      at_cap=int(sum(1 for _, st in v if st == lbm.BATCH_MAXSTEPS)),
                      stalled=int(sum(1 for _, st in v if st == lbm.BATCH_STALLED)),
                      unstable=int(sum(1 for _, st in v if st in (lbm.BATCH_UNSTABLE,
                                                                    lbm.BATCH_DROPPED))))
            for key, v in sorted(out.items())}


TOLERANCES = dict(rho_l=0.01, rho_v=0.01, sigma=0.03, W=0.03)


def benchmark(n_train: int = 2000, n_held: int = 256, seed_train: int = 5, seed_held: int = 6,
              epochs: int = 400, crossings: float = 8.0, max_steps: int = 200000,
              train_size=(64, 8, 128), log=None):
    """Surrogate-seeded against plain calibration on held-out tuples.

    Trains the surrogate on equilibria of n_train sampled tuples (small
    lattices), then calibrates n_held held-out tuples (one flat and one
    droplet lattice each, L drawn from 64..512) twice: plain (Maxwell
    densities, width w, run to the convergence rule) and surrogate-seeded
    (run_seeded_calibration).  Returns a JSON-ready dict with wall times,
    converged tuples per second and the errors of the seeded labels and of
    the bare predictions against the plain labels."""
    import time

    import torch
    say = log or (lambda *a: None)
    t0 = time.perf_counter()
    train_tiles, train_tile_table = autotune_batch_tiles(
        counts=class_counts(sample_tuples(n_train, seed_train), [train_size] * n_train), log=say)
    train_tune_s = time.perf_counter() - t0
    say(f"training set tiles tuned in {train_tune_s:.1f} s")
    t0 = time.perf_counter()
    x, y, info_t = training_set(n_train, seed_train, size=train_size, max_steps=max_steps,
                                tiles=train_tiles)
    gen_s = time.perf_counter() - t0
    say(f"training set: {len(x)} valid of {n_train} tuples in {gen_s:.1f} s")
    sur = lbm.Surrogate(inputs.mlp_initial_params(0))
    sur.set_target_scaling(y)
    t1 = time.perf_counter()
    losses = sur.fit(x, y, epochs=epochs, batch=256, lr=3e-3, seed=1, lr_final=1e-4)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    say(f"training: {train_s:.2f} s, loss {losses[0]:.4f} -> {losses[-1]:.2e}")
    tup = sample_tuples(n_held, seed_held)
    sizes = sample_sizes(n_held, seed_held)
    feats = features(tup)
    sur.predict(feats[:1])  # first call loads the kernels
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pred_only = sur.predict(feats)
    infer_s = time.perf_counter() - t2
    t3 = time.perf_counter()
    tiles, tile_table = autotune_batch_tiles(counts=class_counts(tup, sizes), log=say)
    tune_s = time.perf_counter() - t3
    lab_p, inf_p = run_calibration(tup, sizes, max_steps=max_steps, tiles=tiles)
    say(f"plain: {inf_p['seconds']:.1f} s, {inf_p['converged_units']} tuples")
    # the reproducibility floor: the plain method again from other starts
    # (interfaces 1.6 times wider), to the same convergence rule
    other = [(rl, rv, 1.6 * W) for rl, rv, W in (initial_guess(t) for t in tup)]
    lab_b, inf_b = run_calibration(tup, sizes, max_steps=max_steps, tiles=tiles, guesses=other)
    say(f"plain from other starts: {inf_b['seconds']:.1f} s, {inf_b['converged_units']} tuples")
    rel_pp, m_pp = compare(lab_p, lab_b)
    lab_s, inf_s = run_seeded_calibration(tup, sizes, sur, max_steps=max_steps,
                                          crossings=crossings, tiles=tiles)
    say(f"seeded: {inf_s['seconds']:.1f} s, {inf_s['converged_units']} tuples, "
        f"{inf_s['accepted']} accepted after verification")
    rel, m = compare(lab_p, lab_s)
    big = by_size(rel, m, sizes)["128_and_up"]
    if big["tuples"]:
        say(f"seeded vs plain, L >= 128 ({big['tuples']} tuples): sigma within 3 %: "
            f"{100 * big['sigma_within_3pct']:.1f} %, rho_v within 1 %: "
            f"{100 * big['rho_v_within_1pct']:.1f} %")
    pred = pred_only
    yp = targets(lab_p)
    mp = valid(lab_p)
    prel = np.abs(pred[mp] / yp[mp] - 1)
    names = ("rho_l", "rho_v", "sigma", "W")
    return dict(
        held_out=dict(tuples=n_held, lattices=2 * n_held, seed=seed_held,
                      sizes="L x L, L uniform in {64,128,256,512}; flat slab + droplet R = L/5",
                      precision="fp32_shifted"),
        training=dict(tuples=n_train, valid=int(len(x)), lattices=2 * n_train,
                      size=list(train_size), generation_s=gen_s, train_s=train_s,
                      tile_tuning_s=train_tune_s, tiles=train_tile_table,
                      epochs=epochs, loss_first=float(losses[0]), loss_last=float(losses[-1])),
        plain=dict(seconds=inf_p["seconds"], tuples_converged=inf_p["converged_units"],
                   tuples_per_s=inf_p["units_per_second"], lockstep_steps=inf_p["steps"],
                   batch=inf_p["batch"]),
        seeded=dict(seconds=inf_s["seconds"], tuples_converged=inf_s["converged_units"],
                    tuples_per_s=inf_s["units_per_second"], lockstep_steps=inf_s["steps"],
                    accepted_after_verification=inf_s["accepted"],
                    lattices_accepted_after_verification=inf_s["accepted_lattices"],
                    fallback=inf_s["fallback"], verification_crossings=crossings,
                    batch=inf_s["batch"]),
        speedup=inf_p["seconds"] / inf_s["seconds"],
        batch_tiles=dict(seconds=tune_s, classes=tile_table,
                         note="tile shape per size class, timed on batches of that class "
                              "before both legs (autotune_batch_tiles); not in either leg's time"),
        surrogate_only=dict(seconds=infer_s, tuples=n_held,
                            speedup_vs_plain=inf_p["seconds"] / infer_s if infer_s > 0 else None,
                            note="labels predicted directly by the trained network (BF16 "
                                 "inputs, FP32 accumulate) in place of the plain runs; "
                                 "accuracy in surrogate_vs_plain"),
        seeded_vs_plain={k: _stats(rel[k], TOLERANCES[k]) for k in names},
        seeded_vs_plain_by_size=by_size(rel, m, sizes),
        plain_vs_plain_by_size=by_size(rel_pp, m_pp, sizes),
        plain_vs_plain=dict(
            note="the plain calibration run a second time from starts with 1.6 times wider "
                 "interfaces: how reproducible the labels of the method itself are",
            tuples=int(m_pp.sum()), seconds=inf_b["seconds"],
            sigma_within_1pct=_stats(rel_pp["sigma"], 0.01)["frac_within"],
            **{k: _stats(rel_pp[k], TOLERANCES[k]) for k in names}),
        plain_steps_by_class=steps_by_class(tup, sizes, inf_p),
        seeded_vs_plain_tuples=int(m.sum()),
        surrogate_vs_plain={k: _stats(prel[:, i], TOLERANCES[k]) for i, k in enumerate(names)},
    )

