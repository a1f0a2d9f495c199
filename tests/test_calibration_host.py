"""Host logic of the calibration driver (no device work): the seed of each
model and the per-lattice verification rule."""
import math

import numpy as np

from oracle import theory as th
from paper_2403_11167_amd import calibration as cal
from paper_2403_11167_amd import lbm


def test_free_energy_seed_takes_maxwell_densities():
    """A free-energy tuple is seeded with the Maxwell densities (the model
    meets the Maxwell rule, Sec. 5.1) and the predicted width and sigma; a
    pseudopotential tuple with all four predictions."""
    tuples = [cal.Tuple4(lbm.MODEL_FE, 0.8, 4.0, 1.0), cal.Tuple4(lbm.MODEL_P, 0.8, 4.0, 1.0)]
    pred = np.array([[0.31, 0.012, 0.02, 5.5], [0.32, 0.011, 0.03, 4.5]])
    g = cal.seeded_guesses(pred, tuples=tuples)
    T = 0.8 * cal.critical_T()
    rl, rv, _ = th.maxwell(th.CS, cal.A, cal.B, cal.RGAS, T)
    assert math.isclose(g[0][0], rl, rel_tol=1e-9) and math.isclose(g[0][1], rv, rel_tol=1e-9)
    assert g[0][2:] == (5.5, 0.02)
    assert g[1] == (0.32, 0.011, 4.5, 0.03)
    # without tuples every seed is the prediction
    assert cal.seeded_guesses(pred)[0] == (0.31, 0.012, 5.5, 0.02)


def test_lattice_verification_rule():
    p = (0.30, 0.010, 0.020, 5.0)
    flat = dict(rho_l=0.3025, rho_v=0.01009, W=5.2)
    assert cal.lattice_agrees("flat", flat, p)
    assert not cal.lattice_agrees("flat", dict(flat, rho_v=0.0102), p)  # 2 %
    assert not cal.lattice_agrees("flat", dict(flat, W=5.3), p)         # 6 %
    assert not cal.lattice_agrees("flat", dict(flat, rho_l=math.nan), p)
    drop = dict(sigma=0.0205, drop_contrast=0.25)
    assert cal.lattice_agrees("droplet", drop, p)
    assert not cal.lattice_agrees("droplet", dict(drop, sigma=0.0207), p)   # 3.5 %
    # a droplet that dissolved measures no surface tension
    assert not cal.lattice_agrees("droplet", dict(drop, drop_contrast=0.1), p)


def test_each_tuple_is_one_unit():
    """pair_units pairs the flat and the droplet lattice of each tuple, and
    nothing else."""
    class Rec:
        def __init__(self):
            self.pairs = []

        def set_partner(self, i, j):
            self.pairs.append((i, j))

    meta = [(0, "flat"), (0, "droplet"), (1, "flat"), (1, "droplet"), (2, "flat"), (2, "droplet")]
    r = Rec()
    cal.pair_units(r, meta)
    assert r.pairs == [(0, 1), (2, 3), (4, 5)]


def test_class_counts_cover_both_lattices_of_each_tuple():
    """The tile autotuner times each size class at the number of lattices it
    has in the batch: one flat and one droplet lattice per tuple, keyed by
    (model, nx, ny)."""
    tuples = [cal.Tuple4(lbm.MODEL_P, 0.8, 5.0, 1.0), cal.Tuple4(lbm.MODEL_FE, 0.8, 5.0, 1.0),
              cal.Tuple4(lbm.MODEL_P, 0.7, 4.0, 1.5)]
    counts = cal.class_counts(tuples, [256, 64, (64, 8, 128)])
    assert counts == {(lbm.MODEL_P, 256, 256): 2, (lbm.MODEL_FE, 64, 64): 2,
                      (lbm.MODEL_P, 64, 8): 1, (lbm.MODEL_P, 128, 128): 1}
    held = cal.sample_tuples(64, 6)
    sizes = cal.sample_sizes(64, 6)
    assert sum(cal.class_counts(held, sizes).values()) == 2 * 64


def test_parallel_p_match_equals_serial_calls():
    """The pseudopotential matching of a tuple (sigma^Li, kappa^P, kappa^Li,
    App. B and C) computed on a thread pool ahead of the configs equals the
    library call made directly, for every tuple."""
    tuples = [t for t in cal.sample_tuples(40, 21) if t.model == lbm.MODEL_P]
    assert len(tuples) > 5
    cal._P_MATCH.clear()
    cal.prefill_p_match(tuples, workers=4)
    for t in tuples:
        direct = lbm.match_p_to_fe(cal.EOS, cal.A, cal.B, cal.RGAS, t.Tr * cal.critical_T(),
                                   cal.kappa_fe(t), t.w)
        assert cal.p_match(t.Tr, cal.kappa_fe(t), t.w) == direct
    cfg = cal.model_config(tuples[0], 64, 64, lbm.FP32_SHIFTED)
    assert (cfg.sigma_li, cfg.kappa_p, cfg.kappa_li) == cal.p_match(
        tuples[0].Tr, cal.kappa_fe(tuples[0]), tuples[0].w)


def test_agreement_by_lattice_size():
    """by_size splits the label comparison by each tuple's lattice size and
    adds L >= 128; fractions count relative differences within tolerance."""
    def lab(s):
        return dict(rho_l=5.0, rho_v=0.5, W=6.0, sigma=s, ok=True)
    a = [lab(1.0), lab(1.0), lab(1.0), lab(1.0)]
    b = [lab(1.005), lab(1.05), lab(1.0), lab(1.02)]
    b[2]["ok"] = False
    rel, m = cal.compare(a, b)
    out = cal.by_size(rel, m, [64, 64, 128, 256])
    assert out["64"]["tuples"] == 2 and out["64"]["sigma_within_3pct"] == 0.5
    assert out["64"]["sigma_within_1pct"] == 0.5 and out["64"]["rho_v_within_1pct"] == 1.0
    assert "128" not in out  # its only tuple is not valid in both
    assert out["256"]["sigma_within_3pct"] == 1.0 and out["256"]["sigma_within_1pct"] == 0.0
    assert out["128_and_up"]["tuples"] == 1
