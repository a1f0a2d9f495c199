"""What the trained surrogate gains over the method without it: trained by
the library's own kernels on equilibria the batched lattices compute, it
predicts held-out calibration results in a fraction of a second, to the
accuracy the plain runs themselves are reproducible to."""
import time

import numpy as np
import pytest

from paper_2403_11167_amd import calibration as cal
from paper_2403_11167_amd import inputs, lbm

pytestmark = pytest.mark.gpu


def test_surrogate_replaces_calibration_runs():
    import torch
    x, y, info = cal.training_set(600, 15, size=(64, 8, 96), max_steps=60000)
    assert len(x) > 250
    sur = lbm.Surrogate(inputs.mlp_initial_params(0))
    sur.set_target_scaling(y)
    losses = sur.fit(x, y, epochs=400, batch=128, lr=3e-3, seed=1, lr_final=1e-4)
    assert losses[-1] < 0.02 * losses[0]
    # held-out tuples, calibrated by the plain method on the training geometry
    tup = cal.sample_tuples(48, 16)
    labels, plain = cal.run_calibration(tup, [(64, 8, 96)] * 48, max_steps=60000)
    m = cal.valid(labels)
    assert m.sum() >= 15
    feats = cal.features(tup)
    sur.predict(feats[:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = sur.predict(feats)
    infer = time.perf_counter() - t0
    rel = np.abs(pred[m] / cal.targets(labels)[m] - 1)
    # rho_l and W: within 1 % and 3 % for (nearly) every tuple; rho_v and
    # sigma: median within 1 % and 3 %
    assert np.mean(rel[:, 0] < 0.01) >= 0.95
    assert np.mean(rel[:, 3] < 0.03) >= 0.9
    assert np.median(rel[:, 1]) < 0.01
    assert np.median(rel[:, 2]) < 0.03
    # the prediction replaces runs that take seconds
    assert infer < 0.05 * plain["seconds"], (infer, plain["seconds"])
