"""Plain FP64 reference of the calibration surrogate: an MLP 4 -> 128 -> 128
-> 128 -> 4 with GELU after each hidden layer, its squared-error loss, the
gradient of that loss by explicit back-propagation, and one Adam update.

TEST INFRASTRUCTURE ONLY: the GPU library never imports this module; only
the test suite, the smoke check and the benchmark's CPU leg do.

Definitions (the GPU kernels implement the same ones independently):
  parameters  one float vector, per layer l = 1..4 the weight matrix stored
              input-major, W_l[k, j] at offset off_l + k * n_out + j, then the
              bias b_l[j]; sizes 4x128, 128x128, 128x128, 128x4 (34180 values);
  inputs      xh = (x - x_shift) * x_scale (x = model, Tr, w, kappa);
  outputs     out = a3 W4 + b4 in log space; the physical prediction is
              y = exp(out * y_scale + y_shift);
  hidden      z_l = a_{l-1} W_l + b_l, a_l = GELU(z_l) = z_l Phi(z_l) with
              Phi the standard normal CDF (Hendrycks and Gimpel, 2016);
  loss        mean over samples and the 4 outputs of (out - t)^2 with the
              target t = (log y - y_shift) / y_scale;
  BF16 mode   every product operand is rounded to bfloat16 (round to nearest,
              ties to even) before it is multiplied: the layer inputs a_l
              (including xh) and the weights W_l; biases, sums and the
              back-propagated errors stay unrounded.  The gradient treats the
              rounding of W as the identity (straight-through);
  Adam        Kingma and Ba (2015), Algorithm 1, with bias correction.
"""
from __future__ import annotations

import math

import numpy as np

H = 128
IN = 4
OUT = 4
SIZES = [(IN, H), (H, H), (H, H), (H, OUT)]


def layout():
    """[(weight offset, bias offset, n_in, n_out)] per layer, total count."""
    out, off = [], 0
    for n_in, n_out in SIZES:
        out.append((off, off + n_in * n_out, n_in, n_out))
        off += n_in * n_out + n_out
    return out, off


LAYOUT, NPARAMS = layout()


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    return [(theta[w:w + a * b].reshape(a, b), theta[bo:bo + b]) for w, bo, a, b in LAYOUT]


def bf16_round(v):
    """Round to the nearest bfloat16 value (ties to even), returned as
    float64.  Works on the float32 bit pattern: add 0x7FFF plus the lowest
    kept bit, then clear the low 16 bits."""
    f = np.asarray(v, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    from scipy.special import erf
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def normalise_inputs(x, norm):
    return (np.asarray(x, np.float64) - norm["x_shift"]) * norm["x_scale"]


def targets(y, norm):
    return (np.log(np.asarray(y, np.float64)) - norm["y_shift"]) / norm["y_scale"]


def forward(theta, x, norm, bf16=False):
    """(out in log space, cache of (a_in, z) per layer)."""
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, np.float64))
    a = rnd(normalise_inputs(x, norm))
    cache = []
    layers = unpack(theta)
    for l, (W, b) in enumerate(layers):
        z = a @ rnd(W) + b
        cache.append((a, z))
        if l < len(layers) - 1:
            a = rnd(gelu(z))
    return z, cache


def predict(theta, x, norm, bf16=False):
    out, _ = forward(theta, x, norm, bf16)
    return np.exp(out * norm["y_scale"] + norm["y_shift"])


def loss_and_grad(theta, x, y, norm, bf16=False):
    """Mean squared error in normalised log space and its gradient with
    respect to every parameter (same layout as theta)."""
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, np.float64))
    out, cache = forward(theta, x, norm, bf16)
    t = targets(y, norm)
    n = out.shape[0]
    r = out - t
    loss = float(np.sum(r * r) / (n * OUT))
    grad = np.zeros(NPARAMS)
    layers = unpack(theta)
    d = 2.0 * r / (n * OUT)  # dL/dz of the output layer
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        a_in, _ = cache[l]
        w_off, b_off, n_in, n_out = LAYOUT[l]
        grad[w_off:w_off + n_in * n_out] = (a_in.T @ d).ravel()
        grad[b_off:b_off + n_out] = d.sum(axis=0)
        if l > 0:
            da = d @ rnd(W).T
            d = da * gelu_prime(cache[l - 1][1])
    return loss, grad


def adam(theta, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
