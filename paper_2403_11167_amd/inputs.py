"""Seeded synthetic initial density fields.

This module holds no lattice Boltzmann arithmetic: it only draws the
initial density fields rho0 that both the GPU library and the CPU oracle
start from (each side then builds its own equilibrium populations).  Phase
densities are passed in as numbers.

Shapes follow the paper's workloads (Sec. 5.1, 5.2) and the throughput
workload:
  * planar slab: liquid between two tanh interfaces (Sec. 5.1);
  * droplet: a tanh disc of radius R at the box centre (Sec. 5.2);
  * spinodal: mean density with seeded uniform multiplicative noise.
"""
from __future__ import annotations

import numpy as np


def planar_slab(nx: int, ny: int, rho_l: float, rho_v: float, width: float = 5.0,
                x_lo: float | None = None, x_hi: float | None = None,
                noise: float = 0.0, seed: int = 1) -> np.ndarray:
    """rho(x) = rho_v + (rho_l - rho_v)/2 [tanh(2(x - x_lo)/W) - tanh(2(x - x_hi)/W)],
    liquid between the two interfaces.  Defaults put the interfaces at the
    quarter points (x_lo = nx/4 - 1/2, x_hi = 3 nx/4 - 1/2), so the liquid
    nodes are exactly [nx/4, 3 nx/4).  Optional additive uniform noise
    noise * U(-1, 1) drawn from numpy's default_rng(seed)."""
    if x_lo is None:
        x_lo = nx / 4 - 0.5
    if x_hi is None:
        x_hi = 3 * nx / 4 - 0.5
    x = np.arange(nx, dtype=np.float64)
    prof = rho_v + 0.5 * (rho_l - rho_v) * (np.tanh(2 * (x - x_lo) / width)
                                              - np.tanh(2 * (x - x_hi) / width))
    rho = np.broadcast_to(prof, (ny, nx)).copy()
    if noise:
        rng = np.random.default_rng(seed)
        rho += noise * rng.uniform(-1.0, 1.0, size=rho.shape)
    return rho


def layered(nx: int, ny: int, rho_l: float, rho_v: float, width: float = 5.0,
            y_i: float | None = None) -> np.ndarray:
    """rho(y) = (rho_l + rho_v)/2 + (rho_l - rho_v)/2 tanh(2 (y - y_i)/W):
    vapour below, liquid above one interface parallel to the x axis (the
    channel between two walls, Sec. 5.3).  Default y_i = (ny - 1)/2, the
    mid-plane between wall rows 0 and ny - 1."""
    if y_i is None:
        y_i = 0.5 * (ny - 1)
    y = np.arange(ny, dtype=np.float64)
    prof = 0.5 * (rho_l + rho_v) + 0.5 * (rho_l - rho_v) * np.tanh(2 * (y - y_i) / width)
    return np.broadcast_to(prof[:, None], (ny, nx)).copy()


def droplet(nx: int, ny: int, rho_l: float, rho_v: float, radius: float,
            width: float = 5.0, cx: float | None = None, cy: float | None = None) -> np.ndarray:
    """rho = (rho_l + rho_v)/2 - (rho_l - rho_v)/2 tanh(2 (r - R)/W), centred
    at (nx/2, ny/2) by default."""
    if cx is None:
        cx = nx / 2
    if cy is None:
        cy = ny / 2
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2 * (r - radius) / width)


def droplets(nx: int, ny: int, rho_l: float, rho_v: float, radius: float,
             centres, width: float = 5.0) -> np.ndarray:
    """Several droplets of the same radius (the collision of Sec. 5.4): the
    pointwise maximum of the single-droplet tanh profiles centred at each
    (cx, cy) of centres (no periodic images)."""
    return np.max([droplet(nx, ny, rho_l, rho_v, radius, width, cx, cy) for cx, cy in centres],
                  axis=0)


def spinodal(nx: int, ny: int, rho_mean: float, amplitude: float = 0.01,
             seed: int = 3) -> np.ndarray:
    """rho = rho_mean (1 + amplitude U(-1, 1)), numpy default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return rho_mean * (1.0 + amplitude * rng.uniform(-1.0, 1.0, size=(ny, nx)))


def uniform(nx: int, ny: int, rho: float) -> np.ndarray:
    return np.full((ny, nx), float(rho))


MLP_LAYER_SIZES = ((4, 128), (128, 128), (128, 128), (128, 4))


def mlp_initial_params(seed: int) -> np.ndarray:
    """Initial surrogate parameters as one float32 vector: per layer the
    n_in x n_out weights (input-major) drawn from
    U(-sqrt(6 / n_in), sqrt(6 / n_in)) / 2, then n_out zero biases;
    numpy default_rng(seed)."""
    rng = np.random.default_rng(seed)
    parts = []
    for n_in, n_out in MLP_LAYER_SIZES:
        lim = 0.5 * np.sqrt(6.0 / n_in)
        parts.append(rng.uniform(-lim, lim, size=n_in * n_out))
        parts.append(np.zeros(n_out))
    return np.concatenate(parts).astype(np.float32)
