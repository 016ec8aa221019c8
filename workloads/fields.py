"""Smooth blur-width fields s(x) on a grid (seeded)."""
import numpy as np


def cosine_field(shape, lo, hi, n_modes, kmax, seed=None, rng=None):
    """Random low-frequency cosine field, min-max normalised to [lo, hi].

    Draw order per mode j (fixed so runs are reproducible): integer wave
    vector k_j in [1, kmax]^d, phase theta_j in [0, 2 pi), amplitude a_j in
    [0.5, 1).  m(x) = sum_j a_j cos(2 pi sum_i k_ji x_i / n_i + theta_j), with
    x the integer grid index (axis 0 first).
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    shape = tuple(int(n) for n in shape)
    d = len(shape)
    axes = [np.arange(n, dtype=np.float64) for n in shape]
    grids = np.meshgrid(*axes, indexing="ij")
    m = np.zeros(shape, dtype=np.float64)
    params = []
    for _ in range(n_modes):
        k = rng.integers(1, kmax + 1, size=d)
        th = rng.uniform(0.0, 2.0 * np.pi)
        a = rng.uniform(0.5, 1.0)
        phase = sum(2.0 * np.pi * k[i] * grids[i] / shape[i] for i in range(d))
        m += a * np.cos(phase + th)
        params.append({"k": [int(v) for v in k], "theta": float(th), "a": float(a)})
    mn, mx = m.min(), m.max()
    s = lo + (hi - lo) * (m - mn) / (mx - mn)
    return s, params


def cfg0_sigma(n=64):
    """s(x) = 2 + 4 (0.5 + 0.5 sin(2 pi x1/n) cos(2 pi x2/n)); x1 = axis 0."""
    x1, x2 = np.meshgrid(np.arange(n, dtype=np.float64),
                         np.arange(n, dtype=np.float64), indexing="ij")
    return 2.0 + 4.0 * (0.5 + 0.5 * np.sin(2 * np.pi * x1 / n) * np.cos(2 * np.pi * x2 / n))
