"""Helpers for the library tests (inputs, tolerances, tiny cases)."""
import numpy as np

from workloads import make_config, cosine_field
from tests.tilings import hanging_2d, hanging_3d, const_blur, workload_from, tensor, unequal_radii_3x3

# Per-vector relative L2 bars against the FP64 oracle.
TOL = {0: 1e-5, 1: 1e-12}     # PC_F32, PC_F64


def relerr(got, ref):
    got = np.asarray(got, dtype=np.float64).reshape(ref.shape)
    num = np.linalg.norm((got - ref).reshape(ref.shape[0], -1), axis=1)
    den = np.linalg.norm(ref.reshape(ref.shape[0], -1), axis=1)
    return num / np.maximum(den, 1e-300)


def small_cases():
    """(name, workload) pairs spanning several tiles, ragged tails, hanging
    nodes, 1-D, rectangles and boundary-clipped patches."""
    cases = [("cfg0", make_config(0))]
    lo, hi = hanging_2d(33, corner=(32, 0), levels=3)
    x0, x1 = np.meshgrid(np.arange(33), np.arange(33), indexing="ij")
    s = 0.8 + 1.5 * (x0 + x1) / 64
    cases.append(("hanging33", workload_from(np.stack([s, s]), lo, hi)))
    lo = np.array([[0], [9], [13], [30], [77]])
    hi = np.array([[9], [13], [30], [77], [100]])
    x = np.arange(101)
    s1 = 1.0 + 2.0 * np.sin(x / 17.0) ** 2
    cases.append(("1d", workload_from(s1[None, :], lo, hi)))
    lo, hi = tensor((45, 301), 4)
    cases.append(("rect45x301", const_blur((45, 301), 1.6, lo, hi)))
    lo, hi = tensor((70, 70), 2)                     # one leaf: a big single patch
    x0, x1 = np.meshgrid(np.arange(70), np.arange(70), indexing="ij")
    s = 2.0 + 3.0 * (x0 / 69.0)
    cases.append(("oneleaf70", workload_from(np.stack([s, s]), lo, hi)))
    cases.append(("cfg1_small", make_config(1, scale=0.25)))
    # the unequal-radii extension golden's tiling (radii 1, 2, 3 side by side)
    cases.append(("unequal3x3", unequal_radii_3x3()))
    return cases


def small_cases_3d():
    """3-D (name, workload) pairs: a rectangular box with per-axis widths
    varying along their own axes, a cube with cosine width fields (the 3-D
    workload's recipe at 24^3, 4 x 4 x 4 points) and a 17^3 tiling refined
    towards one corner (hanging nodes, broken facets)."""
    lo, hi = tensor((12, 17, 23), 3)
    x0, x1, x2 = np.meshgrid(np.arange(12), np.arange(17), np.arange(23), indexing="ij")
    s0 = 0.7 + 0.8 * x0 / 11
    s1 = 1.0 + 0.5 * np.cos(x1 / 4.0)
    s2 = 0.9 + 0.6 * x2 / 22
    cases = [("rect3d", workload_from(np.stack([s0, s1, s2]), lo, hi))]
    n = 24
    rng = np.random.default_rng(2)
    f = [cosine_field((n, n, n), 0.8, 3.0, 2, 2, rng=rng)[0] for _ in range(3)]
    lo, hi = tensor((n, n, n), 4)
    cases.append(("cube24", workload_from(np.stack(f), lo, hi)))
    # hanging nodes: 17^3 refined towards one corner (broken facets)
    m = 17
    x0, x1, x2 = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    lo, hi = hanging_3d(m, min_width=4)
    sig = np.stack([0.7 + 0.5 * x0 / 16, 0.9 + 0.3 * np.cos(x1 / 5.0), 0.8 + 0.4 * x2 / 16])
    cases.append(("hang3d", workload_from(sig, lo, hi)))
    return cases
