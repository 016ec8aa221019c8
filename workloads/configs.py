"""The synthetic workloads (exact seeds and sizes).

0: 2-D 64^2, uniform 5x5 sample grid, s(x) = 2 + 4(0.5 + 0.5 sin cos), B = 1
   (one N(0,1) vector, seed 0); FP64 primary.
1: 2-D 1024^2, s in [2, 12] from 2 cosine modes (kmax 3, seed 1), quadtree
   refined where |grad s| is large (about 600 points), B = 64 N(0,1)
   vectors (seed 101), FP32.
2: 3-D 128^3, per-axis widths s_i in [1.5, 6] (one 2-mode field per axis,
   kmax 2, seed 2), 9^3 tensor sample grid, B = 16 (seed 102).
3: 2-D 2048^2, s in [2, 16] (seed 3), start from a 4x4 sample grid, q = 32
   Rademacher probes (seed 103).
Small variants (``scale`` < 1) keep the structure at test-friendly sizes.
"""
from dataclasses import dataclass, field
import numpy as np

from .fields import cosine_field, cfg0_sigma
from .grids import uniform_nodes, tensor_leaves, corner_points, tune_quadtree, quadtree_leaves
from .blur import BlurOperator


@dataclass
class Workload:
    name: str
    d: int
    shape: tuple
    leaf_lo: np.ndarray
    leaf_hi: np.ndarray
    points: np.ndarray
    radius: np.ndarray
    phi: np.ndarray
    phi_off: np.ndarray
    op: BlurOperator
    batch: int
    vec_seed: int
    params: dict = field(default_factory=dict)

    @property
    def N(self):
        return int(np.prod(self.shape))

    @property
    def r(self):
        return int(self.points.shape[0])

    def vectors(self, B=None, dtype=np.float64, seed=None):
        """B standard-normal vectors, shape (B, N), rounded to ``dtype``."""
        B = self.batch if B is None else B
        rng = np.random.default_rng(self.vec_seed if seed is None else seed)
        U = rng.standard_normal((B,) + tuple(self.shape))
        return U.reshape(B, -1).astype(dtype)

    def rademacher(self, q, seed):
        rng = np.random.default_rng(seed)
        return (rng.integers(0, 2, size=(q, self.N)) * 2 - 1).astype(np.float64)


def _finish(name, s_axes, leaf_lo, leaf_hi, batch, vec_seed, params):
    op = BlurOperator(s_axes)
    pts = corner_points(leaf_lo, leaf_hi)
    radius, phi, off = op.impulse_responses(pts)
    return Workload(name, op.d, tuple(op.shape), leaf_lo, leaf_hi, pts, radius, phi, off,
                    op, batch, vec_seed, params)


def make_config(idx, scale=1.0):
    """Build workload ``idx``; ``scale`` < 1 shrinks the grid for quick tests."""
    if idx == 0:
        n = 64
        s = cfg0_sigma(n)
        nodes = uniform_nodes(n, 5)
        lo, hi = tensor_leaves([nodes, nodes])
        return _finish("blur2d_64_uniform5x5", np.stack([s, s]), lo, hi, 1, 0,
                       {"nodes": nodes})
    if idx == 1:
        n = max(32, int(round(1024 * scale)))
        s, modes = cosine_field((n, n), 2.0, 12.0, 2, 3, seed=1)
        r_target = 600 if scale >= 1.0 else max(9, int(600 * scale * scale))
        t, lo, hi, r = tune_quadtree(s, int(r_target * 0.95), int(r_target * 1.05) + 1,
                                     min_width=max(4, int(16 * min(1.0, scale * 4))))
        return _finish(f"blur2d_{n}_quadtree", np.stack([s, s]), lo, hi, 64, 101,
                       {"modes": modes, "theta": t})
    if idx == 2:
        n = max(16, int(round(128 * scale)))
        rng = np.random.default_rng(2)
        fields = []
        allm = []
        for _ in range(3):
            f, m = cosine_field((n, n, n), 1.5, 6.0, 2, 2, rng=rng)
            fields.append(f)
            allm.append(m)
        nodes = uniform_nodes(n, 9)
        lo, hi = tensor_leaves([nodes, nodes, nodes])
        return _finish(f"blur3d_{n}_tensor9", np.stack(fields), lo, hi, 16, 102,
                       {"modes": allm, "nodes": nodes})
    if idx == 3:
        n = max(32, int(round(2048 * scale)))
        s, modes = cosine_field((n, n), 2.0, 16.0, 2, 3, seed=3)
        nodes = uniform_nodes(n, 4)
        lo, hi = tensor_leaves([nodes, nodes])
        return _finish(f"blur2d_{n}_start4x4", np.stack([s, s]), lo, hi, 32, 103,
                       {"modes": modes, "nodes": nodes})
    raise ValueError(f"unknown config {idx}")


def make_serving_ops(sizes=None, with_3d=False, sizes3=None):
    """The resident operators of the serving workload.

    2-D: grids 256^2 to 2048^2 with 25 to about 2000 sample points (s in
    [2, 12], s in [2, 16] on the largest), uniform grids for the two smallest,
    quadtrees otherwise (seeds 40 + i).
    3-D (with_3d): tensor grids 64^3 / 3^3, 80^3 / 5^3, 96^3 / 7^3, 128^3 / 9^3
    (the 3-D workload's operator), 144^3 / 10^3 and 160^3 / 12^3 points, per-axis
    widths in [1.5, 6] (one two-mode field per axis, kmax 2, seeds 50 + i).
    ``sizes`` / ``sizes3`` keep only the listed grid sizes."""
    specs = [(256, 25, 0), (512, 100, 0), (768, 300, 1), (1024, 600, 1), (1536, 1000, 1), (2048, 2000, 1)]
    out = []
    for i, (n, r_target, adaptive) in enumerate(specs):
        if sizes is not None and n not in sizes:
            continue
        hi_s = 16.0 if n == 2048 else 12.0
        s, modes = cosine_field((n, n), 2.0, hi_s, 2, 3, seed=40 + i)
        if not adaptive:
            m = int(round(np.sqrt(r_target)))
            nodes = uniform_nodes(n, m)
            lo, hi = tensor_leaves([nodes, nodes])
            name = f"blur2d_{n}_uniform{m}x{m}"
        else:
            _, lo, hi, _ = tune_quadtree(s, int(r_target * 0.9), int(r_target * 1.1) + 1)
            name = f"blur2d_{n}_quadtree"
        out.append(_finish(name, np.stack([s, s]), lo, hi, 32, 104 + i, {"modes": modes}))
    if not with_3d:
        return out
    specs3 = [(64, 3), (80, 5), (96, 7), (128, 9), (144, 10), (160, 12)]
    for i, (n, m) in enumerate(specs3):
        if sizes3 is not None and n not in sizes3:
            continue
        if n == 128:
            w = make_config(2)
            w.batch, w.vec_seed = 32, 110 + i
            out.append(w)
            continue
        rng = np.random.default_rng(50 + i)
        fields = [cosine_field((n, n, n), 1.5, 6.0, 2, 2, rng=rng)[0] for _ in range(3)]
        nodes = uniform_nodes(n, m)
        lo, hi = tensor_leaves([nodes, nodes, nodes])
        out.append(_finish(f"blur3d_{n}_tensor{m}", np.stack(fields), lo, hi, 32, 110 + i, {}))
    return out
