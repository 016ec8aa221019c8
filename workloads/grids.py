"""Leaf tilings of a box domain and their corner points (inputs only).

Boxes are inclusive integer boxes: a leaf is (lo, hi) with lo[i] <= hi[i]; two
neighbouring leaves share their common facet, as the cells of the paper's
binary cell tree do (Sec. 2.2).  The sample points handed to the library are the
sorted union of all leaf corners (axis 0 most significant).
"""
import itertools
import numpy as np


def uniform_nodes(n, m):
    """m tensor-grid node positions on [0, n-1]: floor(i (n-1)/(m-1) + 1/2)."""
    return [int(np.floor(i * (n - 1) / (m - 1) + 0.5)) for i in range(m)]


def tensor_leaves(node_lists):
    """Leaves of a tensor grid given per-axis sorted node positions."""
    d = len(node_lists)
    spans = [list(zip(nl[:-1], nl[1:])) for nl in node_lists]
    lo, hi = [], []
    for combo in itertools.product(*spans):
        lo.append([c[0] for c in combo])
        hi.append([c[1] for c in combo])
    return np.array(lo, dtype=np.int64).reshape(-1, d), np.array(hi, dtype=np.int64).reshape(-1, d)


def _grad_norm(s):
    g = np.gradient(s)
    if s.ndim == 1:
        g = [g]
    return np.sqrt(sum(gi * gi for gi in g))


def quadtree_leaves(s, theta, min_width=16):
    """Refine the root box at its midpoint (all axes at once) while the cell is
    wider than ``min_width`` and width * max_cell |grad s| exceeds ``theta``.

    The midpoint is floor((lo + hi) / 2) per axis; children share the facet.
    """
    shape = s.shape
    d = s.ndim
    gn = _grad_norm(s)
    root = (tuple([0] * d), tuple(n - 1 for n in shape))
    stack = [root]
    leaves = []
    while stack:
        lo, hi = stack.pop()
        width = max(hi[i] - lo[i] for i in range(d))
        sl = tuple(slice(lo[i], hi[i] + 1) for i in range(d))
        if width > min_width and width * float(gn[sl].max()) > theta:
            mid = [(lo[i] + hi[i]) // 2 for i in range(d)]
            for bits in itertools.product((0, 1), repeat=d):
                clo = tuple(lo[i] if b == 0 else mid[i] for i, b in enumerate(bits))
                chi = tuple(mid[i] if b == 0 else hi[i] for i, b in enumerate(bits))
                stack.append((clo, chi))
        else:
            leaves.append((lo, hi))
    leaves.sort()
    lo = np.array([l[0] for l in leaves], dtype=np.int64)
    hi = np.array([l[1] for l in leaves], dtype=np.int64)
    return lo, hi


def corner_points(leaf_lo, leaf_hi):
    """Sorted unique union of the corners of all leaves, shape (r, d)."""
    d = leaf_lo.shape[1]
    pts = set()
    for lo, hi in zip(leaf_lo, leaf_hi):
        for bits in itertools.product((0, 1), repeat=d):
            pts.add(tuple(int(hi[i] if b else lo[i]) for i, b in enumerate(bits)))
    return np.array(sorted(pts), dtype=np.int64).reshape(-1, d)


def tune_quadtree(s, r_lo, r_hi, min_width=16, iters=60):
    """Bisect the refinement threshold so the point count lands in [r_lo, r_hi]."""
    t_lo, t_hi = 1e-3, 1e4   # small threshold -> many points
    best = None
    for _ in range(iters):
        t = np.sqrt(t_lo * t_hi)
        lo, hi = quadtree_leaves(s, t, min_width)
        r = corner_points(lo, hi).shape[0]
        best = (t, lo, hi, r)
        if r < r_lo:
            t_hi = t
        elif r > r_hi:
            t_lo = t
        else:
            return best
    return best
