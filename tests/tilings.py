"""Small hand-made tilings for the CPU tests (inputs only)."""
import numpy as np

from workloads import BlurOperator, corner_points, tensor_leaves, uniform_nodes
from workloads.configs import Workload


def refine(shape, rule):
    """Quadtree-style tiling: split a box at its midpoint (all live axes) while
    ``rule(lo, hi)`` is true."""
    d = len(shape)
    stack = [(tuple([0] * d), tuple(n - 1 for n in shape))]
    leaves = []
    while stack:
        lo, hi = stack.pop()
        if rule(lo, hi):
            mid = [(l + h) // 2 for l, h in zip(lo, hi)]
            live = [i for i in range(d) if hi[i] - lo[i] >= 2]
            import itertools
            for bits in itertools.product((0, 1), repeat=len(live)):
                clo, chi = list(lo), list(hi)
                for b, i in zip(bits, live):
                    if b == 0:
                        chi[i] = mid[i]
                    else:
                        clo[i] = mid[i]
                stack.append((tuple(clo), tuple(chi)))
        else:
            leaves.append((lo, hi))
    leaves.sort()
    return (np.array([l for l, _ in leaves], dtype=np.int64),
            np.array([h for _, h in leaves], dtype=np.int64))


def hanging_2d(n=17, corner=(0, 0), levels=2):
    """n x n domain refined towards one corner: produces hanging nodes."""
    corner = np.array(corner)

    def rule(lo, hi):
        w = max(h - l for l, h in zip(lo, hi))
        if w <= max(2, (n - 1) >> levels):
            return False
        return bool(np.all(np.array(lo) <= corner) and np.all(np.array(hi) >= corner)) or w >= n - 1
    return refine((n, n), rule)


def workload_from(sig_axes, lo, hi, name="t"):
    op = BlurOperator(sig_axes)
    pts = corner_points(lo, hi)
    radius, phi, off = op.impulse_responses(pts)
    return Workload(name, op.d, tuple(op.shape), lo, hi, pts, radius, phi, off, op, 1, 0, {})


def const_blur(shape, s, lo, hi):
    sig = np.full((len(shape),) + tuple(shape), float(s))
    return workload_from(sig, lo, hi, "const")


def tensor(shape, m):
    return tensor_leaves([uniform_nodes(n, m) for n in shape])
