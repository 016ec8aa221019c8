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


def hanging_3d(n=9, min_width=2):
    """n^3 domain refined (all axes at once) towards the corner (0, 0, 0) down
    to leaves of width min_width: every face between the refined octants and
    the coarse leaves is broken."""
    def rule(lo, hi):
        w = max(h - l for l, h in zip(lo, hi))
        return w > min_width and (w >= n - 1 or all(l == 0 for l in lo))
    return refine((n, n, n), rule)


def extrude(lo2, hi2, znodes):
    """3-D tiling: every 2-D leaf times every interval between z nodes."""
    lo, hi = [], []
    for a, b in zip(lo2, hi2):
        for z0, z1 in zip(znodes[:-1], znodes[1:]):
            lo.append([a[0], a[1], z0])
            hi.append([b[0], b[1], z1])
    lo, hi = np.array(lo, dtype=np.int64), np.array(hi, dtype=np.int64)
    order = np.lexsort(lo.T[::-1])
    return lo[order], hi[order]


def unequal_radii_3x3(radii=(1, 2, 3, 2, 3, 1, 3, 1, 2), c=3):
    """Omega = [0,2]^2 with four 1x1 leaves and the 3x3 sample points; point
    k = 3a + b at (a, b) has the patch phi_k[z] = 100 (k+1) + 10 (z0+c) +
    (z1+c) on the box |z_i| <= R_k (the extension goldens' tiling)."""
    lo, hi = tensor_leaves([[0, 1, 2], [0, 1, 2]])
    pts = corner_points(lo, hi)
    R = np.repeat(np.asarray(radii, dtype=np.int64)[:, None], 2, axis=1)
    phi, off = [], [0]
    for j in range(9):
        r = int(radii[j])
        z0, z1 = np.meshgrid(np.arange(-r, r + 1), np.arange(-r, r + 1), indexing="ij")
        blk = 100.0 * (j + 1) + 10.0 * (z0 + c) + (z1 + c)
        phi.append(blk.ravel())
        off.append(off[-1] + blk.size)
    return Workload("unequal3x3", 2, (3, 3), lo, hi, pts, R, np.concatenate(phi),
                    np.array(off, dtype=np.int64), None, 1, 0, {})
