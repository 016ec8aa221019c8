"""Cell-tree bookkeeping of the refinement loop (Sec. 2.2, Sec. 2.7,
Algorithm 1): sample points of a tiling, the subdivision direction of a leaf,
splitting, and the keys that tell which terms of the sum a refinement
changed.  Pure NumPy: no device code, usable without a GPU.

Subdivision direction (Sec. 2.7).  For each axis i along which the leaf is
wider than 2, the paper averages the impulse responses of the leaf's corners
on its front face (phi^{i+}) and on its back face (phi^{i-}) and measures the
change ||phi^{i+} - phi^{i-}|| over the offsets z with c_mid + z in Omega;
the leaf is split along the axis with the largest change.  Sampled at the two
faces only, that change vanishes when phi_p varies along the axis with a
period close to the leaf's width (the faces see the same phase), and the leaf
is then split along the other axes over and over.  Here the change is
measured along the path back face -> midplane -> front face:
    ||phi^{i+} - phi^{i0}|| + ||phi^{i0} - phi^{i-}||,
with phi^{i0} the average of the impulse responses at the midpoints of the
leaf's edges along axis i (the points that splitting along i creates).  When
phi_p changes linearly along the axis this equals the paper's quantity; when
the faces alias, the midplane term sees the change.  The corner-only rule is
kept as rule="faces".
"""
import itertools

import numpy as np


def corner_points(lo, hi):
    """Sorted (axis 0 most significant) union of the leaves' corners."""
    d = lo.shape[1]
    pts = set()
    for a, b in zip(lo, hi):
        for bits in itertools.product((0, 1), repeat=d):
            pts.add(tuple(int(b[i] if bit else a[i]) for i, bit in enumerate(bits)))
    return np.array(sorted(pts), dtype=np.int64).reshape(-1, d)


def _average(patches, R):
    """Mean of centred patches embedded in the box prod [-R_j, R_j]."""
    d = len(R)
    acc = np.zeros(tuple(2 * R + 1))
    for P in patches:
        r = np.array(P.shape) // 2
        sl = tuple(slice(int(R[j] - r[j]), int(R[j] + r[j] + 1)) for j in range(d))
        acc[sl] += P
    return acc / len(patches)


def split_direction(lo, hi, shape, patch_of, rule="midplane"):
    """Axis along which the impulse responses change the most across the
    leaf [lo, hi] (None if no axis is wider than 2).  patch_of(point) returns
    the point's centred impulse-response patch."""
    d = len(lo)
    mid = [(int(lo[i]) + int(hi[i])) // 2 for i in range(d)]
    best, best_axis = -1.0, None
    for i in range(d):
        if hi[i] - lo[i] <= 2:
            continue
        front, back, middle = [], [], []
        for bits in itertools.product((0, 1), repeat=d):
            p = [int(hi[j] if bits[j] else lo[j]) for j in range(d)]
            (front if bits[i] else back).append(patch_of(p))
            if rule == "midplane" and not bits[i]:
                m = list(p)
                m[i] = mid[i]          # midpoint of the edge along axis i
                middle.append(patch_of(m))
        R = np.max([np.array(P.shape) // 2 for P in front + back + middle], axis=0)
        # offsets z with c_mid + z inside Omega
        sl = tuple(slice(int(max(0, R[j] - mid[j])), int(min(2 * R[j] + 1, R[j] + shape[j] - mid[j])))
                   for j in range(d))
        a, b = _average(front, R), _average(back, R)
        if rule == "midplane":
            c = _average(middle, R)
            val = float(np.sqrt(np.sum((a - c)[sl] ** 2))) + float(np.sqrt(np.sum((c - b)[sl] ** 2)))
        elif rule == "faces":
            val = float(np.sqrt(np.sum((a - b)[sl] ** 2)))
        else:
            raise ValueError(f"unknown rule {rule!r}")
        if val > best:
            best, best_axis = val, i
    return best_axis


def split_leaf(lo, hi, axis):
    """The two children of a leaf split at its midpoint along axis."""
    mid = (lo[axis] + hi[axis]) // 2
    a_hi = hi.copy()
    a_hi[axis] = mid
    b_lo = lo.copy()
    b_lo[axis] = mid
    return (lo.copy(), a_hi), (b_lo, hi.copy())


def split_round(lo, hi, eta, frac, shape, patch_of, rule="midplane"):
    """One refinement round: the leaves with the largest eta_C (one leaf if
    frac <= 0, as Algorithm 1; else that fraction, at least one; ties to the
    lower index) are split along their split_direction.  Returns the new
    leaves sorted by lower corner, or None if no leaf can be split."""
    order = np.argsort(-eta, kind="stable")
    refinable = [c for c in order if np.any(hi[c] - lo[c] > 2)]
    if not refinable:
        return None
    n_take = 1 if frac <= 0 else max(1, int(np.ceil(frac * len(lo))))
    chosen = set(int(c) for c in refinable[:n_take])
    new_lo, new_hi = [], []
    for c in range(len(lo)):
        if c in chosen:
            axis = split_direction(lo[c], hi[c], shape, patch_of, rule)
            (alo, ahi), (blo, bhi) = split_leaf(lo[c], hi[c], axis)
            new_lo += [alo, blo]
            new_hi += [ahi, bhi]
        else:
            new_lo.append(lo[c])
            new_hi.append(hi[c])
    order = np.lexsort(np.array(new_lo).T[::-1])
    return np.array(new_lo)[order], np.array(new_hi)[order]


def leaf_point_sets(lo, hi, pts):
    """For every leaf, the indices of the points on its closed box (pts sorted
    with axis 0 most significant, as corner_points returns them)."""
    x0 = pts[:, 0]
    a = np.searchsorted(x0, lo[:, 0], side="left")
    b = np.searchsorted(x0, hi[:, 0], side="right")
    out = []
    for c in range(len(lo)):
        cand = pts[a[c]:b[c], 1:]
        inside = np.all((cand >= lo[c, 1:]) & (cand <= hi[c, 1:]), axis=1)
        out.append(a[c] + np.nonzero(inside)[0])
    return out


def term_keys(lo, hi, pts):
    """A key per point that is equal between two tilings iff the point's term
    of the sum is the same: the point, and the boxes of the leaves containing
    it with the points on each (they fix U_k, w_k, nbrs(k) and phi_k^E)."""
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    sets = leaf_point_sets(lo, hi, pts)
    leaf_key = [lo[c].astype(np.int64).tobytes() + hi[c].astype(np.int64).tobytes() + pts[sc].tobytes()
                for c, sc in enumerate(sets)]
    cells = [[] for _ in range(len(pts))]
    for c, sc in enumerate(sets):
        for k in sc.tolist():
            cells[k].append(leaf_key[c])
    return [(pts[k].tobytes(), tuple(sorted(cells[k]))) for k in range(len(pts))]
