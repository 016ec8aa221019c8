"""Adaptive grid structure (Sec. 2.2).

A leaf cell is an inclusive integer box (lo, hi).  The sample points are the
corners of all cells of the tree; since a refined cell's corners are corners
of its children, that is the union of the leaves' corners.  cells(p) is the set
of leaves containing p, the blocky neighbourhood U_k is their union, and
nbrs(k) is the set of sample points sharing a leaf with p_k (k included).
"""
import itertools
import numpy as np


class TilingError(ValueError):
    pass


class Grid:
    def __init__(self, shape, leaf_lo, leaf_hi, points=None):
        self.shape = tuple(int(n) for n in shape)
        self.d = len(self.shape)
        self.leaf_lo = np.asarray(leaf_lo, dtype=np.int64).reshape(-1, self.d)
        self.leaf_hi = np.asarray(leaf_hi, dtype=np.int64).reshape(-1, self.d)
        self._validate_tiling()
        pts = self._corners()
        if points is not None:
            points = np.asarray(points, dtype=np.int64).reshape(-1, self.d)
            if points.shape != pts.shape or np.any(points != pts):
                raise TilingError("sample points are not the sorted union of leaf corners")
        self.points = pts
        self.r = pts.shape[0]
        self.index = {tuple(int(v) for v in p): k for k, p in enumerate(pts)}
        # cells(p_k): leaves that contain p_k
        self.cells = [[] for _ in range(self.r)]
        # points lying in each leaf (corners and hanging nodes)
        self.leaf_points = []
        for c in range(self.leaf_lo.shape[0]):
            inside = np.nonzero(np.all((pts >= self.leaf_lo[c]) & (pts <= self.leaf_hi[c]), axis=1))[0]
            self.leaf_points.append(inside)
            for k in inside:
                self.cells[k].append(c)
        self.nbrs = []
        for k in range(self.r):
            s = set()
            for c in self.cells[k]:
                s.update(int(j) for j in self.leaf_points[c])
            self.nbrs.append(sorted(s))
        # bounding box of U_k
        self.u_lo = np.array([self.leaf_lo[self.cells[k]].min(axis=0) for k in range(self.r)])
        self.u_hi = np.array([self.leaf_hi[self.cells[k]].max(axis=0) for k in range(self.r)])

    # -- tiling checks -----------------------------------------------------
    def _validate_tiling(self):
        lo, hi, d = self.leaf_lo, self.leaf_hi, self.d
        n = np.array(self.shape)
        if lo.shape[0] == 0:
            raise TilingError("no leaves")
        if np.any(lo < 0) or np.any(hi > n - 1) or np.any(lo > hi):
            raise TilingError("leaf outside the domain or inverted")
        live = n > 1                      # axes of extent 1 are trivial
        if np.any((hi - lo)[:, live] == 0):
            raise TilingError("degenerate leaf (zero width along a live axis)")
        vol = np.prod(np.where(live, hi - lo, 1), axis=1).astype(np.float64)
        if abs(vol.sum() - float(np.prod(np.where(live, n - 1, 1)))) > 0.5:
            raise TilingError("leaf volumes do not add up to the domain volume")
        # pairwise interiors disjoint: open intervals (lo, hi) overlap on all live axes
        L = lo.shape[0]
        for c in range(L):
            ov = np.ones(L, dtype=bool)
            for i in range(d):
                if not live[i]:
                    continue
                ov &= (np.minimum(hi[:, i], hi[c, i]) - np.maximum(lo[:, i], lo[c, i])) > 0
            ov[c] = False
            if ov.any():
                raise TilingError("leaf interiors overlap")

    def _corners(self):
        pts = set()
        for lo, hi in zip(self.leaf_lo, self.leaf_hi):
            for bits in itertools.product((0, 1), repeat=self.d):
                pts.add(tuple(int(hi[i] if b else lo[i]) for i, b in enumerate(bits)))
        return np.array(sorted(pts), dtype=np.int64).reshape(-1, self.d)

    def facet_parts(self, c, axis, side):
        """The facet of leaf c normal to ``axis`` (side 0: at lo, 1: at hi) as
        the union of (d-1)-dimensional boxes (Sec. 2.4): where the leaves on
        the other side are smaller the facet is broken into their facets
        (clipped to it); a facet on the domain boundary, or facing one larger
        leaf, is a single box.  Returns a list of (lo, hi) with lo[axis] =
        hi[axis] = the facet's coordinate."""
        lo, hi = self.leaf_lo[c], self.leaf_hi[c]
        v = hi[axis] if side else lo[axis]
        flo, fhi = lo.copy(), hi.copy()
        flo[axis] = fhi[axis] = v
        other = self.leaf_lo[:, axis] == v if side else self.leaf_hi[:, axis] == v
        parts = []
        for e in np.nonzero(other)[0]:
            if e == c:
                continue
            plo = np.maximum(flo, self.leaf_lo[e])
            phi = np.minimum(fhi, self.leaf_hi[e])
            plo[axis] = phi[axis] = v
            ok = all(phi[i] > plo[i] for i in range(self.d) if i != axis and fhi[i] > flo[i])
            if ok:
                parts.append((plo, phi))
        return parts if parts else [(flo, fhi)]

    def leaf_of_each_point_mask(self):
        """Boolean (L, N) membership of grid points in leaves (tiny grids only)."""
        N = int(np.prod(self.shape))
        coords = np.array(np.unravel_index(np.arange(N), self.shape)).T
        return np.array([np.all((coords >= l) & (coords <= h), axis=1)
                         for l, h in zip(self.leaf_lo, self.leaf_hi)])
