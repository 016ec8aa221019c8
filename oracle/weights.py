"""Harmonic partition-of-unity weighting functions w_k (Sec. 2.4).

On every leaf C and for every sample point p_k in C, w_k restricted to C is
built recursively in dimension: at sample points w_k is 1 at p_k and 0 at all
other sample points; on each 1-D box (an edge cut at every sample point lying
on it) it solves the discrete 1-D Laplace equation, i.e. it is linear between
consecutive cuts; on each higher-dimensional box it solves the discrete
Laplace equation (the positive definite graph Laplacian, i.e. the Kronecker-sum
finite-difference Laplacian) with the already computed lower-dimensional
values as Dirichlet data.  w_k is zero off U_k.

In 3-D a facet that contains hanging nodes (a broken facet) is replaced by
the smaller boxes it is made of, the facets of the smaller leaves on its
other side (Sec. 2.4); each of those boxes is solved on its own.
"""
import itertools
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _laplace_dirichlet(box):
    """Fill the interior of ``box`` (shape S + (nrhs,), boundary filled) with the
    discrete harmonic extension of its boundary values."""
    S = box.shape[:-1]
    live = [i for i, n in enumerate(S) if n > 1]
    inner = tuple(n - 2 if i in live else n for i, n in enumerate(S))
    if any(n <= 0 for n in inner):
        return box
    sl_in = tuple(slice(1, -1) if i in live else slice(None) for i in range(len(S)))
    nin = int(np.prod(inner))
    # Kronecker-sum Laplacian over the live axes of the interior
    mats = []
    for i in live:
        T = sp.diags([-np.ones(inner[i] - 1), 2 * np.ones(inner[i]), -np.ones(inner[i] - 1)],
                     [-1, 0, 1], format="csr")
        parts = [sp.identity(inner[j], format="csr") for j in range(len(S))]
        parts[i] = T
        K = parts[0]
        for P in parts[1:]:
            K = sp.kron(K, P, format="csr")
        mats.append(K)
    L = mats[0]
    for K in mats[1:]:
        L = L + K
    # right-hand side: Dirichlet neighbours
    nrhs = box.shape[-1]
    rhs = np.zeros(inner + (nrhs,))
    for i in live:
        lo_face = [slice(1, -1) if j in live else slice(None) for j in range(len(S))]
        hi_face = list(lo_face)
        lo_face[i] = slice(0, 1)
        hi_face[i] = slice(S[i] - 1, S[i])
        tgt_lo = [slice(None)] * len(S)
        tgt_hi = [slice(None)] * len(S)
        tgt_lo[i] = slice(0, 1)
        tgt_hi[i] = slice(inner[i] - 1, inner[i])
        rhs[tuple(tgt_lo)] += box[tuple(lo_face)]
        rhs[tuple(tgt_hi)] += box[tuple(hi_face)]
    lu = spla.splu(sp.csc_matrix(L))
    sol = lu.solve(rhs.reshape(nin, nrhs))
    box[sl_in] = sol.reshape(inner + (nrhs,))
    return box


def harmonic_on_box(lo, hi, pts, vals, facet_parts=None):
    """Recursive harmonic extension on the inclusive box [lo, hi].

    pts: (P, d) sample points lying in the box; vals: (P, nrhs) prescribed
    values there.  facet_parts(i, side) -> list of (lo, hi) boxes making up
    the facet normal to axis i (for a 3-D box with broken facets); None: every
    facet is one box.  Returns an array of shape (hi-lo+1) + (nrhs,).
    """
    lo = np.asarray(lo)
    hi = np.asarray(hi)
    d = lo.size
    S = tuple(int(h - l + 1) for l, h in zip(lo, hi))
    nrhs = vals.shape[1]
    live = [i for i in range(d) if hi[i] > lo[i]]
    out = np.zeros(S + (nrhs,))
    if not live:
        m = np.all(pts == lo, axis=1)
        if m.sum() != 1:
            raise ValueError("0-dimensional box is not a sample point")
        out[(0,) * d] = vals[np.nonzero(m)[0][0]]
        return out
    if len(live) == 1:
        i = live[0]
        pos = pts[:, i]
        order = np.argsort(pos)
        pos, v = pos[order], vals[order]
        if pos[0] != lo[i] or pos[-1] != hi[i]:
            raise ValueError("edge endpoints are not sample points")
        xs = np.arange(lo[i], hi[i] + 1)
        line = np.stack([np.interp(xs, pos, v[:, j]) for j in range(nrhs)], axis=1)
        shp = [1] * d
        shp[i] = S[i]
        return line.reshape(tuple(shp) + (nrhs,)) * np.ones(S + (1,))
    # boundary: every facet (or the boxes a broken facet is made of), recursively
    for i in live:
        for sd, side in ((0, lo[i]), (1, hi[i])):
            if facet_parts is not None and len(live) >= 3:
                parts = facet_parts(i, sd)
            else:
                flo = lo.copy()
                fhi = hi.copy()
                flo[i] = side
                fhi[i] = side
                parts = [(flo, fhi)]
            for plo, phi in parts:
                on = np.all((pts >= plo) & (pts <= phi), axis=1)
                fv = harmonic_on_box(plo, phi, pts[on], vals[on])
                sl = tuple(slice(int(plo[j] - lo[j]), int(phi[j] - lo[j] + 1)) for j in range(d))
                out[sl] = fv
    return _laplace_dirichlet(out)


def multilinear_on_box(lo, hi, pts):
    """Closed form for a leaf whose only sample points are its 2^d corners:
    the multilinear hat of each corner (used as a fast path and pinned against
    the Laplace solve in the tests)."""
    d = len(lo)
    S = tuple(int(h - l + 1) for l, h in zip(lo, hi))
    out = np.zeros(S + (pts.shape[0],))
    grids = np.meshgrid(*[np.arange(l, h + 1, dtype=np.float64) for l, h in zip(lo, hi)], indexing="ij")
    for j, p in enumerate(pts):
        w = np.ones(S)
        for i in range(d):
            if hi[i] == lo[i]:
                continue
            w = w * (1.0 - np.abs(grids[i] - p[i]) / float(hi[i] - lo[i]))
        out[..., j] = w
    return out


def leaf_weights(grid, c, closed_form=True):
    """Weights on leaf c of all sample points in it: (pts_idx, array S + (P,))."""
    lo, hi = grid.leaf_lo[c], grid.leaf_hi[c]
    idx = grid.leaf_points[c]
    pts = grid.points[idx]
    d = grid.d
    ncorner = 2 ** sum(1 for i in range(d) if hi[i] > lo[i])
    if closed_form and len(idx) == ncorner:
        return idx, multilinear_on_box(lo, hi, pts)
    vals = np.eye(len(idx))
    return idx, harmonic_on_box(lo, hi, pts, vals, facet_parts=lambda i, sd: grid.facet_parts(c, i, sd))


def harmonic_weights(grid, closed_form=True):
    """w_k on bbox(U_k) for every k (zero on bbox(U_k) \\ U_k)."""
    W = [np.zeros(tuple(int(v) for v in (grid.u_hi[k] - grid.u_lo[k] + 1))) for k in range(grid.r)]
    for c in range(grid.leaf_lo.shape[0]):
        idx, vals = leaf_weights(grid, c, closed_form)
        lo, hi = grid.leaf_lo[c], grid.leaf_hi[c]
        for j, k in enumerate(idx):
            off = lo - grid.u_lo[k]
            sl = tuple(slice(int(off[i]), int(off[i] + hi[i] - lo[i] + 1)) for i in range(grid.d))
            W[k][sl] = vals[..., j]
    return W
