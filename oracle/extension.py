"""Extended impulse responses phi_k^E (Sec. 2.5).

phi_j is defined on its domain of definition Omega - p_j.  The caller supplies
it on the box prod [-R_j, R_j]; inside the domain of definition and outside
that box it is zero (the blur is truncated there).

With the counting function c_k = 1_{Omega-p_k} + sum_{j in nbrs(k), j != k}
1_{(Omega-p_j) \\ (Omega-p_k)}, v_k = 1/c_k on supp(c_k), and the split
weights v_k^(j) (eq. (2.7)), the extension is
phi_k^E = sum_{j in nbrs(k)} v_k^(j) . phi_j: phi_k itself where defined, the
plain average of the neighbours defined there elsewhere, 0 where none is.

phi_k^E is only ever evaluated at offsets y - x with y in Omega and x in U_k,
so it is stored on Zbox_k = (Omega - bbox(U_k)) intersected with the union of
the neighbours' patch boxes; it is zero outside.

Where neighbours were supplied on boxes of unequal radii, a neighbour counts
in the average wherever its domain of definition covers the offset, also where
its supplied box does not (it contributes 0 there): Sec. 2.5 states
supp(phi_j) = Omega - p_j for the counting function c_k.  Pinned by
hand-derived values with equal and with unequal radii (tests/golden).
"""
import numpy as np


def _patch(phi, phi_off, radius, j):
    R = radius[j]
    shape = tuple(int(2 * v + 1) for v in R)
    return phi[phi_off[j]:phi_off[j + 1]].reshape(shape)


def _defined_mask(shape, p, zlo, zshape):
    """1_{Omega - p} on the offset box starting at zlo."""
    d = len(shape)
    m = np.ones(zshape, dtype=bool)
    for i in range(d):
        z = np.arange(zlo[i], zlo[i] + zshape[i])
        ok = (p[i] + z >= 0) & (p[i] + z <= shape[i] - 1)
        sh = [1] * d
        sh[i] = zshape[i]
        m &= ok.reshape(sh)
    return m


def _values(phi, phi_off, radius, j, zlo, zshape):
    """phi_j on the offset box (zero outside its supplied patch)."""
    d = len(zlo)
    R = radius[j]
    P = _patch(phi, phi_off, radius, j)
    out = np.zeros(zshape)
    src, dst = [], []
    for i in range(d):
        a = max(zlo[i], -R[i])
        b = min(zlo[i] + zshape[i] - 1, R[i])
        if a > b:
            return out
        src.append(slice(int(a + R[i]), int(b + R[i] + 1)))
        dst.append(slice(int(a - zlo[i]), int(b - zlo[i] + 1)))
    out[tuple(dst)] = P[tuple(src)]
    return out


def extended_kernels(grid, radius, phi, phi_off, extend=True):
    """Return (zlo[k], phiE[k]) for every k: phi_k^E on the offset box Zbox_k."""
    shape = grid.shape
    d = grid.d
    radius = np.asarray(radius, dtype=np.int64).reshape(-1, d)
    n = np.array(shape)
    zlos, kernels = [], []
    for k in range(grid.r):
        nb = grid.nbrs[k] if extend else [k]
        rmax = radius[nb].max(axis=0)
        # offsets reachable from U_k into Omega, cut to the neighbours' patches
        zlo = np.maximum(-rmax, 0 - grid.u_hi[k])
        zhi = np.minimum(rmax, n - 1 - grid.u_lo[k])
        zshape = tuple(int(v) for v in np.maximum(zhi - zlo + 1, 0))
        pk = grid.points[k]
        own = _defined_mask(shape, pk, zlo, zshape)
        out = np.where(own, _values(phi, phi_off, radius, k, zlo, zshape), 0.0)
        if extend:
            count = np.zeros(zshape)
            acc = np.zeros(zshape)
            for j in nb:
                if j == k:
                    continue
                mj = _defined_mask(shape, grid.points[j], zlo, zshape) & ~own
                count += mj
                acc += np.where(mj, _values(phi, phi_off, radius, j, zlo, zshape), 0.0)
            fill = (~own) & (count > 0)
            out = np.where(fill, acc / np.where(count > 0, count, 1.0), out)
        zlos.append(zlo.astype(np.int64))
        kernels.append(out)
    return zlos, kernels


def split_weights(grid, k, zlo, zshape):
    """v_k^(j) for j in nbrs(k) on an offset box (eq. (2.7)); used by the
    tests of Lemma 2 and Prop. 1."""
    shape = grid.shape
    own = _defined_mask(shape, grid.points[k], zlo, zshape)
    c = own.astype(np.float64).copy()
    masks = {}
    for j in grid.nbrs[k]:
        if j == k:
            continue
        mj = _defined_mask(shape, grid.points[j], zlo, zshape) & ~own
        masks[j] = mj
        c += mj
    v = np.where(c > 0, 1.0 / np.where(c > 0, c, 1.0), 0.0)
    out = {k: v * own}
    for j, mj in masks.items():
        out[j] = v * mj
    return out
