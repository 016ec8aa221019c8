"""Pins of the oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks a property that a
mistake in the weights, the extension or the sums would break (partition of
unity, closed forms, hand-derived values, exactness for convolutions, the
a-priori bound of Thm. 1, a library convolution, brute force on tiny grids).
"""
import os
import numpy as np
import pytest
import scipy.signal

from oracle import OracleOperator, Grid, TilingError, estimate, harmonic_weights
from oracle.extension import extended_kernels, split_weights
from oracle.weights import leaf_weights, harmonic_on_box
from workloads import make_config, BlurOperator, uniform_nodes, tensor_leaves
from tests.tilings import (hanging_2d, hanging_3d, extrude, const_blur, workload_from, tensor, refine,
                           unequal_radii_3x3)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _pu_check(op, tol=1e-14):
    g = op.grid
    total = np.zeros(op.shape)
    for k in range(g.r):
        sl = tuple(slice(int(g.u_lo[k, i]), int(g.u_hi[k, i] + 1)) for i in range(op.d))
        assert op.W[k].min() >= -1e-15
        total[sl] += op.W[k]
        for j in range(g.r):            # w_k[p_j] = delta_kj where p_j in bbox(U_k)
            p = g.points[j]
            if np.all(p >= g.u_lo[k]) and np.all(p <= g.u_hi[k]):
                assert abs(op.W[k][tuple(p - g.u_lo[k])] - (1.0 if j == k else 0.0)) < 1e-15
    assert np.abs(total - 1.0).max() < tol


# ---------------------------------------------------------------- weights (Sec. 2.4)
@pytest.mark.parametrize("case", ["cfg0", "hanging", "hanging_solve", "1d", "3d", "3d_hanging"])
def test_partition_of_unity(case):
    if case == "cfg0":
        op = OracleOperator.from_workload(make_config(0))
    elif case in ("hanging", "hanging_solve"):
        lo, hi = hanging_2d(17, levels=3)
        w = const_blur((17, 17), 1.0, lo, hi)
        op = OracleOperator.from_workload(w, closed_form_weights=(case == "hanging"))
    elif case == "1d":
        lo = np.array([[0], [5], [7], [15]])
        hi = np.array([[5], [7], [15], [20]])
        op = OracleOperator.from_workload(const_blur((21,), 1.0, lo, hi))
    elif case == "3d":
        lo, hi = tensor((9, 8, 7), 3)
        op = OracleOperator.from_workload(const_blur((9, 8, 7), 0.8, lo, hi), closed_form_weights=False)
    else:
        lo, hi = hanging_3d(9)
        op = OracleOperator.from_workload(const_blur((9, 9, 9), 0.8, lo, hi))
    _pu_check(op)


def test_golden_hanging_node_weights():
    """Hand-derived values on a leaf with a hanging node (tests/golden)."""
    lo = np.array([[0, 0], [0, 2], [1, 2]])
    hi = np.array([[2, 2], [1, 4], [2, 4]])
    g = Grid((3, 5), lo, hi)
    W = harmonic_weights(g, closed_form=True)
    rows = np.loadtxt(os.path.join(GOLD, "hanging_node_weights_3x5.txt"))
    for k, y0, y1, val in rows:
        k = int(k)
        y = np.array([int(y0), int(y1)])
        assert np.all(y >= g.u_lo[k]) and np.all(y <= g.u_hi[k])
        assert abs(W[k][tuple(y - g.u_lo[k])] - val) < 1e-15, (k, y, val)


def test_closed_form_equals_laplace_on_conforming_cells():
    """Multilinear functions are discrete-harmonic for the Kronecker-sum
    Laplacian, so on conforming cells the solve must give the hat."""
    for lo, hi in [((0, 0), (6, 9)), ((3, 1, 2), (7, 5, 5)), ((2,), (11,))]:
        lo, hi = np.array(lo), np.array(hi)
        import itertools
        pts = np.array(sorted({tuple(int(hi[i] if b else lo[i]) for i, b in enumerate(bits))
                               for bits in itertools.product((0, 1), repeat=len(lo))}))
        sol = harmonic_on_box(lo, hi, pts, np.eye(len(pts)))
        from oracle.weights import multilinear_on_box
        ml = multilinear_on_box(lo, hi, pts)
        assert np.abs(sol - ml).max() < 1e-13


def test_hanging_cell_is_discrete_harmonic():
    """Interior 5-point residual of every weight on hanging-node cells."""
    lo, hi = hanging_2d(33, levels=3)
    g = Grid((33, 33), lo, hi)
    nhang = 0
    for c in range(len(lo)):
        idx, vals = leaf_weights(g, c, closed_form=True)
        if len(idx) == 4:
            continue
        nhang += 1
        v = vals
        res = (v[2:, 1:-1] + v[:-2, 1:-1] + v[1:-1, 2:] + v[1:-1, :-2] - 4 * v[1:-1, 1:-1])
        assert np.abs(res).max() < 1e-12
        # edges: piecewise linear between the sample points lying on them
        for e in (v[0], v[-1], v[:, 0], v[:, -1]):
            second = e[2:] - 2 * e[1:-1] + e[:-2]
            kinks = np.abs(second) > 1e-12
            assert kinks.sum() <= 2 * len(idx)
    assert nhang > 0


def test_3d_broken_facets_extruded_tiling_is_2d_times_hat():
    """A 3-D tiling made of a 2-D hanging-node tiling times z intervals: its
    harmonic weights are the 2-D weights times the linear hats in z (the
    product of a discrete-harmonic 2-D function and a linear function is
    discrete-harmonic for the Kronecker-sum Laplacian, and the extension is
    unique).  Ties the 3-D face and volume solves to the pinned 2-D ones."""
    lo2, hi2 = hanging_2d(17, corner=(16, 0), levels=2)
    zn = [0, 3, 8]
    lo, hi = extrude(lo2, hi2, zn)
    g3 = Grid((17, 17, 9), lo, hi)
    g2 = Grid((17, 17), lo2, hi2)
    assert any(len(ix) > 8 for ix in g3.leaf_points)          # broken facets present
    W3 = harmonic_weights(g3, closed_form=False)
    W2 = harmonic_weights(g2, closed_form=False)
    for k, p in enumerate(g3.points):
        k2 = g2.index[(int(p[0]), int(p[1]))]
        z = np.arange(g3.u_lo[k, 2], g3.u_hi[k, 2] + 1)
        j = zn.index(int(p[2]))
        hat = np.zeros(z.size)
        for a, b in zip(zn[:-1], zn[1:]):
            m = (z >= a) & (z <= b)
            if p[2] == a:
                hat[m] = np.maximum(hat[m], 1.0 - (z[m] - a) / (b - a))
            elif p[2] == b:
                hat[m] = np.maximum(hat[m], (z[m] - a) / (b - a))
        assert j >= 0
        sl = tuple(slice(int(g3.u_lo[k, i] - g2.u_lo[k2, i]), int(g3.u_hi[k, i] - g2.u_lo[k2, i] + 1))
                   for i in range(2))
        ref = W2[k2][sl][:, :, None] * hat[None, None, :]
        assert np.abs(W3[k] - ref).max() < 1e-12, k


def test_3d_broken_facets_are_discrete_harmonic_and_continuous():
    """Octant-refined 9^3 tiling: on every leaf the weights satisfy the
    7-point Laplacian in the interior and the 5-point one inside each box a
    facet is made of; adjacent leaves give the same values on shared facets;
    sample-point values are delta."""
    lo, hi = hanging_3d(9)
    g = Grid((9, 9, 9), lo, hi)
    per_leaf = {c: leaf_weights(g, c, closed_form=False) for c in range(len(lo))}
    nbroken = 0
    for c, (idx, v) in per_leaf.items():
        res = (v[2:, 1:-1, 1:-1] + v[:-2, 1:-1, 1:-1] + v[1:-1, 2:, 1:-1] + v[1:-1, :-2, 1:-1] +
               v[1:-1, 1:-1, 2:] + v[1:-1, 1:-1, :-2] - 6 * v[1:-1, 1:-1, 1:-1])
        assert np.abs(res).max() < 1e-12 if res.size else True
        for i in range(3):
            for sd in (0, 1):
                parts = g.facet_parts(c, i, sd)
                nbroken += len(parts) > 1
                for plo, phi in parts:
                    sl = tuple(slice(int(plo[j] - lo[c][j]), int(phi[j] - lo[c][j] + 1)) for j in range(3))
                    f = np.squeeze(v[sl], axis=i)
                    if min(f.shape[:2]) >= 3:
                        r2 = f[2:, 1:-1] + f[:-2, 1:-1] + f[1:-1, 2:] + f[1:-1, :-2] - 4 * f[1:-1, 1:-1]
                        assert np.abs(r2).max() < 1e-12
        pts = g.points[idx]
        for j, p in enumerate(pts):
            assert abs(v[tuple(p - lo[c])][j] - 1.0) < 1e-14
    assert nbroken > 0
    # continuity: values of each point's weight agree on the intersection of two leaves
    for c in range(len(lo)):
        for e in range(c + 1, len(lo)):
            a = np.maximum(lo[c], lo[e])
            b = np.minimum(hi[c], hi[e])
            if np.any(a > b):
                continue
            ic, vc = per_leaf[c]
            ie, ve = per_leaf[e]
            for j, k in enumerate(ic):
                if k not in ie:
                    continue
                je = int(np.nonzero(ie == k)[0][0])
                sc = tuple(slice(int(a[i] - lo[c][i]), int(b[i] - lo[c][i] + 1)) for i in range(3))
                se = tuple(slice(int(a[i] - lo[e][i]), int(b[i] - lo[e][i] + 1)) for i in range(3))
                assert np.abs(vc[sc][..., j] - ve[se][..., je]).max() < 1e-12


# ---------------------------------------------------------------- extension (Sec. 2.5)
def _golden_extension_case(radii, c):
    w = unequal_radii_3x3(radii, c)
    return Grid(w.shape, w.leaf_lo, w.leaf_hi), w.radius, w.phi, w.phi_off


def _check_golden_extension(fname, radii, c):
    g, R, phi, off = _golden_extension_case(radii, c)
    rows = np.loadtxt(os.path.join(GOLD, fname))
    for extend, col in ((True, 3), (False, 4)):
        zlo, K = extended_kernels(g, R, phi, off, extend=extend)
        for row in rows:
            k, z = int(row[0]), np.array([int(row[1]), int(row[2])])
            idx = z - zlo[k]
            if np.any(idx < 0) or np.any(idx >= np.array(K[k].shape)):
                val = 0.0
            else:
                val = K[k][tuple(idx)]
            assert val == row[col], (fname, extend, k, z, val, row[col])


UNEQUAL_RADII = [1, 2, 3, 2, 3, 1, 3, 1, 2]


@pytest.mark.parametrize("fname,radii,c", [("extension_2d_3x3.txt", [2] * 9, 2),
                                           ("extension_unequal_radii.txt", UNEQUAL_RADII, 3)])
def test_golden_extension_values(fname, radii, c):
    """Hand-derived phi_k^E (Sec. 2.5, eq. (2.7)-(2.8)) with equal and with
    unequal neighbour radii (tests/golden)."""
    _check_golden_extension(fname, radii, c)


def test_golden_unequal_radii_rejects_box_support(monkeypatch):
    """Planting the other reading in the oracle (a neighbour counts only where
    its supplied box covers z) must break the unequal-radii golden: the pin
    fixes the paper's supp(phi_j) = Omega - p_j."""
    import oracle.extension as ext
    g, R, _, _ = _golden_extension_case(UNEQUAL_RADII, 3)
    rad = {tuple(int(v) for v in g.points[j]): int(R[j, 0]) for j in range(g.r)}
    plain = ext._defined_mask

    def box_mask(shape, p, zlo, zshape):
        m = plain(shape, p, zlo, zshape)
        r = rad[tuple(int(v) for v in p)]
        for i in range(len(zlo)):
            z = np.arange(zlo[i], zlo[i] + zshape[i])
            sh = [1] * len(zlo)
            sh[i] = zshape[i]
            m = m & (np.abs(z) <= r).reshape(sh)
        return m

    monkeypatch.setattr(ext, "_defined_mask", box_mask)
    with pytest.raises(AssertionError):
        _check_golden_extension("extension_unequal_radii.txt", UNEQUAL_RADII, 3)


def test_lemma2_split_weights_sum():
    """Lemma 2: sum_j v_k^(j) = 1 exactly on Omega - U_k and 0 elsewhere."""
    lo, hi = hanging_2d(17, levels=3)
    g = Grid((17, 17), lo, hi)
    n = np.array(g.shape)
    for k in range(g.r):
        zlo = -n + 1
        zshape = tuple(2 * n - 1)
        v = split_weights(g, k, zlo, zshape)
        total = sum(v.values())
        # brute-force Minkowski difference Omega - U_k over U_k's points
        inU = np.zeros(g.shape, dtype=bool)
        for c in g.cells[k]:
            inU[tuple(slice(int(g.leaf_lo[c, i]), int(g.leaf_hi[c, i] + 1)) for i in range(2))] = True
        xs = np.argwhere(inU)
        diff = np.zeros(zshape, dtype=bool)
        for x in xs:
            # y - x for y in Omega covers the box [-x, n-1-x]
            a = -x - zlo
            diff[a[0]:a[0] + n[0], a[1]:a[1] + n[1]] = True
        assert np.abs(total[diff] - 1.0).max() < 1e-15
        assert np.abs(total[~diff]).max() == 0.0


def test_prop1_product_partition_of_unity():
    """Prop. 1(2): W_k[y,x] = sum_{j in nbrs(k)} w_j[x] v_j^(k)[y-x] sums to 1
    over k for every (y, x) in Omega x Omega."""
    lo, hi = hanging_2d(9, levels=2)
    w = const_blur((9, 9), 0.7, lo, hi)
    op = OracleOperator.from_workload(w)
    g = op.grid
    n = np.array(g.shape)
    N = op.N
    zlo = -n + 1
    zshape = tuple(2 * n - 1)
    V = [split_weights(g, j, zlo, zshape) for j in range(g.r)]
    coords = np.array(np.unravel_index(np.arange(N), g.shape)).T
    S = np.zeros((N, N))
    for j in range(g.r):
        wj = np.zeros(g.shape)
        sl = tuple(slice(int(g.u_lo[j, i]), int(g.u_hi[j, i] + 1)) for i in range(2))
        wj[sl] = op.W[j]
        wj = wj.ravel()
        for k, vjk in V[j].items():
            # S[y, x] += w_j[x] v_j^(k)[y - x]
            dz = coords[:, None, :] - coords[None, :, :] - zlo   # (y, x, 2)
            S += wj[None, :] * vjk[dz[..., 0], dz[..., 1]]
    assert np.abs(S - 1.0).max() < 1e-14


# ---------------------------------------------------------------- apply (eq. (2.5))
@pytest.mark.parametrize("case", ["1d", "2d_uniform", "2d_hanging", "3d", "3d_hanging"])
def test_exact_for_convolutions(case):
    """Thm. 1 with F = 0: a restricted convolution is reproduced exactly by any
    tiling, hanging nodes included (no boundary artifacts)."""
    rng = np.random.default_rng(7)
    if case == "1d":
        lo = np.array([[0], [9], [13], [30]])
        hi = np.array([[9], [13], [30], [40]])
        w = const_blur((41,), 2.2, lo, hi)
    elif case == "2d_uniform":
        lo, hi = tensor((20, 23), 4)
        w = const_blur((20, 23), 1.6, lo, hi)
    elif case == "2d_hanging":
        lo, hi = hanging_2d(25, corner=(24, 0), levels=3)
        w = const_blur((25, 25), 1.9, lo, hi)
    elif case == "3d_hanging":
        lo, hi = hanging_3d(9)
        w = const_blur((9, 9, 9), 0.8, lo, hi)
    else:
        lo, hi = tensor((9, 10, 8), 3)
        w = const_blur((9, 10, 8), 0.9, lo, hi)
    op = OracleOperator.from_workload(w)
    for _ in range(2):
        u = rng.standard_normal(op.N)
        ref = w.op.apply(u)
        assert np.linalg.norm(op.apply(u) - ref) <= 1e-13 * np.linalg.norm(ref)
        assert np.linalg.norm(op.apply_adjoint(u) - w.op.apply(u, adjoint=True)) <= 1e-13 * np.linalg.norm(ref)
    # zero extension shows boundary artifacts on the same operator
    op0 = OracleOperator.from_workload(w, extend=False)
    u = rng.standard_normal(op.N)
    ref = w.op.apply(u)
    assert np.linalg.norm(op0.apply(u) - ref) > 1e-3 * np.linalg.norm(ref)


def test_fig2_one_dimensional_boundary_artifacts():
    """Fig. 2: A is a Gaussian convolution restricted to [0, N-1], sample points
    at both ends.  Extension by zero gives artifacts; the neighbour extension
    reproduces A exactly."""
    n = 40
    w = const_blur((n,), 3.0, np.array([[0]]), np.array([[n - 1]]))
    A = w.op.dense()
    At = OracleOperator.from_workload(w).dense()
    A0 = OracleOperator.from_workload(w, extend=False).dense()
    assert np.abs(At - A).max() < 1e-15
    assert np.abs(A0 - A).max() > 1e-2


def test_identity_operator():
    """phi_k = delta (radius 0): A~ = sum_k w_k . f = f by the partition of unity."""
    lo, hi = hanging_2d(17, levels=3)
    g_pts = Grid((17, 17), lo, hi).points
    r = len(g_pts)
    op = OracleOperator((17, 17), lo, hi, g_pts, np.zeros((r, 2), dtype=np.int64),
                        np.ones(r), np.arange(r + 1))
    u = np.random.default_rng(1).standard_normal(op.N)
    assert np.abs(op.apply(u) - u).max() < 1e-14
    assert np.abs(op.apply_adjoint(u) - u).max() < 1e-14


def test_single_leaf_matches_library_convolution():
    """One leaf (Omega itself) and a convolution kernel: A~ f equals
    scipy.signal.convolve(f, psi) cropped to Omega."""
    n0, n1, s = 20, 24, 1.5
    w = const_blur((n0, n1), s, np.array([[0, 0]]), np.array([[n0 - 1, n1 - 1]]))
    op = OracleOperator.from_workload(w)
    psi = w.op.patch((0, 0))
    R = (psi.shape[0] - 1) // 2
    u = np.random.default_rng(3).standard_normal((n0, n1))
    ref = scipy.signal.convolve(u, psi, mode="full", method="direct")[R:R + n0, R:R + n1]
    assert np.abs(op.apply(u).reshape(n0, n1) - ref).max() < 1e-14
    v = np.random.default_rng(4).standard_normal((n0, n1))
    refa = scipy.signal.correlate(v, psi, mode="full", method="direct")[R:R + n0, R:R + n1]
    assert np.abs(op.apply_adjoint(v).reshape(n0, n1) - refa).max() < 1e-14


def _varying_case(n=11):
    lo, hi = hanging_2d(n, levels=2)
    x0, x1 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    s = 0.6 + 0.5 * (x0 + 0.5 * x1) / n
    return workload_from(np.stack([s, s]), lo, hi)


def test_dense_entries_and_adjoint_consistency():
    """Matrix entries (Sec. 3.1) times f equal the convolution sum; the adjoint
    apply equals the transpose (eq. (1.6))."""
    w = _varying_case()
    op = OracleOperator.from_workload(w)
    A = op.dense()
    rng = np.random.default_rng(9)
    u, v = rng.standard_normal(op.N), rng.standard_normal(op.N)
    assert np.abs(A @ u - op.apply(u)).max() < 1e-14
    assert np.abs(A.T @ v - op.apply_adjoint(v)).max() < 1e-14
    assert abs(np.dot(op.apply(u), v) - np.dot(u, op.apply_adjoint(v))) < 1e-13 * np.linalg.norm(u) * np.linalg.norm(v)
    for (y, x) in [((3, 4), (2, 2)), ((0, 10), (1, 9)), ((7, 7), (7, 7))]:
        yi = np.ravel_multi_index(y, op.shape)
        xi = np.ravel_multi_index(x, op.shape)
        assert abs(op.entry(np.array(y), np.array(x)) - A[yi, xi]) < 1e-15


def test_theorem1_pointwise_bound():
    """Thm. 1: |A~ - A| <= F pointwise (hence in Frobenius norm), with
    F[y,x] = max over k with (y,x) in mu_k^E of |A[y-x+p_k, p_k] - A[y,x]|."""
    w = _varying_case(13)
    op = OracleOperator.from_workload(w)
    g = op.grid
    A = w.op.dense()
    At = op.dense()
    N, shape = op.N, op.shape
    coords = np.array(np.unravel_index(np.arange(N), shape)).T
    inU = []
    for k in range(g.r):
        m = np.zeros(shape, dtype=bool)
        for c in g.cells[k]:
            m[tuple(slice(int(g.leaf_lo[c, i]), int(g.leaf_hi[c, i] + 1)) for i in range(2))] = True
        inU.append(m.ravel())
    F = np.full((N, N), -1.0)
    for k in range(g.r):
        UE = np.zeros(N, dtype=bool)
        for j in g.nbrs[k]:
            UE |= inU[j]
        pk = g.points[k]
        tgt = coords[:, None, :] - coords[None, :, :] + pk          # y - x + p_k
        ok = np.all((tgt >= 0) & (tgt < np.array(shape)), axis=2) & UE[None, :]
        ti = np.ravel_multi_index((np.clip(tgt[..., 0], 0, shape[0] - 1),
                                   np.clip(tgt[..., 1], 0, shape[1] - 1)), shape)
        Fk = np.abs(A[ti, np.ravel_multi_index(tuple(pk), shape)] - A)
        F = np.where(ok, np.maximum(F, Fk), F)
    assert F.min() >= 0.0                                           # every (y,x) is covered
    err = np.abs(At - A)
    assert np.all(err <= F + 1e-15)
    assert np.linalg.norm(At - A) <= np.linalg.norm(F) + 1e-14
    assert np.linalg.norm(At - A) > 1e-3                            # the case is not trivial


def test_locally_constant_kernel_columns_exact():
    """If every impulse response a column x touches is the same kernel and
    A's column x has that kernel too, A~[:, x] = A[:, x] (the zero final error
    of Sec. 5.1)."""
    n = 33
    lo, hi = tensor((n, n), 5)
    x0, _ = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    s = np.where(x0 < 16, 1.0, 1.6)
    w = workload_from(np.stack([s, s]), lo, hi)
    op = OracleOperator.from_workload(w)
    g = op.grid
    A, At = w.op.dense(), op.dense()
    ps = np.array([w.op.width_at(p)[0] for p in g.points])
    good = bad = 0
    for xf in range(op.N):
        x = np.array(np.unravel_index(xf, op.shape))
        ks = [k for k in range(g.r) if np.all(x >= g.u_lo[k]) and np.all(x <= g.u_hi[k])
              and op.W[k][tuple(x - g.u_lo[k])] > 0]
        widths = {ps[j] for k in ks for j in g.nbrs[k]} | {s[tuple(x)]}
        if len(widths) == 1:
            assert np.abs(At[:, xf] - A[:, xf]).max() < 1e-15
            good += 1
        else:
            bad += int(np.abs(At[:, xf] - A[:, xf]).max() > 1e-6)
    assert good > 100 and bad > 10


# ---------------------------------------------------------------- estimator (Sec. 2.6)
def test_estimator_matches_dense_computation():
    w = _varying_case(11)
    op = OracleOperator.from_workload(w)
    A, At = w.op.dense(), op.dense()
    rng = np.random.default_rng(11)
    q = 7
    Z = rng.standard_normal((q, op.N))
    Y = (A.T @ Z.T).T
    eta, eta_om, eta_rel, Yt = estimate(op, Z, Y)
    D = (At.T - A.T) @ Z.T                                          # (N, q)
    g = op.grid
    for c in range(len(g.leaf_lo)):
        m = np.zeros(op.shape, dtype=bool)
        m[tuple(slice(int(g.leaf_lo[c, i]), int(g.leaf_hi[c, i] + 1)) for i in range(2))] = True
        assert abs(eta[c] - np.linalg.norm(D[m.ravel()]) / np.sqrt(q)) < 1e-13
    assert abs(eta_om - np.linalg.norm(D) / np.sqrt(q)) < 1e-13
    assert abs(eta_rel - np.linalg.norm(D) / np.linalg.norm(Y)) < 1e-13


def test_estimator_is_unbiased_for_cell_errors():
    """eq. (2.10): eta_C^2 -> e_C^2 = ||(A~ - A)[Omega, C]||_F^2 as q grows."""
    w = _varying_case(9)
    op = OracleOperator.from_workload(w)
    A, At = w.op.dense(), op.dense()
    q = 3000
    Z = np.random.default_rng(12).standard_normal((q, op.N))
    Y = (A.T @ Z.T).T
    eta, *_ = estimate(op, Z, Y)
    g = op.grid
    for c in range(len(g.leaf_lo)):
        m = np.zeros(op.shape, dtype=bool)
        m[tuple(slice(int(g.leaf_lo[c, i]), int(g.leaf_hi[c, i] + 1)) for i in range(2))] = True
        e2 = np.linalg.norm((At - A)[:, m.ravel()]) ** 2
        assert abs(eta[c] ** 2 - e2) <= 5 * np.sqrt(2.0 / q) * e2 + 1e-30


# ---------------------------------------------------------------- grid (Sec. 2.2)
def test_tiling_validation():
    lo, hi = tensor((9, 9), 3)
    Grid((9, 9), lo, hi)
    with pytest.raises(TilingError):                  # gap
        Grid((9, 9), lo[:-1], hi[:-1])
    with pytest.raises(TilingError):                  # overlap
        Grid((9, 9), np.vstack([lo, [[1, 1]]]), np.vstack([hi, [[3, 3]]]))
    with pytest.raises(TilingError):                  # outside
        Grid((9, 9), lo, hi + 1)
    g = Grid((9, 9), lo, hi)
    with pytest.raises(TilingError):                  # points != corners
        Grid((9, 9), lo, hi, g.points[:-1])


def test_neighbourhoods_on_hanging_grid():
    lo = np.array([[0, 0], [0, 2], [1, 2]])
    hi = np.array([[2, 2], [1, 4], [2, 4]])
    g = Grid((3, 5), lo, hi)
    k = g.index[(1, 2)]                               # hanging node on C1's edge
    assert sorted(g.cells[k]) == [0, 1, 2]
    assert g.nbrs[k] == list(range(8))
    assert list(g.u_lo[k]) == [0, 0] and list(g.u_hi[k]) == [2, 4]
    k0 = g.index[(0, 0)]
    assert g.nbrs[k0] == sorted([g.index[p] for p in [(0, 0), (0, 2), (1, 2), (2, 0), (2, 2)]])


def test_c_core_matches_numpy_loops():
    w = make_config(0)
    op = OracleOperator.from_workload(w)
    u = w.vectors()[0]
    a = op.apply(u, backend="numpy")
    b = op.apply(u, backend="c")
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()
    assert np.abs(op.apply_adjoint(u, backend="numpy") - op.apply_adjoint(u, backend="c")).max() < 1e-13
    ys = np.array([[0, 0], [63, 63], [31, 7], [5, 60]])
    assert np.abs(op.apply_at(u, ys) - a.reshape(64, 64)[ys[:, 0], ys[:, 1]]).max() < 1e-13


@pytest.mark.parametrize("name", ["cfg0", "hanging33", "rect45x301", "cube24", "hang3d"])
def test_window_applies_match_full_applies(name):
    """apply_window / apply_adjoint_window (the C core restricted to a box of
    outputs, used for the full-size checks over whole rows and planes) equal
    the NumPy-loop full applies restricted to the box, for boxes inside,
    touching the edges of, and covering Omega."""
    from tests.libhelpers import small_cases, small_cases_3d
    w = dict(small_cases() + small_cases_3d())[name]
    op = OracleOperator.from_workload(w)
    u = np.random.default_rng(23).standard_normal(op.N)
    full = op.apply(u, backend="numpy").reshape(op.shape)
    fulla = op.apply_adjoint(u, backend="numpy").reshape(op.shape)
    n = np.array(op.shape)
    boxes = [(n // 3, n // 3 + n // 4), (np.zeros_like(n), n - 1), (n - 1, n - 1), (np.zeros_like(n), n // 5)]
    for lo, hi in boxes:
        sl = tuple(slice(int(a), int(b) + 1) for a, b in zip(lo, hi))
        scale = np.abs(full).max()
        assert np.abs(op.apply_window(u, lo, hi) - full[sl].ravel()).max() <= 1e-13 * scale
        assert np.abs(op.apply_adjoint_window(u, lo, hi) - fulla[sl].ravel()).max() <= 1e-13 * np.abs(fulla).max()


def test_sampled_adjoint_matches_full_adjoint():
    """apply_adjoint_at (used for full-size sampled checks) against the full
    adjoint, itself pinned by the transpose and exactness tests."""
    w = _varying_case(13)
    op = OracleOperator.from_workload(w)
    v = np.random.default_rng(21).standard_normal(op.N)
    full = op.apply_adjoint(v).reshape(op.shape)
    xs = np.array([[0, 0], [12, 12], [3, 7], [12, 0], [6, 6]])
    assert np.abs(op.apply_adjoint_at(v, xs) - full[xs[:, 0], xs[:, 1]]).max() < 1e-13


def test_term_subsets_partition_the_sum():
    """Sums over complementary subsets of the terms add up to the full apply
    (each term counted once), forward and adjoint (Sec. 2.8 recomputes only a
    subset of the terms after a refinement)."""
    w = make_config(0)
    op = OracleOperator.from_workload(w)
    rng = np.random.default_rng(12)
    S = rng.permutation(w.r)[:11]
    Sc = np.setdiff1d(np.arange(w.r), S)
    u = rng.standard_normal(w.N)
    for adj in (False, True):
        fn = op.apply_adjoint if adj else op.apply
        full = fn(u)
        part = fn(u, patches=S) + fn(u, patches=Sc)
        assert np.abs(part - full).max() <= 1e-13 * np.abs(full).max()
        assert np.all(fn(u, patches=[]) == 0.0)
