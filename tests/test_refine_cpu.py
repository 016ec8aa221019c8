"""The estimator-driven refinement loop on the CPU, judged by the oracle
(Sec. 2.3, Sec. 2.6, Sec. 2.7, Algorithm 1).

Workload: the 2048^2 refinement recipe at 128^2 (widths in [2, 16], two
cosine modes with wave numbers up to 3, a 4 x 4 start grid whose spacing is
a third of the domain).  Each round the oracle's estimator (eq. (2.11), four
Rademacher probes, Y = A* Z from the exact blur) picks the leaves and
tiling.split_round splits them.  The judge is the oracle's relative error
estimate with eight fresh probes: the adaptive tiling must beat the uniform
tiling with at least as many points, and the corner-only direction rule,
which aliases on this recipe, must be beaten by the midplane rule."""
import numpy as np
import pytest

from oracle import OracleOperator, estimate
from workloads import make_config, uniform_nodes, tensor_leaves
from paper_1805_06018_amd.tiling import corner_points, split_direction, split_round


@pytest.fixture(scope="module")
def recipe():
    w = make_config(3, scale=1 / 16)
    Z = w.rademacher(4, 103)
    Y = np.stack([w.op.apply(z, adjoint=True) for z in Z])
    Zj = w.rademacher(8, 977)
    Yj = np.stack([w.op.apply(z, adjoint=True) for z in Zj])
    return w, Z, Y, Zj, Yj


def _oracle(w, lo, hi):
    pts = corner_points(lo, hi)
    radius, phi, off = w.op.impulse_responses(pts)
    return OracleOperator(w.shape, lo, hi, pts, radius, phi, off), len(pts)


def _loop(w, Z, Y, rule, max_points):
    lo, hi = w.leaf_lo.copy(), w.leaf_hi.copy()
    while True:
        ora, npts = _oracle(w, lo, hi)
        if npts >= max_points:
            return ora, npts
        eta, _, _, _ = estimate(ora, Z, Y)
        lo, hi = split_round(lo, hi, eta, 0.1, w.shape, w.op.patch, rule)


def test_midplane_rule_sees_the_aliased_axis(recipe):
    """The start leaves are a third of the domain wide, the period of the
    k = 3 mode: along axis 0 their faces see the same phase, so the
    corner-only rule picks axis 1 on every start leaf; the midplane rule
    picks axis 0 on some."""
    w = recipe[0]
    axes = {rule: [split_direction(lo, hi, w.shape, w.op.patch, rule) for lo, hi in zip(w.leaf_lo, w.leaf_hi)]
            for rule in ("faces", "midplane")}
    assert set(axes["faces"]) == {1}, axes
    assert set(axes["midplane"]) == {0, 1}, axes


def test_adaptive_refinement_beats_uniform(recipe):
    w, Z, Y, Zj, Yj = recipe
    ora, npts = _loop(w, Z, Y, "midplane", 240)
    err_adaptive = estimate(ora, Zj, Yj)[2]
    m = int(np.ceil(np.sqrt(npts)))              # uniform m x m nodes, m^2 >= npts
    nodes = uniform_nodes(w.shape[0], m)
    ulo, uhi = tensor_leaves([nodes, nodes])
    ora_u, npts_u = _oracle(w, ulo, uhi)
    err_uniform = estimate(ora_u, Zj, Yj)[2]
    ora_f, npts_f = _loop(w, Z, Y, "faces", 240)
    err_faces = estimate(ora_f, Zj, Yj)[2]
    print(f"points adaptive {npts} uniform {npts_u} faces {npts_f}; "
          f"rel. error adaptive {err_adaptive:.4f} uniform {err_uniform:.4f} faces {err_faces:.4f}")
    assert npts_u >= npts
    assert err_adaptive < 0.8 * err_uniform
    assert err_adaptive < 0.5 * err_faces
