"""GPU tests of the estimator-driven refinement loop (Sec. 2.3, 2.6, 2.7)."""
import numpy as np
import pytest
import torch

from oracle import OracleOperator, estimate
from workloads import make_config, BlurOperator, corner_points
from tests.tilings import workload_from, tensor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible HIP device")
    from paper_1805_06018_amd import _lib, refine
    from workloads.blur_gpu import GpuBlurAdjoint
    return _lib, refine, GpuBlurAdjoint


def test_exact_blur_adjoint_matches_cpu(mods):
    _, _, GpuBlurAdjoint = mods
    n0, n1 = 23, 31
    x0, x1 = np.meshgrid(np.arange(n0), np.arange(n1), indexing="ij")
    s0 = 0.8 + 1.5 * x0 / n0
    s1 = 1.2 + 0.7 * np.cos(x1 / 5.0)
    op = BlurOperator(np.stack([s0, s1]))
    V = np.random.default_rng(3).standard_normal((3, n0 * n1))
    ref = np.stack([op.apply(v, adjoint=True) for v in V])
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 2e-6)):
        g = GpuBlurAdjoint(op, dtype=dt)
        out = g(torch.from_numpy(V).to(device="cuda", dtype=dt)).cpu().numpy()
        err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
        assert err < tol, (dt, err)


def test_exact_blur_adjoint_3d_matches_cpu(mods):
    _, _, GpuBlurAdjoint = mods
    n = (9, 11, 13)
    x0, x1, x2 = np.meshgrid(*(np.arange(v) for v in n), indexing="ij")
    sig = np.stack([0.7 + 0.9 * x0 / 8, 1.1 + 0.4 * np.sin(x1 / 3.0), 0.8 + 0.7 * x2 / 12])
    op = BlurOperator(sig)
    V = np.random.default_rng(4).standard_normal((10, int(np.prod(n))))
    ref = np.stack([op.apply(v, adjoint=True) for v in V])
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 2e-6)):
        g = GpuBlurAdjoint(op, dtype=dt)
        out = g(torch.from_numpy(V).to(device="cuda", dtype=dt)).cpu().numpy()
        err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
        assert err < tol, (dt, err)


def test_refinement_loop_converges_and_matches_oracle(mods):
    _lib, refine, GpuBlurAdjoint = mods
    # 256^2 with widths scaled like the grid (s in [1, 4]), 4 x 4 start
    from workloads import cosine_field, uniform_nodes, tensor_leaves
    n = 256
    s, _ = cosine_field((n, n), 1.0, 4.0, 2, 3, seed=3)
    nodes = uniform_nodes(n, 4)
    lo0, hi0 = tensor_leaves([nodes, nodes])
    w = workload_from(np.stack([s, s]), lo0, hi0)
    q = 8
    Zh = w.rademacher(q, 7)
    Z = torch.from_numpy(Zh.astype(np.float32)).cuda()
    Y = GpuBlurAdjoint(w.op)(Z)
    torch.cuda.synchronize()
    lo, hi, rounds = refine.refine(w.shape, w.leaf_lo, w.leaf_hi, w.op.impulse_responses, w.op.patch, Z, Y,
                                   tol=2e-2, max_points=800, frac=0.15)
    errs = [r["eta_rel"] for r in rounds]
    print("rounds", len(rounds), "points", [r["points"] for r in rounds], "eta_rel", errs, flush=True)
    assert rounds[-1]["points"] >= 800 or errs[-1] < 2e-2
    assert errs[-1] < 0.8 * errs[0]
    # final grid: the GPU estimate against the oracle's on the same Z and Y
    pts = corner_points(lo, hi)
    radius, phi, off = w.op.impulse_responses(pts)
    op = _lib.PcOperator(2, w.shape, lo, hi, pts, radius, phi, off, dtype=_lib.PC_F32)
    eta, eabs, erel = op.error_estimate(Z, Y)
    ora = OracleOperator(w.shape, lo, hi, pts, radius, phi, off)
    eta_o, eabs_o, erel_o, _ = estimate(ora, Zh, Y.cpu().numpy().astype(np.float64))
    assert abs(erel - erel_o) <= 1e-3 * erel_o, (erel, erel_o)
    assert np.abs(eta - eta_o).max() <= 1e-3 * eta_o.max()
