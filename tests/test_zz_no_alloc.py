"""The allocation-free batched apply (pc_apply_batch_noalloc) through the C
ABI: on two calls in a row, the second with a smaller batch and new input,
its output equals pc_apply_batch's bit for bit and the FP64 oracle's within
the per-vector bars (FP32 1e-5, FP64 1e-12 relative L2).  2-D operators run
it both ways: colour launches (no work area needed) and the staged schedule
(PC_TUNE_DIRECT = 0), whose staging lives in the fixed work area.  Operators
whose staging for one vector exceeds the work area are refused before
anything is enqueued."""
import sys

import numpy as np
import pytest
import torch

from oracle import OracleOperator
from workloads import make_config
from tests.libhelpers import small_cases, small_cases_3d, relerr, TOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible HIP device")
    from paper_1805_06018_amd import _lib
    return _lib


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _two_calls(lib, w, dtype, sizes, seed, oracle_rows, direct=1):
    tdt = torch.float64 if dtype == lib.PC_F64 else torch.float32
    ndt = np.float64 if dtype == lib.PC_F64 else np.float32
    op = lib.PcOperator.from_workload(w, dtype=dtype)
    op.set_tuning(lib.PC_TUNE_DIRECT, direct)
    ora = OracleOperator.from_workload(w)
    rng = np.random.default_rng(seed)
    for call, B in enumerate(sizes):
        _note(f"noalloc {w.name} dtype={dtype} direct={direct} call={call} B={B}")
        U = rng.standard_normal((B, w.N)).astype(ndt)
        Ud = torch.from_numpy(U).cuda()
        got = torch.full_like(Ud, float("nan"))
        op.apply_batch_noalloc(Ud, got)
        ref = torch.full_like(Ud, float("nan"))
        op.apply_batch(Ud, ref)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (w.name, call)
        rows = [j for j in oracle_rows if j < B]
        want = ora.apply_batch(U[rows].astype(np.float64))
        e = relerr(got.cpu().numpy()[rows], want)
        assert e.max() <= TOL[dtype], (w.name, call, e)
    op.close()


@pytest.mark.parametrize("name", ["hanging33", "cfg1_small", "rect45x301"])
def test_noalloc_2d_small(lib, name):
    w = dict(small_cases())[name]
    w.name = name
    for dtype in (lib.PC_F32, lib.PC_F64):
        for direct in (0, 1):
            _two_calls(lib, w, dtype, (7, 3), 71, range(7), direct)


@pytest.mark.parametrize("name", ["cube24", "hang3d"])
def test_noalloc_3d_small(lib, name):
    w = dict(small_cases_3d())[name]
    w.name = name
    for dtype in (lib.PC_F32, lib.PC_F64):
        _two_calls(lib, w, dtype, (3, 1), 73, range(3))


def test_noalloc_blur1024(lib):
    """The 1024^2 workload in FP32, staged: 65 MB of staging per vector, so
    the work area takes two vectors per chunk; 5 vectors then 2."""
    w = make_config(1)
    _two_calls(lib, w, lib.PC_F32, (5, 2), 75, (0,), direct=0)


def test_noalloc_refuses_what_does_not_fit(lib):
    """The 1024^2 workload with an FP64 operator, staged, needs 252 MB of
    staging per vector: PC_ERR_UNSUPPORTED, output untouched."""
    w = make_config(1)
    op = lib.PcOperator.from_workload(w, dtype=lib.PC_F64)
    op.set_tuning(lib.PC_TUNE_DIRECT, 0)
    U = torch.zeros((1, w.N), dtype=torch.float64, device="cuda")
    out = torch.full_like(U, 3.0)
    with pytest.raises(lib.PcError) as ei:
        op.apply_batch_noalloc(U, out)
    assert ei.value.status == lib.PC_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert torch.all(out == 3.0)
    op.close()
