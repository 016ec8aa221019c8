"""GPU parity of the HIP library against the FP64 oracle, through the C ABI.

Bars (per-vector relative L2 against the FP64 oracle on the same
dtype-rounded inputs): FP32 <= 1e-5, FP64 <= 1e-12.  Small cases compare
every output; the full-size workloads compare all of Omega (1024^2, 8 of
the 64 vectors), complete 8-row slabs (2048^2) or complete axis-0 planes
(128^3), the relative L2 taken over the compared outputs.  Integer/layout
properties (batch vs single apply, plain vs fused, repeat runs) are checked
bitwise.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import OracleOperator, estimate
from workloads import make_config
from tests.libhelpers import small_cases, relerr, TOL

pytestmark = pytest.mark.gpu


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible HIP device")


@pytest.fixture(scope="module")
def lib():
    _require_gpu()
    from paper_1805_06018_amd import _lib
    return _lib


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dt(dtype):
    return (torch.float64, np.float64) if dtype == 1 else (torch.float32, np.float32)


@pytest.mark.parametrize("idx", range(7))
def test_small_cases_parity(lib, idx):
    name, w = small_cases()[idx]
    rng = np.random.default_rng(200 + idx)
    U = rng.standard_normal((5, w.N))
    for flags in (0, lib.PC_NO_EXTEND, lib.PC_PLAN_SMALLEST_FFT):
        ora = OracleOperator.from_workload(w, extend=((flags & lib.PC_NO_EXTEND) == 0))
        for dtype in (lib.PC_F64, lib.PC_F32):
            _note(f"case={name} flags={flags} dtype={dtype}")
            tdt, ndt = _dt(dtype)
            op = lib.PcOperator.from_workload(w, dtype=dtype, flags=flags)
            Ur = U.astype(ndt)
            Ud = torch.from_numpy(Ur).cuda()
            for adj in (False, True):
                out = torch.full_like(Ud, float("nan"))
                (op.apply_adjoint_batch if adj else op.apply_batch)(Ud, out)
                torch.cuda.synchronize()
                ref = ora.apply_batch(Ur.astype(np.float64), adjoint=adj)
                e = relerr(out.cpu().numpy(), ref)
                assert e.max() <= TOL[dtype], (name, flags, dtype, adj, e)
            op.close()


def test_batch_column_equals_single_apply_and_plain(lib):
    w = make_config(1, scale=0.25)
    op = lib.PcOperator.from_workload(w, dtype=lib.PC_F32)
    U = torch.from_numpy(w.vectors(7, dtype=np.float32)).cuda()
    out = torch.zeros_like(U)
    op.apply_batch(U, out)
    plain = torch.zeros_like(U)
    op.apply_batch_plain(U, plain)
    single = torch.zeros(w.N, dtype=torch.float32, device="cuda")
    again = torch.zeros_like(U)
    op.apply_batch(U, again)
    torch.cuda.synchronize()
    assert torch.equal(out, again)                   # repeat run: bitwise
    assert torch.equal(out, plain)                   # plain path: same sums, same order
    for j in (0, 3, 6):
        op.apply(U[j].contiguous(), single)
        torch.cuda.synchronize()
        assert torch.equal(single, out[j])           # column j of the batch
    # empty batch is a no-op; strided rows are honoured
    empty = torch.zeros((0, w.N), dtype=torch.float32, device="cuda")
    op.apply_batch(empty, empty)
    Ubig = torch.zeros((3, w.N + 64), dtype=torch.float32, device="cuda")
    Ubig[:, :w.N] = U[:3]
    Obig = torch.full((3, w.N + 64), 7.0, dtype=torch.float32, device="cuda")
    op.apply_batch(Ubig[:, :w.N], Obig[:, :w.N])
    torch.cuda.synchronize()
    assert torch.equal(Obig[:, :w.N], out[:3])
    assert torch.all(Obig[:, w.N:] == 7.0)
    # colour launches (outputs zeroed, each colour's disjoint boxes added in
    # place, vector chunks on 1, 2 or 4 streams): the same bits, forward and
    # adjoint, also into strided outputs
    adj_ref = torch.zeros_like(U)
    op.apply_adjoint_batch(U, adj_ref)
    op.set_tuning(lib.PC_TUNE_DIRECT, 1)
    for streams, chunk in ((1, 0), (2, 0), (4, 2), (4, 0)):
        op.set_tuning(lib.PC_TUNE_STREAMS, streams)
        op.set_tuning(lib.PC_TUNE_CHUNK, chunk)
        got = torch.full_like(U, float("nan"))
        op.apply_batch(U, got)
        gota = torch.full_like(U, float("nan"))
        op.apply_adjoint_batch(U, gota)
        Ob = torch.full((3, w.N + 64), 7.0, dtype=torch.float32, device="cuda")
        op.apply_batch(Ubig[:, :w.N], Ob[:, :w.N])
        torch.cuda.synchronize()
        assert torch.equal(got, out) and torch.equal(gota, adj_ref), (streams, chunk)
        assert torch.equal(Ob[:, :w.N], out[:3]) and torch.all(Ob[:, w.N:] == 7.0)
    op.set_tuning(lib.PC_TUNE_DIRECT, 0)
    op.set_tuning(lib.PC_TUNE_CHUNK, 0)
    # persistent convolution launches (units from per-XCD queues), the
    # item-major block order and one launch for all items (no two-per-CU
    # part for the small items): the same bits
    for key, val in ((lib.PC_TUNE_PERSISTENT, 1), (lib.PC_TUNE_XCD_ORDER, 1), (lib.PC_TUNE_SPLIT, 0)):
        op.set_tuning(key, val)
        for chunk in (0, 3):
            op.set_tuning(lib.PC_TUNE_CHUNK, chunk)
            got = torch.full_like(U, float("nan"))
            op.apply_batch(U, got)
            gota = torch.full_like(U, float("nan"))
            op.apply_adjoint_batch(U, gota)
            torch.cuda.synchronize()
            assert torch.equal(got, out) and torch.equal(gota, adj_ref), (key, chunk)
        op.set_tuning(key, 1 - val)
    op.set_tuning(lib.PC_TUNE_CHUNK, 0)


def test_profiling_times_every_launch(lib):
    """pc_set_profiling / pc_read_profile: every convolution and reduction
    launch of a timed call is counted with a positive duration, whichever
    launch form runs (two-part staged launch and single launch time through
    events carried by their dispatches, the persistent form through events
    around its launches, the plain path per item), and timing changes no
    bit of the result."""
    w = make_config(1, scale=0.25)
    _note(f"profiling: r={w.r}")
    op = lib.PcOperator.from_workload(w, dtype=lib.PC_F32)
    n_items = op.stats()["n_items"]
    U = torch.from_numpy(w.vectors(7, dtype=np.float32)).cuda()
    ref = torch.zeros_like(U)
    op.apply_batch(U, ref)
    torch.cuda.synchronize()
    op.read_profile()
    for key, val, off in ((lib.PC_TUNE_SPLIT, 1, 1), (lib.PC_TUNE_SPLIT, 0, 1), (lib.PC_TUNE_PERSISTENT, 1, 0)):
        op.set_tuning(key, val)
        for chunk, launches in ((0, 1), (3, 3)):
            op.set_tuning(lib.PC_TUNE_CHUNK, chunk)
            op.set_profiling(True)
            for adj in (False, True):
                got = torch.full_like(U, float("nan"))
                (op.apply_adjoint_batch if adj else op.apply_batch)(U, got)
            op.set_profiling(False)
            pr = op.read_profile()
            torch.cuda.synchronize()
            assert pr["conv_launches"] == 2 * launches and pr["reduce_launches"] == 2 * launches, (key, val, pr)
            assert pr["conv_vectors"] == 2 * 7 and pr["conv_ms"] > 0 and pr["reduce_ms"] > 0, (key, val, pr)
            out = torch.zeros_like(U)
            op.apply_batch(U, out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (key, val, chunk)
        op.set_tuning(key, off)
    op.set_tuning(lib.PC_TUNE_CHUNK, 0)
    # the plain path: one timed launch per item and vector
    op.set_profiling(True)
    plain = torch.zeros_like(U)
    op.apply_batch_plain(U, plain)
    op.set_profiling(False)
    pr = op.read_profile()
    assert pr["conv_launches"] == 7 * n_items and pr["reduce_launches"] == 7, pr
    assert torch.equal(plain, ref)
    # nothing left over once read
    pr = op.read_profile()
    assert pr["conv_launches"] == 0 and pr["reduce_launches"] == 0
    op.close()


FULL_VECTORS = tuple(range(0, 64, 9))   # 8 of the 64 vectors: 0, 9, ..., 63


def _rel_l2(got, ref):
    return float(np.linalg.norm(np.asarray(got, dtype=np.float64) - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("adjoint", [False, True])
def test_full_size_blur1024_batch64(lib, adjoint):
    """The benchmark workload (1024^2, ~600 points, B = 64, FP32) in the
    launch configuration the benchmark times: 8 of the 64 vectors (first,
    last and every 9th) against full oracle applies (adjoint: A~* of the
    same batch), per-vector relative L2 over all of Omega <= 1e-5."""
    w = make_config(1)
    _note(f"blur1024: r={w.r} adjoint={adjoint}")
    op = lib.PcOperator.from_workload(w, dtype=lib.PC_F32)
    U = w.vectors(64, dtype=np.float32)
    Ud = torch.from_numpy(U).cuda()
    out = torch.zeros_like(Ud)
    (op.apply_adjoint_batch if adjoint else op.apply_batch)(Ud, out)
    # the persistent form of the launch and the single launch for all items
    # give the same bits
    for key, val in ((lib.PC_TUNE_PERSISTENT, 1), (lib.PC_TUNE_SPLIT, 0)):
        op.set_tuning(key, val)
        again = torch.full_like(Ud, float("nan"))
        (op.apply_adjoint_batch if adjoint else op.apply_batch)(Ud, again)
        torch.cuda.synchronize()
        assert torch.equal(again, out), key
        op.set_tuning(key, 1 - val)
    got = out.cpu().numpy()
    assert np.all(np.isfinite(got))
    ora = OracleOperator.from_workload(w)
    fn = ora.apply_adjoint if adjoint else ora.apply
    errs = {}
    for j in FULL_VECTORS:
        _note(f"oracle {'adjoint' if adjoint else 'apply'} of vector {j}")
        errs[j] = _rel_l2(got[j], fn(U[j].astype(np.float64)))
    _note(f"rel-L2 per vector: {errs}")
    assert max(errs.values()) <= TOL[lib.PC_F32], errs


def test_full_size_blur1024_fp64(lib):
    """The 1024^2 workload with an FP64 operator (512-thread kernel, FP64 row
    pieces): 9 vectors, so the default 8-vector launches end with a ragged
    1-vector launch; vectors 0, 1 and 8 forward and 0 and 8 adjoint against
    full oracle applies, relative L2 <= 1e-12."""
    w = make_config(1)
    _note(f"blur1024 fp64: r={w.r}")
    op = lib.PcOperator.from_workload(w, dtype=lib.PC_F64)
    U = w.vectors(9, dtype=np.float64)
    Ud = torch.from_numpy(U).cuda()
    out = torch.zeros_like(Ud)
    op.apply_batch(Ud, out)
    outa = torch.zeros_like(Ud)
    op.apply_adjoint_batch(Ud, outa)
    torch.cuda.synchronize()
    got, gota = out.cpu().numpy(), outa.cpu().numpy()
    assert np.all(np.isfinite(got)) and np.all(np.isfinite(gota))
    ora = OracleOperator.from_workload(w)
    errs = {}
    for j in (0, 1, 8):
        _note(f"oracle apply of vector {j}")
        errs[("fwd", j)] = _rel_l2(got[j], ora.apply(U[j]))
    for j in (0, 8):
        _note(f"oracle adjoint of vector {j}")
        errs[("adj", j)] = _rel_l2(gota[j], ora.apply_adjoint(U[j]))
    _note(f"rel-L2: {errs}")
    assert max(errs.values()) <= TOL[lib.PC_F64], errs


class _DevView:
    """A device array view built from a raw pointer (for the callback)."""

    def __init__(self, ptr, rows, cols, ld, typestr, esz):
        self.__cuda_array_interface__ = {"shape": (rows, cols), "typestr": typestr, "data": (ptr, False),
                                         "version": 2, "strides": (ld * esz, esz)}


@pytest.mark.parametrize("dtype", [1, 0])
def test_error_estimate_matches_oracle(lib, dtype):
    from tests.tilings import hanging_2d, workload_from
    n = 33
    lo, hi = hanging_2d(n, corner=(0, 32), levels=3)
    x0, x1 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    s = 0.7 + 1.2 * (x0 + 2 * x1) / (3 * n)
    w = workload_from(np.stack([s, s]), lo, hi)
    tdt, ndt = _dt(dtype)
    A = w.op.dense()
    q = 6
    Z = np.random.default_rng(31).standard_normal((q, w.N)).astype(ndt)
    Y = np.ascontiguousarray((A.T @ Z.astype(np.float64).T).T.astype(ndt))
    ora = OracleOperator.from_workload(w)
    eta_o, eom_o, erel_o, _ = estimate(ora, Z.astype(np.float64), Y.astype(np.float64))
    op = lib.PcOperator.from_workload(w, dtype=dtype)
    Zd = torch.from_numpy(Z).cuda()
    Yd = torch.from_numpy(Y).cuda()
    eta, eom, erel = op.error_estimate(Zd, Yd)
    # Tolerances from the apply's own bar.  The estimate differs from the
    # oracle's only through Y~ (Y and Z are the same numbers on both sides):
    # with E = Y~_gpu - Y~_oracle, the reverse triangle inequality gives
    # |eta_C - eta_C,o| <= q^-1/2 ||E_C||_F, the same for eta_Omega over all
    # of Omega, and |eta_rel - eta_rel,o| <= ||E||_F / ||Y||_F.  The per-vector
    # bar ||e_i|| <= delta ||y~_i|| bounds ||E||_F <= delta ||Y~_o||_F.  The
    # GPU Y~ (the same adjoint launch as inside the estimate) is checked
    # against the bar first, then the estimate against both the bound from
    # delta and the tighter one from the measured E (FP64 sums: slack 1e-12).
    delta = TOL[dtype]
    Yt_o = ora.apply_batch(Z.astype(np.float64), adjoint=True)
    Ytd = torch.zeros_like(Zd)
    op.apply_adjoint_batch(Zd, Ytd)
    torch.cuda.synchronize()
    Yt_g = Ytd.cpu().numpy().astype(np.float64)
    assert relerr(Yt_g, Yt_o).max() <= delta
    E = Yt_g - Yt_o
    fro_t = np.linalg.norm(Yt_o)
    fro_y = np.linalg.norm(Y.astype(np.float64))
    Eg = E.reshape((q,) + tuple(w.shape))
    leaf_E = np.array([np.linalg.norm(Eg[(slice(None),) + tuple(slice(int(a), int(b) + 1) for a, b in zip(lo_c, hi_c))])
                       for lo_c, hi_c in zip(ora.grid.leaf_lo, ora.grid.leaf_hi)])
    slack = 1e-12
    assert np.all(np.abs(eta - eta_o) <= delta * fro_t / np.sqrt(q) + slack * eta_o.max())
    assert np.all(np.abs(eta - eta_o) <= leaf_E / np.sqrt(q) + slack * eta_o.max())
    assert abs(eom - eom_o) <= min(delta * fro_t, np.linalg.norm(E)) / np.sqrt(q) + slack * eom_o
    assert abs(erel - erel_o) <= min(delta * fro_t, np.linalg.norm(E)) / fro_y + slack * erel_o
    # exact adjoint supplied through the callback instead of Y: the estimate
    # then also moves by the callback's own rounding, dY = Y_cb - Y, so the
    # bound becomes q^-1/2 (||E_C||_F + ||dY_C||_F)
    At = torch.from_numpy(A.astype(ndt)).cuda()
    esz = 8 if dtype == 1 else 4
    typestr = "<f8" if dtype == 1 else "<f4"
    calls = []

    def cb(B, iptr, ldi, optr, ldo, sptr):
        zin = torch.as_tensor(_DevView(iptr, B, w.N, ldi, typestr, esz), device="cuda")
        yout = torch.as_tensor(_DevView(optr, B, w.N, ldo, typestr, esz), device="cuda")
        yout.copy_(zin @ At)
        torch.cuda.synchronize()
        calls.append(yout.cpu().numpy().astype(np.float64))
        return 0

    eta2, eom2, erel2 = op.error_estimate(Zd, None, exact_adjoint=cb)
    assert len(calls) == 1 and calls[0].shape == (q, w.N)
    dY = (calls[0] - Y.astype(np.float64)).reshape((q,) + tuple(w.shape))
    leaf_dY = np.array([np.linalg.norm(dY[(slice(None),) + tuple(slice(int(a), int(b) + 1) for a, b in zip(lo_c, hi_c))])
                        for lo_c, hi_c in zip(ora.grid.leaf_lo, ora.grid.leaf_hi)])
    assert np.all(np.abs(eta2 - eta_o) <= (leaf_E + leaf_dY) / np.sqrt(q) + slack * eta_o.max())
    # a failing callback reports PC_ERR_CALLBACK and leaves the operator usable
    with pytest.raises(lib.PcError) as ei:
        op.error_estimate(Zd, None, exact_adjoint=lambda *a: 3)
    assert ei.value.status == lib.PC_ERR_CALLBACK
    eta3, _, _ = op.error_estimate(Zd, Yd)
    assert np.array_equal(eta3, eta)


def test_apply_argument_errors(lib):
    w = make_config(0)
    op = lib.PcOperator.from_workload(w, dtype=lib.PC_F64)
    U = torch.zeros((2, w.N - 1), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.PcError) as ei:
        op.apply_batch(U, U)
    assert ei.value.status == lib.PC_ERR_ARG
    with pytest.raises(TypeError):
        op.apply_batch(torch.zeros((1, w.N), dtype=torch.float32, device="cuda"),
                       torch.zeros((1, w.N), dtype=torch.float32, device="cuda"))


def test_work_buffer_budget_and_device_sums(lib):
    """PC_TUNE_BUDGET: a call whose staging would take the operator's work
    buffers beyond the budget returns PC_ERR_BUDGET and leaves its output
    untouched; within the budget it runs, and buffers grow in stream order
    (a larger batch after a smaller one on another stream).  The estimator
    sums left on the device give the same numbers as pc_estimate_sums."""
    w = make_config(1, scale=0.25)
    op = lib.PcOperator.from_workload(w, dtype=lib.PC_F32)
    op.set_tuning(lib.PC_TUNE_DIRECT, 0)                 # the staged schedule (colour launches need no buffer)
    per = op.stats()["slot_elems_fwd"] * 4
    op.set_tuning(lib.PC_TUNE_BUDGET, 2 * per)
    U = torch.from_numpy(w.vectors(6, dtype=np.float32)).cuda()
    out = torch.full_like(U, 5.0)
    with pytest.raises(lib.PcError) as ei:
        op.apply_batch(U, out)
    assert ei.value.status == lib.PC_ERR_BUDGET
    torch.cuda.synchronize()
    assert torch.all(out == 5.0)
    op.apply_batch(U[:2], out[:2])                       # fits: 2 vectors of staging
    op.set_tuning(lib.PC_TUNE_BUDGET, 0)
    assert op.device_bytes() >= op.stats()["device_bytes"] + 2 * per
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        op.apply_batch(U, out, stream=side)              # grows the staging on another stream
    torch.cuda.synchronize()
    ref = torch.zeros_like(U)
    op.apply_batch_plain(U, ref)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    Y = torch.from_numpy(w.vectors(4, dtype=np.float32, seed=9)).cuda()
    eta, ea, er = op.estimate_sums(U[:4], Y)
    sums = torch.full((op.n_leaves + 2,), float("nan"), dtype=torch.float64, device="cuda")
    op.estimate_sums_device(U[:4], Y, sums)
    torch.cuda.synchronize()
    eta2, ea2, er2 = op.eta_from_sums(sums.cpu().numpy(), 4)
    assert np.array_equal(eta, eta2) and ea == ea2 and er == er2
    op.close()


def test_large_pieces_blur2048_start_grid(lib):
    """2048^2 start grid (16 points, cells 683 wide, kernels up to 129^2): every
    patch is cut into a grid of row x column pieces.  Forward and adjoint of
    two vectors against the oracle on seven 8-row slabs of complete rows
    (the domain edges, the cell boundaries at 682 / 1365 and between),
    relative L2 per slab <= 1e-5."""
    w = make_config(3)
    op = lib.PcOperator.from_workload(w, dtype=lib.PC_F32)
    _note(f"blur2048 start: items={op.stats()['n_items']}")
    U = w.vectors(2, dtype=np.float32)
    Ud = torch.from_numpy(U).cuda()
    fwd = torch.zeros_like(Ud)
    adj = torch.zeros_like(Ud)
    op.apply_batch(Ud, fwd)
    op.apply_adjoint_batch(Ud, adj)
    torch.cuda.synchronize()
    n = w.shape[0]
    fwd = fwd.cpu().numpy().reshape(2, n, n)
    adj = adj.cpu().numpy().reshape(2, n, n)
    ora = OracleOperator.from_workload(w)
    errs = {}
    for r0 in (0, 340, 678, 1020, 1361, 1700, n - 8):
        lo, hi = (r0, 0), (r0 + 7, n - 1)
        for j in range(2):
            u = U[j].astype(np.float64)
            errs[("fwd", r0, j)] = _rel_l2(fwd[j, r0:r0 + 8].ravel(), ora.apply_window(u, lo, hi))
            errs[("adj", r0, j)] = _rel_l2(adj[j, r0:r0 + 8].ravel(), ora.apply_adjoint_window(u, lo, hi))
    _note(f"max rel-L2 over slabs: {max(errs.values()):.3e}")
    assert max(errs.values()) <= TOL[lib.PC_F32], errs


# ------------------------------------------------------------------- 3-D
@pytest.mark.parametrize("idx", range(3))
def test_small_cases_3d_parity(lib, idx):
    from tests.libhelpers import small_cases_3d
    name, w = small_cases_3d()[idx]
    rng = np.random.default_rng(300 + idx)
    U = rng.standard_normal((3, w.N))
    for flags in (0, lib.PC_NO_EXTEND, lib.PC_PLAN_SMALLEST_FFT):
        ora = OracleOperator.from_workload(w, extend=((flags & lib.PC_NO_EXTEND) == 0))
        for dtype in (lib.PC_F64, lib.PC_F32):
            _note(f"case={name} flags={flags} dtype={dtype}")
            tdt, ndt = _dt(dtype)
            op = lib.PcOperator.from_workload(w, dtype=dtype, flags=flags)
            Ur = U.astype(ndt)
            Ud = torch.from_numpy(Ur).cuda()
            for adj in (False, True):
                out = torch.full_like(Ud, float("nan"))
                (op.apply_adjoint_batch if adj else op.apply_batch)(Ud, out)
                torch.cuda.synchronize()
                ref = ora.apply_batch(Ur.astype(np.float64), adjoint=adj)
                e = relerr(out.cpu().numpy(), ref)
                assert e.max() <= TOL[dtype], (name, flags, dtype, adj, e)
            op.close()


def test_3d_schedules_are_bitwise_equal(lib):
    """Batch vs single vector, plain per-item launches, vector chunks of one
    and item groups of one item (tiny scratch) all give the same bits."""
    from tests.libhelpers import small_cases_3d
    _, w = small_cases_3d()[1]
    op = lib.PcOperator.from_workload(w, dtype=lib.PC_F32)
    U = torch.from_numpy(np.random.default_rng(4).standard_normal((4, w.N)).astype(np.float32)).cuda()
    for adj in (False, True):
        fn = op.apply_adjoint_batch if adj else op.apply_batch
        ref = torch.zeros_like(U)
        fn(U, ref)
        torch.cuda.synchronize()
        if not adj:
            plain = torch.zeros_like(U)
            op.apply_batch_plain(U, plain)
            single = torch.zeros(w.N, dtype=torch.float32, device="cuda")
            op.apply(U[2].contiguous(), single)
            torch.cuda.synchronize()
            assert torch.equal(plain, ref)
            assert torch.equal(single, ref[2])
        op.set_tuning(lib.PC_TUNE_SCRATCH, 1)     # every group holds one item
        op.set_tuning(lib.PC_TUNE_CHUNK, 1)
        other = torch.zeros_like(U)
        fn(U, other)
        torch.cuda.synchronize()
        op.set_tuning(lib.PC_TUNE_SCRATCH, 0)
        op.set_tuning(lib.PC_TUNE_CHUNK, 0)
        assert torch.equal(other, ref), adj


def test_error_estimate_3d_matches_oracle(lib):
    from tests.libhelpers import small_cases_3d
    _, w = small_cases_3d()[0]
    ora = OracleOperator.from_workload(w)
    q = 4
    Z = np.random.default_rng(41).standard_normal((q, w.N))
    Y = np.stack([w.op.apply(z, adjoint=True) for z in Z])
    eta_o, eom_o, erel_o, _ = estimate(ora, Z, Y)
    op = lib.PcOperator.from_workload(w, dtype=lib.PC_F64)
    eta, eom, erel = op.error_estimate(torch.from_numpy(Z).cuda(), torch.from_numpy(Y).cuda())
    assert eta.shape == eta_o.shape
    assert np.abs(eta - eta_o).max() <= 1e-10 * eta_o.max()
    assert abs(erel - erel_o) <= 1e-10 * erel_o


PLANES_128 = tuple(range(0, 128, 8)) + (127,)     # every 8th axis-0 plane and the last


@pytest.mark.parametrize("dtype", [0, 1])
def test_full_size_blur3d_128(lib, dtype):
    """The 3-D workload (128^3, 9^3 points): FP32 with B = 16 in the batched
    launch configuration, FP64 with B = 2.  Complete axis-0 planes against
    the oracle (every 8th plane and the last; a full oracle apply is out of
    reach): forward of the first and last vector, adjoint of vector 0,
    relative L2 over the planes <= 1e-5 (FP32) / 1e-12 (FP64)."""
    w = make_config(2)
    B = 16 if dtype == 0 else 2
    tdt, ndt = _dt(dtype)
    op = lib.PcOperator.from_workload(w, dtype=dtype)
    _note(f"blur3d: dtype={dtype} items={op.stats()['n_items']}")
    U = w.vectors(B, dtype=ndt)
    Ud = torch.from_numpy(U).cuda()
    fwd = torch.zeros_like(Ud)
    adj = torch.zeros_like(Ud)
    op.apply_batch(Ud, fwd)
    op.apply_adjoint_batch(Ud[:2], adj[:2])
    torch.cuda.synchronize()
    n = w.shape[0]
    fwd = fwd.cpu().numpy().reshape(B, n, n * n)
    adj = adj.cpu().numpy().reshape(B, n, n * n)
    assert np.all(np.isfinite(fwd))
    ora = OracleOperator.from_workload(w)
    planes = list(PLANES_128)
    errs = {}
    for kind, j in (("fwd", 0), ("fwd", B - 1), ("adj", 0)):
        _note(f"oracle {kind} of vector {j} on {len(planes)} planes")
        u = U[j].astype(np.float64)
        fn = ora.apply_adjoint_window if kind == "adj" else ora.apply_window
        got = adj[j] if kind == "adj" else fwd[j]
        ref = np.concatenate([fn(u, (q, 0, 0), (q, n - 1, n - 1)) for q in planes])
        errs[(kind, j)] = _rel_l2(got[planes].ravel(), ref)
    _note(f"rel-L2: {errs}")
    assert max(errs.values()) <= TOL[dtype], errs


# ------------------------------------------------------------ matrix entries
@pytest.mark.parametrize("name", ["cfg0", "hanging33", "cube24", "hang3d"])
def test_entries_match_oracle(lib, name):
    """pc_entries (Sec. 3.1) against the oracle's entry formula, FP64 and
    FP32; out-of-range pairs give NaN; entries agree with applies to unit
    vectors (columns of A~)."""
    from tests.libhelpers import small_cases_3d
    w = dict(small_cases() + small_cases_3d())[name]
    ora = OracleOperator.from_workload(w)
    rng = np.random.default_rng(21)
    n = np.array(w.shape)
    xs = rng.integers(0, n, (500, w.d))
    xs[:30] = w.points[rng.integers(0, w.r, 30)]
    ys = np.clip(xs + rng.integers(-8, 9, (500, w.d)), 0, n - 1)
    ref = np.array([ora.entry(y, x) for y, x in zip(ys, xs)])
    scale = np.abs(ref).max()
    for dtype, tol in ((lib.PC_F64, 1e-13), (lib.PC_F32, 2e-6)):
        op = lib.PcOperator.from_workload(w, dtype=dtype)
        got = op.entries(torch.from_numpy(ys).cuda(), torch.from_numpy(xs).cuda()).cpu().numpy()
        assert np.abs(got - ref).max() <= tol * scale, (name, dtype)
        bad = op.entries(torch.tensor([list(n)], dtype=torch.int64).cuda(),
                         torch.zeros((1, w.d), dtype=torch.int64).cuda()).cpu().numpy()
        assert np.isnan(bad[0])
        if dtype == lib.PC_F64:
            # column x of A~ from an apply to the unit vector at x
            x = xs[5]
            e = torch.zeros(w.N, dtype=torch.float64, device="cuda")
            e[int(np.ravel_multi_index(tuple(x), w.shape))] = 1.0
            col = torch.zeros_like(e)
            op.apply(e, col)
            allys = np.stack(np.unravel_index(np.arange(w.N), w.shape), axis=1)
            ent = op.entries(torch.from_numpy(allys).cuda(),
                             torch.from_numpy(np.repeat(x[None, :], w.N, axis=0)).cuda())
            torch.cuda.synchronize()
            assert (ent - col).abs().max().item() <= 1e-13 * col.abs().max().item()
        op.close()


# -------------------------------------------------------------- block apply
def _block(shape, lo, hi, full):
    sl = tuple(slice(int(a), int(b) + 1) for a, b in zip(lo, hi))
    return full.reshape((full.shape[0],) + tuple(shape))[(slice(None),) + sl].reshape(full.shape[0], -1)


@pytest.mark.parametrize("dtype", [0, 1])
def test_block_apply_equals_restricted_full_apply(lib, dtype):
    """A~[T, S] U_S (and the adjoint block) equal the full apply of the
    zero-extended vectors restricted to T: the clipped work items see the same
    values and the dropped ones contribute exact zeros.  Several box pairs on
    the quarter-scale 1024^2 workload, 5 vectors; plus a small case against
    the oracle."""
    tdt, ndt = _dt(dtype)
    w = make_config(1, scale=0.25)
    op = lib.PcOperator.from_workload(w, dtype=dtype)
    n = np.array(w.shape)
    rng = np.random.default_rng(41)
    pairs = [((np.zeros(2, int), n - 1), (np.zeros(2, int), n - 1)),
             ((np.array([10, 20]), np.array([60, 200])), (np.array([30, 0]), np.array([200, 90]))),
             ((np.array([0, 0]), np.array([40, 40])), (np.array([200, 200]), np.array([255, 255]))),
             ((np.array([100, 100]), np.array([101, 180])), (np.array([90, 95]), np.array([130, 140])))]
    for t_box, s_box in pairs:
        full = torch.from_numpy(rng.standard_normal((5, w.N)).astype(ndt)).cuda()
        ext = torch.zeros_like(full).reshape((5,) + tuple(w.shape))
        sl = tuple(slice(int(a), int(b) + 1) for a, b in zip(*s_box))
        ext[(slice(None),) + sl] = full.reshape((5,) + tuple(w.shape))[(slice(None),) + sl]
        ext = ext.reshape(5, -1)
        US = _block(w.shape, *s_box, full).contiguous()
        for adj in (False, True):
            ref_full = torch.zeros_like(full)
            (op.apply_adjoint_batch if adj else op.apply_batch)(ext, ref_full)
            nT = int(np.prod(t_box[1] - t_box[0] + 1))
            got = torch.full((5, nT), float("nan"), dtype=tdt, device="cuda")
            op.apply_block(t_box, s_box, US, got, adjoint=adj)
            torch.cuda.synchronize()
            ref = _block(w.shape, *t_box, ref_full)
            assert torch.equal(got, ref), (dtype, adj, t_box, s_box)
    # small case against the oracle
    w0 = make_config(0)
    ora = OracleOperator.from_workload(w0)
    op0 = lib.PcOperator.from_workload(w0, dtype=lib.PC_F64)
    t_box, s_box = (np.array([5, 10]), np.array([40, 63])), (np.array([20, 0]), np.array([63, 30]))
    u = rng.standard_normal(w0.N)
    ext = np.zeros(w0.N)
    ext.reshape(64, 64)[20:64, 0:31] = u.reshape(64, 64)[20:64, 0:31]
    US = torch.from_numpy(np.ascontiguousarray(u.reshape(64, 64)[20:64, 0:31]).reshape(1, -1)).cuda()
    got = torch.zeros((1, 36 * 54), dtype=torch.float64, device="cuda")
    op0.apply_block(t_box, s_box, US, got)
    ref = ora.apply(ext).reshape(64, 64)[5:41, 10:64].ravel()
    assert np.abs(got.cpu().numpy()[0] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["cube24", "hang3d"])
def test_block_apply_3d_equals_restricted_full_apply(lib, name):
    from tests.libhelpers import small_cases_3d
    w = dict(small_cases_3d())[name]
    n = np.array(w.shape)
    rng = np.random.default_rng(43)
    pairs = [((np.zeros(3, int), n - 1), (np.zeros(3, int), n - 1)),
             ((np.array([2, 3, 1]), np.array([12, 15, 9])), (np.array([5, 0, 4]), np.array([14, 10, 16]))),
             ((np.array([0, 0, 0]), np.array([4, 4, 4])), (n - 5, n - 1))]
    for dtype in (lib.PC_F32, lib.PC_F64):
        tdt, ndt = _dt(dtype)
        op = lib.PcOperator.from_workload(w, dtype=dtype)
        for t_box, s_box in pairs:
            full = torch.from_numpy(rng.standard_normal((3, w.N)).astype(ndt)).cuda()
            sl = (slice(None),) + tuple(slice(int(a), int(b) + 1) for a, b in zip(*s_box))
            ext = torch.zeros_like(full).reshape((3,) + tuple(w.shape))
            ext[sl] = full.reshape((3,) + tuple(w.shape))[sl]
            ext = ext.reshape(3, -1)
            US = full.reshape((3,) + tuple(w.shape))[sl].reshape(3, -1).contiguous()
            tl = (slice(None),) + tuple(slice(int(a), int(b) + 1) for a, b in zip(*t_box))
            nT = int(np.prod(t_box[1] - t_box[0] + 1))
            for adj in (False, True):
                ref_full = torch.zeros_like(full)
                (op.apply_adjoint_batch if adj else op.apply_batch)(ext, ref_full)
                got = torch.full((3, nT), float("nan"), dtype=tdt, device="cuda")
                op.apply_block(t_box, s_box, US, got, adjoint=adj)
                torch.cuda.synchronize()
                ref = ref_full.reshape((3,) + tuple(w.shape))[tl].reshape(3, -1)
                assert torch.equal(got, ref), (name, dtype, adj, t_box, s_box)
        op.close()


@pytest.mark.parametrize("name", ["hanging33", "rect3d"])
def test_graph_replays_equal_eager_applies(lib, name):
    """A batched apply (and adjoint apply) recorded into a HIP graph by stream
    capture: every replay, with new input in the captured buffer and eager
    work on the same operator in between, equals the eager apply bitwise and
    the oracle within the FP32 tolerance."""
    from tests.libhelpers import small_cases_3d
    w = dict(small_cases() + small_cases_3d())[name]
    ora = OracleOperator.from_workload(w)
    rng = np.random.default_rng(61)
    op = lib.PcOperator.from_workload(w, dtype=lib.PC_F32)
    for adj in (False, True):
        _note(f"case={name} graph adjoint={adj}")
        U = torch.zeros((3, w.N), dtype=torch.float32, device="cuda")
        OUT = torch.zeros_like(U)
        g = op.graph(U, OUT, adjoint=adj)
        eager = op.apply_adjoint_batch if adj else op.apply_batch
        for rep in range(3):
            Un = rng.standard_normal((3, w.N)).astype(np.float32)
            U.copy_(torch.from_numpy(Un))
            E = torch.empty_like(U)
            eager(U, E)                       # eager work on the operator between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(OUT, E), (name, adj, rep)
            ref = ora.apply_batch(Un.astype(np.float64), adjoint=adj)
            assert relerr(OUT.cpu().numpy(), ref).max() <= TOL[lib.PC_F32], (name, adj, rep)
        del g
    op.close()


def test_calls_that_synchronise_refuse_capture(lib):
    """Block applies and the estimator return host data or copy tables
    synchronously: under stream capture they fail with PC_ERR_ARG before
    enqueuing anything, and the capture stays usable."""
    w = small_cases()[0][1]
    op = lib.PcOperator.from_workload(w, dtype=lib.PC_F32)
    U = torch.zeros((2, w.N), dtype=torch.float32, device="cuda")
    OUT = torch.zeros_like(U)
    op.apply_batch(U, OUT)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    errs = []
    with torch.cuda.graph(g):
        op.apply_batch(U, OUT)
        box = (np.zeros(w.d, int), np.array(w.shape) - 1)
        try:
            op.apply_block(box, box, U, OUT)
        except lib.PcError as e:
            errs.append(e.status)
        try:
            op.estimate_sums(U, OUT)
        except lib.PcError as e:
            errs.append(e.status)
    assert errs == [lib.PC_ERR_ARG, lib.PC_ERR_ARG]
    U.copy_(torch.from_numpy(np.random.default_rng(3).standard_normal((2, w.N)).astype(np.float32)))
    E = torch.empty_like(U)
    op.apply_batch(U, E)
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(OUT, E)
    op.close()
