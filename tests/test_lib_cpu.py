"""CPU tests of the HIP library: exported symbols, argument validation (all
of which happens before any HIP call), and the kernel phases run by the CPU
emulation build against the oracle (with an AddressSanitizer pass)."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from oracle import OracleOperator
from workloads import make_config
from tests.libhelpers import small_cases, small_cases_3d, relerr, TOL
from tests.tilings import refine, workload_from

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1805_06018_amd")


def _declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "pc.h")).read()
    return sorted(set(re.findall(r"^(?:pc_status|size_t|const char\*)\s+(pc_\w+)\s*\(", hdr, re.M)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(PKG, "libpc.so"))
    syms = _declared_symbols()
    assert "pc_create" in syms and "pc_error_estimate" in syms and len(syms) >= 11
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_lists_every_symbol():
    from paper_1805_06018_amd import _lib
    assert sorted(_lib.EXPORTED) == _declared_symbols()


# ------------------------------------------------------------- validation
def _args(w):
    return dict(d=w.d, shape=w.shape, leaf_lo=w.leaf_lo, leaf_hi=w.leaf_hi, points=w.points,
                radius=w.radius, phi=w.phi, phi_off=w.phi_off)


def test_create_rejects_bad_input():
    from paper_1805_06018_amd._lib import raw_create, PC_ERR_ARG, PC_ERR_GRID, PC_ERR_UNSUPPORTED
    w = make_config(0)
    a = _args(w)
    st, msg = raw_create(**{**a, "leaf_lo": a["leaf_lo"][:-1], "leaf_hi": a["leaf_hi"][:-1]})
    assert st == PC_ERR_GRID, msg                          # gap in the tiling
    lo = np.vstack([a["leaf_lo"], [[1, 1]]])
    hi = np.vstack([a["leaf_hi"], [[5, 5]]])
    st, msg = raw_create(**{**a, "leaf_lo": lo, "leaf_hi": hi})
    assert st == PC_ERR_GRID, msg                          # overlap
    pts = a["points"].copy()
    pts[3] += 1
    st, msg = raw_create(**{**a, "points": pts})
    assert st == PC_ERR_GRID, msg                          # points != corners
    rad = a["radius"].copy()
    rad[0, 0] = -1
    st, msg = raw_create(**{**a, "radius": rad})
    assert st == PC_ERR_ARG, msg                           # negative radius
    off = a["phi_off"].copy()
    off[5] += 1
    st, msg = raw_create(**{**a, "phi_off": off})
    assert st == PC_ERR_ARG, msg                           # phi_off inconsistent
    st, msg = raw_create(**{**a, "d": 4})
    assert st == PC_ERR_ARG, msg
    st, msg = raw_create(**a, dtype=7)
    assert st == PC_ERR_ARG, msg
    st, msg = raw_create(**a, flags=1 << 5)
    assert st == PC_ERR_ARG, msg
    # a 3-D patch beyond the FFT lengths of the kernels (no pieces in 3-D)
    x = np.full((3, 300, 6, 6), 1.2)
    lo3, hi3 = np.array([[0, 0, 0]]), np.array([[299, 5, 5]])
    st, msg = raw_create(**_args(workload_from(x, lo3, hi3)))
    assert st == PC_ERR_UNSUPPORTED and "FFT" in msg, msg


# ------------------------------------------------------------- CPU emulation
def _emu_lib(path=os.path.join(PKG, "libpc_emu.so")):
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.pc_emu_create.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, ctypes.c_int64, P, P, P, P,
                                  ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(P)]
    lib.pc_emu_create_patches.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, ctypes.c_int64, P, P, P, P,
                                          ctypes.c_int, ctypes.c_uint32, ctypes.c_int64, P, ctypes.POINTER(P)]
    lib.pc_emu_apply.argtypes = [P, ctypes.c_int, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64]
    lib.pc_emu_apply_direct.argtypes = [P, ctypes.c_int, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64]
    lib.pc_emu_items.argtypes = [P, P]
    lib.pc_emu_items.restype = ctypes.c_int64
    lib.pc_emu_order.argtypes = [P, ctypes.c_int, P]
    lib.pc_emu_order.restype = ctypes.c_int64
    lib.pc_emu_destroy.argtypes = [P]
    lib.pc_emu_last_error.restype = ctypes.c_char_p
    return lib


def emu_apply(lib, w, U, dtype, flags=0, adj=False, patches=None, direct=False):
    k = [np.ascontiguousarray(v, dtype=np.int64) for v in (w.shape, w.leaf_lo, w.leaf_hi, w.points, w.radius)]
    phi = np.ascontiguousarray(w.phi, dtype=np.float64)
    off = np.ascontiguousarray(w.phi_off, dtype=np.int64)
    h = ctypes.c_void_p()
    if patches is None:
        rc = lib.pc_emu_create(w.d, k[0].ctypes.data, len(w.leaf_lo), k[1].ctypes.data, k[2].ctypes.data,
                               len(w.points), k[3].ctypes.data, k[4].ctypes.data, phi.ctypes.data, off.ctypes.data,
                               dtype, flags, ctypes.byref(h))
    else:
        sel = np.ascontiguousarray(patches, dtype=np.int64)
        rc = lib.pc_emu_create_patches(w.d, k[0].ctypes.data, len(w.leaf_lo), k[1].ctypes.data, k[2].ctypes.data,
                                       len(w.points), k[3].ctypes.data, k[4].ctypes.data, phi.ctypes.data,
                                       off.ctypes.data, dtype, flags, sel.size, sel.ctypes.data, ctypes.byref(h))
    assert rc == 0, lib.pc_emu_last_error()
    dt = np.float64 if dtype == 1 else np.float32
    U = np.ascontiguousarray(U, dtype=dt)
    out = np.zeros_like(U)
    fn = lib.pc_emu_apply_direct if direct else lib.pc_emu_apply
    assert fn(h, int(adj), U.shape[0], U.ctypes.data, U.shape[1], out.ctypes.data, out.shape[1]) == 0
    lib.pc_emu_destroy(h)
    return out


@pytest.mark.parametrize("idx", range(10))
def test_emulated_kernels_match_oracle(idx):
    name, w = (small_cases() + small_cases_3d())[idx]
    lib = _emu_lib()
    rng = np.random.default_rng(100 + idx)
    U = rng.standard_normal((3, w.N))
    for flags in (0, 1, 4):     # default, PC_NO_EXTEND, PC_PLAN_SMALLEST_FFT
        op = OracleOperator.from_workload(w, extend=((flags & 1) == 0))
        for dtype in (1, 0):
            Ur = U.astype(np.float32).astype(np.float64) if dtype == 0 else U
            for adj in (False, True):
                got = emu_apply(lib, w, Ur, dtype, flags, adj)
                ref = op.apply_batch(Ur, adjoint=adj)
                e = relerr(got, ref)
                assert e.max() <= TOL[dtype], (name, flags, dtype, adj, e)


@pytest.mark.parametrize("name", ["cfg0", "hanging33", "cube24", "hang3d"])
def test_emulated_term_subsets_match_oracle(name):
    """Operators restricted to a subset of the terms (pc_create_patches) against
    the oracle's sum over the same terms; the empty subset gives zero."""
    w = dict(small_cases() + small_cases_3d())[name]
    lib = _emu_lib()
    rng = np.random.default_rng(7)
    U = rng.standard_normal((2, w.N))
    ora = OracleOperator.from_workload(w)
    for sel in (rng.permutation(w.r)[: max(1, w.r // 3)], np.array([w.r - 1]), np.zeros(0, dtype=np.int64)):
        for adj in (False, True):
            got = emu_apply(lib, w, U, 1, 0, adj, patches=sel)
            ref = ora.apply_batch(U, adjoint=adj, patches=sel)
            if sel.size == 0:
                assert np.all(got == 0.0)
            else:
                assert relerr(got, ref).max() <= TOL[1], (name, sel.size, adj)


@pytest.mark.parametrize("idx", range(7))
def test_colour_launches_equal_staged_reduction(idx):
    """The colour-launch path (outputs zeroed, items of each colour adding
    their written boxes in place, colour after colour) gives the same bits as
    staging every box and summing in the reduction, FP32 and FP64, forward
    and adjoint; and the items of one colour write pairwise disjoint boxes,
    so their adds cannot race on the GPU."""
    name, w = small_cases()[idx]
    lib = _emu_lib()
    U = np.random.default_rng(500 + idx).standard_normal((2, w.N))
    for dtype in (0, 1):
        for adj in (False, True):
            staged = emu_apply(lib, w, U, dtype, 0, adj)
            direct = emu_apply(lib, w, U, dtype, 0, adj, direct=True)
            assert np.array_equal(staged, direct), (name, dtype, adj)
    h = _emu_handle(lib, w)
    n = int(lib.pc_emu_items(h, None))
    for adj in (0, 1):
        tab = np.zeros((n, 6), dtype=np.int32)
        n_col = lib.pc_emu_order(h, adj, tab.ctypes.data)
        assert n_col >= 1 and sorted(tab[:, 0]) == list(range(n)) and np.all(np.diff(tab[:, 1]) >= 0)
        for c in range(n_col):
            boxes = tab[tab[:, 1] == c][:, 2:]
            cover = np.zeros((max(1, w.shape[0]) if w.d == 2 else 1, w.shape[-1]), dtype=np.int32)
            for r0, c0, n0, n1 in boxes:
                cover[r0:r0 + n0, c0:c0 + n1] += 1
            assert cover.max() <= 1, (name, adj, c)
    lib.pc_emu_destroy(h)


def test_create_patches_rejects_bad_selection():
    from paper_1805_06018_amd._lib import raw_create, PC_ERR_ARG
    w = make_config(0)
    for bad in ([0, 0], [w.r], [-1]):
        st, msg = raw_create(**_args(w), patches=bad)
        assert st == PC_ERR_ARG and "distinct" in msg, (bad, msg)
    st, msg = raw_create(**_args(w), n_sel=-1)
    assert st == PC_ERR_ARG, msg


def _emu_handle(lib, w, dtype=1, patches=None):
    k = [np.ascontiguousarray(v, dtype=np.int64) for v in (w.shape, w.leaf_lo, w.leaf_hi, w.points, w.radius)]
    phi = np.ascontiguousarray(w.phi, dtype=np.float64)
    off = np.ascontiguousarray(w.phi_off, dtype=np.int64)
    h = ctypes.c_void_p()
    if patches is None:
        rc = lib.pc_emu_create(w.d, k[0].ctypes.data, len(w.leaf_lo), k[1].ctypes.data, k[2].ctypes.data,
                               len(w.points), k[3].ctypes.data, k[4].ctypes.data, phi.ctypes.data, off.ctypes.data,
                               dtype, 0, ctypes.byref(h))
    else:
        sel = np.ascontiguousarray(patches, dtype=np.int64)
        rc = lib.pc_emu_create_patches(w.d, k[0].ctypes.data, len(w.leaf_lo), k[1].ctypes.data, k[2].ctypes.data,
                                       len(w.points), k[3].ctypes.data, k[4].ctypes.data, phi.ctypes.data,
                                       off.ctypes.data, dtype, 0, sel.size, sel.ctypes.data, ctypes.byref(h))
    assert rc == 0, lib.pc_emu_last_error()
    return h


def _emu_entries(lib, h, ys, xs):
    lib.pc_emu_entries.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p]
    ys = np.ascontiguousarray(ys, dtype=np.int64)
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    out = np.zeros(len(ys))
    lib.pc_emu_entries(h, len(ys), ys.ctypes.data, xs.ctypes.data, out.ctypes.data)
    return out


@pytest.mark.parametrize("name", ["cfg0", "hanging33", "1d", "rect3d", "hang3d"])
def test_emulated_entries_match_oracle(name):
    """Matrix entries (Sec. 3.1) from the library's entry function against
    the oracle's entry formula: random pairs with y near x (inside the kernel
    boxes), pairs on leaf edges and corners, and pairs outside Omega (NaN)."""
    w = dict(small_cases() + small_cases_3d())[name]
    lib = _emu_lib()
    h = _emu_handle(lib, w)
    ora = OracleOperator.from_workload(w)
    rng = np.random.default_rng(9)
    n = np.array(w.shape)
    xs = rng.integers(0, n, (300, w.d))
    xs[:20] = w.points[rng.integers(0, w.r, 20)]             # on sample points / leaf corners
    ys = np.clip(xs + rng.integers(-6, 7, (300, w.d)), 0, n - 1)
    got = _emu_entries(lib, h, ys, xs)
    ref = np.array([ora.entry(y, x) for y, x in zip(ys, xs)])
    assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()), name
    bad = _emu_entries(lib, h, np.vstack([n, n - 1]), np.vstack([n - 1, -np.ones(w.d, dtype=np.int64)]))
    assert np.all(np.isnan(bad))
    # entries of a term subset + its complement = the full entries
    S = rng.permutation(w.r)[: w.r // 2]
    Sc = np.setdiff1d(np.arange(w.r), S)
    hs, hc = _emu_handle(lib, w, patches=S), _emu_handle(lib, w, patches=Sc)
    part = _emu_entries(lib, hs, ys, xs) + _emu_entries(lib, hc, ys, xs)
    assert np.abs(part - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    for x in (h, hs, hc):
        lib.pc_emu_destroy(x)


def test_emulated_entries_form_the_dense_matrix():
    """On the 1-D case every entry (N^2 pairs) equals the oracle's dense A~."""
    w = dict(small_cases())["1d"]
    lib = _emu_lib()
    h = _emu_handle(lib, w)
    N = w.N
    yy, xx = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    got = _emu_entries(lib, h, yy.reshape(-1, 1), xx.reshape(-1, 1)).reshape(N, N)
    ref = OracleOperator.from_workload(w).dense()
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    lib.pc_emu_destroy(h)


def _box_vec(shape, lo, hi, full):
    sl = tuple(slice(int(a), int(b) + 1) for a, b in zip(lo, hi))
    return np.ascontiguousarray(full.reshape(shape)[sl]).ravel()


def _emu_block(lib, h, adj, t_box, s_box, US):
    lib.pc_emu_apply_block.argtypes = [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 4 + \
        [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64]
    b = [np.ascontiguousarray(v, dtype=np.int64) for v in (t_box[0], t_box[1], s_box[0], s_box[1])]
    nT = int(np.prod(b[1] - b[0] + 1))
    US = np.ascontiguousarray(US, dtype=np.float64)
    out = np.full((US.shape[0], nT), np.nan)
    rc = lib.pc_emu_apply_block(h, int(adj), b[0].ctypes.data, b[1].ctypes.data, b[2].ctypes.data,
                                b[3].ctypes.data, US.shape[0], US.ctypes.data, US.shape[1], out.ctypes.data, nT)
    return rc, out


@pytest.mark.parametrize("name", ["cfg0", "hanging33", "1d", "rect45x301", "rect3d", "hang3d"])
def test_emulated_block_apply_matches_oracle(name):
    """Block applies (Sec. 3.3): A~[T, S] u_S and A~*[T, S] v_S equal the
    oracle's full apply of the zero-extended vector restricted to T, for
    overlapping, disjoint, nested and whole-domain boxes (2-D and 3-D)."""
    w = dict(small_cases() + small_cases_3d())[name]
    lib = _emu_lib()
    h = _emu_handle(lib, w)
    ora = OracleOperator.from_workload(w)
    n = np.array(w.shape)
    rng = np.random.default_rng(31)
    boxes = [((np.zeros(w.d, int), n - 1), (np.zeros(w.d, int), n - 1))]
    for _ in range(4):
        a, b = np.sort(rng.integers(0, n, (2, w.d)), axis=0)
        c, e = np.sort(rng.integers(0, n, (2, w.d)), axis=0)
        boxes.append(((a, b), (c, e)))
    for t_box, s_box in boxes:
        full = rng.standard_normal(w.N)
        ext = np.zeros(w.N)
        sl = tuple(slice(int(x), int(y) + 1) for x, y in zip(*s_box))
        ext.reshape(w.shape)[sl] = full.reshape(w.shape)[sl]
        US = _box_vec(w.shape, *s_box, full)[None, :]
        for adj in (False, True):
            rc, got = _emu_block(lib, h, adj, t_box, s_box, US)
            assert rc == 0
            ref = _box_vec(w.shape, *t_box, (ora.apply_adjoint if adj else ora.apply)(ext))
            scale = max(np.abs(ref).max(), 1e-300)
            assert np.abs(got[0] - ref).max() <= 1e-12 * max(scale, 1.0), (name, adj, t_box, s_box)
    # boxes outside Omega are rejected
    rc, _ = _emu_block(lib, h, False, (np.zeros(w.d, int), n), (np.zeros(w.d, int), n - 1),
                       np.zeros((1, w.N)))
    assert rc != 0
    lib.pc_emu_destroy(h)


def test_emulated_kernels_under_address_sanitizer():
    """Same emulation built with AddressSanitizer, run in a child process with
    the sanitizer runtime preloaded: any out-of-range index aborts it."""
    asan_rt = "/opt/rocm/lib/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so"
    lib = os.path.join(PKG, "libpc_emu_asan.so")
    if not (os.path.exists(asan_rt) and os.path.exists(lib)):
        pytest.skip("sanitizer runtime or ASan emulation build not present")
    code = (
        "import sys, numpy as np; sys.path.insert(0, %r)\n"
        "from tests.test_lib_cpu import _emu_lib, emu_apply\n"
        "from tests.libhelpers import small_cases, small_cases_3d\n"
        "lib = _emu_lib(%r)\n"
        "from tests.test_lib_cpu import _emu_handle, _emu_entries, _emu_block\n"
        "for name, w in small_cases() + small_cases_3d():\n"
        "    U = np.random.default_rng(1).standard_normal((2, w.N))\n"
        "    h = _emu_handle(lib, w)\n"
        "    xs = np.random.default_rng(2).integers(0, np.array(w.shape), (50, w.d))\n"
        "    _emu_entries(lib, h, np.clip(xs + 3, 0, np.array(w.shape) - 1), xs)\n"
        "    if True:\n"
        "        lo = np.array(w.shape) // 4; hi = np.array(w.shape) - 2\n"
        "        _emu_block(lib, h, 0, (lo, hi), (lo // 2, hi - 1), np.ones((1, int(np.prod(hi - lo // 2)))))\n"
        "        _emu_block(lib, h, 1, (lo, hi), (lo // 2, hi - 1), np.ones((1, int(np.prod(hi - lo // 2)))))\n"
        "    lib.pc_emu_destroy(h)\n"
        "    for dt in (0, 1):\n"
        "        for fl in (0, 1):\n"
        "            for adj in (0, 1): emu_apply(lib, w, U, dt, fl, adj)\n"
        "            if w.d < 3:\n"
        "                for adj in (0, 1): emu_apply(lib, w, U, dt, fl, adj, direct=True)\n"
        "print('ASAN-CLEAN')\n" % (ROOT, lib))
    env = dict(os.environ, LD_PRELOAD=asan_rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0 and "ASAN-CLEAN" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]


def test_autotune_candidates():
    """The autotuner's candidate schedules: the library default first, no
    duplicates, 3-D candidates vary chunk and scratch, 2-D colour launches
    against staging, persistent launches, chunk and overlap."""
    import types
    from paper_1805_06018_amd import _lib, tune
    defaults = {_lib.PC_TUNE_DIRECT: 0, _lib.PC_TUNE_STREAMS: 4, _lib.PC_TUNE_SPLIT: 1}
    for d, keys in ((2, {_lib.PC_TUNE_CHUNK, _lib.PC_TUNE_OVERLAP, _lib.PC_TUNE_DIRECT, _lib.PC_TUNE_STREAMS,
                         _lib.PC_TUNE_PERSISTENT, _lib.PC_TUNE_XCD_ORDER, _lib.PC_TUNE_SPLIT}),
                    (3, {_lib.PC_TUNE_CHUNK, _lib.PC_TUNE_SCRATCH})):
        c = tune.candidates(types.SimpleNamespace(d=d), 16)
        assert all(v == defaults.get(k, 0) for k, v in c[0].items())
        varied = {k for x in c for k, v in x.items() if v != c[0][k]}
        assert varied == keys, (d, varied)
        assert len({tuple(sorted(x.items())) for x in c}) == len(c)
        assert all(1 <= x[_lib.PC_TUNE_CHUNK] <= 16 for x in c if x[_lib.PC_TUNE_CHUNK])


def test_debug_fail_launches_validates_arguments():
    """The failure-injection hook rejects a null operator and bad ranges (no
    device work is needed to check the validation)."""
    from paper_1805_06018_amd import _lib
    assert _lib._lib.pc_debug_fail_launches(None, 1, 1) == _lib.PC_ERR_ARG
