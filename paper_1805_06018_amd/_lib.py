"""ctypes binding of libpc.so (argument marshalling only).

Names follow the C ABI in include/pc.h.  Device arrays are torch tensors on a
HIP device; their data pointers and torch's current stream are passed
through.  Every step of the apply runs in the HIP library: if libpc.so is
missing this module raises on import instead of falling back to anything.
"""
import ctypes
import os

import numpy as np
import torch   # loads the HIP runtime first so libpc.so binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpc.so")

PC_OK, PC_ERR_ARG, PC_ERR_GRID, PC_ERR_OOM, PC_ERR_BUDGET, PC_ERR_DEVICE, PC_ERR_CALLBACK, PC_ERR_UNSUPPORTED = range(8)
PC_F32, PC_F64 = 0, 1
PC_NO_EXTEND = 1
PC_PLAN_HALF_LDS = 2
PC_PLAN_SMALLEST_FFT = 4

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(python -m paper_1805_06018_amd.build)")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
MATVEC_FN = ctypes.CFUNCTYPE(ctypes.c_int, _P, _I64, _P, _I64, _P, _I64, _P)


class PcStats(ctypes.Structure):
    _fields_ = [("n", _I64), ("r", _I64), ("n_leaves", _I64), ("n_items", _I64),
                ("sum_fft_points", _I64), ("alg_flops_per_rhs", ctypes.c_double),
                ("kernel_elems", _I64), ("spectrum_bytes", _I64), ("weight_bytes", _I64),
                ("slot_elems_fwd", _I64), ("slot_elems_adj", _I64), ("device_bytes", _I64),
                ("dtype", ctypes.c_int32), ("max_lds_bytes", ctypes.c_int32)]


class PcProfile(ctypes.Structure):
    _fields_ = [("conv_ms", ctypes.c_double), ("reduce_ms", ctypes.c_double), ("conv_launches", _I64),
                ("reduce_launches", _I64), ("conv_vectors", _I64)]


_lib.pc_create.argtypes = [ctypes.c_int, _P, _I64, _P, _P, _I64, _P, _P, _P, _P, ctypes.c_int,
                           ctypes.c_uint32, _P, ctypes.POINTER(_P)]
_lib.pc_create.restype = ctypes.c_int
_lib.pc_create_patches.argtypes = [ctypes.c_int, _P, _I64, _P, _P, _I64, _P, _P, _P, _P, ctypes.c_int,
                                   ctypes.c_uint32, _I64, _P, _P, ctypes.POINTER(_P)]
_lib.pc_create_patches.restype = ctypes.c_int
_lib.pc_apply.argtypes = [_P, _P, _P, _P]
_lib.pc_apply.restype = ctypes.c_int
for _name in ("pc_apply_batch", "pc_apply_adjoint_batch", "pc_apply_batch_plain", "pc_apply_batch_noalloc"):
    getattr(_lib, _name).argtypes = [_P, _I64, _P, _I64, _P, _I64, _P]
    getattr(_lib, _name).restype = ctypes.c_int
for _name in ("pc_apply_batch_axpy", "pc_apply_adjoint_batch_axpy"):
    getattr(_lib, _name).argtypes = [_P, _I64, _P, _I64, ctypes.c_double, _P, _I64, _P]
    getattr(_lib, _name).restype = ctypes.c_int
_lib.pc_apply_block.argtypes = [_P, ctypes.c_int, _P, _P, _P, _P, _I64, _P, _I64, _P, _I64, _P]
_lib.pc_apply_block.restype = ctypes.c_int
_lib.pc_entries.argtypes = [_P, _I64, _P, _P, _P, _P]
_lib.pc_entries.restype = ctypes.c_int
_lib.pc_estimate_sums.argtypes = [_P, _I64, _P, _I64, _P, _I64, _P, _P, _P, _P]
_lib.pc_estimate_sums.restype = ctypes.c_int
_lib.pc_estimate_sums_device.argtypes = [_P, _I64, _P, _I64, _P, _I64, _P, _P]
_lib.pc_estimate_sums_device.restype = ctypes.c_int
_lib.pc_error_estimate.argtypes = [_P, _I64, _P, _I64, _P, _I64, MATVEC_FN, _P, _P, _P, _P, _P]
_lib.pc_error_estimate.restype = ctypes.c_int
_lib.pc_get_stats.argtypes = [_P, ctypes.POINTER(PcStats)]
_lib.pc_get_stats.restype = ctypes.c_int
_lib.pc_debug_fail_launches.argtypes = [_P, _I64, _I64]
_lib.pc_debug_fail_launches.restype = ctypes.c_int
_lib.pc_set_profiling.argtypes = [_P, ctypes.c_int]
_lib.pc_set_profiling.restype = ctypes.c_int
_lib.pc_set_tuning.argtypes = [_P, ctypes.c_int, _I64]
_lib.pc_set_tuning.restype = ctypes.c_int
(PC_TUNE_CHUNK, PC_TUNE_OVERLAP, PC_TUNE_SCRATCH, PC_TUNE_BUDGET, PC_TUNE_DIRECT, PC_TUNE_STREAMS,
 PC_TUNE_PERSISTENT, PC_TUNE_XCD_ORDER, PC_TUNE_SPLIT) = 1, 2, 3, 4, 5, 6, 7, 8, 9
_lib.pc_read_profile.argtypes = [_P, ctypes.POINTER(PcProfile)]
_lib.pc_read_profile.restype = ctypes.c_int
_lib.pc_device_bytes.argtypes = [_P]
_lib.pc_device_bytes.restype = ctypes.c_size_t
_lib.pc_destroy.argtypes = [_P]
_lib.pc_destroy.restype = ctypes.c_int
_lib.pc_status_string.argtypes = [ctypes.c_int]
_lib.pc_status_string.restype = ctypes.c_char_p
_lib.pc_last_error.argtypes = []
_lib.pc_last_error.restype = ctypes.c_char_p

EXPORTED = ["pc_create", "pc_create_patches", "pc_apply", "pc_apply_batch", "pc_apply_adjoint_batch",
            "pc_apply_batch_plain", "pc_apply_batch_noalloc", "pc_apply_batch_axpy", "pc_apply_adjoint_batch_axpy", "pc_apply_block", "pc_entries",
            "pc_estimate_sums", "pc_estimate_sums_device",
            "pc_error_estimate", "pc_get_stats", "pc_debug_fail_launches", "pc_set_profiling", "pc_set_tuning", "pc_read_profile", "pc_device_bytes",
            "pc_destroy", "pc_status_string", "pc_last_error"]


class PcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_lib.pc_status_string(status).decode()}: {msg}")
        self.status = status


def _check(st):
    if st != PC_OK:
        raise PcError(st, _lib.pc_last_error().decode())


def _i64(a):
    return np.ascontiguousarray(np.asarray(a), dtype=np.int64)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a torch tensor on a HIP device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _ld(t, name):
    """Leading dimension of a (B, N) tensor whose rows are contiguous."""
    if t.dim() == 1:
        return t.numel()
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be 1-D or 2-D with contiguous rows")
    return t.stride(0)


class PcOperator:
    """Owner of a pc_op handle.  Construction = pc_create (host arrays are
    copied); the apply methods take torch tensors on the device."""

    def __init__(self, d, shape, leaf_lo, leaf_hi, points, radius, phi, phi_off,
                 dtype=PC_F32, flags=0, stream=None, patches=None):
        """patches: None for the full operator, else the point indices whose
        terms the operator keeps (pc_create_patches)."""
        self._keep = [_i64(shape), _i64(leaf_lo), _i64(leaf_hi), _i64(points), _i64(radius),
                      np.ascontiguousarray(phi, dtype=np.float64), _i64(phi_off)]
        k = self._keep
        h = _P()
        if patches is None:
            st = _lib.pc_create(int(d), k[0].ctypes.data, int(k[1].size // d), k[1].ctypes.data,
                                k[2].ctypes.data, int(k[3].size // d), k[3].ctypes.data, k[4].ctypes.data,
                                k[5].ctypes.data, k[6].ctypes.data, int(dtype), int(flags),
                                _stream(stream), ctypes.byref(h))
        else:
            sel = _i64(patches).ravel()
            st = _lib.pc_create_patches(int(d), k[0].ctypes.data, int(k[1].size // d), k[1].ctypes.data,
                                        k[2].ctypes.data, int(k[3].size // d), k[3].ctypes.data, k[4].ctypes.data,
                                        k[5].ctypes.data, k[6].ctypes.data, int(dtype), int(flags), int(sel.size),
                                        sel.ctypes.data, _stream(stream), ctypes.byref(h))
        _check(st)
        self._h = h
        self.d = int(d)
        self.shape = tuple(int(v) for v in shape)
        self.N = int(np.prod(self.shape))
        self.dtype = int(dtype)
        self.torch_dtype = torch.float64 if dtype == PC_F64 else torch.float32
        self.n_leaves = int(k[1].size // d)
        self._keep = None

    @classmethod
    def from_workload(cls, w, dtype=PC_F32, flags=0, stream=None):
        return cls(w.d, w.shape, w.leaf_lo, w.leaf_hi, w.points, w.radius, w.phi, w.phi_off,
                   dtype=dtype, flags=flags, stream=stream)

    # -- applies ------------------------------------------------------------
    def apply(self, u, out, stream=None):
        _check(_lib.pc_apply(self._h, _dev(u, self.torch_dtype, "u"), _dev(out, self.torch_dtype, "out"),
                             _stream(stream)))
        return out

    def _batch(self, fn, U, OUT, stream):
        B = 1 if U.dim() == 1 else U.shape[0]
        _check(fn(self._h, B, _dev(U, self.torch_dtype, "U"), _ld(U, "U"),
                  _dev(OUT, self.torch_dtype, "OUT"), _ld(OUT, "OUT"), _stream(stream)))
        return OUT

    def apply_batch(self, U, OUT, stream=None):
        return self._batch(_lib.pc_apply_batch, U, OUT, stream)

    def apply_adjoint_batch(self, V, OUT, stream=None):
        return self._batch(_lib.pc_apply_adjoint_batch, V, OUT, stream)

    def apply_batch_plain(self, U, OUT, stream=None):
        return self._batch(_lib.pc_apply_batch_plain, U, OUT, stream)

    def apply_batch_noalloc(self, U, OUT, stream=None):
        """pc_apply_batch_noalloc: the batched apply on the device's fixed
        work area (no allocation in the call)."""
        return self._batch(_lib.pc_apply_batch_noalloc, U, OUT, stream)

    def graph(self, U, OUT, adjoint=False):
        """Records one batched apply (adjoint: A~* apply) from U into OUT as a
        torch.cuda.CUDAGraph.  One eager call first sizes the operator's work
        buffers; each replay recomputes OUT from the current contents of U."""
        fn = self.apply_adjoint_batch if adjoint else self.apply_batch
        fn(U, OUT)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn(U, OUT)
        return g

    def _axpy(self, fn, U, alpha, OUT, stream):
        B = 1 if U.dim() == 1 else U.shape[0]
        _check(fn(self._h, B, _dev(U, self.torch_dtype, "U"), _ld(U, "U"), float(alpha),
                  _dev(OUT, self.torch_dtype, "OUT"), _ld(OUT, "OUT"), _stream(stream)))
        return OUT

    def apply_batch_axpy(self, U, alpha, OUT, stream=None):
        """OUT += alpha * A~ U."""
        return self._axpy(_lib.pc_apply_batch_axpy, U, alpha, OUT, stream)

    def apply_adjoint_batch_axpy(self, V, alpha, OUT, stream=None):
        """OUT += alpha * A~* V."""
        return self._axpy(_lib.pc_apply_adjoint_batch_axpy, V, alpha, OUT, stream)

    def apply_block(self, t_box, s_box, U, OUT, adjoint=False, stream=None):
        """OUT_T = A~[T, S] U_S (adjoint: A~*[T, S] U_S), pc_apply_block.
        t_box, s_box: (lo, hi) pairs of d inclusive coordinates; U: (B, |S|)
        and OUT: (B, |T|) device tensors, row-major over the boxes."""
        tlo, thi = _i64(t_box[0]).ravel(), _i64(t_box[1]).ravel()
        slo, shi = _i64(s_box[0]).ravel(), _i64(s_box[1]).ravel()
        B = 1 if U.dim() == 1 else U.shape[0]
        _check(_lib.pc_apply_block(self._h, int(bool(adjoint)), tlo.ctypes.data, thi.ctypes.data, slo.ctypes.data,
                                   shi.ctypes.data, B, _dev(U, self.torch_dtype, "U"), _ld(U, "U"),
                                   _dev(OUT, self.torch_dtype, "OUT"), _ld(OUT, "OUT"), _stream(stream)))
        return OUT

    def entries(self, ys, xs, out=None, stream=None):
        """Matrix entries A~[ys[i], xs[i]] (pc_entries); ys, xs: (n, d) int64
        device tensors.  Returns a device tensor of the operator's dtype."""
        if ys.dtype != torch.int64 or xs.dtype != torch.int64 or ys.shape != xs.shape:
            raise TypeError("ys and xs must be int64 tensors of the same shape (n, d)")
        ys = ys.reshape(-1, self.d).contiguous()
        xs = xs.reshape(-1, self.d).contiguous()
        n = ys.shape[0]
        if out is None:
            out = torch.empty(n, dtype=self.torch_dtype, device=ys.device)
        _check(_lib.pc_entries(self._h, n, _dev(ys, torch.int64, "ys"), _dev(xs, torch.int64, "xs"),
                               _dev(out, self.torch_dtype, "out"), _stream(stream)))
        return out

    def estimate_sums(self, Yt, Y, stream=None):
        """Estimator of Sec. 2.6 from a given Y~ (pc_estimate_sums):
        (eta_leaf[n_leaves], eta_abs, eta_rel)."""
        q = 1 if Yt.dim() == 1 else Yt.shape[0]
        eta = np.zeros(self.n_leaves)
        ea = ctypes.c_double()
        er = ctypes.c_double()
        _check(_lib.pc_estimate_sums(self._h, q, _dev(Yt, self.torch_dtype, "Yt"), _ld(Yt, "Yt"),
                                     _dev(Y, self.torch_dtype, "Y"), _ld(Y, "Y"), eta.ctypes.data,
                                     ctypes.byref(ea), ctypes.byref(er), _stream(stream)))
        return eta, ea.value, er.value

    def estimate_sums_device(self, Yt, Y, sums, stream=None):
        """pc_estimate_sums_device: the estimator's FP64 sums into the device
        tensor sums (float64, n_leaves + 2), without synchronising."""
        q = 1 if Yt.dim() == 1 else Yt.shape[0]
        if sums.numel() < self.n_leaves + 2:
            raise ValueError("sums needs n_leaves + 2 elements")
        _check(_lib.pc_estimate_sums_device(self._h, q, _dev(Yt, self.torch_dtype, "Yt"), _ld(Yt, "Yt"),
                                            _dev(Y, self.torch_dtype, "Y"), _ld(Y, "Y"),
                                            _dev(sums, torch.float64, "sums"), _stream(stream)))
        return sums

    @staticmethod
    def eta_from_sums(sums, q):
        """(eta_leaf, eta_abs, eta_rel) from host sums of estimate_sums_device."""
        s = np.asarray(sums, dtype=np.float64)
        L = s.size - 2
        eta_rel = float(np.sqrt(s[L]) / np.sqrt(s[L + 1])) if s[L + 1] > 0 else float("inf")
        return np.sqrt(s[:L] / q), float(np.sqrt(s[L] / q)), eta_rel

    def error_estimate(self, Z, Y=None, exact_adjoint=None, stream=None):
        """Returns (eta_leaf[n_leaves], eta_abs, eta_rel).  exact_adjoint, if
        given, is called as f(B, in_ptr, ldin, out_ptr, ldout, stream_ptr) -> int."""
        q = 1 if Z.dim() == 1 else Z.shape[0]
        eta = np.zeros(self.n_leaves)
        ea = ctypes.c_double()
        er = ctypes.c_double()
        if exact_adjoint is not None:
            cb = MATVEC_FN(lambda user, B, i, li, o, lo, s: int(exact_adjoint(B, i, li, o, lo, s)))
        else:
            cb = MATVEC_FN()
        yp = _dev(Y, self.torch_dtype, "Y") if Y is not None else _P()
        ly = _ld(Y, "Y") if Y is not None else 0
        _check(_lib.pc_error_estimate(self._h, q, _dev(Z, self.torch_dtype, "Z"), _ld(Z, "Z"), yp, ly,
                                      cb, None, eta.ctypes.data, ctypes.byref(ea), ctypes.byref(er),
                                      _stream(stream)))
        return eta, ea.value, er.value

    # -- info ---------------------------------------------------------------
    def stats(self):
        st = PcStats()
        _check(_lib.pc_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in PcStats._fields_}

    def debug_fail_launches(self, first, count=1):
        """Test hook: convolution launches first .. first + count - 1 from
        now on fail with PcError (PC_ERR_DEVICE) before they are enqueued;
        the operator stays usable.  count = 0 disables."""
        _check(_lib.pc_debug_fail_launches(self._h, int(first), int(count)))

    def set_profiling(self, enable=True):
        _check(_lib.pc_set_profiling(self._h, int(bool(enable))))

    def set_tuning(self, key, value):
        _check(_lib.pc_set_tuning(self._h, int(key), int(value)))

    def read_profile(self):
        pr = PcProfile()
        _check(_lib.pc_read_profile(self._h, ctypes.byref(pr)))
        return {f: getattr(pr, f) for f, _ in PcProfile._fields_}

    def device_bytes(self):
        return int(_lib.pc_device_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.pc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def raw_create(d, shape, leaf_lo, leaf_hi, points, radius, phi, phi_off, dtype=PC_F32, flags=0,
               n_leaves=None, r=None, patches=None, n_sel=None):
    """pc_create (or pc_create_patches when patches / n_sel is given) with
    explicit counts, for argument-validation tests.  Returns (status, message)."""
    k = [_i64(shape), _i64(leaf_lo), _i64(leaf_hi), _i64(points), _i64(radius),
         np.ascontiguousarray(phi, dtype=np.float64), _i64(phi_off)]
    h = _P()
    L = int(k[1].size // max(d, 1)) if n_leaves is None else n_leaves
    R = int(k[3].size // max(d, 1)) if r is None else r
    if patches is None and n_sel is None:
        st = _lib.pc_create(int(d), k[0].ctypes.data, L, k[1].ctypes.data, k[2].ctypes.data, R,
                            k[3].ctypes.data, k[4].ctypes.data, k[5].ctypes.data, k[6].ctypes.data,
                            int(dtype), int(flags), None, ctypes.byref(h))
    else:
        sel = _i64(patches if patches is not None else []).ravel()
        ns = int(sel.size) if n_sel is None else int(n_sel)
        st = _lib.pc_create_patches(int(d), k[0].ctypes.data, L, k[1].ctypes.data, k[2].ctypes.data, R,
                                    k[3].ctypes.data, k[4].ctypes.data, k[5].ctypes.data, k[6].ctypes.data,
                                    int(dtype), int(flags), ns, sel.ctypes.data, None, ctypes.byref(h))
    msg = _lib.pc_last_error().decode()
    if st == PC_OK:
        _lib.pc_destroy(h)
    return st, msg
