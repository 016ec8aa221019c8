"""Exact blur adjoint on the GPU (the black-box A* of the error estimator).

ctypes wrapper of workloads/libblur.so (built by the package build step).
Device arrays are torch tensors; torch is imported first so the library binds
to the same HIP runtime.
"""
import ctypes
import os

import numpy as np
import torch

_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libblur.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise ImportError(f"{_LIB} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.blur_adjoint.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int64, P,
                                     ctypes.c_int64, ctypes.c_int, P]
        lib.blur_adjoint.restype = ctypes.c_int
        lib.blur_adjoint3.argtypes = [ctypes.c_int, P, P, P, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P,
                                      ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int, P]
        lib.blur_adjoint3.restype = ctypes.c_int
        lib.blur_forward.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int, P]
        lib.blur_forward.restype = ctypes.c_int
        _lib = lib
    return _lib


class GpuBlurAdjoint:
    """Holds the width and radius fields of a BlurOperator on the device."""

    def __init__(self, op, dtype=torch.float32, device="cuda"):
        self.d3 = op.d == 3
        if self.d3:
            self.n = tuple(int(v) for v in op.shape)
            self.N = int(np.prod(self.n))
            self.s = [torch.from_numpy(np.ascontiguousarray(op.sig[i]).ravel()).to(device=device, dtype=dtype)
                      for i in range(3)]
            self.r = [torch.from_numpy(np.ascontiguousarray(op.radius[i], dtype=np.int32).ravel()).to(device)
                      for i in range(3)]
            self.dtype = dtype
            self.code = 1 if dtype == torch.float64 else 0
            return
        if op.d == 1:
            s0 = np.ones(op.shape)
            s1 = op.sig[0]
            r0 = np.zeros(op.shape, dtype=np.int32)
            r1 = op.radius[0]
            self.n0, self.n1 = 1, int(op.shape[0])
        else:
            s0, s1 = op.sig[0], op.sig[1]
            r0, r1 = op.radius[0], op.radius[1]
            self.n0, self.n1 = int(op.shape[0]), int(op.shape[1])
        self.N = self.n0 * self.n1
        self.dtype = dtype
        self.s0 = torch.from_numpy(np.ascontiguousarray(s0).ravel()).to(device=device, dtype=dtype)
        self.s1 = torch.from_numpy(np.ascontiguousarray(s1).ravel()).to(device=device, dtype=dtype)
        self.r0 = torch.from_numpy(np.ascontiguousarray(r0, dtype=np.int32).ravel()).to(device)
        self.r1 = torch.from_numpy(np.ascontiguousarray(r1, dtype=np.int32).ravel()).to(device)
        self.code = 1 if dtype == torch.float64 else 0

    def raw(self, B, in_ptr, ldin, out_ptr, ldout, stream_ptr):
        """Callback form: pointers and leading dimensions as plain ints."""
        if self.d3:
            return _load().blur_adjoint3(self.code, *(t.data_ptr() for t in self.s), *(t.data_ptr() for t in self.r),
                                         *self.n, in_ptr, ldin, out_ptr, ldout, B, stream_ptr)
        return _load().blur_adjoint(self.code, self.s0.data_ptr(), self.s1.data_ptr(), self.r0.data_ptr(),
                                    self.r1.data_ptr(), self.n0, self.n1, in_ptr, ldin, out_ptr, ldout, B,
                                    stream_ptr)

    def __call__(self, V, OUT=None):
        V = V.reshape(-1, self.N)
        if OUT is None:
            OUT = torch.empty_like(V)
        rc = self.raw(V.shape[0], V.data_ptr(), V.stride(0), OUT.data_ptr(), OUT.stride(0),
                      torch.cuda.current_stream().cuda_stream)
        if rc != 0:
            raise RuntimeError("blur_adjoint launch failed")
        return OUT


class GpuBlur:
    """Exact forward blur A (2-D or 1-D BlurOperator) on the GPU."""

    def __init__(self, op, dtype=torch.float32, device="cuda"):
        if op.d == 3:
            raise NotImplementedError("the exact forward blur is provided for 1-D and 2-D operators")
        if op.d == 1:
            s0, s1 = np.ones(op.shape), op.sig[0]
            r0, r1 = np.zeros(op.shape, dtype=np.int32), op.radius[0]
            self.n0, self.n1 = 1, int(op.shape[0])
        else:
            s0, s1 = op.sig[0], op.sig[1]
            r0, r1 = op.radius[0], op.radius[1]
            self.n0, self.n1 = int(op.shape[0]), int(op.shape[1])
        self.N = self.n0 * self.n1
        # 1 / Z(x): the Gaussian summed over the full radius box (separable)
        def axis_sum(sv, rv):
            sv, rv = np.ravel(sv).astype(np.float64), np.ravel(rv)
            tot = np.ones_like(sv)
            for a in range(1, int(rv.max()) + 1):
                tot += np.where(a <= rv, 2.0 * np.exp(-a * a / (2.0 * sv * sv)), 0.0)
            return tot
        z = axis_sum(s0, r0) * axis_sum(s1, r1)
        self.rmax0, self.rmax1 = int(np.max(r0)), int(np.max(r1))
        to = lambda a: torch.from_numpy(np.ascontiguousarray(a).ravel()).to(device=device, dtype=dtype)
        self.s0, self.s1, self.inv_z = to(s0), to(s1), to(1.0 / z)
        self.r0 = torch.from_numpy(np.ascontiguousarray(r0, dtype=np.int32).ravel()).to(device)
        self.r1 = torch.from_numpy(np.ascontiguousarray(r1, dtype=np.int32).ravel()).to(device)
        self.code = 1 if dtype == torch.float64 else 0
        self.dtype = dtype

    def __call__(self, U, OUT=None):
        U = U.reshape(-1, self.N)
        if OUT is None:
            OUT = torch.empty_like(U)
        rc = _load().blur_forward(self.code, self.s0.data_ptr(), self.s1.data_ptr(), self.r0.data_ptr(),
                                  self.r1.data_ptr(), self.inv_z.data_ptr(), self.n0, self.n1, self.rmax0,
                                  self.rmax1, U.data_ptr(), U.stride(0), OUT.data_ptr(), OUT.stride(0), U.shape[0],
                                  torch.cuda.current_stream().cuda_stream)
        if rc != 0:
            raise RuntimeError("blur_forward launch failed")
        return OUT
