"""The product-convolution operator and its adjoint, by direct summation.

Forward (eq. (2.5)):  (A~ f)[y] = sum_k sum_{x in U_k} w_k[x] f[x] phi_k^E[y - x],  y in Omega.
Adjoint (eq. (1.6)):  (A~* g)[x] = sum_k w_k[x] sum_{y in Omega} phi_k^E[y - x] g[y].
Matrix entries (Sec. 3.1): A~[y, x] = sum_{k : x in U_k} w_k[x] phi_k^E[y - x].

Everything is FP64 and summed over k in ascending order (optionally over a
subset of the terms only).  The per-patch
convolution is a plain double loop (NumPy over the input box for each kernel
offset, or the C core in ``direct`` for larger grids); no FFT is used.
"""
import numpy as np

from .grid import Grid
from .weights import harmonic_weights
from .extension import extended_kernels


class OracleOperator:
    def __init__(self, shape, leaf_lo, leaf_hi, points, radius, phi, phi_off,
                 extend=True, closed_form_weights=True):
        self.grid = Grid(shape, leaf_lo, leaf_hi, points)
        self.shape = self.grid.shape
        self.d = self.grid.d
        self.N = int(np.prod(self.shape))
        self.radius = np.asarray(radius, dtype=np.int64).reshape(-1, self.d)
        self.phi = np.asarray(phi, dtype=np.float64)
        self.phi_off = np.asarray(phi_off, dtype=np.int64)
        if np.any(self.radius < 0):
            raise ValueError("negative patch radius")
        self.extend = extend
        self.W = harmonic_weights(self.grid, closed_form=closed_form_weights)
        self.zlo, self.K = extended_kernels(self.grid, self.radius, self.phi, self.phi_off, extend)
        self.u_lo = self.grid.u_lo
        self.u_hi = self.grid.u_hi

    @classmethod
    def from_workload(cls, w, extend=True, **kw):
        return cls(w.shape, w.leaf_lo, w.leaf_hi, w.points, w.radius, w.phi, w.phi_off,
                   extend=extend, **kw)

    # -- one patch ------------------------------------------------------------
    def _conv_patch(self, k, t, out, backend):
        """out[y] += sum_x t[x] phi_k^E[y - x] for x in bbox(U_k), y in Omega."""
        if backend == "c":
            from . import direct
            direct.conv_add(t, self.u_lo[k], self.K[k], self.zlo[k], out)
            return
        d, n = self.d, self.shape
        K, zlo, ulo = self.K[k], self.zlo[k], self.u_lo[k]
        m = t.shape
        for zf in np.ndindex(K.shape):
            c = K[zf]
            if c == 0.0:
                continue
            z = np.array(zf) + zlo
            ylo = ulo + z
            a = np.maximum(ylo, 0)
            b = np.minimum(ylo + np.array(m) - 1, np.array(n) - 1)
            if np.any(a > b):
                continue
            dst = tuple(slice(int(a[i]), int(b[i] + 1)) for i in range(d))
            src = tuple(slice(int(a[i] - ylo[i]), int(b[i] - ylo[i] + 1)) for i in range(d))
            out[dst] += c * t[src]

    def _corr_patch(self, k, g, backend):
        """c[x] = sum_y phi_k^E[y - x] g[y] for x in bbox(U_k)."""
        m = tuple(int(v) for v in (self.u_hi[k] - self.u_lo[k] + 1))
        if backend == "c":
            from . import direct
            return direct.corr(g, self.u_lo[k], m, self.K[k], self.zlo[k])
        d, n = self.d, self.shape
        K, zlo, ulo = self.K[k], self.zlo[k], self.u_lo[k]
        c_out = np.zeros(m)
        for zf in np.ndindex(K.shape):
            c = K[zf]
            if c == 0.0:
                continue
            z = np.array(zf) + zlo
            ylo = ulo + z
            a = np.maximum(ylo, 0)
            b = np.minimum(ylo + np.array(m) - 1, np.array(n) - 1)
            if np.any(a > b):
                continue
            src = tuple(slice(int(a[i]), int(b[i] + 1)) for i in range(d))
            dst = tuple(slice(int(a[i] - ylo[i]), int(b[i] - ylo[i] + 1)) for i in range(d))
            c_out[dst] += c * g[src]
        return c_out

    # -- operator actions -----------------------------------------------------
    def _backend(self, backend):
        if backend is None:
            return "c" if self.N > 8192 else "numpy"
        return backend

    def _terms(self, patches):
        """Ascending point indices of the terms summed: all, or a subset (the
        terms Sec. 2.8 recomputes after a refinement)."""
        if patches is None:
            return range(self.grid.r)
        return sorted(int(k) for k in patches)

    def apply(self, f, backend=None, patches=None):
        backend = self._backend(backend)
        f = np.asarray(f, dtype=np.float64).reshape(self.shape)
        out = np.zeros(self.shape)
        for k in self._terms(patches):
            sl = tuple(slice(int(self.u_lo[k, i]), int(self.u_hi[k, i] + 1)) for i in range(self.d))
            t = self.W[k] * f[sl]
            self._conv_patch(k, t, out, backend)
        return out.ravel()

    def apply_adjoint(self, g, backend=None, patches=None):
        backend = self._backend(backend)
        g = np.asarray(g, dtype=np.float64).reshape(self.shape)
        out = np.zeros(self.shape)
        for k in self._terms(patches):
            sl = tuple(slice(int(self.u_lo[k, i]), int(self.u_hi[k, i] + 1)) for i in range(self.d))
            out[sl] += self.W[k] * self._corr_patch(k, g, backend)
        return out.ravel()

    def apply_window(self, f, lo, hi):
        """(A~ f)[y] for every y of the box [lo, hi] (inclusive), by the direct
        sums of eq. (2.5) over the ascending terms whose outputs reach the
        box; returned row-major over the box (full-size checks of whole rows,
        planes or slabs)."""
        from . import direct
        lo = np.asarray(lo, dtype=np.int64).ravel()
        hi = np.asarray(hi, dtype=np.int64).ravel()
        f = np.asarray(f, dtype=np.float64).reshape(self.shape)
        out = np.zeros(tuple(int(v) for v in hi - lo + 1))
        for k in range(self.grid.r):
            zlo = self.zlo[k]
            zhi = zlo + np.array(self.K[k].shape) - 1
            if np.any(self.u_lo[k] + zlo > hi) or np.any(self.u_hi[k] + zhi < lo):
                continue
            sl = tuple(slice(int(self.u_lo[k, i]), int(self.u_hi[k, i] + 1)) for i in range(self.d))
            direct.conv_add(self.W[k] * f[sl], self.u_lo[k], self.K[k], zlo, out, olo=lo)
        return out.ravel()

    def apply_adjoint_window(self, g, lo, hi):
        """(A~* g)[x] for every x of the box [lo, hi] (eq. (1.6)), row-major
        over the box: per ascending term, the correlation with phi_k^E on the
        part of bbox(U_k) inside the box, times w_k."""
        from . import direct
        lo = np.asarray(lo, dtype=np.int64).ravel()
        hi = np.asarray(hi, dtype=np.int64).ravel()
        g = np.asarray(g, dtype=np.float64).reshape(self.shape)
        out = np.zeros(tuple(int(v) for v in hi - lo + 1))
        for k in range(self.grid.r):
            a = np.maximum(self.u_lo[k], lo)
            b = np.minimum(self.u_hi[k], hi)
            if np.any(a > b):
                continue
            c = direct.corr(g, a, b - a + 1, self.K[k], self.zlo[k])
            wsl = tuple(slice(int(a[i] - self.u_lo[k, i]), int(b[i] - self.u_lo[k, i] + 1)) for i in range(self.d))
            osl = tuple(slice(int(a[i] - lo[i]), int(b[i] - lo[i] + 1)) for i in range(self.d))
            out[osl] += self.W[k][wsl] * c
        return out.ravel()

    def apply_batch(self, F, adjoint=False, backend=None, patches=None):
        F = np.asarray(F, dtype=np.float64).reshape(-1, self.N)
        fn = self.apply_adjoint if adjoint else self.apply
        return np.stack([fn(f, backend, patches) for f in F])

    def entry(self, y, x):
        """A~[y, x] from the matrix-entry formula (Sec. 3.1)."""
        y = np.asarray(y)
        x = np.asarray(x)
        s = 0.0
        for k in range(self.grid.r):
            if np.any(x < self.u_lo[k]) or np.any(x > self.u_hi[k]):
                continue
            wk = self.W[k][tuple(x - self.u_lo[k])]
            if wk == 0.0:
                continue
            z = y - x - self.zlo[k]
            if np.any(z < 0) or np.any(z >= np.array(self.K[k].shape)):
                continue
            s += wk * self.K[k][tuple(z)]
        return s

    def dense(self):
        """Dense N x N matrix from the matrix-entry formula (tiny grids)."""
        N = self.N
        A = np.zeros((N, N))
        coords = [np.array(np.unravel_index(i, self.shape)) for i in range(N)]
        for xf in range(N):
            x = coords[xf]
            for k in range(self.grid.r):
                if np.any(x < self.u_lo[k]) or np.any(x > self.u_hi[k]):
                    continue
                wk = self.W[k][tuple(x - self.u_lo[k])]
                if wk == 0.0:
                    continue
                K, zlo = self.K[k], self.zlo[k]
                for zf in np.ndindex(K.shape):
                    if K[zf] == 0.0:
                        continue
                    y = x + np.array(zf) + zlo
                    if np.all(y >= 0) and np.all(y < np.array(self.shape)):
                        A[np.ravel_multi_index(tuple(y), self.shape), xf] += wk * K[zf]
        return A

    def apply_at(self, f, ys):
        """(A~ f)[y] for a list of output points (for sampled checks at full size)."""
        f = np.asarray(f, dtype=np.float64).reshape(self.shape)
        ys = np.asarray(ys, dtype=np.int64).reshape(-1, self.d)
        out = np.zeros(len(ys))
        for k in range(self.grid.r):
            ulo, uhi = self.u_lo[k], self.u_hi[k]
            K, zlo = self.K[k], self.zlo[k]
            zhi = zlo + np.array(K.shape) - 1
            # outputs touched by this patch
            hit = np.all((ys >= ulo + zlo) & (ys <= uhi + zhi), axis=1)
            for q in np.nonzero(hit)[0]:
                y = ys[q]
                a = np.maximum(ulo, y - zhi)
                b = np.minimum(uhi, y - zlo)
                if np.any(a > b):
                    continue
                xs = tuple(slice(int(a[i]), int(b[i] + 1)) for i in range(self.d))
                wsl = tuple(slice(int(a[i] - ulo[i]), int(b[i] - ulo[i] + 1)) for i in range(self.d))
                # phi^E[y - x] for x in [a, b]: reversed slice of K
                ksl = tuple(slice(int(y[i] - a[i] - zlo[i]), int(y[i] - b[i] - zlo[i]) - 1 if int(y[i] - b[i] - zlo[i]) > 0 else None, -1)
                            for i in range(self.d))
                out[q] += float(np.sum(self.W[k][wsl] * f[xs] * K[ksl]))
        return out

    def apply_adjoint_at(self, g, xs):
        """(A~* g)[x] for a list of points x (eq. (1.6)), by direct summation."""
        g = np.asarray(g, dtype=np.float64).reshape(self.shape)
        xs = np.asarray(xs, dtype=np.int64).reshape(-1, self.d)
        n = np.array(self.shape)
        out = np.zeros(len(xs))
        for k in range(self.grid.r):
            ulo, uhi = self.u_lo[k], self.u_hi[k]
            K, zlo = self.K[k], self.zlo[k]
            for q in np.nonzero(np.all((xs >= ulo) & (xs <= uhi), axis=1))[0]:
                x = xs[q]
                wk = self.W[k][tuple(x - ulo)]
                if wk == 0.0:
                    continue
                # y = x + z for z in the kernel box, y inside Omega
                a = np.maximum(zlo, -x)
                b = np.minimum(zlo + np.array(K.shape) - 1, n - 1 - x)
                if np.any(a > b):
                    continue
                ksl = tuple(slice(int(a[i] - zlo[i]), int(b[i] - zlo[i] + 1)) for i in range(self.d))
                gsl = tuple(slice(int(x[i] + a[i]), int(x[i] + b[i] + 1)) for i in range(self.d))
                out[q] += wk * float(np.sum(K[ksl] * g[gsl]))
        return out
