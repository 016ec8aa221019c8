"""Spatially varying Gaussian blur: the operator whose impulse responses feed
the product-convolution approximation (the black-box A of the method).

A[y, x] = exp(-sum_i (y_i-x_i)^2 / (2 s_i(x)^2)) / Z(x) if |y_i - x_i| <= R_i(x)
for all i, else 0, with R_i(x) = ceil(4 s_i(x)) and
Z(x) = sum over the full box |xi_i| <= R_i(x) of exp(-sum_i xi_i^2 / (2 s_i(x)^2)),
independent of the domain, so that a constant s gives an exact convolution
restricted to the domain.

The impulse response at p (eq. (1.2), (2.6)) is phi_p[z] = A[p+z, p]:
it is handed to the library on the full box |z_i| <= R_i(p); entries with
p + z outside the domain are ignored by the consumer.
"""
import numpy as np


class BlurOperator:
    """Blur with per-axis widths ``sig`` of shape (d, *shape) (isotropic fields
    are broadcast to every axis)."""

    def __init__(self, sig):
        sig = np.asarray(sig, dtype=np.float64)
        self.sig = sig
        self.d = sig.shape[0]
        self.shape = sig.shape[1:]
        self.radius = np.ceil(4.0 * sig).astype(np.int64)   # (d, *shape)

    @classmethod
    def isotropic(cls, s):
        s = np.asarray(s, dtype=np.float64)
        return cls(np.broadcast_to(s, (s.ndim,) + s.shape).copy())

    def width_at(self, p):
        p = tuple(int(v) for v in p)
        return np.array([self.sig[(i,) + p] for i in range(self.d)])

    def radius_at(self, p):
        p = tuple(int(v) for v in p)
        return np.array([int(self.radius[(i,) + p]) for i in range(self.d)], dtype=np.int64)

    @staticmethod
    def _column(sv, R):
        """Normalised Gaussian on the box prod [-R_i, R_i] (separable)."""
        parts = []
        for i in range(len(R)):
            xi = np.arange(-R[i], R[i] + 1, dtype=np.float64)
            parts.append(np.exp(-xi * xi / (2.0 * sv[i] * sv[i])))
        g = parts[0]
        for q in parts[1:]:
            g = np.multiply.outer(g, q)
        return g / g.sum()

    def patch(self, p):
        """phi_p on prod [-R_i(p), R_i(p)], row-major, centre at offset 0."""
        return self._column(self.width_at(p), self.radius_at(p))

    def impulse_responses(self, points):
        """Concatenated patches for each point: (radius[r, d], phi(flat), offsets[r+1])."""
        radii, blocks, offs = [], [], [0]
        for p in points:
            R = self.radius_at(p)
            g = self.patch(p)
            radii.append(R)
            blocks.append(g.ravel())
            offs.append(offs[-1] + g.size)
        return (np.array(radii, dtype=np.int64).reshape(-1, self.d),
                np.concatenate(blocks) if blocks else np.zeros(0),
                np.array(offs, dtype=np.int64))

    # --- exact operator (black box), FP64, for tests -------------------------
    def dense(self):
        """Dense N x N matrix (tiny grids only), row-major flattening of the domain."""
        shape = self.shape
        N = int(np.prod(shape))
        A = np.zeros((N, N))
        for xf in range(N):
            x = np.unravel_index(xf, shape)
            R = self.radius_at(x)
            g = self._column(self.width_at(x), R)
            for zf in range(g.size):
                z = np.array(np.unravel_index(zf, g.shape)) - R
                y = np.array(x) + z
                if np.all(y >= 0) and np.all(y < np.array(shape)):
                    A[np.ravel_multi_index(tuple(y), shape), xf] = g.flat[zf]
        return A

    def apply(self, u, adjoint=False):
        """Exact A u (or A^T u) by direct summation over columns, FP64."""
        shape = self.shape
        u = np.asarray(u, dtype=np.float64).reshape(shape)
        out = np.zeros(shape)
        d = self.d
        for xf in range(u.size):
            x = np.unravel_index(xf, shape)
            R = self.radius_at(x)
            g = self._column(self.width_at(x), R)
            lo = [max(0, x[i] - R[i]) for i in range(d)]
            hi = [min(shape[i] - 1, x[i] + R[i]) for i in range(d)]
            ys = tuple(slice(lo[i], hi[i] + 1) for i in range(d))
            gs = tuple(slice(lo[i] - x[i] + R[i], hi[i] - x[i] + R[i] + 1) for i in range(d))
            if adjoint:
                out[x] += float(np.sum(g[gs] * u[ys]))
            else:
                out[ys] += g[gs] * u[x]
        return out.ravel()
