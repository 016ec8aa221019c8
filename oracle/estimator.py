"""Randomized a-posteriori error estimator (Sec. 2.6).

With probe vectors Z (q columns), Y = A* Z (exact adjoint) and Y~ = A~* Z:
  eta_C     = q^{-1/2} || (Y~ - Y)[C, :] ||_F   for every leaf C
              (C's own point set: points on shared facets count in each cell);
  eta_Omega = q^{-1/2} || Y~ - Y ||_F           (every grid point once);
  eta_rel   = || Y~ - Y ||_F / || Y ||_F.
The sample-average identity ||M||_F^2 = E ||M zeta||^2 (eq. (2.10)) makes
eta_C^2 an unbiased estimate of e_C^2 = ||(A~ - A)[Omega, C]||_F^2.
"""
import numpy as np


def estimate(op, Z, Y, backend=None):
    """op: OracleOperator; Z, Y: (q, N).  Returns (eta_leaf[L], eta_omega, eta_rel, Ytilde)."""
    Z = np.asarray(Z, dtype=np.float64).reshape(-1, op.N)
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, op.N)
    q = Z.shape[0]
    Yt = op.apply_batch(Z, adjoint=True, backend=backend)
    D = (Yt - Y).reshape((q,) + op.shape)
    sq = np.sum(D * D, axis=0)          # sum over probes, per grid point
    g = op.grid
    eta = np.zeros(g.leaf_lo.shape[0])
    for c in range(g.leaf_lo.shape[0]):
        sl = tuple(slice(int(g.leaf_lo[c, i]), int(g.leaf_hi[c, i] + 1)) for i in range(op.d))
        eta[c] = np.sqrt(np.sum(sq[sl]) / q)
    tot = float(np.sum(sq))
    eta_omega = np.sqrt(tot / q)
    eta_rel = np.sqrt(tot) / np.sqrt(float(np.sum(Y * Y)))
    return eta, eta_omega, eta_rel, Yt
