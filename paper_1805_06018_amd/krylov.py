"""Krylov solves preconditioned with the product-convolution approximation,
without hierarchical matrices.

The paper uses A~ to precondition Krylov solves with operators that are
expensive to apply (Sec. 1, Sec. 5.2, Sec. 5.3), through a hierarchical-matrix
factorisation of A~.  Here A~ enters through its fast applies instead:

    problem:         (A* A + alpha I) x = A* b      (Tikhonov-regularised
                     deblurring with the exact blur A; symmetric positive
                     definite; CG)
    preconditioner:  y = P(r) ~ (A~* A~ + alpha I)^{-1} r by a fixed number of
                     inner CG iterations on the approximation's normal
                     operator (two library applies per inner iteration)

The preconditioner changes with its argument (an inner iteration), so the
outer solve is flexible CG (beta from (z_{k+1}, r_{k+1} - r_k)).  Operator
applies run in the HIP kernels (the library for A~, the workloads' direct
blur for A); the vector updates and inner products of the Krylov recurrence
are plain device tensor operations.
"""
import json
import time

import numpy as np
import torch

from . import _lib


def _dot(a, b):
    return float(torch.dot(a.reshape(-1), b.reshape(-1)))


def cg(apply, b, tol=1e-8, maxit=500, x0=None, precond=None, flexible=False):
    """(Flexible) preconditioned CG on a symmetric positive definite apply.
    Returns x and the list of relative residual norms (one per iteration)."""
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    r = b - apply(x) if x0 is not None else b.clone()
    nb = float(torch.linalg.vector_norm(b))
    z = precond(r) if precond else r
    p = z.clone()
    rz = _dot(r, z)
    hist = [float(torch.linalg.vector_norm(r)) / nb]
    for _ in range(maxit):
        if hist[-1] < tol:
            break
        q = apply(p)
        alpha = rz / _dot(p, q)
        x += alpha * p
        r_old = r.clone() if flexible else None
        r -= alpha * q
        hist.append(float(torch.linalg.vector_norm(r)) / nb)
        if hist[-1] < tol:
            break
        z = precond(r) if precond else r
        rz_new = _dot(r, z)
        beta = (rz_new - _dot(r_old, z)) / rz if flexible else rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, hist


class NormalOps:
    """(A* A + alpha I) for the exact blur and for the approximation."""

    def __init__(self, forward, adjoint, pc, alpha):
        self.fwd, self.adj, self.pc, self.alpha = forward, adjoint, pc, alpha
        self.n_exact = 0
        self.n_approx = 0

    def exact(self, x):
        self.n_exact += 2
        return self.adj(self.fwd(x[None, :]))[0] + self.alpha * x

    def approx(self, x):
        self.n_approx += 2
        t = torch.empty_like(x)
        self.pc.apply(x, t)
        s = torch.empty_like(x)
        self.pc.apply_adjoint_batch(t[None, :], s[None, :])
        return s + self.alpha * x

    def precond(self, inner):
        def p(r):
            y, _ = cg(self.approx, r, tol=0.0, maxit=inner)
            return y
        return p


def solve_demo(w, alpha, inner=10, tol=1e-8, maxit=400, dtype=torch.float64, seed=7, log=None):
    """Deblur a seeded image on workload w: plain CG on the exact normal
    operator against flexible CG preconditioned with inner solves on the
    approximation.  Returns a dict of iteration counts, applies and times."""
    from workloads.blur_gpu import GpuBlur, GpuBlurAdjoint
    A = GpuBlur(w.op, dtype=dtype)
    At = GpuBlurAdjoint(w.op, dtype=dtype)
    pc_dtype = _lib.PC_F64 if dtype == torch.float64 else _lib.PC_F32
    op = _lib.PcOperator.from_workload(w, dtype=pc_dtype)
    rng = np.random.default_rng(seed)
    x_true = torch.from_numpy(rng.standard_normal(w.N)).to(device="cuda", dtype=dtype)
    b = A(x_true[None, :])[0]
    ops = NormalOps(A, At, op, alpha)
    rhs = At(b[None, :])[0]
    torch.cuda.synchronize()
    out = {"workload": w.name, "N": w.N, "points": w.r, "alpha": alpha, "inner": inner, "tol": tol}
    t0 = time.time()
    x_cg, h_cg = cg(ops.exact, rhs, tol=tol, maxit=maxit)
    torch.cuda.synchronize()
    out.update({"cg_iterations": len(h_cg) - 1, "cg_exact_applies": ops.n_exact, "cg_s": time.time() - t0,
                "cg_final_res": h_cg[-1]})
    ops.n_exact = ops.n_approx = 0
    t0 = time.time()
    x_p, h_p = cg(ops.exact, rhs, tol=tol, maxit=maxit, precond=ops.precond(inner), flexible=True)
    torch.cuda.synchronize()
    out.update({"pcg_iterations": len(h_p) - 1, "pcg_exact_applies": ops.n_exact,
                "pcg_approx_applies": ops.n_approx, "pcg_s": time.time() - t0, "pcg_final_res": h_p[-1],
                "solution_diff_rel": float(torch.linalg.vector_norm(x_p - x_cg) / torch.linalg.vector_norm(x_cg))})
    if log:
        log(out)
    return out, h_cg, h_p


def main(argv=None):
    import argparse
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from workloads import cosine_field, tune_quadtree
    from workloads.configs import _finish

    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--points", type=int, default=300)
    ap.add_argument("--alpha", type=str, default="1e-2,1e-3")
    ap.add_argument("--inner", type=int, default=10)
    ap.add_argument("--tol", type=float, default=1e-8)
    args = ap.parse_args(argv)
    s, _ = cosine_field((args.n, args.n), 2.0, 8.0, 2, 3, seed=5)
    _, lo, hi, _ = tune_quadtree(s, int(args.points * 0.9), int(args.points * 1.1) + 1)
    w = _finish(f"blur2d_{args.n}_quadtree", np.stack([s, s]), lo, hi, 1, 0, {})
    for a in (float(v) for v in args.alpha.split(",")):
        solve_demo(w, a, inner=args.inner, tol=args.tol, log=lambda r: print(json.dumps(r), flush=True))


if __name__ == "__main__":
    main()
