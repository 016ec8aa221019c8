"""Adaptive refinement driven by the randomized error estimator (Sec. 2.3,
Sec. 2.6, Sec. 2.7, Sec. 2.8, Algorithm 1).

Y = A* Z is computed once (Sec. 2.8) by the caller's exact adjoint.  Each
round estimates eta_C for every leaf and the relative error
||Y~ - Y||_F / ||Y||_F and stops when the relative error is below the
tolerance or the point budget is reached.  Otherwise it refines the worst
leaves: Algorithm 1 refines one leaf per iteration (frac = 0 here); frac > 0
refines that fraction of the leaves with the largest eta_C per round.

Two ways to keep Y~ = A~* Z current:
  - rebuild: the whole operator is built again every round and Y~ recomputed
    (pc_create + pc_error_estimate);
  - incremental (Sec. 2.8): Y~ stays on the device; after a refinement only
    the terms of the sum that changed are convolved: those of new points and
    of points whose cells, weights or neighbours changed.  The old terms are
    subtracted with an operator holding only them on the old tiling, the new
    ones added with one holding only them on the new tiling
    (pc_create_patches + pc_apply_adjoint_batch_axpy), and the estimator sums
    are formed from the updated Y~ (pc_estimate_sums).  Impulse responses are
    requested only for new points.

Subdivision direction (Sec. 2.7): tiling.split_direction, the paper's
front/back comparison of corner impulse responses with the change measured
through the leaf's midplane as well (see that module).
"""
import json
import sys
import time

import numpy as np
import torch

from . import _lib
from .tiling import corner_points, split_round, term_keys


class _ImpulseCache:
    """Impulse responses per point, computed once per point (Sec. 2.8: A is
    applied to point sources at new sample points only)."""

    def __init__(self, impulse_responses):
        self.fn = impulse_responses
        self.cache = {}
        self.n_new = 0

    def __call__(self, pts):
        new = [p for p in map(tuple, pts) if p not in self.cache]
        if new:
            radius, phi, off = self.fn(np.array(new, dtype=np.int64))
            for i, p in enumerate(new):
                self.cache[p] = (radius[i], phi[off[i]:off[i + 1]])
            self.n_new += len(new)
        rad = np.array([self.cache[tuple(p)][0] for p in pts], dtype=np.int64)
        blocks = [self.cache[tuple(p)][1] for p in pts]
        off = np.zeros(len(pts) + 1, dtype=np.int64)
        off[1:] = np.cumsum([b.size for b in blocks])
        return rad, np.concatenate(blocks), off


def refine(shape, leaf_lo, leaf_hi, impulse_responses, patch_of, Z, Y, tol=1e-2, max_points=4000,
           frac=0.1, max_rounds=200, dtype=_lib.PC_F32, log=None, incremental=False, yt_out=None,
           rule="midplane"):
    """Run the loop.  impulse_responses(points) -> (radius, phi, phi_off);
    patch_of(point) -> the point's impulse-response patch (for the split
    direction); Z, Y: (q, N) device tensors, Y = A* Z.  frac = 0 refines one
    leaf per round (Algorithm 1).  rule: the subdivision-direction rule of
    tiling.split_direction ("midplane", or the corner-only "faces").
    Returns the final leaves and per-round records; with yt_out (a list),
    the final Y~ is appended to it."""
    lo = np.array(leaf_lo, dtype=np.int64)
    hi = np.array(leaf_hi, dtype=np.int64)
    d = lo.shape[1]
    imp = _ImpulseCache(impulse_responses)
    rounds = []
    Yt = None
    prev = None          # (lo, hi, pts, radius, phi, off, keys) of the previous tiling
    for it in range(max_rounds):
        t0 = time.time()
        pts = corner_points(lo, hi)
        radius, phi, off = imp(pts)
        t1 = time.time()
        rec = {"round": it, "points": int(len(pts)), "leaves": int(len(lo))}
        if not incremental or prev is None:
            op = _lib.PcOperator(d, shape, lo, hi, pts, radius, phi, off, dtype=dtype)
            t2 = time.time()
            if incremental:
                Yt = torch.zeros_like(Y)
                op.apply_adjoint_batch(Z, Yt)
                eta, eabs, erel = op.estimate_sums(Yt, Y)
            else:
                eta, eabs, erel = op.error_estimate(Z, Y)
            keys = term_keys(lo, hi, pts) if incremental else None
            rec["terms_convolved"] = int(len(pts))
        else:
            keys = term_keys(lo, hi, pts)
            plo, phi_, ppts, prad, pphi, poff, pkeys = prev
            kn, ko = set(keys), set(pkeys)
            s_old = [k for k in range(len(ppts)) if pkeys[k] not in kn]
            s_new = [k for k in range(len(pts)) if keys[k] not in ko]
            op_old = _lib.PcOperator(d, shape, plo, phi_, ppts, prad, pphi, poff, dtype=dtype, patches=s_old)
            op = _lib.PcOperator(d, shape, lo, hi, pts, radius, phi, off, dtype=dtype, patches=s_new)
            t2 = time.time()
            op_old.apply_adjoint_batch_axpy(Z, -1.0, Yt)
            op.apply_adjoint_batch_axpy(Z, 1.0, Yt)
            eta, eabs, erel = op.estimate_sums(Yt, Y)
            op_old.close()
            rec["terms_convolved"] = int(len(s_old) + len(s_new))
        t3 = time.time()
        rec.update({"eta_rel": erel, "eta_abs": eabs, "t_impulse_s": t1 - t0, "t_create_s": t2 - t1,
                    "t_estimate_s": t3 - t2, "new_impulse_responses": imp.n_new})
        rounds.append(rec)
        if log:
            log(rec)
        op.close()
        if incremental:
            prev = (lo, hi, pts, radius, phi, off, keys)
        if erel < tol or len(pts) >= max_points or it == max_rounds - 1:
            break        # the returned tiling is the one the last estimate is for
        nxt = split_round(lo, hi, eta, frac, shape, patch_of, rule)
        if nxt is None:
            break
        lo, hi = nxt
    if yt_out is not None and Yt is not None:
        yt_out.append(Yt)
    return lo, hi, rounds


def main(argv=None):
    """Run the loop on a seeded blur workload (inputs from the workloads package)."""
    import argparse
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from workloads import make_config
    from workloads.blur_gpu import GpuBlurAdjoint

    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--q", type=int, default=32)
    ap.add_argument("--tol", type=float, default=1e-2)
    ap.add_argument("--frac", type=float, default=0.1, help="0: one leaf per round (Algorithm 1)")
    ap.add_argument("--max-points", type=int, default=20000)
    ap.add_argument("--max-rounds", type=int, default=200)
    ap.add_argument("--incremental", action="store_true", help="update Y~ with the changed terms only")
    ap.add_argument("--rule", choices=["midplane", "faces"], default="midplane",
                    help="subdivision-direction rule (tiling.split_direction)")
    ap.add_argument("--drift-check", action="store_true",
                    help="at the end, compare the incremental Y~ with a full recomputation")
    ap.add_argument("--q-check", type=str, default="",
                    help="comma list of probe counts (e.g. 5,100): on the final tiling, estimate with "
                         "fresh probe sets of each size")
    args = ap.parse_args(argv)
    w = make_config(args.config, scale=args.scale)
    Z = torch.from_numpy(w.rademacher(args.q, w.vec_seed).astype(np.float32)).cuda()
    exact = GpuBlurAdjoint(w.op)
    t0 = time.time()
    Y = exact(Z)
    torch.cuda.synchronize()
    cmd = "python -m paper_1805_06018_amd.refine " + " ".join(sys.argv[1:] if argv is None else argv)
    print(json.dumps({"command": cmd.strip(), "workload": w.name, "N": w.N, "q": args.q,
                      "incremental": args.incremental,
                      "frac": args.frac, "rule": args.rule, "t_exact_adjoint_s": time.time() - t0}), flush=True)
    yts = []
    t0 = time.time()
    lo, hi, rounds = refine(w.shape, w.leaf_lo, w.leaf_hi, w.op.impulse_responses, w.op.patch, Z, Y,
                            tol=args.tol, max_points=args.max_points, frac=args.frac, max_rounds=args.max_rounds,
                            incremental=args.incremental, yt_out=yts, rule=args.rule,
                            log=lambda r: print(json.dumps(r), flush=True))
    t_loop = time.time() - t0
    out = {"final_points": rounds[-1]["points"], "final_eta_rel": rounds[-1]["eta_rel"], "rounds": len(rounds),
           "t_loop_s": t_loop, "terms_convolved": int(sum(r["terms_convolved"] for r in rounds))}
    need_full = args.drift_check or args.q_check
    if need_full:
        pts = corner_points(lo, hi)
        radius, phi, off = w.op.impulse_responses(pts)
        op = _lib.PcOperator(w.d, w.shape, lo, hi, pts, radius, phi, off)
    if args.drift_check and yts:
        full = torch.zeros_like(Y)
        op.apply_adjoint_batch(Z, full)
        torch.cuda.synchronize()
        out["yt_drift_rel"] = float((yts[0] - full).double().norm() / full.double().norm())
        _, _, erel_full = op.estimate_sums(full, Y)
        out["eta_rel_full_recompute"] = erel_full
    if args.q_check:
        for i, qc in enumerate(int(v) for v in args.q_check.split(",")):
            Zc = torch.from_numpy(w.rademacher(qc, w.vec_seed + 7000 + i).astype(np.float32)).cuda()
            Yc = exact(Zc)
            _, _, er = op.error_estimate(Zc, Yc)
            out[f"eta_rel_q{qc}"] = er
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
