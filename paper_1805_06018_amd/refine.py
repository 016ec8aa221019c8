"""Adaptive refinement driven by the randomized error estimator (Sec. 2.3,
Sec. 2.6, Sec. 2.7, Algorithm 1), rebuilding the operator every round.

Y = A* Z is computed once (Sec. 2.8) by the caller's exact adjoint.  Each
round builds the product-convolution operator on the current leaves
(pc_create), estimates eta_C for every leaf and the relative error
||Y~ - Y||_F / ||Y||_F (pc_error_estimate), and stops when the relative
error is below the tolerance or the point budget is reached.  Otherwise it
refines the worst leaves: Algorithm 1 refines one leaf per iteration; this
driver refines a fraction of the leaves with the largest eta_C per round, so
that a grid of a few thousand points is reached in a few dozen rebuilds.

Subdivision direction (Sec. 2.7): for each axis along which the leaf is wider
than 2, the impulse responses of the corners on the front and on the back of
the leaf are averaged, and the leaf is split at its midpoint along the axis
where the two averages differ most in l2 over the offsets z with
c_mid + z in Omega.  The impulse responses used are the supplied patches
(zero outside their boxes).
"""
import itertools
import json
import sys
import time

import numpy as np
import torch

from . import _lib


def corner_points(lo, hi):
    d = lo.shape[1]
    pts = set()
    for a, b in zip(lo, hi):
        for bits in itertools.product((0, 1), repeat=d):
            pts.add(tuple(int(b[i] if bit else a[i]) for i, bit in enumerate(bits)))
    return np.array(sorted(pts), dtype=np.int64).reshape(-1, d)


def split_direction(lo, hi, shape, patch_of):
    """Axis along which the corner impulse responses change the most."""
    d = len(lo)
    mid = [(lo[i] + hi[i]) // 2 for i in range(d)]
    best, best_axis = -1.0, None
    for i in range(d):
        if hi[i] - lo[i] <= 2:
            continue
        groups = {}
        for side, val in (("+", hi[i]), ("-", lo[i])):
            pats = []
            for bits in itertools.product((0, 1), repeat=d):
                p = tuple(int(hi[j] if bits[j] else lo[j]) for j in range(d))
                if p[i] == val:
                    pats.append(patch_of(p))
            groups[side] = pats
        R = np.max([np.array(P.shape) // 2 for P in groups["+"] + groups["-"]], axis=0)

        def avg(pats):
            acc = np.zeros(tuple(2 * R + 1))
            for P in pats:
                r = np.array(P.shape) // 2
                sl = tuple(slice(int(R[j] - r[j]), int(R[j] + r[j] + 1)) for j in range(d))
                acc[sl] += P
            return acc / len(pats)

        diff = avg(groups["+"]) - avg(groups["-"])
        # restrict to offsets z with c_mid + z inside the domain
        sl = tuple(slice(int(max(0, R[j] - mid[j])), int(min(2 * R[j] + 1, R[j] + shape[j] - mid[j])))
                   for j in range(d))
        val = float(np.sqrt(np.sum(diff[sl] ** 2)))
        if val > best:
            best, best_axis = val, i
    return best_axis


def split_leaf(lo, hi, axis):
    mid = (lo[axis] + hi[axis]) // 2
    a_hi = hi.copy()
    a_hi[axis] = mid
    b_lo = lo.copy()
    b_lo[axis] = mid
    return (lo.copy(), a_hi), (b_lo, hi.copy())


def refine(shape, leaf_lo, leaf_hi, impulse_responses, patch_of, Z, Y, tol=1e-2, max_points=4000,
           frac=0.1, max_rounds=200, dtype=_lib.PC_F32, log=None):
    """Run the loop.  impulse_responses(points) -> (radius, phi, phi_off);
    patch_of(point) -> the point's impulse-response patch (for the split
    direction); Z, Y: (q, N) device tensors, Y = A* Z.  Returns the final
    leaves and per-round records."""
    lo = np.array(leaf_lo, dtype=np.int64)
    hi = np.array(leaf_hi, dtype=np.int64)
    d = lo.shape[1]
    rounds = []
    for it in range(max_rounds):
        t0 = time.time()
        pts = corner_points(lo, hi)
        radius, phi, off = impulse_responses(pts)
        t1 = time.time()
        op = _lib.PcOperator(d, shape, lo, hi, pts, radius, phi, off, dtype=dtype)
        t2 = time.time()
        eta, eabs, erel = op.error_estimate(Z, Y)
        t3 = time.time()
        rec = {"round": it, "points": int(len(pts)), "leaves": int(len(lo)), "eta_rel": erel, "eta_abs": eabs,
               "t_impulse_s": t1 - t0, "t_create_s": t2 - t1, "t_estimate_s": t3 - t2}
        rounds.append(rec)
        if log:
            log(rec)
        op.close()
        if erel < tol or len(pts) >= max_points:
            break
        order = np.argsort(-eta, kind="stable")
        refinable = [c for c in order if np.any(hi[c] - lo[c] > 2)]
        if not refinable:
            break
        take = refinable[:max(1, int(np.ceil(frac * len(lo))))]
        chosen = set(int(c) for c in take)
        new_lo, new_hi = [], []
        for c in range(len(lo)):
            if c in chosen:
                axis = split_direction(lo[c], hi[c], shape, patch_of)
                (alo, ahi), (blo, bhi) = split_leaf(lo[c], hi[c], axis)
                new_lo += [alo, blo]
                new_hi += [ahi, bhi]
            else:
                new_lo.append(lo[c])
                new_hi.append(hi[c])
        order = np.lexsort(np.array(new_lo).T[::-1])
        lo = np.array(new_lo)[order]
        hi = np.array(new_hi)[order]
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
    ap.add_argument("--frac", type=float, default=0.1)
    ap.add_argument("--max-points", type=int, default=4000)
    args = ap.parse_args(argv)
    w = make_config(args.config, scale=args.scale)
    Z = torch.from_numpy(w.rademacher(args.q, w.vec_seed).astype(np.float32)).cuda()
    exact = GpuBlurAdjoint(w.op)
    t0 = time.time()
    Y = exact(Z)
    torch.cuda.synchronize()
    print(json.dumps({"workload": w.name, "N": w.N, "q": args.q, "t_exact_adjoint_s": time.time() - t0}),
          flush=True)
    lo, hi, rounds = refine(w.shape, w.leaf_lo, w.leaf_hi, w.op.impulse_responses, w.op.patch, Z, Y,
                            tol=args.tol, max_points=args.max_points, frac=args.frac,
                            log=lambda r: print(json.dumps(r), flush=True))
    print(json.dumps({"final_points": rounds[-1]["points"], "final_eta_rel": rounds[-1]["eta_rel"],
                      "rounds": len(rounds)}), flush=True)


if __name__ == "__main__":
    main()
