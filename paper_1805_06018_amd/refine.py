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


def leaf_point_sets(lo, hi, pts):
    """For every leaf, the indices of the points on its closed box (pts sorted
    with axis 0 most significant, as corner_points returns them)."""
    x0 = pts[:, 0]
    a = np.searchsorted(x0, lo[:, 0], side="left")
    b = np.searchsorted(x0, hi[:, 0], side="right")
    out = []
    for c in range(len(lo)):
        cand = pts[a[c]:b[c], 1:]
        inside = np.all((cand >= lo[c, 1:]) & (cand <= hi[c, 1:]), axis=1)
        out.append(a[c] + np.nonzero(inside)[0])
    return out


def term_keys(lo, hi, pts):
    """A key per point that is equal between two tilings iff the point's term
    of the sum is the same: the point, and the boxes of the leaves containing
    it with the points on each (they fix U_k, w_k, nbrs(k) and phi_k^E)."""
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    sets = leaf_point_sets(lo, hi, pts)
    leaf_key = [lo[c].astype(np.int64).tobytes() + hi[c].astype(np.int64).tobytes() + pts[sc].tobytes()
                for c, sc in enumerate(sets)]
    cells = [[] for _ in range(len(pts))]
    for c, sc in enumerate(sets):
        for k in sc.tolist():
            cells[k].append(leaf_key[c])
    return [(pts[k].tobytes(), tuple(sorted(cells[k]))) for k in range(len(pts))]


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


def _split_round(lo, hi, eta, frac, shape, patch_of):
    order = np.argsort(-eta, kind="stable")
    refinable = [c for c in order if np.any(hi[c] - lo[c] > 2)]
    if not refinable:
        return None
    n_take = 1 if frac <= 0 else max(1, int(np.ceil(frac * len(lo))))
    chosen = set(int(c) for c in refinable[:n_take])
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
    return np.array(new_lo)[order], np.array(new_hi)[order]


def refine(shape, leaf_lo, leaf_hi, impulse_responses, patch_of, Z, Y, tol=1e-2, max_points=4000,
           frac=0.1, max_rounds=200, dtype=_lib.PC_F32, log=None, incremental=False, yt_out=None):
    """Run the loop.  impulse_responses(points) -> (radius, phi, phi_off);
    patch_of(point) -> the point's impulse-response patch (for the split
    direction); Z, Y: (q, N) device tensors, Y = A* Z.  frac = 0 refines one
    leaf per round (Algorithm 1).  Returns the final leaves and per-round
    records; with yt_out (a list), the final Y~ is appended to it."""
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
        nxt = _split_round(lo, hi, eta, frac, shape, patch_of)
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
    ap.add_argument("--max-points", type=int, default=4000)
    ap.add_argument("--max-rounds", type=int, default=200)
    ap.add_argument("--incremental", action="store_true", help="update Y~ with the changed terms only")
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
    print(json.dumps({"workload": w.name, "N": w.N, "q": args.q, "incremental": args.incremental,
                      "frac": args.frac, "t_exact_adjoint_s": time.time() - t0}), flush=True)
    yts = []
    t0 = time.time()
    lo, hi, rounds = refine(w.shape, w.leaf_lo, w.leaf_hi, w.op.impulse_responses, w.op.patch, Z, Y,
                            tol=args.tol, max_points=args.max_points, frac=args.frac, max_rounds=args.max_rounds,
                            incremental=args.incremental, yt_out=yts,
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
