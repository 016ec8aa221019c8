"""Continuous-batching request loop over resident product-convolution
operators.

Requests (apply, or error-estimate with probe vectors) arrive on a Poisson
clock for one of several resident operators.  The server keeps every
operator's spectra on the device and runs a loop that
  - moves arrived requests into a queue;
  - retires finished batches (their events have fired);
  - admits work while a stream slot is free and the HBM budget allows it: all
    queued apply requests for the operator with the oldest waiting request are
    merged into one fused pc_apply_batch launch (continuous batching across
    requests; the apply of each vector is independent of the batch, so every
    result is bitwise the same alone and in the mix); an estimate request is
    stream-ordered too: the adjoint apply of its probes and the estimator
    sums (pc_estimate_sums_device) are enqueued with a copy of the sums to
    pinned host memory, and eta is formed once its event has fired, so the
    loop never blocks on the device.
Batches for different operators run on different streams and overlap on the
device; one operator has at most one batch in flight (its work buffers are
shared).  Each request reads its own rows of the operator's input pool (an
offset that depends on its id), so a result handed to the wrong request
shows.  Modes: "batched" (the above), "sequential" (one request at a time,
fused kernels) and "plain" (one request at a time, one launch per patch and
vector).  Latency = completion time observed by the loop - arrival time.
"""
import json
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib


@dataclass
class Request:
    rid: int
    op: int
    kind: str            # "apply" or "estimate"
    B: int
    arrival: float       # seconds after the start of the run
    t_done: float = None
    result: object = None
    retried: bool = False    # its batch failed once; it runs alone next
    solo: bool = False
    failed: bool = False     # failed again alone: result holds the error


@dataclass
class Resident:
    name: str
    pc: object           # _lib.PcOperator
    N: int
    U: torch.Tensor      # (POOL_ROWS, N) input pool: a request reads B rows from its own offset
    Z: torch.Tensor      # (q, N) probes for estimate requests
    Y: torch.Tensor      # (q, N) exact adjoint of Z
    work_bytes: int = 0  # resident operator data + staging estimate


POOL_ROWS = 64


def input_rows(q):
    """First pool row of request q's input (its B rows follow)."""
    return (q.rid * 13) % (POOL_ROWS - q.B + 1)


def poisson_requests(n_req, n_ops, rate, seed=104, max_b=32, p_estimate=0.2, q=8):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_req):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        op = int(rng.integers(0, n_ops))
        kind = "estimate" if rng.uniform() < p_estimate else "apply"
        B = q if kind == "estimate" else int(rng.integers(1, max_b + 1))
        out.append(Request(i, op, kind, B, t))
    return out


class _Batch:
    def __init__(self, op, reqs, stream, nbytes, finish=None):
        self.op, self.reqs, self.stream, self.nbytes = op, reqs, stream, nbytes
        self.finish = finish          # called once the event has fired
        self.large = False
        self.event = torch.cuda.Event()


class Server:
    def __init__(self, residents, hbm_budget=16 << 30, max_batch=64, n_streams=4, large_work=128 << 20):
        """max_batch: vectors merged into one launch; large_work: requests
        whose work (_work) exceeds it run alone, and merged batches stay
        below it."""
        self.ops = residents
        self.budget = hbm_budget
        self.max_batch = max_batch
        self.large_work = large_work
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.resident_bytes = sum(r.work_bytes for r in residents)
        if self.resident_bytes > self.budget:
            raise ValueError("resident operators exceed the HBM budget")
        self.launch_failures = 0

    def _work(self, B, op):
        """Relative cost of B vectors on an operator: grid points, a 3-D
        point weighted 10 (the 3-D apply runs about ten times fewer grid
        points per second than the 2-D one)."""
        r = self.ops[op]
        return B * r.N * (10 if r.pc.d == 3 else 1)

    def _large(self, q):
        return self._work(q.B, q.op) > self.large_work

    def _failed(self, reqs, err, pending, t):
        """A launch failed: nothing of it was enqueued and the operator stays
        valid.  Every request of the batch goes back to the front of the
        queue to run alone once more; a request whose own retry fails is
        reported failed."""
        self.launch_failures += 1
        for q in reversed(reqs):
            if q.retried:
                q.result = f"failed: {err}"
                q.failed = True
                q.t_done = t
            else:
                q.retried = True
                q.solo = True
                pending.appendleft(q)

    def _launch_apply(self, op, reqs, stream, plain=False):
        r = self.ops[op]
        Bt = sum(q.B for q in reqs)
        with torch.cuda.stream(stream):
            rows = [(input_rows(q), q.B) for q in reqs]
            if len(reqs) == 1:
                inp = r.U[rows[0][0]:rows[0][0] + Bt]
            else:
                inp = torch.cat([r.U[a:a + b] for a, b in rows], dim=0)
            out = torch.empty((Bt, r.N), dtype=torch.float32, device="cuda")
            (r.pc.apply_batch_plain if plain else r.pc.apply_batch)(inp, out, stream=stream)
        o = 0
        for q in reqs:
            q.result = out[o:o + q.B]
            o += q.B
        b = _Batch(op, reqs, stream, 2 * Bt * r.N * 4)
        b.large = self._work(Bt, op) > self.large_work
        b.event.record(stream)
        return b

    def _launch_estimate(self, q, stream):
        """Enqueues Y~ = A~* Z, the estimator sums and their copy to pinned
        host memory on the stream; eta is formed after the event."""
        r = self.ops[q.op]
        with torch.cuda.stream(stream):
            Yt = torch.empty((q.B, r.N), dtype=torch.float32, device="cuda")
            r.pc.apply_adjoint_batch(r.Z[:q.B], Yt, stream=stream)
            sums = torch.empty(r.pc.n_leaves + 2, dtype=torch.float64, device="cuda")
            r.pc.estimate_sums_device(Yt, r.Y[:q.B], sums, stream=stream)
            host = torch.empty(sums.shape, dtype=torch.float64, pin_memory=True)
            host.copy_(sums, non_blocking=True)

        def finish():
            q.result = r.pc.eta_from_sums(host.numpy(), q.B)

        b = _Batch(q.op, [q], stream, q.B * r.N * 4, finish)
        b.large = self._large(q)
        b.event.record(stream)
        return b

    def run(self, requests, mode="batched"):
        reqs = sorted(requests, key=lambda q: q.arrival)
        pending = deque()
        inflight = []
        busy_ops = set()
        inflight_bytes = 0
        peak = self.resident_bytes
        batches = []
        i = 0
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        while i < len(reqs) or pending or inflight:
            t = now()
            while i < len(reqs) and reqs[i].arrival <= t:
                pending.append(reqs[i])
                i += 1
            for b in list(inflight):
                if b.event.query():
                    if b.finish:
                        b.finish()
                    td = now()
                    for q in b.reqs:
                        q.t_done = td
                    inflight.remove(b)
                    busy_ops.discard(b.op)
                    inflight_bytes -= b.nbytes
            if mode != "batched" and inflight:
                continue
            if not pending:
                if not inflight and i < len(reqs):
                    time.sleep(max(0.0, min(reqs[i].arrival - now(), 1e-3)))
                continue
            if len(inflight) >= len(self.streams):
                continue
            free = [s for s in self.streams if all(b.stream is not s for b in inflight)]
            stream = free[0]
            if mode != "batched":
                q = pending.popleft()
                try:
                    if q.kind == "estimate":
                        b = self._launch_estimate(q, stream)
                    else:
                        b = self._launch_apply(q.op, [q], stream, plain=(mode == "plain"))
                except _lib.PcError as e:
                    self._failed([q], e, pending, now())
                    continue
                inflight.append(b)
                batches.append(1)
                continue
            # batched: the oldest waiting request whose operator is free.  A
            # large request (work above large_work) is served as in the
            # sequential loop - it waits for the device to drain, then runs
            # alone - so the requests that set the latency tail are never
            # slowed by sharing the device; small requests are merged and
            # overlapped, and do not overtake a large request at the head
            if any(b.large for b in inflight):
                continue
            # a large request at the head of the queue is served next, whatever
            # operator it needs: nothing behind it is admitted while it waits
            head = pending[0] if self._large(pending[0]) else next(
                (q for q in pending if q.op not in busy_ops), None)
            if head is None:
                continue
            if self._large(head):
                if inflight:
                    continue
                pending.remove(head)
                try:
                    b = (self._launch_estimate(head, stream) if head.kind == "estimate"
                         else self._launch_apply(head.op, [head], stream))
                except _lib.PcError as e:
                    self._failed([head], e, pending, now())
                    continue
                inflight.append(b)
                busy_ops.add(head.op)
                inflight_bytes += b.nbytes
                peak = max(peak, self.resident_bytes + inflight_bytes)
                batches.append(1)
                continue
            r = self.ops[head.op]
            if head.kind == "estimate":
                nb = head.B * r.N * 4
                if self.resident_bytes + inflight_bytes + nb > self.budget:
                    if not inflight:
                        pending.remove(head)
                        head.result = "rejected: exceeds the HBM budget"
                        head.t_done = now()
                    continue
                pending.remove(head)
                try:
                    b = self._launch_estimate(head, stream)
                except _lib.PcError as e:
                    self._failed([head], e, pending, now())
                    continue
                inflight.append(b)
                busy_ops.add(head.op)
                inflight_bytes += b.nbytes
                peak = max(peak, self.resident_bytes + inflight_bytes)
                batches.append(1)
                continue
            take, vecs = [], 0
            for q in pending:
                if q.op != head.op or q.kind != "apply":
                    continue
                if take and (q.solo or head.solo):   # a retried request runs alone
                    break
                nb = 2 * (vecs + q.B) * r.N * 4
                if take and self._work(vecs + q.B, head.op) > self.large_work:
                    break
                if vecs + q.B > self.max_batch or self.resident_bytes + inflight_bytes + nb > self.budget:
                    break
                take.append(q)
                vecs += q.B
            if not take:
                if not inflight:   # it cannot fit even with nothing else admitted
                    pending.remove(head)
                    head.result = "rejected: exceeds the HBM budget"
                    head.t_done = now()
                # otherwise wait until in-flight batches free memory
                continue
            for q in take:
                pending.remove(q)
            try:
                b = self._launch_apply(head.op, take, stream)
            except _lib.PcError as e:
                self._failed(take, e, pending, now())
                continue
            inflight.append(b)
            busy_ops.add(head.op)
            inflight_bytes += b.nbytes
            peak = max(peak, self.resident_bytes + inflight_bytes)
            batches.append(len(take))
        t_end = now()
        out = summarize(reqs, t_end, batches, self.ops)
        out["peak_admitted_bytes"] = int(peak)
        out["launch_failures"] = self.launch_failures
        out["failed"] = sum(1 for q in reqs if q.failed)
        return out


def summarize(reqs, t_end, batches, ops):
    lat = {k: [] for k in ("apply", "estimate")}
    vec = 0
    pts = 0
    rejected = 0
    for q in reqs:
        if q.failed:
            continue
        if isinstance(q.result, str):
            rejected += 1
            continue
        lat[q.kind].append(q.t_done - q.arrival)
        vec += q.B
        pts += q.B * ops[q.op].N
    out = {"requests": len(reqs), "wall_s": t_end, "req_per_s": len(reqs) / t_end,
           "grid_points_per_s": pts / t_end, "vectors_per_s": vec / t_end,
           "mean_batch_requests": float(np.mean(batches)) if batches else 0.0, "rejected": rejected}
    for k, v in lat.items():
        if v:
            out[f"{k}_p50_ms"] = 1e3 * float(np.percentile(v, 50))
            out[f"{k}_p99_ms"] = 1e3 * float(np.percentile(v, 99))
    return out


def build_residents(workloads, q=8, dtype=_lib.PC_F32, max_batch=64, log=None):
    """Creates every operator, its input pool, probes and exact adjoint, and
    runs one apply of max_batch vectors and one estimate so that the work
    buffers reach their full size; work_bytes is then the operator's whole
    device footprint (pc_device_bytes)."""
    from workloads.blur_gpu import GpuBlurAdjoint
    res = []
    for w in workloads:
        op = _lib.PcOperator.from_workload(w, dtype=dtype)
        U = torch.from_numpy(w.vectors(POOL_ROWS, dtype=np.float32)).cuda()
        Z = torch.from_numpy(w.rademacher(q, w.vec_seed + 1000).astype(np.float32)).cuda()
        Y = GpuBlurAdjoint(w.op)(Z)
        tmp = torch.zeros((max_batch, w.N), dtype=torch.float32, device="cuda")
        op.apply_batch(tmp, tmp.clone())
        op.error_estimate(Z, Y)
        op.estimate_sums_device(Z, Y, torch.empty(op.n_leaves + 2, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        del tmp
        res.append(Resident(w.name, op, w.N, U, Z, Y, op.device_bytes()))
        if log:
            log({"op": w.name, "points": w.r, "device_gib": res[-1].work_bytes / 2**30})
    torch.cuda.synchronize()
    return res


def main(argv=None):
    import argparse
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from workloads import make_serving_ops

    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--budget-gib", type=float, default=0.0,
                    help="HBM budget (operators + in-flight); 0: resident footprint + 4 GiB")
    ap.add_argument("--ops", choices=["2d", "all"], default="all")
    ap.add_argument("--plain-requests", type=int, default=40)
    ap.add_argument("--loads", type=str, default="0.5,0.8,1.0")
    ap.add_argument("--large-mwork", type=float, default=128.0,
                    help="requests whose work (vectors x grid points, 3-D points x 10) exceeds this many "
                         "million run alone in the batched loop")
    args = ap.parse_args(argv)
    cmd = "python -m paper_1805_06018_amd.serve " + " ".join(sys.argv[1:] if argv is None else argv)
    print(json.dumps({"command": cmd.strip()}), flush=True)
    t0 = time.time()
    res = build_residents(make_serving_ops(with_3d=(args.ops == "all")),
                          log=lambda r: print(json.dumps(r), flush=True))
    resident = sum(r.work_bytes for r in res)
    budget = int(args.budget_gib * 2**30) if args.budget_gib > 0 else resident + (4 << 30)
    print(json.dumps({"ops": [r.name for r in res], "setup_s": time.time() - t0,
                      "resident_gib": resident / 2**30, "budget_gib": budget / 2**30}), flush=True)
    srv = Server(res, hbm_budget=budget, large_work=int(args.large_mwork * 2**20))
    # warm-up, then the saturated rate of one-request-at-a-time fused applies
    srv.run(poisson_requests(24, len(res), 0.0), mode="sequential")
    sat = srv.run(poisson_requests(args.requests // 4, len(res), 0.0), mode="sequential")
    rate = sat["req_per_s"]
    print(json.dumps({"mode": "sequential", "load": "saturated", **sat}), flush=True)
    satb = srv.run(poisson_requests(args.requests // 4, len(res), 0.0), mode="batched")
    print(json.dumps({"mode": "batched", "load": "saturated", **satb}), flush=True)
    if args.plain_requests > 0:
        pl = srv.run(poisson_requests(args.plain_requests, len(res), 0.0), mode="plain")
        print(json.dumps({"mode": "plain", "load": "saturated", **pl}), flush=True)
    for f in [float(x) for x in args.loads.split(",")]:
        for mode in ("sequential", "batched"):
            out = srv.run(poisson_requests(args.requests, len(res), f * rate), mode=mode)
            print(json.dumps({"mode": mode, "load": f, "rate_req_per_s": f * rate, **out}), flush=True)


if __name__ == "__main__":
    main()
