"""Autotuner of the apply schedule.

The library's schedule knobs (pc_set_tuning) change how a batched apply is
cut into launches, never what it computes: colour launches adding into the
outputs or staged boxes and a reduction (PC_TUNE_DIRECT, 1-D/2-D
operators), staged convolutions as one workgroup per unit (whole items
per XCD or item-major, PC_TUNE_XCD_ORDER; small items two workgroups per
CU, PC_TUNE_SPLIT) or as a fixed grid taking units from queues
(PC_TUNE_PERSISTENT), vectors per
convolution launch (PC_TUNE_CHUNK), reduction
overlapped on a second stream (PC_TUNE_OVERLAP, staged 1-D/2-D) and the
plane-spectrum scratch per item group (PC_TUNE_SCRATCH, 3-D operators).
autotune() times each candidate setting on the caller's own vectors, times
the fastest few again in alternating rounds, checks that every schedule
gives the bitwise same result, applies the one with the least median and
returns both tables.  Results can
be cached in a JSON file keyed by the operator's shape, size and batch.
"""
import json
import os

import torch

from . import _lib

_MiB = 1 << 20


def candidates(op, B, allow_overlap=True):
    """Candidate settings {key: value} for an operator and batch size; the
    first one is the library default.  allow_overlap=False keeps every
    reduction on the caller's stream (each kernel then runs alone, which is
    what per-kernel timing needs)."""
    default = {_lib.PC_TUNE_CHUNK: 0, _lib.PC_TUNE_OVERLAP: 0, _lib.PC_TUNE_SCRATCH: 0}
    if op.d < 3:
        default[_lib.PC_TUNE_DIRECT] = 0
        default[_lib.PC_TUNE_STREAMS] = 4
        default[_lib.PC_TUNE_PERSISTENT] = 0
        default[_lib.PC_TUNE_XCD_ORDER] = 0
        default[_lib.PC_TUNE_SPLIT] = 1
    out = [dict(default)]
    # powers of two and the sizes in between (for B = 64: 8, 10, 12, 16, 20,
    # 22, 24, 28, 32, 64); a batch that a chunk does not divide ends with a
    # shorter launch
    chunks = sorted({c for c in (B * k // 64 for k in (8, 10, 12, 16, 20, 22, 24, 28, 32, 64)) if 1 <= c <= B})
    if op.d == 3:
        for scratch in (0, 128 * _MiB, 256 * _MiB, 1024 * _MiB):
            for chunk in [0] + [c for c in chunks if c >= 2]:
                c = dict(default)
                c[_lib.PC_TUNE_CHUNK] = chunk
                c[_lib.PC_TUNE_SCRATCH] = scratch
                if c != default:
                    out.append(c)
    else:
        for overlap in ((0, 1) if allow_overlap else (0,)):   # staged boxes and a reduction
            # one workgroup per unit (whole items per XCD with the small
            # items two per CU or not, or item-major), or unit queues
            for persistent, xcd, split in ((0, 0, 1), (0, 0, 0), (0, 1, 0), (1, 0, 0)):
                for chunk in [0] + chunks:
                    c = dict(default)
                    c[_lib.PC_TUNE_CHUNK] = chunk
                    c[_lib.PC_TUNE_OVERLAP] = overlap
                    c[_lib.PC_TUNE_PERSISTENT] = persistent
                    c[_lib.PC_TUNE_XCD_ORDER] = xcd
                    c[_lib.PC_TUNE_SPLIT] = split
                    if c != default:
                        out.append(c)
        for streams in (4, 2, 1):               # colour launches
            for chunk in [0] + [x for x in chunks if x <= max(1, B // 2)]:
                c = dict(default)
                c[_lib.PC_TUNE_DIRECT] = 1
                c[_lib.PC_TUNE_STREAMS] = streams
                c[_lib.PC_TUNE_CHUNK] = chunk
                out.append(c)
    return out


def _key(op, B, adjoint):
    st = op.stats()
    return f"d{op.d}_N{op.N}_items{st['n_items']}_dt{int(op.torch_dtype == torch.float64)}_B{B}_adj{int(adjoint)}"


def _apply_settings(op, setting):
    for k, v in setting.items():
        op.set_tuning(int(k), int(v))


def _time(fn, U, OUT, reps):
    """Durations (ms) of reps back-to-back calls, each bracketed by events."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for i in range(reps):
        fn(U, OUT)
        ev[i + 1].record()
    torch.cuda.synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]


def autotune(op, U, OUT, adjoint=False, reps=3, cache_path=None, allow_overlap=True, confirm=4, confirm_reps=8,
             confirm_rounds=2):
    """Times every candidate schedule for applying op (adjoint: its adjoint)
    to the batch U into OUT (the least of reps calls each), then times the
    confirm fastest again in confirm_rounds alternating rounds of
    confirm_reps calls, leaves the one with the least median set on op and
    returns {"best": {key: value}, "best_ms": its median, "default_ms": t0,
    "table": [first pass], "confirm": [second pass]}.  A single pass of a
    few calls lets run-to-run noise choose among schedules within a percent
    of each other; the second pass is what decides.  Raises if two
    schedules disagree bitwise."""
    B = 1 if U.dim() == 1 else U.shape[0]
    key = _key(op, B, adjoint) + ("" if allow_overlap else "_noovl")
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            best = {int(k): v for k, v in cache[key]["best"].items()}
            _apply_settings(op, best)
            return cache[key]
    fn = op.apply_adjoint_batch if adjoint else op.apply_batch
    ref = None
    table = []
    cands = candidates(op, B, allow_overlap)
    for setting in cands:
        _apply_settings(op, setting)
        fn(U, OUT)   # sizes the work buffers for this schedule
        torch.cuda.synchronize()
        if ref is None:
            ref = OUT.clone()
        elif not torch.equal(OUT, ref):
            raise RuntimeError(f"schedule {setting} changed the result")
        ms = min(_time(fn, U, OUT, reps))
        table.append({"setting": {str(k): v for k, v in setting.items()}, "ms": ms})
    top = sorted(range(len(table)), key=lambda i: table[i]["ms"])[:max(1, confirm)]
    runs = {i: [] for i in top}
    for _ in range(max(1, confirm_rounds)):
        for i in top:
            _apply_settings(op, cands[i])
            fn(U, OUT)
            runs[i] += _time(fn, U, OUT, max(1, confirm_reps))
            if not torch.equal(OUT, ref):
                raise RuntimeError(f"schedule {cands[i]} changed the result")
    med = {i: sorted(runs[i])[len(runs[i]) // 2] for i in top}
    bi = min(top, key=lambda i: med[i])
    res = {"best": table[bi]["setting"], "best_ms": med[bi], "default_ms": table[0]["ms"], "table": table,
           "confirm": [{"setting": table[i]["setting"], "ms": med[i]} for i in top]}
    _apply_settings(op, cands[bi])
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as fh:
                cache = json.load(fh)
        cache[key] = res
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return res


def autotune_plan(make_op, U, OUT, plan_flags=(0, None), adjoint=False, reps=3, allow_overlap=True):
    """Plan-level choices, made at pc_create: make_op(flags) builds the
    operator with the given plan flags.  For each candidate (0: the cost
    model's FFT lengths; PC_PLAN_SMALLEST_FFT: the smallest supported
    lengths) the schedule autotuner runs and the best time is kept.  The
    plans differ in FFT lengths, so their results agree to rounding (each is
    checked against the other within 1e-5 relative L2 per vector), not
    bitwise.  Returns (op, {"plan_flags": f, "plans": [...], **autotune result})
    with the fastest operator kept and the others closed."""
    cands = [0, _lib.PC_PLAN_SMALLEST_FFT] if plan_flags == (0, None) else list(plan_flags)
    best = None
    plans = []
    ref = None
    for f in cands:
        op = make_op(f)
        res = autotune(op, U, OUT, adjoint=adjoint, reps=reps, allow_overlap=allow_overlap)
        torch.cuda.synchronize()
        out = OUT.double()
        if ref is None:
            ref = out.clone()
        else:
            rel = ((out - ref).norm(dim=-1) / ref.norm(dim=-1).clamp_min(1e-300)).max().item()
            if rel > 1e-5:
                raise RuntimeError(f"plan flags {f} changed the result by {rel:.3e}")
        st = op.stats()
        plans.append({"plan_flags": int(f), "items": int(st["n_items"]), "fft_points": int(st["sum_fft_points"]),
                      "best_ms": res["best_ms"]})
        if best is None or res["best_ms"] < best[1]["best_ms"]:
            if best is not None:
                best[0].close()
            best = (op, dict(res, plan_flags=int(f)))
        else:
            op.close()
    op, res = best
    _apply_settings(op, {int(k): v for k, v in res["best"].items()})
    res["plans"] = plans
    return op, res


def names(setting):
    """Readable form of a setting: {"direct": .., "streams": .., "persistent": .., "chunk": .., "overlap": ..,
    "scratch_MiB": ..}."""
    s = {int(k): v for k, v in setting.items()}
    return {"direct": s.get(_lib.PC_TUNE_DIRECT, 0), "streams": s.get(_lib.PC_TUNE_STREAMS, 1),
            "persistent": s.get(_lib.PC_TUNE_PERSISTENT, 0), "item_major": s.get(_lib.PC_TUNE_XCD_ORDER, 0),
            "split": s.get(_lib.PC_TUNE_SPLIT, 1),
            "chunk": s.get(_lib.PC_TUNE_CHUNK, 0),
            "overlap": s.get(_lib.PC_TUNE_OVERLAP, 0), "scratch_MiB": s.get(_lib.PC_TUNE_SCRATCH, 0) // _MiB}
