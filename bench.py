"""Benchmark of the product-convolution apply on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                [--workload blur1024|blur3d] [--dtype f32|f64] [--plan auto|cost|smallest]
                [--no-graph] [--no-autotune]

A step is one pc_apply_batch of the whole hot path (gather with weights,
forward FFT, spectral product, inverse FFT, deterministic scatter-add) with
inputs resident in HBM.  Default workload: the 1024^2 spatially varying blur
with ~600 adaptive sample points and 64 right-hand sides in FP32.  blur3d:
the 128^3 blur with a 9^3 sample grid and 16 right-hand sides.  Prints one
JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VALU = 157.3e12      # MI355X FP32 vector FLOP/s
PEAK_FP64_VALU = 78.6e12       # MI355X FP64 vector FLOP/s
PEAK_HBM = 8.0e12              # MI355X HBM3E B/s

# HBM bytes per convolution launch from the committed counter runs (FETCH_SIZE
# x 2.0 + WRITE_SIZE x 1.0, calibrated on a plain copy), one line per plan,
# launch form (split: the large items' launch and the small items' two-per-CU
# launch of one vector chunk; single: one launch for all items) and launch
# size; valid only while the kernel and planner sources hash to the recorded
# value.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "conv_kernel_blur1024_b64.md")
TRAFFIC_SOURCES = ["paper_1805_06018_amd/csrc/" + f
                   for f in ("pc_kernels.hip", "pc_phases.h", "pc_fft.h", "pc_internal.h", "pc_plan.cpp")]


def measured_traffic(vectors_per_launch, plan_flags=0, launch="split"):
    import hashlib
    import re
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    for m in re.finditer(r"traffic plan_flags=(\d+) launch=(\w+) vectors_per_launch=(\d+) bytes_per_launch=([0-9.eE+]+) "
                         r"sources_sha256=([0-9a-f]{64})", text):
        if ((int(m.group(1)), m.group(2), int(m.group(3))) == (plan_flags, launch, vectors_per_launch)
                and m.group(5) == h.hexdigest()):
            return float(m.group(4))
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--workload", choices=["blur1024", "blur3d"], default="blur1024")
    ap.add_argument("--dtype", choices=["f32", "f64"], default="f32")
    ap.add_argument("--plan", choices=["auto", "cost", "smallest"], default="auto",
                    help="FFT lengths of the 2-D plan: the autotuner's pick of the two (auto), the "
                         "planner's cost model (cost) or the smallest supported lengths (smallest)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default schedule instead of the autotuner's choice")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip timing replays of the apply recorded into a HIP graph (stream capture)")
    ap.add_argument("--cpu-vectors", type=int, default=8,
                    help="vectors of the 1024^2 batch the oracle's CPU baseline applies")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain device copy of the 256 MiB input (a known-size "
                         "reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the library has no multi-GPU mode", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1805_06018_amd import _lib
    from workloads import make_config

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    three_d = args.workload == "blur3d"
    w = make_config(2 if three_d else 1)
    B = w.batch
    f64 = args.dtype == "f64"
    ndt = np.float64 if f64 else np.float32
    esz = 8 if f64 else 4
    plan_flags = _lib.PC_PLAN_SMALLEST_FFT if args.plan == "smallest" else 0
    t0 = time.time()
    op = _lib.PcOperator.from_workload(w, dtype=_lib.PC_F64 if f64 else _lib.PC_F32, flags=plan_flags)
    t_create = time.time() - t0
    st = op.stats()
    U = torch.from_numpy(w.vectors(B, dtype=ndt)).to(dev)
    OUT = torch.empty_like(U)
    print(f"# workload {w.name}: N={w.N} r={w.r} B={B} items={st['n_items']} create={t_create:.2f}s",
          file=sys.stderr, flush=True)

    schedule = {"autotuned": False, "plan_flags": plan_flags}
    if not args.no_autotune:
        from paper_1805_06018_amd import tune
        t_tune = time.time()
        # reductions stay on the launch stream: the convolution kernel then
        # runs alone and its per-launch time is its own
        if three_d or args.plan != "auto":
            res = tune.autotune(op, U, OUT, allow_overlap=False)
            res["plan_flags"], res["plans"] = plan_flags, []
        else:
            op.close()
            op, res = tune.autotune_plan(
                lambda fl: _lib.PcOperator.from_workload(w, dtype=_lib.PC_F64 if f64 else _lib.PC_F32, flags=fl),
                U, OUT, allow_overlap=False)
            st = op.stats()
            plan_flags = res["plan_flags"]
        schedule = {"autotuned": True, "plan_flags": res["plan_flags"], "plans": res["plans"],
                    "chosen": tune.names(res["best"]), "best_ms": res["best_ms"],
                    "default_ms": res["default_ms"], "candidates": len(res["table"]),
                    "confirmed": [dict(tune.names(c["setting"]), ms=c["ms"]) for c in res.get("confirm", [])],
                    "tune_s": time.time() - t_tune}
        print(f"# autotune: {schedule}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        op.apply_batch(U, OUT)
    torch.cuda.synchronize()

    # timed region (kernel events recorded on the same stream)
    op.read_profile()
    op.set_profiling(True)
    # one event between consecutive applies: per-apply latency percentiles
    # and the total come from the same stream timeline
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(args.steps):
        op.apply_batch(U, OUT)
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms_total = ev[0].elapsed_time(ev[-1])
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    op.set_profiling(False)
    prof = op.read_profile()
    ms_step = ms_total / args.steps
    value = w.N * B / (ms_step * 1e-3)

    # dominant kernel: the convolution launches (2-D: one fused launch per
    # vector chunk; 3-D: the plane / axis-0 / plane kernels of each item group)
    conv_avg_s = prof["conv_ms"] / max(prof["conv_launches"], 1) * 1e-3
    achieved = st["alg_flops_per_rhs"] * prof["conv_vectors"] / (prof["conv_ms"] * 1e-3)
    peak = PEAK_FP64_VALU if f64 else PEAK_FP32_VALU
    alg_bytes_step = 2.0 * esz * w.N * B + esz * st["kernel_elems"]

    graph = None
    if not args.no_graph:
        ref_out = OUT.clone()
        g = op.graph(U, OUT)
        for _ in range(3):
            g.replay()
        gev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        gev[0].record()
        for i in range(args.steps):
            g.replay()
            gev[i + 1].record()
        torch.cuda.synchronize()
        glat = np.array([gev[i].elapsed_time(gev[i + 1]) for i in range(args.steps)])
        gms = gev[0].elapsed_time(gev[-1]) / args.steps
        graph = {"ms_per_step": gms, "value": w.N * B / (gms * 1e-3),
                 "p50_ms": float(np.percentile(glat, 50)), "p99_ms": float(np.percentile(glat, 99)),
                 "replays": int(args.steps), "bitwise_equal_to_eager": bool(torch.equal(OUT, ref_out))}
        del g

    if args.copy_probe:
        probe = torch.empty_like(U)
        probe.copy_(U)
        torch.cuda.synchronize()
        print(f"# copy probe: {U.numel() * 4} bytes read and written", file=sys.stderr, flush=True)

    # plain per-patch / per-vector apply (same kernels, one launch each)
    plain_ms = None
    if args.plain_steps > 0:
        OUTp = torch.empty_like(U)
        op.apply_batch_plain(U, OUTp)
        torch.cuda.synchronize()
        t1 = time.time()
        for _ in range(args.plain_steps):
            op.apply_batch_plain(U, OUTp)
        torch.cuda.synchronize()
        plain_ms = (time.time() - t1) * 1e3 / args.plain_steps
        same = bool(torch.equal(OUTp, OUT))
    else:
        same = None

    # context for the HBM readings: the rate of a plain device-to-device copy
    # of 1 GiB (four times the 256 MB last-level cache), read plus write bytes
    cp_src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    cp_dst = torch.empty_like(cp_src)
    for _ in range(3):
        cp_dst.copy_(cp_src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(20):
        cp_dst.copy_(cp_src)
    c1.record()
    torch.cuda.synchronize()
    copy_tbps = 2 * cp_src.numel() * 4 * 20 / (c0.elapsed_time(c1) * 1e-3) / 1e12
    del cp_src, cp_dst

    # per-launch HBM bytes: the committed counter runs cover the FP32 2-D
    # launch sizes of every candidate schedule; a batch that the chunk does
    # not divide ends with a shorter launch, so the bytes are averaged over
    # the launches of one apply (as the launch time is)
    traffic = None
    chosen = schedule.get("chosen", {}) if schedule["autotuned"] else {}
    direct, persistent = chosen.get("direct", 0), chosen.get("persistent", 0)
    if not three_d and not f64 and not direct and not persistent and not chosen.get("item_major", 0):
        per_vec = st["slot_elems_fwd"] * esz
        cap = max(1, (2 << 30) // max(per_vec, 1))          # the library's 2 GiB staging cap
        chunk = schedule.get("chosen", {}).get("chunk", 0) if schedule["autotuned"] else 0
        chunk = min(cap, chunk if chunk > 0 else B)
        sizes = [chunk] * (B // chunk) + ([B % chunk] if B % chunk else [])
        if len(sizes) == prof["conv_launches"] / args.steps:
            launch = "split" if chosen.get("split", 1) else "single"
            per = [measured_traffic(v, plan_flags, launch) for v in sizes]
            if all(x is not None for x in per):
                traffic = sum(per) / len(per)

    if three_d:
        wl = f"blur3d_128x128x128_tensor9_r{w.r}_b{B}"
    else:
        wl = f"blur2d_1024x1024_quadtree_r{w.r}_b{B}"
    rec = {
        "metric": "PC apply grid-points/s (FP32, 1e-5 rel.L2) vs plain apply; HBM %; p50/p99 lat",
        "value": value,
        "unit": "grid-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": wl, "grid": list(w.shape), "r": w.r, "batch": B, "items": st["n_items"],
                   "schedule": schedule},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic},
        "kernels": {"conv_ms_per_launch": conv_avg_s * 1e3, "conv_launches_per_step": prof["conv_launches"] / args.steps,
                    "conv_ms_per_step": prof["conv_ms"] / args.steps,
                    "reduce_ms_per_step": prof["reduce_ms"] / args.steps,
                    "alg_flops_per_vector": st["alg_flops_per_rhs"]},
        "hbm_alg_frac": alg_bytes_step / (ms_step * 1e-3) / PEAK_HBM,
        "hbm_copy_TBps": copy_tbps,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "applies": int(lat.size)},
        "graph": graph,
        "plain": {"ms_per_step": plain_ms, "value": (w.N * B / (plain_ms * 1e-3)) if plain_ms else None,
                  "bitwise_equal_to_fused": same},
    }

    cpu_model = None
    try:
        with open("/proc/cpuinfo") as fh:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    if not args.no_cpu_baseline and not three_d:
        from oracle import OracleOperator
        ora = OracleOperator.from_workload(w)
        nv = max(1, min(args.cpu_vectors, B))
        rows = [int(j * B / nv) for j in range(nv)]          # spread over the batch
        Uh = U[rows].cpu().numpy().astype(np.float64)
        got = OUT[rows].cpu().numpy().astype(np.float64)
        t2 = time.time()
        refs = [ora.apply(Uh[i], backend="c") for i in range(nv)]
        t_cpu = time.time() - t2
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        errs = [float(np.linalg.norm(got[i] - refs[i]) / np.linalg.norm(refs[i])) for i in range(nv)]
        rec["cpu_baseline"] = {"value": w.N * nv / t_cpu, "unit": "grid-points/s", "cores": cores, "kind": "oracle",
                               "cpu_model": cpu_model,
                               "sample": f"{nv} of {B} vectors (rows {rows}), full 1024^2 outputs, FP64 direct "
                                         "summation (C core, OpenMP); the whole batch would take "
                                         f"{t_cpu * B / nv:.0f} s (extrapolated)"}
        rec["rel_l2_vs_oracle"] = {"max": max(errs), "median": float(np.median(errs)), "vectors": rows}
    elif not args.no_cpu_baseline:
        # a full FP64 oracle apply of one 3-D vector is ~3e12 multiply-adds:
        # time the oracle's direct summation at a bounded set of outputs
        from oracle import OracleOperator
        ora = OracleOperator.from_workload(w)
        u0 = U[0].cpu().numpy().astype(np.float64)
        n = w.shape[0]
        ys = np.random.default_rng(17).integers(0, n, (2000, 3))
        t2 = time.time()
        ref = ora.apply_at(u0, ys)
        t_cpu = time.time() - t2
        flat = (ys[:, 0] * n + ys[:, 1]) * n + ys[:, 2]
        got = OUT[0].cpu().numpy().astype(np.float64)[flat]
        rec["cpu_baseline"] = {"value": len(ys) / t_cpu, "unit": "grid-points/s", "cores": 1, "kind": "oracle",
                               "cpu_model": cpu_model,
                               "sample": f"2000 random output points of 1 of {B} vectors, FP64 direct "
                                         "summation (NumPy, one thread)"}
        rec["rel_l2_vs_oracle_vec0_sampled"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
