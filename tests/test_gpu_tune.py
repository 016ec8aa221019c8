"""Autotuner of the apply schedule (GPU): every candidate schedule gives the
bitwise same result, the fastest is left set, and the cache round-trips."""
import json
import os
import sys

import numpy as np
import pytest
import torch

from oracle import OracleOperator
from tests.libhelpers import small_cases, small_cases_3d, relerr, TOL

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["hanging33", "cube24"])
def test_autotune_keeps_result_and_sets_fastest(name, tmp_path):
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible HIP device")
    from paper_1805_06018_amd import _lib, tune
    w = dict(small_cases() + small_cases_3d())[name]
    print(f"case={name} autotune", flush=True)
    op = _lib.PcOperator.from_workload(w, dtype=_lib.PC_F32)
    Un = np.random.default_rng(9).standard_normal((8, w.N)).astype(np.float32)
    U = torch.from_numpy(Un).cuda()
    OUT = torch.empty_like(U)
    cache = str(tmp_path / "tune.json")
    res = tune.autotune(op, U, OUT, reps=2, cache_path=cache)
    assert len(res["table"]) == len(tune.candidates(op, 8))
    # the second pass re-times the fastest of the first and keeps its winner
    first = sorted(r["ms"] for r in res["table"])[:len(res["confirm"])]
    assert sorted(r["ms"] for r in res["table"] if r["setting"] in [c["setting"] for c in res["confirm"]]) == first
    assert res["best_ms"] == min(c["ms"] for c in res["confirm"])
    assert res["best"] in [c["setting"] for c in res["confirm"] if c["ms"] == res["best_ms"]]
    # the chosen schedule is the one now set: same result as the oracle
    OUT2 = torch.empty_like(U)
    op.apply_batch(U, OUT2)
    torch.cuda.synchronize()
    assert torch.equal(OUT2, OUT)
    ref = OracleOperator.from_workload(w).apply_batch(Un.astype(np.float64))
    assert relerr(OUT2.cpu().numpy(), ref).max() <= TOL[_lib.PC_F32]
    # second call: read from the cache, nothing re-timed
    with open(cache) as fh:
        assert len(json.load(fh)) == 1
    res2 = tune.autotune(op, U, OUT, reps=2, cache_path=cache)
    assert res2["best"] == res["best"] and res2["table"] == res["table"]
    op.close()
