"""GPU tests of the continuous-batching request loop."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible HIP device")
    from paper_1805_06018_amd import serve
    from workloads import make_serving_ops
    # three 2-D operators and the smallest 3-D one (64^3, 27 points)
    res = serve.build_residents(make_serving_ops(sizes=(256, 512, 768), with_3d=True, sizes3=(64,)))
    return serve, res


def _alone(serve, r, q):
    """The request's result computed alone, from its own rows of the pool."""
    a = serve.input_rows(q)
    out = torch.empty((q.B, r.N), dtype=torch.float32, device="cuda")
    r.pc.apply_batch(r.U[a:a + q.B], out)
    torch.cuda.synchronize()
    return out


def test_results_same_alone_and_in_the_mix(served):
    """Every request reads its own rows of its operator's pool; merged into
    batches with other requests (2-D and 3-D operators, four streams) each
    result equals the request's alone result bit for bit, and a stream-ordered
    estimate equals the synchronous pc_error_estimate."""
    serve, res = served
    srv = serve.Server(res, hbm_budget=24 << 30)
    reqs = serve.poisson_requests(60, len(res), 0.0, seed=5)
    out = srv.run(reqs, mode="batched")
    assert out["mean_batch_requests"] > 1.0          # requests were merged
    assert len({serve.input_rows(q) for q in reqs}) > 10
    assert {res[q.op].pc.d for q in reqs} == {2, 3}
    for q in reqs:
        r = res[q.op]
        if q.kind == "apply":
            assert torch.equal(_alone(serve, r, q), q.result), q.rid
        else:
            eta, ea, er = r.pc.error_estimate(r.Z[:q.B], r.Y[:q.B])
            assert np.array_equal(eta, q.result[0]) and ea == q.result[1] and er == q.result[2]


def test_hbm_budget_admission(served):
    serve, res = served
    resident = sum(r.work_bytes for r in res)
    with pytest.raises(ValueError):
        serve.Server(res, hbm_budget=resident // 2)
    # room for about eight vectors of the largest grid in flight
    room = 2 * 8 * max(r.N for r in res) * 4
    srv = serve.Server(res, hbm_budget=resident + room)
    reqs = serve.poisson_requests(40, len(res), 0.0, seed=6, max_b=8)
    out = srv.run(reqs, mode="batched")
    assert all(q.t_done is not None for q in reqs)
    assert out["peak_admitted_bytes"] <= resident + room
    for q in reqs:
        if q.kind == "apply":
            assert torch.equal(_alone(serve, res[q.op], q), q.result)


def test_failed_launch_is_isolated(served):
    """Two injected launch failures on one operator (host-side test hook, no
    kernel runs for them): the batch that hits the first is retried request
    by request, the request whose retry hits the second is reported failed,
    every other request completes with its alone result, and the operator
    keeps working."""
    serve, res = served
    srv = serve.Server(res, hbm_budget=24 << 30)
    reqs = serve.poisson_requests(40, len(res), 0.0, seed=8)
    target = next(q.op for q in reqs if q.kind == "apply")
    res[target].pc.debug_fail_launches(1, 2)
    try:
        out = srv.run(reqs, mode="batched")
    finally:
        res[target].pc.debug_fail_launches(0, 0)
    assert out["launch_failures"] == 2 and out["failed"] == 1
    failed = [q for q in reqs if q.failed]
    assert failed[0].op == target and failed[0].result.startswith("failed:")
    for q in reqs:
        if q.failed:
            continue
        r = res[q.op]
        if q.kind == "apply":
            assert torch.equal(_alone(serve, r, q), q.result), q.rid
        else:
            eta, ea, er = r.pc.error_estimate(r.Z[:q.B], r.Y[:q.B])
            assert np.array_equal(eta, q.result[0]) and ea == q.result[1] and er == q.result[2]
    # the operator still applies correctly after the injected failures
    q = failed[0]
    r = res[q.op]
    a = torch.empty((q.B, r.N), dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    r.pc.apply_batch(r.U[:q.B], a)
    r.pc.apply_batch_plain(r.U[:q.B], b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
