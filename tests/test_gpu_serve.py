"""Served requests: each result is the same alone and in the mix; admission
never exceeds the budget; an oversize request is rejected, not stuck."""
import numpy as np
import pytest

from helpers import assert_same_csc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def store_and_pool(spx):
    from paper_1109_3739_amd import serve
    pool = serve.make_pool(12, seed=5, scales=range(8, 12), degrees=range(2, 9))
    store = serve.ResidentStore()
    scales = {}
    for key, (s, M) in enumerate(pool):
        store.add(key, M)
        scales[key] = s
    store.host = {key: M for key, (s, M) in enumerate(pool)}  # host copies for the oracle
    return store, scales


def oracle_result(store, r):
    """The oracle's answer to a served request: the FP32 product of the two
    resident matrices, or the extraction A(I, J) of the int64 edge ids."""
    import oracle
    M = store.host[r.a]
    if r.kind == "spgemm":
        return oracle.spgemm_csc(M, store.host[r.b])
    E = M.with_values(np.arange(M.nnz, dtype=np.int64))
    return oracle.spref(E, r.I.cpu().numpy(), r.J.cpu().numpy())


def run(spx, store, scales, mode, n=60, qps=1e6, budget=64 << 30, seed=1):
    from paper_1109_3739_amd import serve
    reqs = serve.make_requests(store, scales, n, qps, seed=seed)
    srv = serve.Server(store, mode=mode, budget_bytes=budget)
    srv.run(reqs, keep_results=True)
    return reqs, srv


def test_results_same_alone_and_in_the_mix(spx, store_and_pool):
    store, scales = store_and_pool
    reqs, srv = run(spx, store, scales, "batched")
    assert srv.rounds < len(reqs)  # requests were really batched
    for r in reqs:
        assert r.status == "ok"
        if r.kind == "spgemm":
            alone = spx.spgemm(store.f32[r.a], store.f32[r.b])
        else:
            alone = spx.spref(store.i64[r.a], r.I, r.J)
        got = r.result.to_host_csc()
        assert_same_csc(got, oracle_result(store, r), exact_values=(r.kind == "spref"),
                        what=f"request {r.rid} ({r.kind}) against the oracle")
        assert_same_csc(got, alone.to_host_csc(), exact_values=(r.kind == "spref"),
                        what=f"request {r.rid} ({r.kind}) alone and in the mix")


def test_plain_mode_matches(spx, store_and_pool):
    store, scales = store_and_pool
    a, _ = run(spx, store, scales, "plain", n=20, seed=2)
    b, _ = run(spx, store, scales, "batched", n=20, seed=2)
    for x, y in zip(a, b):
        assert_same_csc(x.result.to_host_csc(), y.result.to_host_csc(), exact_values=(x.kind == "spref"))


def test_continuous_admission_overlaps_lanes(spx, store_and_pool):
    """At a load the lanes cannot absorb one request at a time, requests that
    arrive while earlier batches run are admitted onto free lanes before
    those batches finish, batches of different lanes overlap, and every
    result still equals the oracle's."""
    store, scales = store_and_pool
    reqs, srv = run(spx, store, scales, "batched", n=120, qps=4000, seed=4)
    assert all(r.status == "ok" for r in reqs)
    assert srv.max_busy_lanes >= 2 and srv.rounds > 1
    # some request started while a request admitted earlier was still running
    by_start = sorted(reqs, key=lambda r: r.start)
    assert any(b.start < a.done and b.start > a.start for a, b in zip(by_start, by_start[1:]))
    for r in reqs:
        assert_same_csc(r.result.to_host_csc(), oracle_result(store, r), exact_values=(r.kind == "spref"),
                        what=f"request {r.rid} ({r.kind})")


def test_per_request_completion(spx, store_and_pool):
    """Extractions of one batch complete, and release their share, one by
    one: their completion times are not all the batch's end."""
    store, scales = store_and_pool
    reqs, srv = run(spx, store, scales, "batched", n=40, qps=1e6, seed=5)
    refs = [r for r in reqs if r.kind == "spref"]
    assert len(refs) > 2 and len({r.done for r in refs}) > 1


def test_drawn_memory_stays_within_budget(spx, store_and_pool):
    """The device memory actually drawn while serving (outputs and every
    plan's scratch, through the caching allocator) never exceeds the budget,
    with admission binding: the budget holds only a few requests at once."""
    import torch
    from paper_1109_3739_amd import serve
    store, scales = store_and_pool
    reqs = serve.make_requests(store, scales, 60, 1e6, seed=6)
    ests = sorted(serve.estimate_bytes(store, r) for r in reqs)
    budget = max(ests[-1], sum(ests) // 8)
    assert sum(ests) > 4 * budget  # admission must hold requests back
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    srv = serve.Server(store, mode="batched", budget_bytes=budget)
    srv.run(reqs)
    torch.cuda.synchronize()
    assert all(r.status == "ok" for r in reqs)
    assert srv.max_used <= budget
    assert torch.cuda.max_memory_allocated() - base <= budget


def test_admission_budget_and_rejection(spx, store_and_pool):
    from paper_1109_3739_amd import serve
    store, scales = store_and_pool
    reqs = serve.make_requests(store, scales, 40, 1e6, seed=3)
    ests = sorted(serve.estimate_bytes(store, r) for r in reqs)
    budget = ests[len(ests) // 2]  # the larger half cannot be admitted at all
    srv = serve.Server(store, mode="batched", budget_bytes=budget)
    srv.run(reqs)
    assert srv.max_used <= budget
    assert all(r.status in ("ok", "rejected") for r in reqs)
    assert any(r.status == "rejected" for r in reqs) and any(r.status == "ok" for r in reqs)
    for r in reqs:
        assert (r.status == "rejected") == (r.est_bytes > budget)
