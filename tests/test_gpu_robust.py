"""Error paths and determinism on the GPU.

* SPX_FAULT=alloc:N makes the N-th device allocation of the library fail:
  every entry point must then return SPX_ENOMEM, release what it had drawn
  (the caching allocator's live bytes return to where they were) and leave
  the library usable; the server must finish every request (ok or failed)
  without hanging.
* Integer and (min,+) results are bit-identical from run to run.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import assert_same_csc

pytestmark = pytest.mark.gpu


@pytest.fixture
def fault():
    """Sets SPX_FAULT for the duration of a test and clears it afterwards."""
    def set_spec(spec):
        if spec is None:
            os.environ.pop("SPX_FAULT", None)
        else:
            os.environ["SPX_FAULT"] = spec
    yield set_spec
    os.environ.pop("SPX_FAULT", None)


def each_fault_point(spx, fault, call, limit=400):
    """Runs `call` with the N-th allocation failing for N = 1, 2, ... until
    three runs in a row succeed (N past the call's allocations; an
    allocation with a fallback, such as the stored row bitmaps, succeeds on
    its own).  Every failed run must raise SPX_ENOMEM and leave the live
    device memory as it was.  Returns (allocations of a run, its output,
    number of failed runs)."""
    import torch
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    streak, failures, out = 0, 0, None
    for n in range(1, limit):
        fault(f"alloc:{n}")
        out = None  # the previous run's output is not live memory of this one
        try:
            out = call()
        except spx.SpxError as e:
            assert e.code == spx.SPX_ENOMEM, f"allocation {n}: {e}"
            assert "SPX_FAULT" in str(e)
            torch.cuda.synchronize()
            assert torch.cuda.memory_allocated() == base, f"allocation {n}: memory not released"
            streak, failures = 0, failures + 1
            continue
        streak += 1
        if streak == 3:
            fault(None)
            assert failures > 0
            return n - 3, out, failures
    raise AssertionError("the call kept allocating")


def test_alloc_faults_spgemm_plan_and_one_shot(spx, fault):
    A = W.rmat(16, 8, seed=81)  # large enough for scratch buffers of their own beside the shared blocks
    dA = spx.from_host(A)
    ref = oracle.spgemm_csc(A, A)

    def plan_exec():
        p = spx.GemmPlan(dA, dA)
        try:
            return p.execute()
        finally:
            p.close()

    nalloc, C, _ = each_fault_point(spx, fault, plan_exec)
    assert nalloc >= 3
    assert_same_csc(C.to_host_csc(), ref, what="after the faults")
    # the C one-shot entry point: its outputs come from ctx->alloc as well
    import ctypes
    lib = spx.load()
    ctx = spx.make_ctx()
    a = dA.desc()

    def one_shot():
        out = spx.spx_mat()
        rc = lib.spx_spgemm(ctypes.byref(ctx), ctypes.byref(a), ctypes.byref(a), 0, 0, ctypes.byref(out))
        if rc != spx.SPX_OK:
            raise spx.SpxError(rc, lib.spx_last_error().decode())
        for ptr in (out.cp, out.ir, out.num):
            spx._free_cb(ptr, None)
        return out

    n2, out, _ = each_fault_point(spx, fault, one_shot)
    assert n2 == nalloc + 3  # plus the three output buffers


def test_alloc_faults_index_batch_and_contraction(spx, fault):
    import torch
    E = W.rmat(12, 8, seed=82, values="edge_id")
    # device index vectors, so that the calls allocate nothing outside the library
    I = torch.from_numpy(W.index_vector(700, E.m, seed=83)).cuda()
    J = torch.from_numpy(W.index_vector(600, E.n, seed=84)).cuda()
    Bn = W.erdos_renyi(700, 600, 3, seed=85, values="id40")
    dE, dB = spx.from_host(E), spx.from_host(Bn)
    each_fault_point(spx, fault, lambda: spx.spref(dE, I, J))
    each_fault_point(spx, fault, lambda: spx.spasgn(dE, I, J, dB))
    each_fault_point(spx, fault, lambda: spx.extend_add(dE, I, J, dB))
    L = [spx.from_host(W.laplacian7(n)) for n in (4, 6, 8)]
    P = [spx.from_host(W.aggregation(n)) for n in (4, 6, 8)]
    each_fault_point(spx, fault, lambda: spx.batch_spgemm(L, P))
    A = spx.from_host(W.rmat(11, 8, seed=86))
    agg = spx.restriction_map(A.n, 4)
    each_fault_point(spx, fault, lambda: spx.contract(A, agg, A.n // 4, agg, A.n // 4))
    _, S, _ = each_fault_point(spx, fault, lambda: spx.spgemm_sum([A, A], [A, A]))
    assert S.nnz > 0


def test_server_survives_alloc_faults(spx, fault):
    """From some allocation on, every allocation fails: each mode still
    finishes every request, as failed or ok, and serves normally again once
    the fault is cleared."""
    from paper_1109_3739_amd import serve
    pool = serve.make_pool(8, seed=87, scales=range(8, 12), degrees=range(2, 6))
    store = serve.ResidentStore()
    scales = {}
    for key, (s, M) in enumerate(pool):
        store.add(key, M)
        scales[key] = s
    for mode in ("batched", "plain"):
        reqs = serve.make_requests(store, scales, 40, 20000, seed=88)
        fault("alloc:30+")
        serve.Server(store, mode=mode).run(reqs)
        fault(None)
        assert all(r.status in ("ok", "failed") for r in reqs), mode
        assert any(r.status == "failed" for r in reqs), mode
        assert all(r.done >= r.arrival for r in reqs)
        again = serve.make_requests(store, scales, 20, 20000, seed=89)
        serve.Server(store, mode=mode).run(again)
        assert all(r.status == "ok" for r in again), mode


def test_results_are_bitwise_repeatable(spx):
    """int64 (+,x) and f64 (min,+) products, 20 runs in one process, on every
    path (R-MAT: tiny, hash and bitmap columns, multi-part columns): each run
    equals the first bit for bit; stops at the first difference."""
    A = W.rmat(15, 8, seed=90, values="f64")
    Ai = A.with_values(np.random.default_rng(91).integers(-3, 4, size=A.nnz).astype(np.int64))
    for M, sr in ((Ai, "plus_times"), (A, "min_plus")):
        dM = spx.from_host(M)
        first = spx.spgemm(dM, dM, sr).to_host_csc()
        assert_same_csc(first, oracle.spgemm_csc(M, M, sr), exact_values=True, what=sr)
        for run in range(19):
            got = spx.spgemm(dM, dM, sr).to_host_csc()
            assert np.array_equal(got.cp, first.cp) and np.array_equal(got.ir, first.ir), f"{sr} run {run + 2}"
            assert np.array_equal(got.num.view(np.uint64), first.num.view(np.uint64)), f"{sr} run {run + 2}"
