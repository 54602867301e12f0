"""The entry point that allocates nothing (spx_csc_to_dcsc_noalloc), called
through the C ABI: its output equals spx_csc_to_dcsc's on two calls in a row,
the second with a smaller input, and it never calls the allocator."""
import ctypes
import gc

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _reference(spx, A):
    return spx.csc_to_dcsc(A)


def _noalloc(spx, lib, A, nzc, counter):
    import torch

    @spx.ALLOC_FN
    def alloc(nbytes, user):
        counter[0] += 1
        return None  # any call would fail the conversion

    @spx.FREE_FN
    def free(ptr, user):
        counter[1] += 1

    ctx = spx.spx_ctx(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), alloc, free, None, 0, 0)
    out = spx.SpMat(A.m, A.n, torch.full((nzc + 1,), -7, dtype=A.cp.dtype, device="cuda"), A.ir, A.num,
                    torch.full((nzc,), -7, dtype=torch.int32, device="cuda"), spx.DCSC)
    nzc_dev = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    a, d = A.desc(), out.desc()
    # the cyclic collector stays off across the call, so that no tensor freed by a
    # collection of earlier tests' garbage moves the allocator's count meanwhile
    gc.collect()
    gc.disable()
    try:
        before = torch.cuda.memory_allocated()
        rc = lib.spx_csc_to_dcsc_noalloc(ctypes.byref(ctx), ctypes.byref(a), ctypes.byref(d),
                                         ctypes.c_void_p(nzc_dev.data_ptr()))
        after = torch.cuda.memory_allocated()
    finally:
        gc.enable()
    assert rc == spx.SPX_OK, lib.spx_last_error().decode()
    assert after == before
    torch.cuda.synchronize()
    return out, int(nzc_dev.item()), d


@pytest.mark.parametrize("ptr", ["int64", "int32"])
def test_noalloc_matches_the_allocating_entry_point(spx, ptr):
    import torch
    lib = spx.load()
    pd = getattr(torch, ptr)
    counter = [0, 0]
    # first a large input (many scan blocks, empty columns), then a smaller one:
    # the second call must not see anything the first left in the scratch
    for M in (W.rmat(20, 4, seed=81), W.rmat(12, 2, seed=82)):
        A = spx.from_host(M, ptr_dtype=pd)
        ref = _reference(spx, A)
        nzc = ref.nzc
        assert nzc < M.n  # the inputs have empty columns
        out, nzc_seen, d = _noalloc(spx, lib, A, nzc, counter)
        assert nzc_seen == nzc
        assert d.fmt == spx.DCSC and d.nnz == M.nnz
        assert torch.equal(out.jc, ref.jc) and torch.equal(out.cp, ref.cp)
        # and against the definition of DCSC (Section 3.2) on the host
        full = np.asarray(M.cp, dtype=np.int64)
        nonempty = np.nonzero(np.diff(full) > 0)[0]
        assert np.array_equal(out.jc.cpu().numpy(), nonempty)
        assert np.array_equal(out.cp.cpu().numpy().astype(np.int64), np.append(full[nonempty], full[-1]))
    assert counter == [0, 0]


def test_noalloc_rejects_too_many_columns(spx):
    import torch
    lib = spx.load()
    n = (1 << 22) + 1
    cp = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    A = spx.SpMat(4, n, cp, torch.zeros(0, dtype=torch.int32, device="cuda"), None)
    ctx = spx.make_ctx()
    out = spx.SpMat(4, n, torch.zeros(1, dtype=torch.int64, device="cuda"), A.ir, None,
                    torch.zeros(0, dtype=torch.int32, device="cuda"), spx.DCSC)
    a, d = A.desc(), out.desc()
    rc = lib.spx_csc_to_dcsc_noalloc(ctypes.byref(ctx), ctypes.byref(a), ctypes.byref(d), None)
    assert rc == spx.SPX_EINVAL
    assert b"at most" in lib.spx_last_error()
