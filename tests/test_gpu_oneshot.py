"""One-shot C-ABI entry points (outputs from the context's allocator) give
the same matrices as the plan/exec pairs, which the parity tests check
against the oracle."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _hip():
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    return hip


def fetch(ptr, count, dtype):
    out = np.empty(max(count, 0), dtype=dtype)
    if count > 0:
        assert _hip().hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2) == 0  # device to host
    return out


def host_of(d, num_dtype):
    """(cp, ir, num) of a CSC descriptor filled by a one-shot call."""
    cp = fetch(d.cp, d.n + 1, np.int64)
    nnz = int(cp[-1])
    ir = fetch(d.ir, nnz, np.int32)
    num = None if num_dtype is None else fetch(d.num, nnz, num_dtype)
    return cp, ir, num


def release(spx, *ptrs):
    for p in ptrs:
        if p:
            spx._free_cb(p, None)


def same(got, ref):
    cp, ir, num = got
    assert np.array_equal(cp, ref.cp.cpu().numpy()) and np.array_equal(ir, ref.ir.cpu().numpy())
    if ref.num is None:
        assert num is None
    else:
        r = ref.num.cpu().numpy()
        assert np.array_equal(num.view(np.uint8), r.view(np.uint8))


def test_one_shot_entry_points(spx):
    import torch
    lib = spx.load()
    A = W.rmat(12, 8, seed=61, values="edge_id")
    dA = spx.from_host(A)
    I = torch.from_numpy(W.index_vector(700, A.m, seed=1)).cuda()
    J = torch.from_numpy(W.index_vector(500, A.n, seed=2)).cuda()
    Bs = spx.from_host(W.erdos_renyi(700, 500, 3, seed=3, values="id40"))
    ctx = spx.make_ctx()
    a, b = dA.desc(), Bs.desc()
    p = ctypes.c_void_p

    out = spx.spx_mat()
    assert lib.spx_spgemm(ctypes.byref(ctx), ctypes.byref(a), ctypes.byref(a), 0, spx.CSC, ctypes.byref(out)) == 0
    torch.cuda.synchronize()
    same(host_of(out, np.int64), spx.spgemm(dA, dA))
    release(spx, out.cp, out.ir, out.num)

    out = spx.spx_mat()
    assert lib.spx_spref(ctypes.byref(ctx), ctypes.byref(a), p(I.data_ptr()), I.numel(), p(J.data_ptr()), J.numel(),
                         ctypes.byref(out)) == 0
    torch.cuda.synchronize()
    same(host_of(out, np.int64), spx.spref(dA, I, J))
    release(spx, out.cp, out.ir, out.num)

    out = spx.spx_mat()
    assert lib.spx_spasgn(ctypes.byref(ctx), ctypes.byref(a), p(I.data_ptr()), I.numel(), p(J.data_ptr()), J.numel(),
                          ctypes.byref(b), ctypes.byref(out)) == 0
    torch.cuda.synchronize()
    same(host_of(out, np.int64), spx.spasgn(dA, I, J, Bs))
    release(spx, out.cp, out.ir, out.num)

    out = spx.spx_mat()
    assert lib.spx_extend_add(ctypes.byref(ctx), ctypes.byref(a), p(I.data_ptr()), I.numel(), p(J.data_ptr()),
                              J.numel(), ctypes.byref(b), 0, ctypes.byref(out)) == 0
    torch.cuda.synchronize()
    same(host_of(out, np.int64), spx.extend_add(dA, I, J, Bs))
    release(spx, out.cp, out.ir, out.num)

    # batch: three products, pools at C[0]
    mats = [spx.from_host(W.erdos_renyi(300 + 50 * i, 300 + 50 * i, 4, seed=70 + i)) for i in range(3)]
    arr = spx.spx_mat * 3
    Ad = arr(*[m.desc() for m in mats])
    Cd = arr()
    assert lib.spx_batch_spgemm(ctypes.byref(ctx), 3, Ad, Ad, 0, None, Cd) == 0
    torch.cuda.synchronize()
    for i, m in enumerate(mats):
        same(host_of(Cd[i], np.float64), spx.spgemm(m, m))
    release(spx, Cd[0].cp, Cd[0].ir, Cd[0].num)

    # errors leave nothing allocated and report the code
    bad = torch.tensor([A.m], dtype=torch.int32, device="cuda")
    out = spx.spx_mat()
    rc = lib.spx_spref(ctypes.byref(ctx), ctypes.byref(a), p(bad.data_ptr()), 1, p(J.data_ptr()), 1, ctypes.byref(out))
    assert rc == spx.SPX_EINVAL and not out.cp
