"""GPU parity of the Sparse SUMMA stage sum C = sum_k A_k B_k (Algorithm 2,
one processor's stages) against the oracle's stage loop."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import assert_same_csc

pytestmark = pytest.mark.gpu


def device(spx, M, dcsc):
    d = spx.from_host(M)
    return spx.csc_to_dcsc(d) if dcsc else d


def stage_sum_check(spx, As, Bs, semiring="plus_times", exact=False, fmts=None, out_fmt=0):
    fmts = fmts or [(False, False)] * len(As)
    dAs = [device(spx, A, fa) for A, (fa, _) in zip(As, fmts)]
    dBs = [device(spx, B, fb) for B, (_, fb) in zip(Bs, fmts)]
    plan = spx.StageSumPlan(dAs, dBs, semiring, out_fmt)
    C = plan.execute()
    info = plan.info()
    plan.close()
    ref = oracle.summa_stages(As, Bs, semiring)
    assert_same_csc(C.to_host_csc(), ref, exact_values=exact, what=f"stage sum {semiring}")
    mults = sum(int(np.diff(A.cp)[B.ir].sum()) for A, B in zip(As, Bs))
    assert info["mults"] == mults and info["nnz"] == ref.cp[-1]
    return C


def blocks_of(A, nb):
    b = A.n // nb
    return [[W.column_block(A, i * b, (i + 1) * b, k * b, (k + 1) * b) for k in range(nb)] for i in range(nb)]


@pytest.mark.parametrize("semiring,values,exact", [
    ("plus_times", "f64", False), ("plus_times", "f32", False), ("plus_times", "i64", True),
    ("min_plus", "f64", True), ("select2nd", "i64", True), ("or_and", "none", True),
])
def test_stage_sum_random_stages(spx, semiring, values, exact):
    rng = np.random.default_rng(71)
    for trial in range(3):
        K = (1, 3, 8)[trial]
        m, n = int(rng.integers(200, 3000)), int(rng.integers(100, 2000))
        bs = [int(x) for x in rng.integers(0, 1500, size=K)]
        bs[-1] = max(bs[-1], 1)
        As, Bs = [], []
        for k, b in enumerate(bs):
            da = min(6, m)
            A = W.erdos_renyi(m, b, da, seed=100 * trial + k, values="f64")
            B = W.erdos_renyi(b, n, min(int(rng.integers(1, 20)), b), seed=100 * trial + 50 + k, values="f64") \
                if b > 0 else W.from_triples([], [], np.empty(0), 0, n)
            for X in (A, B):
                if values == "f32":
                    X.num = X.num.astype(np.float32)
                elif values == "i64":
                    X.num = rng.integers(-1000, 1000, size=X.ir.size).astype(np.int64)
                elif values == "none":
                    X.num = None
            As.append(A)
            Bs.append(B)
        fmts = [(bool(rng.integers(2)), bool(rng.integers(2))) for _ in range(K)]
        stage_sum_check(spx, As, Bs, semiring, exact, fmts, out_fmt=trial % 2)


def test_stage_sum_of_inner_split_is_the_product(spx):
    # sum over an 8-way split of the inner dimension = the whole product
    A = W.rmat(14, 8, seed=72)
    A.num = np.random.default_rng(3).integers(-50, 50, size=A.nnz).astype(np.int64)
    b = A.n // 8
    As = [W.column_block(A, 0, A.m, k * b, (k + 1) * b) for k in range(8)]
    Bs = [W.column_block(A, k * b, (k + 1) * b, 0, A.n) for k in range(8)]
    C = stage_sum_check(spx, As, Bs, "plus_times", exact=True, fmts=[(True, True)] * 8)
    whole = spx.spgemm(spx.from_host(A), spx.from_host(A)).to_host_csc()
    assert_same_csc(C.to_host_csc(), whole, exact_values=True, what="split vs whole")


def test_stage_sum_8x8_summa_block_rmat20(spx):
    """C_00 of 8x8 Sparse SUMMA on R-MAT scale 20: the 8 stage products
    A_0k * A_k0 of 2^17 x 2^17 hypersparse blocks in DCSC, summed."""
    A = W.rmat(20, 8, seed=20)
    bl = blocks_of(A, 8)
    As = [bl[0][k] for k in range(8)]
    Bs = [bl[k][0] for k in range(8)]
    stage_sum_check(spx, As, Bs, "plus_times", False, [(True, True)] * 8, out_fmt=1)


def test_stage_sum_errors(spx):
    A = spx.from_host(W.erdos_renyi(10, 4, 2, seed=1))
    B = spx.from_host(W.erdos_renyi(5, 6, 2, seed=2))
    with pytest.raises(spx.SpxError) as e:
        spx.spgemm_sum([A], [B])
    assert e.value.code == spx.SPX_EINVAL
    with pytest.raises(ValueError):
        spx.spgemm_sum([], [])


def test_stage_sum_int32_pointers_and_empty_stages(spx):
    import torch
    A = W.rmat(12, 8, seed=74, values="edge_id")
    b = A.n // 4
    As = [W.column_block(A, 0, A.m, k * b, (k + 1) * b) for k in range(4)]
    Bs = [W.column_block(A, k * b, (k + 1) * b, 0, A.n) for k in range(4)]
    dAs = [spx.from_host(X, ptr_dtype=torch.int32) for X in As]
    dBs = [spx.from_host(X, ptr_dtype=torch.int32) for X in Bs]
    C = spx.spgemm_sum(dAs, dBs).to_host_csc()
    assert_same_csc(C, oracle.summa_stages(As, Bs), exact_values=True, what="int32 pointers")
    Z = [W.from_triples([], [], np.empty(0, np.int64), 50, 30), W.from_triples([], [], np.empty(0, np.int64), 50, 0)]
    Y = [W.from_triples([], [], np.empty(0, np.int64), 30, 20), W.from_triples([], [], np.empty(0, np.int64), 0, 20)]
    C = stage_sum_check(spx, Z, Y, "plus_times", exact=True)
    assert C.nnz == 0
