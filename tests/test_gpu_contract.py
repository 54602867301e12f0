"""GPU parity of graph contraction / restriction C = S_r A S_c^T (one SpGEMM
pass over A with mapped row ids) against the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import assert_same_csc

pytestmark = pytest.mark.gpu


def contract_check(spx, A, row_agg, mc, col_agg, nc, semiring="plus_times", exact=False, a_dcsc=False,
                   out_fmt=0):
    import torch
    dA = spx.from_host(A)
    if a_dcsc:
        dA = spx.csc_to_dcsc(dA)
    ra = None if row_agg is None else torch.from_numpy(np.asarray(row_agg, np.int32)).cuda()
    ca = None if col_agg is None else torch.from_numpy(np.asarray(col_agg, np.int32)).cuda()
    plan = spx.ContractPlan(dA, ra, mc, ca, nc, semiring, out_fmt)
    C = plan.execute()
    info = plan.info()
    plan.close()
    ref = oracle.contract(A, row_agg, mc, col_agg, nc, semiring)
    assert_same_csc(C.to_host_csc(), ref, exact_values=exact, what=f"contract {semiring}")
    assert info["mults"] == A.ir.size and info["nnz"] == ref.cp[-1]
    return C


@pytest.mark.parametrize("order", [1, 2, 3, 4, 8])
def test_restriction_orders(spx, order):
    A = W.rmat(13, 8, seed=80 + order)
    agg = np.arange(A.n) // order
    nc = -(-A.n // order)
    contract_check(spx, A, agg, nc, agg, nc, "plus_times", out_fmt=order % 2)
    Ai = W.rmat(12, 8, seed=90 + order, values="edge_id")
    agg = np.arange(Ai.n) // order
    nc = -(-Ai.n // order)
    contract_check(spx, Ai, agg, nc, agg, nc, "plus_times", exact=True, a_dcsc=True)
    contract_check(spx, Ai, agg, nc, agg, nc, "min_plus", exact=True)
    contract_check(spx, Ai, agg, nc, agg, nc, "select1st", exact=True)
    contract_check(spx, Ai, agg, nc, agg, nc, "or_and", exact=True)


def test_one_sided_and_unsorted_column_maps(spx):
    rng = np.random.default_rng(83)
    A = W.rmat(12, 8, seed=84, values="edge_id")
    ra = np.sort(rng.integers(0, 700, size=A.m))
    ca = rng.integers(0, 500, size=A.n)
    contract_check(spx, A, ra, 700, None, 0, exact=True)   # S A
    contract_check(spx, A, None, 0, ca, 500, exact=True)   # A S^T, vertices in any order
    contract_check(spx, A, ra, 700, ca, 500, exact=True)
    contract_check(spx, A, None, 0, None, 0, exact=True)   # identity on both sides
    Af = W.rmat(12, 8, seed=85, values="f32")
    contract_check(spx, Af, ra, 700, ca, 500)


def test_contraction_matches_two_explicit_products(spx):
    # S (A S^T) with materialized S and intermediate, on the GPU's own SpGEMM
    A = W.rmat(14, 8, seed=86, values="edge_id")
    agg = np.arange(A.n) // 4
    nc = A.n // 4
    S = W.from_triples(agg, np.arange(A.n), np.ones(A.n, np.int64), nc, A.n)
    St = W.from_triples(np.arange(A.n), agg, np.ones(A.n, np.int64), A.n, nc)
    dS, dSt, dA = spx.from_host(S), spx.from_host(St), spx.from_host(A)
    two = spx.spgemm(dS, spx.spgemm(dA, dSt)).to_host_csc()
    C = contract_check(spx, A, agg, nc, agg, nc, exact=True)
    assert_same_csc(C.to_host_csc(), two, exact_values=True, what="fused vs two products")


def test_restriction_order8_rmat18(spx):
    A = W.rmat(18, 8, seed=87)
    agg = np.arange(A.n) // 8
    contract_check(spx, A, agg, A.n // 8, agg, A.n // 8)


def test_unsorted_row_maps(spx):
    # any row aggregation: the plan sorts A's columns by mapped row (one wave
    # per column up to 64 entries, a workgroup up to 4096) and exec gathers
    # A's values through the permutation
    rng = np.random.default_rng(89)
    A = W.rmat(12, 8, seed=90, values="edge_id")
    agg = rng.integers(0, 600, size=A.n)
    contract_check(spx, A, agg, 600, agg, 600, exact=True)            # graph contraction, random aggregates
    contract_check(spx, A, agg, 600, None, 0, exact=True, a_dcsc=True)
    contract_check(spx, A, np.arange(A.m)[::-1], A.m, None, 0, exact=True)  # a reversal
    Af = W.rmat(12, 8, seed=91, values="f64")
    contract_check(spx, Af, agg, 600, agg, 600, "min_plus", exact=True)
    contract_check(spx, Af, agg, 600, agg, 600, out_fmt=1)
    # columns of 100 to 3000 entries take the workgroup sort
    D = W.erdos_renyi(5000, 40, 3000, seed=92, values="edge_id")
    ragg = rng.integers(0, 70, size=D.m)
    contract_check(spx, D, ragg, 70, np.arange(40) // 4, 10, exact=True)


def test_unsorted_row_map_hub_columns(spx):
    # columns above 4096 entries (hubs) take one global sort each under an
    # unsorted row map; the others the group and workgroup sorts
    rng = np.random.default_rng(96)
    L = W.erdos_renyi(9000, 5, 6000, seed=2, values="edge_id")
    contract_check(spx, L, np.arange(9000)[::-1], 9000, None, 0, exact=True)  # a reversal
    agg = rng.integers(0, 300, size=9000)
    contract_check(spx, L, agg, 300, np.array([0, 1, 0, 2, 1]), 3, exact=True)
    H = W.rmat(16, 16, seed=97, values="f64")  # an R-MAT hub beside short columns
    assert np.diff(H.cp).max() > 4096
    hagg = rng.integers(0, 2000, size=H.m)
    contract_check(spx, H, hagg, 2000, hagg, 2000, "min_plus", exact=True)
    contract_check(spx, H, hagg, 2000, None, 0, a_dcsc=True)


def test_contraction_errors(spx):
    import torch
    A = spx.from_host(W.erdos_renyi(20, 20, 3, seed=1))
    big = torch.full((20,), 7, dtype=torch.int32, device="cuda")
    with pytest.raises(spx.SpxError) as e:
        spx.contract(A, None, 0, big, 5)
    assert e.value.code == spx.SPX_EINVAL


def test_contraction_int32_pointers_and_empty(spx):
    import torch
    A = W.rmat(11, 8, seed=88, values="edge_id")
    agg = np.arange(A.n) // 4
    dA = spx.from_host(A, ptr_dtype=torch.int32)
    ga = torch.from_numpy(agg.astype(np.int32)).cuda()
    C = spx.contract(dA, ga, A.n // 4, ga, A.n // 4).to_host_csc()
    ref = oracle.contract(A, agg, A.n // 4, agg, A.n // 4)
    assert_same_csc(C, ref, exact_values=True, what="int32 pointers")
    E = W.from_triples([], [], np.empty(0, np.int64), 64, 64)
    e = np.arange(64) // 8
    contract_check(spx, E, e, 8, e, 8, exact=True)
    contract_check(spx, E, None, 0, None, 0, exact=True)


def test_unsorted_row_map_wide_ids(spx):
    # mapped rows above 2^26 leave too few bits for a 32-bit (row, position)
    # key in the 64-lane sort, which then takes 64-bit keys
    rng = np.random.default_rng(95)
    m = (1 << 26) + 4096
    A = W.erdos_renyi(m, 64, 40, seed=94, values="edge_id")
    agg = rng.integers(0, m, size=m, dtype=np.int64).astype(np.int32)
    agg[A.ir[:5]] = m - 1  # the largest id, and repeated rows
    contract_check(spx, A, agg, m, None, 0, exact=True)
    contract_check(spx, A, agg, m, np.arange(64) // 2, 32, exact=True)
