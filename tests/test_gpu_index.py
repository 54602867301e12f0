"""GPU parity of SpRef, SpAsgn and the format conversions (bit-exact)."""
import numpy as np
import pytest

import oracle
import workloads as W
from conftest import read_golden
from helpers import assert_same_csc

pytestmark = pytest.mark.gpu


def spref_check(spx, A, I, J, a_dcsc=False):
    dA = spx.from_host(A)
    if a_dcsc:
        dA = spx.csc_to_dcsc(dA)
    B = spx.spref(dA, I, J).to_host_csc()
    ref = oracle.spref(A, I, J)
    assert_same_csc(B, ref, exact_values=True, what="spref")
    return B


def test_spref_small_with_repeats(spx):
    rng = np.random.default_rng(1)
    for trial in range(5):
        A = W.rmat(10, 8, seed=trial, values="edge_id")
        I = rng.integers(0, A.m, size=int(rng.integers(1, 3000))).astype(np.int32)
        J = rng.integers(0, A.n, size=int(rng.integers(1, 3000))).astype(np.int32)
        spref_check(spx, A, I, J, a_dcsc=bool(trial % 2))


def test_spref_long_columns_and_heavy_repeats(spx):
    # a dense column of A and an I with many repeats exercise the medium and
    # long-column paths
    m = 20000
    rows = np.concatenate([np.arange(m), np.arange(0, m, 3)])
    cols = np.concatenate([np.zeros(m, np.int64), np.ones(len(range(0, m, 3)), np.int64)])
    A = W.from_triples(rows, cols, np.arange(rows.size, dtype=np.int64), m, 2)
    rng = np.random.default_rng(2)
    I = rng.integers(0, m, size=9000).astype(np.int32)
    J = np.array([0, 1, 0, 1, 1], dtype=np.int32)
    spref_check(spx, A, I, J)
    I2 = np.concatenate([np.full(200, 5, np.int32), rng.integers(0, m, 100).astype(np.int32)])
    spref_check(spx, A, I2, J)


def test_spref_permutation_roundtrip(spx):
    A = W.rmat(14, 8, seed=3, values="f64")
    p = W.random_permutation(A.n, seed=4)
    pinv = np.empty_like(p)
    pinv[p] = np.arange(p.size, dtype=np.int32)
    dA = spx.from_host(A)
    B = spx.spref(dA, p, p)
    C = spx.spref(B, pinv, pinv).to_host_csc()
    assert_same_csc(C, A, exact_values=True, what="permutation round trip")


def test_fig_scatter_rows(spx):
    g = read_golden("scatter_example.txt")
    I = np.array([int(x) - 1 for x in g["I"]], dtype=np.int32)
    A = W.erdos_renyi(9, 9, 4, seed=5)
    spref_check(spx, A, I, np.arange(9, dtype=np.int32))


def test_spref_errors(spx):
    A = W.erdos_renyi(10, 10, 2, seed=1)
    dA = spx.from_host(A)
    with pytest.raises(spx.SpxError) as e:
        spx.spref(dA, np.array([0, 10], np.int32), np.array([0], np.int32))
    assert e.value.code == spx.SPX_EINVAL
    B = spx.spref(dA, np.zeros(0, np.int32), np.array([1, 2], np.int32))
    assert B.nnz == 0 and B.m == 0 and B.n == 2


def spasgn_check(spx, A, I, J, B):
    C = spx.spasgn(spx.from_host(A), I, J, spx.from_host(B)).to_host_csc()
    ref = oracle.spasgn(A, I, J, B)
    assert_same_csc(C, ref, exact_values=True, what="spasgn")
    return C


def test_spasgn_small_with_repeats(spx):
    rng = np.random.default_rng(9)
    for trial in range(5):
        A = W.rmat(10, 8, seed=10 + trial, values="edge_id")
        lI, lJ = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        I = rng.integers(0, A.m, size=lI).astype(np.int32)
        J = rng.integers(0, A.n, size=lJ).astype(np.int32)
        B = W.erdos_renyi(lI, lJ, min(4, lI), seed=20 + trial, values="id40")
        spasgn_check(spx, A, I, J, B)


def test_spasgn_roundtrip(spx):
    A = W.rmat(12, 8, seed=31, values="edge_id")
    I = W.index_vector(500, A.m, seed=1, repeat_frac=0.0)
    J = W.index_vector(400, A.n, seed=2, repeat_frac=0.0)
    dA = spx.from_host(A)
    sub = spx.spref(dA, I, J)
    C = spx.spasgn(dA, I, J, sub).to_host_csc()
    assert_same_csc(C, A, exact_values=True, what="spasgn(A, I, J, A(I,J))")


def test_formats(spx):
    g = read_golden("fig_csc.txt")
    cp = np.array([int(x) - 1 for x in g["CP"]], dtype=np.int64)
    ir = np.array([int(x) - 1 for x in g["IR"]], dtype=np.int32)
    num = np.array([float(x) for x in g["NUM"]])
    from types import SimpleNamespace
    A = SimpleNamespace(m=9, n=9, cp=cp, ir=ir, num=num)
    dA = spx.from_host(A)
    D = spx.csc_to_dcsc(dA)
    assert D.jc.cpu().tolist() == [int(x) for x in g["JC"]]
    assert D.cp.cpu().tolist() == [int(x) for x in g["DCP"]]
    back = spx.dcsc_to_csc(D)
    assert np.array_equal(back.cp.cpu().numpy(), cp)
    R = W.rmat(12, 4, seed=3)
    dR = spx.from_host(R)
    assert spx.check(dR) and spx.check(spx.csc_to_dcsc(dR))
    jc, dcp = oracle.csc_to_dcsc(R.n, R.cp)
    DR = spx.csc_to_dcsc(dR)
    assert np.array_equal(DR.jc.cpu().numpy(), jc) and np.array_equal(DR.cp.cpu().numpy(), dcp)
    bad = spx.from_host(R)
    bad.ir[1] = bad.ir[0]  # a duplicate row
    assert not spx.check(bad)


@pytest.fixture(scope="module")
def config3():
    A = W.rmat(22, 16, seed=22, values="edge_id")
    I = W.index_vector(1 << 18, A.m, seed=221)
    J = W.index_vector(1 << 18, A.n, seed=222)
    Bp = W.erdos_renyi(1 << 18, 1 << 18, 4, seed=223, values="id40")
    return A, I, J, Bp


def test_config3_spref_full(spx, config3):
    A, I, J, _ = config3
    spref_check(spx, A, I, J)


def test_config3_spasgn_full(spx, config3):
    A, I, J, Bp = config3
    spasgn_check(spx, A, I, J, Bp)
