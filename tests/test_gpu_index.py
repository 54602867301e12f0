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
    # a row index repeated 5000 times, interleaved with others: the transpose of R
    # sorts that row's positions by an ordered pass over I (above the LDS sort's 4096)
    I3 = rng.integers(0, m, 9000).astype(np.int32)
    I3[rng.choice(9000, 5000, replace=False)] = 7
    spref_check(spx, A, I3, J)
    # few outputs from columns that gather thousands of entries (the wide-column path)
    spref_check(spx, A, rng.integers(0, m, 30).astype(np.int32), J)


def test_spref_wide_columns_from_threads(spx):
    """Wide columns (more than 4096 gathered entries, few outputs) are
    extracted on a second stream of the calling thread: three threads, each
    with its own stream, extract at once and repeatedly; every result equals
    the oracle's."""
    import threading
    import torch
    m = 20000
    rng = np.random.default_rng(9)
    rows = [np.arange(m), np.arange(0, m, 3)] + [np.sort(rng.choice(m, 5, replace=False)) for _ in range(50)]
    cols = np.concatenate([np.full(r.size, c, np.int64) for c, r in enumerate(rows)])
    rows = np.concatenate(rows)
    A = W.from_triples(rows, cols, np.arange(rows.size, dtype=np.int64), m, 52)
    dA = spx.from_host(A)
    J = np.concatenate([[0, 1], np.arange(2, 52), [1, 0]]).astype(np.int32)
    cases = [rng.integers(0, m, size=n).astype(np.int32) for n in (30, 200, 1500)]
    refs = [oracle.spref(A, I, J) for I in cases]
    got = [[] for _ in cases]
    errors = []

    def work(k):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for _ in range(4):
                    B = spx.spref(dA, cases[k], J)
                    st.synchronize()
                    got[k].append(B.to_host_csc())
        except Exception as e:  # reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=work, args=(k,)) for k in range(len(cases))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for k, ref in enumerate(refs):
        assert len(got[k]) == 4
        for B in got[k]:
            assert_same_csc(B, ref, exact_values=True, what=f"thread {k}")


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


def test_spasgn_insert_sizes_around_the_wave_limit(spx):
    # inserted rows per column of 1, 64, 65, 100 and 3000 exercise both the
    # one-wave and the workgroup variants of the modified-column kernels
    rng = np.random.default_rng(19)
    A = W.rmat(12, 8, seed=18, values="edge_id")
    I = rng.choice(A.m, 3500, replace=False).astype(np.int32)
    J = rng.choice(A.n, 6, replace=False).astype(np.int32)
    sizes = [1, 64, 65, 100, 3000, 0]
    rows = np.concatenate([np.sort(rng.choice(3500, k, replace=False)) for k in sizes])
    cols = np.repeat(np.arange(6), sizes)
    B = W.from_triples(rows, cols, (1 << 40) + np.arange(rows.size, dtype=np.int64), 3500, 6)
    spasgn_check(spx, A, I, J, B)
    extend_add_check(spx, A, I, J, B)
    Jr = np.concatenate([J, J[:3]]).astype(np.int32)  # repeated columns: landing entries add up
    extra = np.sort(rng.choice(3500, 70, replace=False))  # column 7 lands on J[1] too
    Br = W.from_triples(np.concatenate([rows, extra]), np.concatenate([cols, np.full(70, 7)]),
                        np.arange(rows.size + 70, dtype=np.int64), 3500, 9)
    spasgn_check(spx, A, I, Jr, Br)
    extend_add_check(spx, A, I, Jr, Br)


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
def rmat22_index():
    A = W.rmat(22, 16, seed=22, values="edge_id")
    I = W.index_vector(1 << 18, A.m, seed=221)
    J = W.index_vector(1 << 18, A.n, seed=222)
    Bp = W.erdos_renyi(1 << 18, 1 << 18, 4, seed=223, values="id40")
    return A, I, J, Bp


def test_rmat22_spref_full(spx, rmat22_index):
    A, I, J, _ = rmat22_index
    spref_check(spx, A, I, J)


def test_rmat22_spasgn_full(spx, rmat22_index):
    A, I, J, Bp = rmat22_index
    spasgn_check(spx, A, I, J, Bp)


# ---------------------------------------------------------------- extend-add
def with_values(M, kind, rng):
    """Copy of M with fresh values of ``kind`` (f32, f64, i64 or none)."""
    from types import SimpleNamespace
    nnz = M.ir.size
    num = {"f32": lambda: rng.random(nnz).astype(np.float32),
           "f64": lambda: rng.random(nnz),
           "i64": lambda: rng.integers(-2**40, 2**40, size=nnz),
           "none": lambda: None}[kind]()
    return SimpleNamespace(m=M.m, n=M.n, cp=M.cp, ir=M.ir, num=num)


def extend_add_check(spx, A, I, J, B, semiring="plus_times"):
    C = spx.extend_add(spx.from_host(A), I, J, spx.from_host(B), semiring=semiring).to_host_csc()
    ref = oracle.extend_add(A, I, J, B, semiring=semiring)
    # both sides add in B's storage order, so even float sums are bit-exact
    assert_same_csc(C, ref, exact_values=True, what=f"extend_add {semiring}")
    return C


@pytest.mark.parametrize("kind,semiring", [("f64", "plus_times"), ("f32", "plus_times"), ("i64", "plus_times"),
                                           ("f64", "min_plus"), ("f32", "select2nd"), ("i64", "min_plus"),
                                           ("none", "or_and"), ("none", "plus_times")])
def test_extend_add_small_with_repeats(spx, kind, semiring):
    rng = np.random.default_rng(61)
    for trial in range(4):
        A = with_values(W.rmat(10, 8, seed=40 + trial), kind, rng)
        lI, lJ = int(rng.integers(1, 400)), int(rng.integers(1, 400))
        I = rng.integers(0, A.m, size=lI).astype(np.int32)
        J = rng.integers(0, A.n, size=lJ).astype(np.int32)
        B = with_values(W.erdos_renyi(lI, lJ, min(5, lI), seed=50 + trial), kind, rng)
        extend_add_check(spx, A, I, J, B, semiring)


def test_extend_add_identity_is_sparse_sum_and_edges(spx):
    rng = np.random.default_rng(63)
    A = with_values(W.rmat(11, 8, seed=7), "f64", rng)
    B = with_values(W.rmat(11, 8, seed=8), "f64", rng)
    idx = np.arange(A.m, dtype=np.int32)
    extend_add_check(spx, A, idx, idx, B)
    # no indices, empty B, empty A
    E = W.from_triples([], [], np.empty(0), 0, 0)
    C = extend_add_check(spx, A, np.empty(0, np.int32), np.empty(0, np.int32), E)
    assert np.array_equal(C.ir, A.ir)
    J = rng.integers(0, A.n, size=50).astype(np.int32)
    extend_add_check(spx, A, np.empty(0, np.int32), J, W.from_triples([], [], np.empty(0), 0, 50))
    Z = W.from_triples([], [], np.empty(0), A.m, A.n)
    I = rng.integers(0, A.m, size=300).astype(np.int32)
    extend_add_check(spx, Z, I, J, with_values(W.erdos_renyi(300, 50, 7, seed=9), "f64", rng))


def test_extend_add_crowded_column(spx):
    # One column of C receives 4096 B entries (the LDS limit) from 8 repeated
    # column indices with many repeated rows: a 4096-key sort, 16 scan chunks
    # and long sums.
    rng = np.random.default_rng(65)
    A = with_values(W.erdos_renyi(5000, 3, 900, seed=11), "f64", rng)
    I = rng.integers(0, 5000, size=1024).astype(np.int32)
    J = np.array([1] * 8 + [0, 2], dtype=np.int32)
    rows = np.concatenate([np.arange(512)] * 8 + [np.arange(10), np.arange(20)])
    cols = np.concatenate([np.full(512, q) for q in range(8)] + [np.full(10, 8), np.full(20, 9)])
    B = W.from_triples(rows, cols, rng.random(rows.size), 1024, 10)
    C = extend_add_check(spx, A, I, J, B)
    assert np.diff(C.cp)[1] > 900
    # a 4097th entry moves the column to the global-memory path
    rows2 = np.concatenate([rows, [600]])
    cols2 = np.concatenate([cols, [0]])
    B2 = W.from_triples(rows2, cols2, rng.random(rows2.size), 1024, 10)
    C2 = extend_add_check(spx, A, I, J, B2)
    assert np.array_equal(C2.ir, extend_add_check(spx, A, I, J, B2).ir)


@pytest.mark.parametrize("kind,semiring", [("f64", "plus_times"), ("f32", "plus_times"), ("i64", "plus_times"),
                                           ("f64", "min_plus"), ("none", "or_and")])
def test_extend_add_huge_columns(spx, kind, semiring):
    # columns receiving 4097, 9000 and 70000 landing entries (global key
    # segments of 8192 and 131072 keys: several LDS tiles and global merge
    # stages) from repeated column indices and heavily repeated rows, beside
    # ordinary columns; sums in B's storage order, so bit-exact
    rng = np.random.default_rng(67)
    m = 200_000
    A = with_values(W.erdos_renyi(m, 6, 3000, seed=12), kind, rng)
    lI = 100_000
    I = rng.integers(0, m, size=lI).astype(np.int32)
    I[:5000] = I[5000:10000]  # many repeated rows
    J = np.array([1, 1, 3, 3, 3, 5, 0, 2], dtype=np.int32)
    sizes = [2049, 2048, 3000, 3000, 3000, 70_000, 17, 300]
    rows = np.concatenate([np.sort(rng.choice(lI, k, replace=False)) for k in sizes])
    cols = np.repeat(np.arange(len(sizes)), sizes)
    B = with_values(W.from_triples(rows, cols, np.zeros(rows.size), lI, len(sizes)), kind, rng)
    landing = np.bincount(J, weights=np.array(sizes), minlength=A.n)
    assert landing[1] == 4097 and landing[3] == 9000 and landing[5] == 70_000
    extend_add_check(spx, A, I, J, B, semiring)
    J2 = np.array([5, 5, 4, 4, 4, 5, 0, 2], dtype=np.int32)  # column 5 receives 2049 + 2048 + 70000
    extend_add_check(spx, A, I, J2, B, semiring)


def test_spasgn_huge_columns(spx):
    # columns inserting 4097, 9000 and 70000 rows (distinct rows, last
    # occurrence of repeated indices), beside small and ordinary ones, with
    # int64 and f64 values; the plan sorts the huge columns' keys in global
    # memory
    rng = np.random.default_rng(69)
    m = 300_000
    for vals in ("edge_id", "f64"):
        A = W.erdos_renyi(m, 8, 5000, seed=13, values=vals)
        lI = 120_000
        I = rng.choice(m, lI, replace=False).astype(np.int32)
        I[:1000] = I[1000:2000]  # repeated rows: the later occurrence wins
        J = np.array([0, 1, 2, 3, 3, 5, 6, 7], dtype=np.int32)  # J repeats column 3
        sizes = [4097, 9000, 70_000, 100, 5000, 64, 65, 0]
        rows = np.concatenate([np.sort(rng.choice(lI, k, replace=False)) for k in sizes])
        cols = np.repeat(np.arange(len(sizes)), sizes)
        num = (1 << 40) + np.arange(rows.size, dtype=np.int64)
        if vals == "f64":
            num = rng.random(rows.size)
        B = W.from_triples(rows, cols, num, lI, len(sizes))
        spasgn_check(spx, A, I, J, B)


@pytest.mark.parametrize("a_dcsc,b_dcsc", [(False, True), (True, False), (True, True)])
def test_spasgn_extend_add_dcsc_operands(spx, a_dcsc, b_dcsc):
    # hypersparse operands in DCSC: A with most columns empty, B with empty
    # columns, both as stage blocks would arrive; results equal the CSC ones
    rng = np.random.default_rng(71)
    A = W.column_block(W.rmat(14, 4, seed=72, values="edge_id"), 0, 1 << 14, 0, 1 << 14)
    lI, lJ = 3000, 2000
    I = rng.integers(0, A.m, size=lI).astype(np.int32)
    J = rng.integers(0, A.n, size=lJ).astype(np.int32)
    Bm = W.erdos_renyi(lI, lJ, 3, seed=73, values="id40")
    keep = np.repeat(rng.random(lJ) < 0.3, np.diff(Bm.cp))  # empty most of B's columns
    cols = np.repeat(np.arange(lJ), np.diff(Bm.cp))[keep]
    B = W.from_triples(Bm.ir[keep], cols, Bm.num[keep], lI, lJ)
    dA, dB = spx.from_host(A), spx.from_host(B)
    if a_dcsc:
        dA = spx.csc_to_dcsc(dA)
    if b_dcsc:
        dB = spx.csc_to_dcsc(dB)
    assert (not a_dcsc or dA.nzc < A.n) and (not b_dcsc or dB.nzc < B.n)
    got = spx.spasgn(dA, I, J, dB).to_host_csc()
    assert_same_csc(got, oracle.spasgn(A, I, J, B), exact_values=True, what="spasgn dcsc")
    got = spx.extend_add(dA, I, J, dB).to_host_csc()
    assert_same_csc(got, oracle.extend_add(A, I, J, B), exact_values=True, what="extend_add dcsc")


@pytest.mark.timeout(900)
def test_section52_assignment_rmat21_into_rmat22(spx, rmat22_index):
    """Section 5.2's assignment at one-GPU scale: A(I, J) = B with A the
    scale-22 R-MAT of the SpRef/SpAsgn workload, B an R-MAT of scale 21
    (edge factor 16, int64 ids 2^40 + position, hub columns far above 4096
    entries), I and J of length 2^21 with 10% repeated indices; bit-exact
    against the oracle, and extend-add of the same block."""
    A, _, _, _ = rmat22_index
    L = 1 << 21
    I = W.index_vector(L, A.m, seed=521)
    J = W.index_vector(L, A.n, seed=522)
    B = W.rmat(21, 16, seed=523, values="id40")
    assert np.diff(B.cp).max() > 4096
    spasgn_check(spx, A, I, J, B)
    extend_add_check(spx, A, I, J, B)


def test_extend_add_errors(spx):
    A = W.erdos_renyi(10, 10, 2, seed=1)
    B = W.erdos_renyi(1, 1, 1, seed=2)
    for I, J in (([10], [0]), ([0], [-1])):
        with pytest.raises(spx.SpxError) as e:
            spx.extend_add(spx.from_host(A), np.array(I, np.int32), np.array(J, np.int32), spx.from_host(B))
        assert e.value.code == spx.SPX_EINVAL
    with pytest.raises(spx.SpxError) as e:
        spx.extend_add(spx.from_host(A), np.array([0], np.int32), np.array([0], np.int32), spx.from_host(B),
                       semiring="or_and")
    assert e.value.code == spx.SPX_EUNSUPPORTED


def test_rmat22_extend_add_full(spx, rmat22_index):
    A, I, J, Bp = rmat22_index
    extend_add_check(spx, A, I, J, Bp)


@pytest.mark.parametrize("kind,semiring", [("f32", "plus_times"), ("f64", "min_plus"), ("i64", "plus_times"),
                                           ("none", "or_and")])
def test_register_path_limits(spx, kind, semiring):
    # A columns of 63, 64 and 65 entries and 63, 64 or 65 incoming B entries,
    # one column fed by two B columns (32 + 32) and one by two (10 + 55), with
    # repeated target rows: the register kernels take exactly the columns
    # whose A column and incoming entries fit a wave, the others go to the
    # LDS kernels, and both agree with the oracle bit for bit
    rng = np.random.default_rng(71)
    m = 400
    alens = [63, 64, 65, 64, 0, 64, 30, 5]
    arows = [np.sort(rng.choice(m, k, replace=False)) for k in alens]
    A = W.from_triples(np.concatenate(arows), np.repeat(np.arange(len(alens)), alens),
                       np.arange(sum(alens), dtype=np.int64), m, len(alens))
    A = with_values(A, kind, rng)
    I = rng.integers(0, m, size=200).astype(np.int32)  # repeated rows
    J = np.array([0, 1, 2, 3, 4, 5, 6, 5, 6], dtype=np.int32)
    blens = [64, 64, 63, 65, 64, 32, 10, 32, 55]
    brows = [np.sort(rng.choice(200, k, replace=False)) for k in blens]
    B = W.from_triples(np.concatenate(brows), np.repeat(np.arange(len(blens)), blens),
                       np.arange(sum(blens), dtype=np.int64), 200, len(blens))
    B = with_values(B, kind, rng)
    extend_add_check(spx, A, I, J, B, semiring)
    if kind != "none":
        spasgn_check(spx, A, I, J, B)
