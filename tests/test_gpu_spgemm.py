"""GPU parity of SpGEMM against the CPU oracle (element by element)."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import assert_same_csc

pytestmark = pytest.mark.gpu


def gemm(spx, A, B, semiring="plus_times", out_fmt=0, tuning=None, a_dcsc=False, b_dcsc=False, ptr32=False):
    import torch
    pd = torch.int32 if ptr32 else torch.int64
    dA, dB = spx.from_host(A, ptr_dtype=pd), spx.from_host(B, ptr_dtype=pd)
    if a_dcsc:
        dA = spx.csc_to_dcsc(dA)
    if b_dcsc:
        dB = spx.csc_to_dcsc(dB)
    plan = spx.GemmPlan(dA, dB, semiring, out_fmt, tuning)
    C = plan.execute()
    info = plan.info()
    plan.close()
    return C, info


def check_against_oracle(spx, A, B, semiring, exact=False, **kw):
    C, info = gemm(spx, A, B, semiring, **kw)
    got = C.to_host_csc()
    ref = oracle.spgemm_csc(A, B, semiring)
    assert_same_csc(got, ref, exact_values=exact, what=f"{semiring}")
    mults = int(np.diff(A.cp)[B.ir].sum())
    assert info["mults"] == mults
    assert info["nnz"] == ref.cp[-1] <= mults
    return C, info


def test_er_config_plus_times_and_min_plus(spx):
    A = W.erdos_renyi(4096, 4096, 8, seed=1)
    C, info = check_against_oracle(spx, A, A, "plus_times")
    assert info["mults"] == 262144 and info["cols_tiny"] == 4096
    check_against_oracle(spx, A, A, "min_plus", exact=True)


@pytest.mark.parametrize("d", [4, 8])
@pytest.mark.parametrize("values", ["f64", "f32"])
def test_tiny_columns_add_in_product_order(spx, d, values):
    # columns of at most 64 products (d^2 here) take the one-wave path, which
    # adds each row's products in Algorithm 1's order (B's entries in storage
    # order, then A's rows): the floating-point sums equal the oracle's bitwise.
    # d = 4 pairs two columns per wave, d = 8 gives each column a whole wave.
    A = W.erdos_renyi(4096, 4096, d, seed=30 + d, values=values)
    B = W.erdos_renyi(4096, 4096, d, seed=40 + d, values=values)
    C, info = check_against_oracle(spx, A, B, "plus_times", exact=True)
    assert info["cols_tiny"] == 4096


@pytest.mark.parametrize("semiring,values,exact", [
    ("plus_times", "f64", False), ("plus_times", "f32", False), ("plus_times", "small_int", True),
    ("min_plus", "f64", True), ("min_plus", "f32", True), ("min_plus", "small_int", True),
    ("select2nd", "edge_id", True), ("select1st", "edge_id", True), ("or_and", "none", True),
])
def test_rmat_semirings(spx, semiring, values, exact):
    A = W.rmat(13, 8, seed=5, values="f64")
    rng = np.random.default_rng(7)
    if values == "f32":
        A.num = A.num.astype(np.float32)
    elif values == "small_int":
        A.num = rng.integers(-3, 4, size=A.nnz).astype(np.int64)
    elif values == "edge_id":
        A.num = np.arange(A.nnz, dtype=np.int64)
    elif values == "none":
        A.num = None
    _, info = check_against_oracle(spx, A, A, semiring, exact=exact)
    assert info["cols_heavy"] > 0 and info["cols_medium"] > 0 and info["cols_tiny"] > 0


@pytest.mark.parametrize("tune", [
    dict(tiny_max=0, hash_count_max=0),                   # everything through the bitmap count
    dict(tiny_max=64, hash_count_max=16384),              # no bitmap count
    dict(part_lds_bytes=24 * 1024),                       # many parts, both part modes
    dict(part_lds_bytes=12 * 1024),                       # row blocks of 1024 (f64) / 2048 (f32) rows
    dict(part_lds_bytes=48 * 1024, part_threads=256, count_threads=64, single_part_max=256),
    dict(tiny_max=16, hash_count_max=256, part_lds_bytes=64 * 1024, part_threads=512, single_part_max=64,
         single_threads=64, bitmap_threads=256),
    dict(single_part_max=4096, single_threads=1024),
    dict(tiny_max=0, hash_count_max=0, bitmap_chunk_log2=10, bitmap_threads=256),  # chunked bitmap count
    dict(part_lds_bytes=24 * 1024, xcd_slices=1),        # one shared work queue
    dict(part_lds_bytes=24 * 1024, xcd_slices=3),        # slices not a power of two
    dict(tiny_max=0, hash_count_max=0, bitmap_store_mb=0),  # numeric phase re-marks the bitmap rows
    dict(part_lds_bytes=24 * 1024, bitmap_store_mb=0),
    dict(tiny_max=0, hash_count_max=0, bitmap_store_mb=1),  # over the cap: recomputed
    dict(range_chunk=512),                                 # wide range list in the multi-part launch
    dict(range_chunk=512, part_lds_bytes=24 * 1024),
    dict(range_chunk=256, part_lds_bytes=24 * 1024),
    dict(bucket_parts=1),                                  # parts visit only their bucket of B entries
    dict(bucket_parts=1, part_lds_bytes=24 * 1024, range_chunk=512),
    dict(bucket_parts=1, part_lds_bytes=24 * 1024, xcd_slices=3),
    dict(force_off64=1),                                   # 64-bit gathers (A of 2^29 entries or more)
    dict(force_off64=1, part_lds_bytes=24 * 1024),
    dict(force_off64=1, tiny_max=0, hash_count_max=0, bitmap_store_mb=0),
    dict(force_off64=1, range_chunk=512, bucket_parts=1),
])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_forced_paths(spx, tune, dtype):
    A = W.rmat(14, 8, seed=11, values="f64")
    A.num = A.num.astype(dtype)
    t = spx.default_tuning()
    for k, v in tune.items():
        setattr(t, k, v)
    _, info = check_against_oracle(spx, A, A, "plus_times", tuning=t)
    if "part_lds_bytes" in tune and tune["part_lds_bytes"] <= 24 * 1024:
        assert info["heavy_parts"] > info["cols_heavy"] + info["cols_medium"]


@pytest.mark.parametrize("tune", [
    dict(),
    dict(tiny_max=0, hash_count_max=0),
    dict(tiny_max=64, hash_count_max=16384),
    dict(part_lds_bytes=24 * 1024),
    dict(part_lds_bytes=24 * 1024, bitmap_store_mb=0),
    dict(single_part_max=4096, single_threads=1024),
])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_signed_zeros_follow_algorithm_1(spx, tune, dtype):
    # Products that are all -0.0 (negative A times B values of +0.0) must sum
    # to -0.0, as Algorithm 1 starts each accumulator from its first product;
    # mixed-sign zeros give +0.0.  Checked bitwise on every path.
    A = W.rmat(14, 8, seed=13, values="f64")
    A.num = (-A.num).astype(dtype)
    B = A.with_values(np.zeros(A.nnz, dtype=dtype))
    t = spx.default_tuning()
    for k, v in tune.items():
        setattr(t, k, v)
    C, info = check_against_oracle(spx, A, B, "plus_times", exact=True, tuning=t)
    got = C.to_host_csc()
    assert got.num.size and np.all(got.num == 0) and np.all(np.signbit(got.num))
    B2 = B.with_values(B.num.copy())
    B2.num[::3] = -0.0  # -a * -0 = +0 joins some sums
    C2, _ = check_against_oracle(spx, A, B2, "plus_times", exact=True, tuning=t)
    g2 = C2.to_host_csc().num
    assert np.any(np.signbit(g2)) and np.any(~np.signbit(g2))


def test_min_plus_forced_paths_exact(spx):
    A = W.rmat(14, 8, seed=12, values="f64")
    t = spx.default_tuning()
    t.part_lds_bytes = 24 * 1024
    check_against_oracle(spx, A, A, "min_plus", exact=True, tuning=t)


def test_rectangular_and_independent(spx):
    rng = np.random.default_rng(3)
    A = W.erdos_renyi(3000, 700, 5, seed=4)
    B = W.rmat(10, 6, seed=8)                       # 1024 x 1024 -> need 700 x n
    B = W.column_block(B, 0, 700, 0, 1024)
    check_against_oracle(spx, A, B, "plus_times")
    check_against_oracle(spx, A, B, "min_plus", exact=True)


@pytest.mark.parametrize("tune", [
    dict(tiny_max=0, hash_count_max=0),                            # every column bitmap-counted and stored
    dict(tiny_max=0, hash_count_max=0, bitmap_chunk_log2=10),      # chunks end inside the last word
    dict(tiny_max=0, hash_count_max=0, part_lds_bytes=24 * 1024),  # many parts per stored column
    dict(tiny_max=0, hash_count_max=0, part_lds_bytes=12 * 1024),  # row blocks shorter than a wave's words
])
def test_stored_bitmaps_ragged_rows(spx, tune):
    # m is not a multiple of 64 (nor of a chunk): the stored bitmaps' last word
    # is partial; values f64 and an exact semiring
    A = W.erdos_renyi(50_021, 300, 40, seed=31)
    B = W.erdos_renyi(300, 200, 120, seed=32)
    t = spx.default_tuning()
    for k, v in tune.items():
        setattr(t, k, v)
    _, info = check_against_oracle(spx, A, B, "plus_times", tuning=t)
    assert info["cols_heavy"] == 200
    check_against_oracle(spx, A, B, "min_plus", exact=True, tuning=t)


@pytest.mark.parametrize("d2", [1, 10, 100, 1000, 8000])
def test_tall_skinny_frontier(spx, d2):
    # R-MAT times a tall-skinny Erdos-Renyi matrix, n/k = 8192 (multi-source
    # BFS frontiers of d2 vertices): from a few products per column to
    # columns that cover most rows
    A = W.rmat(14, 8, seed=41)
    F = W.erdos_renyi(A.n, A.n // 8192, d2, seed=42 + d2)
    check_against_oracle(spx, A, F, "plus_times")
    check_against_oracle(spx, A, F, "min_plus", exact=True)


def test_tall_skinny_many_parts(spx):
    # 16 columns of 20000 B entries over 2^17 rows: about ten parts per
    # column and few products per B entry, so the plan picks the wide range
    # list by itself; forced settings (wide list, per-part buckets) agree
    A = W.rmat(17, 8, seed=43)
    F = W.erdos_renyi(A.n, 16, 20000, seed=44)
    check_against_oracle(spx, A, F, "plus_times")
    check_against_oracle(spx, A, F, "min_plus", exact=True)
    for rc, bp in ((256, -1), (512, -1), (256, 1), (512, 1)):
        t = spx.default_tuning()
        t.range_chunk = rc
        t.bucket_parts = bp
        check_against_oracle(spx, A, F, "plus_times", tuning=t)
    t = spx.default_tuning()
    t.range_chunk = 300
    with pytest.raises(spx.SpxError):
        gemm(spx, A, F, "plus_times", tuning=t)


def test_tiny_columns_wide_row_ids(spx):
    # tiny columns whose row ids need more than 25 bits: the wave sort takes
    # 64-bit (row, index) keys instead of 32-bit ones
    A = W.erdos_renyi(40_000_000, 64, 4, seed=51)
    B = W.erdos_renyi(64, 100, 8, seed=52)
    for sr, exact in (("plus_times", False), ("min_plus", True)):
        C, info = gemm(spx, A, B, sr)
        assert info["cols_tiny"] == 100
        ref = oracle.spgemm_csc(A, B, sr, nthreads=1)
        assert_same_csc(C.to_host_csc(), ref, exact_values=exact, what=sr)


def test_tall_hash_parts_sorted_path(spx):
    # A has more than 2^20 rows, so hash-mode parts spanning all rows take the
    # sorted path instead of the two-level rank; a shorter A takes the rank.
    # (The oracle runs on 2 threads: its dense accumulator has m entries.)
    def check(A, B, sr, exact):
        C, info = gemm(spx, A, B, sr)
        ref = oracle.spgemm_csc(A, B, sr, nthreads=2)
        assert_same_csc(C.to_host_csc(), ref, exact_values=exact, what=sr)
        return info
    A = W.erdos_renyi(1_100_000, 96, 24, seed=21)
    B = W.erdos_renyi(96, 64, 48, seed=22)            # multi-launch columns (1152 products)
    B2 = W.erdos_renyi(96, 64, 40, seed=24)           # single-part columns (960 products)
    info = check(A, B, "plus_times", False)
    assert info["cols_medium"] == 64
    check(A, B, "min_plus", True)
    check(A, B2, "plus_times", False)
    A2 = W.erdos_renyi(900_000, 96, 24, seed=23)
    check(A2, B, "plus_times", False)
    check(A2, B2, "min_plus", True)


@pytest.mark.parametrize("out_fmt", [0, 1])
def test_dcsc_stage_blocks(spx, out_fmt):
    """One GPU's share of an 8x8 Sparse SUMMA stage: hypersparse blocks in DCSC."""
    A = W.rmat(15, 8, seed=20)
    b = A.n // 8
    blocks = [[W.column_block(A, i * b, (i + 1) * b, k * b, (k + 1) * b) for k in range(8)] for i in range(8)]
    for k in range(8):
        X, Y = blocks[0][k], blocks[k][0]
        assert np.count_nonzero(np.diff(X.cp)) < X.n  # empty columns: DCSC drops them
        C, info = gemm(spx, X, Y, "plus_times", out_fmt=out_fmt, a_dcsc=True, b_dcsc=True)
        ref = oracle.spgemm_csc(X, Y)
        got = C.to_host_csc()
        assert_same_csc(got, ref, what=f"stage block k={k}")
        if out_fmt == 1:
            jc, dcp = oracle.csc_to_dcsc(ref.n, ref.cp)
            cp, ir, num = C.to_host()
            assert np.array_equal(C.jc.cpu().numpy(), jc) and np.array_equal(cp, dcp)


def test_mixed_formats_and_int32_pointers(spx):
    A = W.rmat(12, 8, seed=30)
    for a_d, b_d in ((True, False), (False, True)):
        check_against_oracle(spx, A, A, "plus_times", a_dcsc=a_d, b_dcsc=b_d)
    check_against_oracle(spx, A, A, "plus_times", ptr32=True)


def test_edge_cases(spx):
    empty = W.from_triples([], [], np.zeros(0), 5, 7)
    other = W.erdos_renyi(7, 3, 2, seed=1)
    check_against_oracle(spx, empty, other, "plus_times")
    one = W.from_triples([0], [0], np.array([2.5]), 1, 1)
    check_against_oracle(spx, one, one, "plus_times")
    # B columns that hit only empty columns of A
    A = W.from_triples([1, 2], [0, 0], np.array([1.0, 2.0]), 3, 3)
    B = W.from_triples([1, 2, 0], [0, 1, 2], np.array([1.0, 1.0, 3.0]), 3, 3)
    check_against_oracle(spx, A, B, "plus_times")
    # zero-column output
    Z = W.from_triples([], [], np.zeros(0), 4, 0)
    X = W.erdos_renyi(6, 4, 2, seed=2)
    C, _ = gemm(spx, X, Z)
    assert C.nnz == 0 and C.n == 0


def test_errors(spx):
    A = W.erdos_renyi(10, 8, 2, seed=1)
    dA = spx.from_host(A)
    with pytest.raises(spx.SpxError) as e:
        spx.spgemm(dA, dA)  # 10x8 times 10x8
    assert e.value.code == spx.SPX_EINVAL
    B = W.erdos_renyi(8, 4, 2, seed=2)
    dB = spx.from_host(B)
    dB.num = dB.num.float()
    with pytest.raises(spx.SpxError) as e:
        spx.spgemm(dA, dB)  # f64 x f32
    assert e.value.code == spx.SPX_EUNSUPPORTED


@pytest.fixture(scope="module")
def rmat20():
    return W.rmat(20, 8, seed=20)


def check_blockwise(A, B, C, semiring="plus_times", block_entries=200_000_000):
    """Every column of a device result C (CSC) against the oracle, in blocks of
    columns copied to the host (the oracle recomputes each column with its
    SPA and compares rows exactly and values within the tolerance)."""
    import torch
    torch.cuda.synchronize()
    cp = C.cp.cpu().numpy().astype(np.int64)
    assert cp[0] == 0 and cp[-1] == C.nnz and np.all(np.diff(cp) >= 0)
    j0, nbad, first = 0, 0, -1
    while j0 < C.n:
        j1 = int(np.searchsorted(cp, cp[j0] + block_entries, side="right")) - 1
        j1 = min(C.n, max(j1, j0 + 1))
        s, e = int(cp[j0]), int(cp[j1])
        gir = C.ir[s:e].cpu().numpy()
        gnum = None if C.num is None else C.num[s:e].cpu().numpy()
        nb, fb = oracle.spgemm_check(A, B, j0, j1, cp[j0:j1 + 1], gir, gnum, semiring)
        if nb and first < 0:
            first = fb
        nbad += nb
        j0 = j1
    assert nbad == 0, f"{nbad} columns differ from the oracle, first {first}"
    return cp


@pytest.mark.timeout(900)
def test_rmat20_full_size_every_column(spx, rmat20):
    """R-MAT scale 20 A*A at full size in the benchmark's configuration
    (default tuning, CSC output, int64 pointers): every one of the 2^20 output
    columns is recomputed by the oracle and compared, rows exactly and values
    within 1e-12 relative, block by block of about 2.4 GB."""
    import torch
    A = rmat20
    dA = spx.from_host(A)
    plan = spx.GemmPlan(dA, dA)
    C = plan.execute()
    info = plan.info()
    plan.close()
    deg = np.diff(A.cp)
    mults = int(deg[A.ir].sum())
    assert info["mults"] == mults
    cp = check_blockwise(A, A, C)
    assert info["nnz"] == C.nnz == cp[-1] <= mults
    del C
    torch.cuda.empty_cache()


@pytest.mark.parametrize("out_fmt", [0, 1])
def test_rmat20_stage_block_dcsc_full_size(spx, rmat20, out_fmt):
    """The benchmark's 8x8 Sparse SUMMA stage block: A00 * A00 of the scale-20
    matrix (2^17 x 2^17, fewer nonzeros than columns), DCSC in and DCSC (or
    CSC) out, every column against the oracle."""
    A = rmat20
    b = A.n // 8
    blk = W.column_block(A, 0, b, 0, b)
    assert blk.nnz < blk.n
    dB = spx.csc_to_dcsc(spx.from_host(blk))
    plan = spx.GemmPlan(dB, dB, out_fmt=out_fmt)
    C = plan.execute()
    info = plan.info()
    plan.close()
    got = C.to_host_csc()
    assert info["mults"] == int(np.diff(blk.cp)[blk.ir].sum())
    ref = oracle.spgemm_csc(blk, blk)
    assert_same_csc(got, ref, what="stage block A00*A00")
    if out_fmt == 1:
        jc, dcp = oracle.csc_to_dcsc(ref.n, ref.cp)
        assert np.array_equal(C.jc.cpu().numpy(), jc) and np.array_equal(C.cp.cpu().numpy(), dcp)


def test_rmat20_forced_64bit_offsets_sampled(spx, rmat20):
    """The gathers through 64-bit positions (taken when A has 2^29 entries or
    more) forced on the scale-20 product: whole columns sampled from every
    bin against the oracle."""
    import torch
    A = rmat20
    dA = spx.from_host(A)
    t = spx.default_tuning()
    t.force_off64 = 1
    plan = spx.GemmPlan(dA, dA, tuning=t)
    C = plan.execute()
    plan.close()
    torch.cuda.synchronize()
    cp = C.cp.cpu().numpy()
    deg = np.diff(A.cp)
    cs = np.concatenate([[0], np.cumsum(deg[A.ir])])
    mults_col = cs[A.cp[1:]] - cs[A.cp[:-1]]
    rng = np.random.default_rng(5)
    order = np.argsort(mults_col)
    nonempty = np.nonzero(mults_col > 0)[0]
    cols = np.unique(np.concatenate([order[-40:], rng.choice(nonempty, 400, replace=False)]))
    rcp, rir, rnum = oracle.spgemm(A, A, cols=cols)
    lens = cp[cols + 1] - cp[cols]
    assert np.array_equal(lens, np.diff(rcp))
    idx = torch.from_numpy(np.concatenate([np.arange(cp[j], cp[j + 1]) for j in cols])).cuda()
    from types import SimpleNamespace
    got = SimpleNamespace(cp=np.concatenate([[0], np.cumsum(lens)]), ir=C.ir[idx].cpu().numpy(),
                          num=C.num[idx].cpu().numpy())
    assert_same_csc(got, SimpleNamespace(cp=rcp, ir=rir, num=rnum), what="64-bit gathers")
    del C
    torch.cuda.empty_cache()
