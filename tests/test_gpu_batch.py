"""GPU parity of the batched SpGEMM (one plan, one persistent launch for many products)."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import assert_same_csc

pytestmark = pytest.mark.gpu


def host(M):
    return M.to_host_csc()


def test_batch_mixed_products_match_oracle_and_single(spx):
    rng = np.random.default_rng(0)
    As, Bs = [], []
    for i in range(12):
        kind = i % 3
        if kind == 0:
            A = W.erdos_renyi(int(rng.integers(50, 400)), int(rng.integers(50, 400)), 3, seed=i)
            B = W.erdos_renyi(A.n, int(rng.integers(1, 300)), 2, seed=100 + i)
        elif kind == 1:
            A = W.rmat(int(rng.integers(8, 12)), 8, seed=i)
            B = A
        else:
            A = W.rmat(10, 4, seed=i)
            B = W.column_block(W.rmat(10, 6, seed=200 + i), 0, A.n, 0, 700)
        As.append(A)
        Bs.append(B)
    dA = [spx.from_host(a) for a in As]
    dB = [spx.from_host(b) for b in Bs]
    Cs = spx.batch_spgemm(dA, dB)
    for i, (A, B, C) in enumerate(zip(As, Bs, Cs)):
        ref = oracle.spgemm_csc(A, B)
        assert_same_csc(host(C), ref, what=f"product {i}")
        single = host(spx.spgemm(dA[i], dB[i]))
        assert np.array_equal(single.cp, host(C).cp) and np.array_equal(single.ir, host(C).ir)


def test_batch_repeated_left_operands(spx):
    # the same left operand (same device arrays) in several products enters
    # the concatenation once; every product still gets its own result
    A1 = W.rmat(10, 8, seed=61)
    A2 = W.erdos_renyi(1024, 1024, 5, seed=62)
    dA1, dA2 = spx.from_host(A1), spx.from_host(A2)
    Bs = [W.erdos_renyi(1024, int(n), d, seed=70 + k) for k, (n, d) in enumerate([(300, 3), (50, 9), (700, 1),
                                                                                     (1, 4), (256, 6), (900, 2)])]
    order = [dA1, dA2, dA1, dA1, dA2, dA1]
    hostA = [A1, A2, A1, A1, A2, A1]
    dB = [spx.from_host(b) for b in Bs]
    for sr, exact in (("plus_times", False), ("min_plus", True)):
        Cs = spx.batch_spgemm(order, dB, sr)
        for i, (A, B, C) in enumerate(zip(hostA, Bs, Cs)):
            assert_same_csc(host(C), oracle.spgemm_csc(A, B, sr), exact_values=exact, what=f"{sr} product {i}")


@pytest.mark.parametrize("semiring", ["min_plus", "or_and"])
def test_batch_other_semirings(spx, semiring):
    As = [W.rmat(9, 8, seed=s) for s in range(5)]
    if semiring == "or_and":
        for a in As:
            a.num = None
    d = [spx.from_host(a) for a in As]
    Cs = spx.batch_spgemm(d, d, semiring)
    for A, C in zip(As, Cs):
        assert_same_csc(host(C), oracle.spgemm_csc(A, A, semiring), exact_values=True, what=semiring)


def galerkin_batch(spx, sizes, dtype):
    import torch
    uniq = sorted(set(int(n) for n in sizes))
    L = {n: spx.from_host(W.laplacian7(n, dtype)) for n in uniq}
    P = {n: spx.from_host(W.aggregation(n, dtype)) for n in uniq}
    PT = {n: spx.from_host(W.aggregation(n, dtype, transpose=True)) for n in uniq}
    As = [L[int(n)] for n in sizes]
    Ps = [P[int(n)] for n in sizes]
    PTs = [PT[int(n)] for n in sizes]
    AP = spx.BatchPlan(As, Ps)
    APs = AP.execute()
    G = spx.BatchPlan(PTs, APs)
    Gs = G.execute()
    torch.cuda.synchronize()
    return AP, G, APs, Gs


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batched_galerkin_closed_form(spx, dtype):
    sizes = W.galerkin_sizes(24, seed=4, lo=4, hi=24)
    AP, G, APs, Gs = galerkin_batch(spx, sizes, dtype)
    for n, C in zip(sizes, Gs):
        ref = W.laplacian7(int(n) // 2, dtype)
        got = host(C)
        assert np.array_equal(got.cp, ref.cp) and np.array_equal(got.ir, ref.ir)
        assert np.array_equal(got.num, 4 * ref.num)  # small integers: exact in any order
    AP.close()
    G.close()


def closed_form_all(spx, sizes, Gs, dtype):
    """Every coarse operator against 4 x the coarse Laplacian, compared on the
    device (small integers: exact in any order); returns the failing ids."""
    import torch
    ref = {}
    for n in sorted(set(int(x) for x in sizes)):
        r = W.laplacian7(n // 2, dtype)
        ref[n] = spx.from_host(r.with_values(4 * r.num))
    bad = []
    for i, (n, C) in enumerate(zip(sizes, Gs)):
        R = ref[int(n)]
        if not (C.nnz == R.nnz and torch.equal(C.cp, R.cp) and torch.equal(C.ir, R.ir)
                and torch.equal(C.num, R.num)):
            bad.append(i)
    return bad


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batched_galerkin_512_every_instance(spx, dtype):
    """The benchmark's Galerkin batch (512 instances, n log-uniform in [16, 96],
    seed 4) under every setting the autotuner may pick for either level: all
    512 coarse operators equal the closed form 4 L_{n/2}."""
    from paper_1109_3739_amd import autotune
    sizes = W.galerkin_sizes(512, seed=4)
    uniq = sorted(set(int(n) for n in sizes))
    L = {n: spx.from_host(W.laplacian7(n, dtype)) for n in uniq}
    P = {n: spx.from_host(W.aggregation(n, dtype)) for n in uniq}
    PT = {n: spx.from_host(W.aggregation(n, dtype, transpose=True)) for n in uniq}
    As = [L[int(n)] for n in sizes]
    Ps = [P[int(n)] for n in sizes]
    PTs = [PT[int(n)] for n in sizes]
    for cand in autotune.CANDIDATES:
        t = autotune.make_tuning(cand)
        p1 = spx.BatchPlan(As, Ps, tuning=t)
        APs = p1.execute()
        p2 = spx.BatchPlan(PTs, APs, tuning=t)
        Gs = p2.execute()
        bad = closed_form_all(spx, sizes, Gs, dtype)
        assert not bad, f"tuning {cand}: instances {bad[:10]} differ from 4 L_(n/2)"
        p1.close()
        p2.close()
        del APs, Gs
    # both levels captured into HIP graphs on one stream and replayed, as the
    # benchmark times them; every replay is checked (eager work in between)
    import torch
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        p1 = spx.BatchPlan(As, Ps, stream=stream)
        APs = p1.execute()
        p2 = spx.BatchPlan(PTs, APs, stream=stream)
        p2.execute()
        p1.capture()
        Gs = p2.capture()
        for rep in range(3):
            torch.zeros(1024, device="cuda").sum().item()  # eager work between replays
            p1.replay()
            p2.replay()
            stream.synchronize()
            bad = closed_form_all(spx, sizes, Gs, dtype)
            assert not bad, f"replay {rep}: instances {bad[:10]} differ from 4 L_(n/2)"
        p1.close()
        p2.close()


def test_batch_graph_replay(spx):
    """Capture the numeric phase once, replay it with new values, with eager
    work and synchronisations between replays; check every replay."""
    import torch
    sizes = [4, 6, 8, 8, 10]
    L = [spx.from_host(W.laplacian7(n)) for n in sizes]
    P = [spx.from_host(W.aggregation(n)) for n in sizes]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = spx.BatchPlan(L, P, stream=stream)
        eager = [host(c) for c in plan.execute()]
        views = plan.capture()
        for rep, scale in enumerate([1.0, 2.0, 0.5, 3.0]):
            for a in L:
                a.num.mul_(scale)  # eager work between replays
            torch.cuda.synchronize()
            plan.replay()
            stream.synchronize()
            total = np.prod([1.0, 2.0, 0.5, 3.0][:rep + 1])
            for e, v in zip(eager, views):
                got = host(v)
                assert np.array_equal(got.cp, e.cp) and np.array_equal(got.ir, e.ir)
                assert np.array_equal(got.num, e.num * total), f"replay {rep}"
        plan.close()


def test_batch_values_in_place(spx):
    """Operand values that already lie back to back in batch order in one
    allocation (as the outputs of an earlier batch do) are read in place.
    Results match the copied path bit for bit and the oracle; an exec and a
    graph replay after the shared values change see the new values; an empty
    operand in the middle and a repeated right operand (not back to back, so
    copied) are handled."""
    import dataclasses
    import torch
    shapes = [(300, 200, 3), (128, 64, 5), (700, 1, 2), (256, 256, 4), (90, 300, 6)]
    As = [W.erdos_renyi(m, k, d, seed=300 + i) for i, (m, k, d) in enumerate(shapes)]
    # B_2 has no entries: its values are never read
    Bs = [W.erdos_renyi(k, n, d, seed=400 + i) for i, (k, n, d) in enumerate([(200, 150, 3), (64, 90, 3), (1, 40, 0),
                                                                              (256, 256, 3), (300, 70, 3)])]
    assert Bs[2].nnz == 0
    dA = [spx.from_host(a) for a in As]
    dB = [spx.from_host(b) for b in Bs]

    def packed(ms):
        vals = torch.cat([m.num for m in ms])
        out, off = [], 0
        for m in ms:
            out.append(dataclasses.replace(m, num=vals[off:off + m.nnz]))
            off += m.nnz
        return vals, out

    avals, pA = packed(dA)
    bvals, pB = packed(dB)
    copied = [host(c) for c in spx.batch_spgemm(dA, dB)]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = spx.BatchPlan(pA, pB, stream=stream)
        got = [host(c) for c in plan.execute()]
        stream.synchronize()
        for i, (g, c) in enumerate(zip(got, copied)):
            assert np.array_equal(g.cp, c.cp) and np.array_equal(g.ir, c.ir) and np.array_equal(g.num, c.num), i
            assert_same_csc(g, oracle.spgemm_csc(As[i], Bs[i]), what=f"in place, product {i}")
        # new values in the shared arrays: a second exec reads them
        avals.mul_(2.0)
        bvals.mul_(0.5)
        stream.synchronize()
        again = [host(c) for c in plan.execute()]
        stream.synchronize()
        for i, (g, c) in enumerate(zip(again, copied)):
            assert np.array_equal(g.ir, c.ir) and np.array_equal(g.num, c.num), f"rescaled, product {i}"
        # captured once, replayed after the values change again
        views = plan.capture()
        bvals.mul_(4.0)
        torch.cuda.synchronize()
        plan.replay()
        stream.synchronize()
        for i, (v, c) in enumerate(zip(views, copied)):
            assert np.array_equal(host(v).num, c.num * 4), f"replay, product {i}"
        plan.close()
    # a repeated right operand breaks the back-to-back layout: values are copied
    rep = [pB[0], pB[1], pB[0]]
    Cs = spx.batch_spgemm([pA[0], pA[1], pA[0]], rep)
    for i, (a, b) in enumerate([(0, 0), (1, 1), (0, 0)]):
        ref = oracle.spgemm_csc(As[a].with_values(2.0 * As[a].num), Bs[b].with_values(2.0 * Bs[b].num))
        assert_same_csc(host(Cs[i]), ref, what=f"repeated operand, product {i}")


def test_batch_errors(spx):
    A = spx.from_host(W.erdos_renyi(10, 8, 2, seed=1))
    with pytest.raises(spx.SpxError):
        spx.batch_spgemm([A], [A])  # 10x8 * 10x8
