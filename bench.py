#!/usr/bin/env python3
"""Benchmark of the SpGEMM hot path on one MI355X.

Workload: C = A*A over (+, x) in FP64 for an R-MAT matrix of scale 20
(2^20 x 2^20, edge factor 8, quadrant probabilities a=.57 b=c=.19 d=.05,
duplicates merged, vertices randomly permuted, values uniform [0,1)).
One step = the whole path for one product: symbolic phase (column lookup,
multiplication counts, binning, exact column counts, int64 scans, part
cutting; one host read-back of the output size) and numeric phase (wave /
LDS accumulation, ordered write-out of IR and NUM, column pointers).  The
input is resident in HBM before timing starts; the 43 GB output buffer is
allocated once and rewritten by every step.  Python's cyclic garbage
collector is frozen over the objects that exist once set-up is done: a full
collection over torch's heap takes ~40 ms and would otherwise land inside
whichever step is running (the host side of a plan); collections of objects
made later still run.

Prints one JSON line: GFLOP/s counted as 2 x multiplications per second,
achieved compulsory GB/s, the roofline of the dominant kernel (HIP events
on the library's stream over the timed steps), and the CPU oracle timed on
a bounded sample of the same product.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-extra] [--no-cpu-baseline]
    python bench.py --extra-only {latency,stages,tall,index,restriction,galerkin,serving}

The other workloads (printed under "extra") give context: launch-bound
latency, the Sparse SUMMA stage block and stage sum, the tall-skinny
product, SpRef / SpAsgn / extend-add, and the restriction S A S^T.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SpGEMM GFLOP/s (2·mults/s) + GB/s on R-MAT s20 A·A; served p50/p99 vs plain"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def csc_bytes(nnz, ncols, vbytes=8, ptr_bytes=8):
    return nnz * (4 + vbytes) + (ncols + 1) * ptr_bytes


def traffic_from_profiles(kernel):
    """HBM bytes per launch from the committed PMC summary, if it was taken
    on the current kernel sources; otherwise None."""
    from paper_1109_3739_amd.profiling import source_digest
    path = os.path.join(ROOT, "profiles", "traffic_spgemm_rmat20.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        if d.get("source_digest") != source_digest():
            return None
        k = d["kernels"].get(kernel)
        return None if k is None else round(float(k["hbm_bytes_per_launch"]))
    except Exception:
        return None


def time_steps(fn, steps, sync):
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) / steps


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, target_s=4.0, reps=3):
    """The oracle (dense-SPA column-wise Gustavson, OpenMP over columns) on
    random samples of the output columns of A*A, at all host threads and at
    one thread: each sample sized for about `target_s` seconds, timed `reps`
    times, median reported.  A sample, not the whole product (which takes
    minutes on one thread); the rate is GFLOP/s = 2 x mults / s of the
    sampled columns."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(1234)
    deg = np.diff(A.cp)
    cs = np.concatenate([[0], np.cumsum(deg[A.ir])])
    mults_col = cs[A.cp[1:]] - cs[A.cp[:-1]]
    order = rng.permutation(A.n)
    cum = np.cumsum(mults_col[order])
    total = float(mults_col.sum())

    def leg(threads):
        # calibrate on a small sample, then size the sample for ~target_s
        n0 = max(64, A.n // (500 if threads > 1 else 8000))
        t0 = time.perf_counter()
        oracle.spgemm(A, A, cols=np.sort(order[:n0]), nthreads=threads)
        rate = max(int(cum[n0 - 1]), 1) / max(time.perf_counter() - t0, 1e-3)
        want = min(rate * target_s, 0.5 * total)
        ncols = int(min(A.n, max(n0, np.searchsorted(cum, want) + 1)))
        cols = np.sort(order[:ncols])
        mults = int(mults_col[cols].sum())
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.spgemm(A, A, cols=cols, nthreads=threads)
            ts.append(time.perf_counter() - t0)
        t = statistics.median(ts)
        return {"gflops": round(2.0 * mults / t / 1e9, 4), "seconds_median": round(t, 3),
                "seconds_all": [round(x, 3) for x in ts], "columns": ncols, "mults": mults,
                "whole_product_s_estimate": round(t * total / mults, 1)}

    threads = oracle.max_threads()
    multi = leg(threads)
    single = leg(1)
    return {
        "value": multi["gflops"],
        "unit": "GFLOP/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "host_logical_cpus": os.cpu_count(),
        "sample": f"a sample, not the whole product: {multi['columns']} of {A.n} output columns drawn uniformly "
                  f"at random (seed 1234), {multi['mults']} mults, median of {reps} runs "
                  f"({multi['seconds_median']} s) at {threads} threads; dense-SPA column-wise Gustavson, "
                  f"OpenMP over columns",
        "all_threads": multi,
        "single_thread": {**single, "cores": 1,
                          "sample": f"{single['columns']} of {A.n} columns (the first of the same random order), "
                                    f"median of {reps} runs at 1 thread"},
    }


def extra_workloads(spx, W, torch, only=None):
    """Latency / bandwidth of the other workloads of the path (context).
    ``only``: run one group (latency, stages, tall, index, restriction)."""
    import numpy as np
    out = {}
    sync = torch.cuda.synchronize

    def want(name):
        return only is None or only == name

    if want("stages") or want("tall"):
        A = W.rmat(20, 8, seed=20)

    if want("latency"):
        # Erdos-Renyi 4096 x 4096, 8 per column: launch-bound latency
        E = W.erdos_renyi(4096, 4096, 8, seed=1)
        dE = spx.from_host(E)
        for sr in ("plus_times", "min_plus"):
            spx.spgemm(dE, dE, sr)
            ts = []
            for _ in range(10):
                sync()
                t0 = time.perf_counter()
                spx.spgemm(dE, dE, sr)
                sync()
                ts.append(time.perf_counter() - t0)
            out[f"er4096_{sr}_ms"] = round(1e3 * statistics.median(ts), 4)

    if want("stages"):
        # one GPU's share of an 8x8 Sparse SUMMA stage: A00 * A00 in DCSC
        b = A.n // 8
        blk = W.column_block(A, 0, b, 0, b)
        dB = spx.csc_to_dcsc(spx.from_host(blk))
        p = spx.GemmPlan(dB, dB, out_fmt=spx.DCSC)
        C = p.execute()
        mults = p.info()["mults"]
        p.close()

        def stage():
            q = spx.GemmPlan(dB, dB, out_fmt=spx.DCSC)
            q.execute(C)
            q.close()

        for _ in range(3):
            stage()
        t = time_steps(stage, 10, sync)
        out["stage_block_dcsc_ms"] = round(1e3 * t, 4)
        out["stage_block_gflops"] = round(2 * mults / t / 1e9, 3)
        out["stage_block_nnz_c"] = int(C.nnz)
        del C

        # all 8 stages of that processor: C_00 = sum_k A_0k * A_k0 as one stage-sum
        # plan, against the 8 stage products formed separately (partials not merged)
        As = [spx.csc_to_dcsc(spx.from_host(W.column_block(A, 0, b, k * b, (k + 1) * b))) for k in range(8)]
        Bs = [spx.csc_to_dcsc(spx.from_host(W.column_block(A, k * b, (k + 1) * b, 0, b))) for k in range(8)]
        sp = spx.StageSumPlan(As, Bs, out_fmt=spx.DCSC)
        S = sp.execute()
        smults = sp.info()["mults"]
        sp.close()

        def stage_sum():
            q = spx.StageSumPlan(As, Bs, out_fmt=spx.DCSC)
            q.execute(S)
            q.close()

        def stages_apart():
            for X, Y in zip(As, Bs):
                q = spx.GemmPlan(X, Y, out_fmt=spx.DCSC)
                q.execute()
                q.close()

        for _ in range(2):
            stage_sum()
            stages_apart()
        t = time_steps(stage_sum, 10, sync)
        t_apart = time_steps(stages_apart, 5, sync)
        out["summa_8x8_c00"] = {"stages": 8, "ms": round(1e3 * t, 4), "gflops": round(2 * smults / t / 1e9, 3),
                                "mults": smults, "nnz_c": int(S.nnz),
                                "stage_products_apart_ms": round(1e3 * t_apart, 4)}
        del S, As, Bs

    if want("tall"):
        # R-MAT scale 20 times a tall-skinny Erdos-Renyi matrix (n/k = 8192, d2
        # nonzeros per column): the multi-source BFS frontier expansion
        dA = spx.from_host(A)
        tall = {}
        for d2 in (1, 10, 100, 1000, 10000, 100000):
            F = W.erdos_renyi(A.n, A.n // 8192, d2, seed=300 + d2)
            dF = spx.from_host(F)
            Cf = spx.spgemm(dA, dF)
            mults = int(np.diff(A.cp)[F.ir].sum())
            t = time_steps(lambda: spx.spgemm(dA, dF), 5, sync)
            tall[str(d2)] = {"ms": round(1e3 * t, 4), "gflops": round(2 * mults / t / 1e9, 3), "mults": mults,
                             "nnz_c": int(Cf.nnz)}
            del Cf, dF
        out["tall_skinny_rmat20_x_er"] = tall

    if want("index"):
        # SpRef / SpAsgn on R-MAT scale 22, edge factor 16, int64 edge ids
        A3 = W.rmat(22, 16, seed=22, values="edge_id")
        I = W.index_vector(1 << 18, A3.m, seed=221)
        J = W.index_vector(1 << 18, A3.n, seed=222)
        Bp = W.erdos_renyi(1 << 18, 1 << 18, 4, seed=223, values="id40")
        dA3, dI, dJ, dBp = spx.from_host(A3), torch.from_numpy(I).cuda(), torch.from_numpy(J).cuda(), spx.from_host(Bp)
        R = spx.spref(dA3, dI, dJ)
        t = time_steps(lambda: spx.spref(dA3, dI, dJ), 5, sync)
        deg = np.diff(A3.cp)
        gathered = int(deg[J].sum())
        ref_bytes = gathered * 12 + R.nnz * 12 + (1 << 18) * 8 * 2 + (1 << 18) * 8
        out["spref_ms"] = round(1e3 * t, 4)
        out["spref_gbs"] = round(ref_bytes / t / 1e9, 2)
        out["spref_nnz"] = int(R.nnz)
        S = spx.spasgn(dA3, dI, dJ, dBp)
        t = time_steps(lambda: spx.spasgn(dA3, dI, dJ, dBp), 5, sync)
        asg_bytes = csc_bytes(A3.nnz, A3.n) + csc_bytes(Bp.nnz, Bp.n) + csc_bytes(S.nnz, A3.n) + (1 << 19) * 4
        out["spasgn_ms"] = round(1e3 * t, 4)
        out["spasgn_gbs"] = round(asg_bytes / t / 1e9, 2)
        out["spasgn_nnz"] = int(S.nnz)
        del S
        E = spx.extend_add(dA3, dI, dJ, dBp)
        t = time_steps(lambda: spx.extend_add(dA3, dI, dJ, dBp), 5, sync)
        ea_bytes = csc_bytes(A3.nnz, A3.n) + csc_bytes(Bp.nnz, Bp.n) + csc_bytes(E.nnz, A3.n) + (1 << 19) * 4
        out["extend_add_ms"] = round(1e3 * t, 4)
        out["extend_add_gbs"] = round(ea_bytes / t / 1e9, 2)
        out["extend_add_nnz"] = int(E.nnz)
        del E, R

    if want("restriction"):
        # restriction S A S^T of orders 2, 4, 8 on R-MAT scale 23: one fused pass
        # over A, against both parenthesizations with S, S^T and the intermediate
        # product materialized
        A23 = W.rmat(23, 8, seed=23)
        dA23 = spx.from_host(A23)
        n23 = A23.n
        res = {}
        for order in (2, 4, 8):
            agg = spx.restriction_map(n23, order)
            nc = n23 // order
            ones = torch.ones(n23, dtype=torch.float64, device="cuda")
            dS = spx.SpMat(nc, n23, torch.arange(n23 + 1, dtype=torch.int64, device="cuda"), agg, ones)
            dSt = spx.SpMat(n23, nc, torch.arange(0, n23 + 1, order, dtype=torch.int64, device="cuda"),
                            torch.arange(n23, dtype=torch.int32, device="cuda"), ones)
            p = spx.ContractPlan(dA23, agg, nc, agg, nc)
            Cr = p.execute()
            p.close()

            def fused():
                q = spx.ContractPlan(dA23, agg, nc, agg, nc)
                q.execute(Cr)
                q.close()

            def left():
                spx.spgemm(spx.spgemm(dS, dA23), dSt)

            def right():
                spx.spgemm(dS, spx.spgemm(dA23, dSt))

            for f in (fused, left, right):
                f()
            t = time_steps(fused, 5, sync)
            byts = csc_bytes(A23.nnz, n23) + csc_bytes(Cr.nnz, nc)
            res[str(order)] = {"ms": round(1e3 * t, 4), "gbs": round(byts / t / 1e9, 2), "nnz_c": int(Cr.nnz),
                               "two_products_left_ms": round(1e3 * time_steps(left, 3, sync), 4),
                               "two_products_right_ms": round(1e3 * time_steps(right, 3, sync), 4)}
            del Cr, dS, dSt
        out["restriction_rmat23"] = {"nnz_a": int(A23.nnz), "orders": res}
    return out


def galerkin(spx, W, torch, count=512, seed=4):
    """Batched Galerkin products P^T (A P) for `count` 7-point Laplacians
    (n^3 grids, n log-uniform in [16, 96]) with 2x2x2 aggregation: one batch
    plan per product level (persistent launches over all instances), against
    2*count separate plan+exec calls on the same GPU, and the numeric phases
    of both levels captured once in HIP graphs and replayed.  Parity: every
    one of the P^T A P must equal 4 x the coarse Laplacian exactly."""
    import numpy as np
    from paper_1109_3739_amd import autotune
    sizes = W.galerkin_sizes(count, seed)
    out = {"instances": count, "n_range": [int(sizes.min()), int(sizes.max())]}
    for dt, name in ((np.float64, "f64"), (np.float32, "f32")):
        uniq = sorted(set(int(n) for n in sizes))
        L = {n: spx.from_host(W.laplacian7(n, dt)) for n in uniq}
        P = {n: spx.from_host(W.aggregation(n, dt)) for n in uniq}
        PT = {n: spx.from_host(W.aggregation(n, dt, transpose=True)) for n in uniq}
        As = [L[int(n)] for n in sizes]
        Ps = [P[int(n)] for n in sizes]
        PTs = [PT[int(n)] for n in sizes]
        mults = int(sum(L[int(n)].nnz + 4 * int(n) ** 3 for n in sizes))  # A*P: nnz(A); P^T*(AP): nnz(AP)
        # each level tuned on its own operands (the levels differ in shape:
        # A*P has 56 products per output column, P^T*(AP) about 32)
        tun, tinfo = autotune.tune_batch(As, Ps)
        p0 = spx.BatchPlan(As, Ps, tuning=tun)
        tun2, tinfo2 = autotune.tune_batch(PTs, p0.execute())
        p0.close()

        def batched():
            p1 = spx.BatchPlan(As, Ps, tuning=tun)
            APs = p1.execute()
            p2 = spx.BatchPlan(PTs, APs, tuning=tun2)
            Gs = p2.execute()
            p1.close()
            p2.close()
            return Gs

        def plain():
            res = []
            for a, p_, pt in zip(As, Ps, PTs):
                ap = spx.spgemm(a, p_)
                res.append(spx.spgemm(pt, ap))
            return res

        refs = {}
        for n in sorted(set(int(x) for x in sizes)):
            r = W.laplacian7(n // 2, dt)
            refs[n] = spx.from_host(r.with_values(4 * r.num))

        def closed_form_ok(Gs):
            # every coarse operator equals 4 L_(n/2) exactly (small integers)
            return all(C.nnz == refs[int(n)].nnz and torch.equal(C.cp, refs[int(n)].cp)
                       and torch.equal(C.ir, refs[int(n)].ir) and torch.equal(C.num, refs[int(n)].num)
                       for n, C in zip(sizes, Gs))

        Gs = batched()
        torch.cuda.synchronize()
        ok = closed_form_ok(Gs)
        del Gs
        t_b = time_steps(batched, 3, torch.cuda.synchronize)
        t_p = time_steps(plain, 1, torch.cuda.synchronize)

        # the pattern is fixed, only values change from call to call (an AMG
        # setup re-run on new coefficients): both levels' numeric phases are
        # captured once into HIP graphs on one stream and replayed; each
        # replay refreshes the values of A and of A P from their arrays
        gstream = torch.cuda.Stream()
        with torch.cuda.stream(gstream):
            # level 2 is planned on level 1's output, so level 1 runs once
            # before it is captured; both capture into the pools of that run
            q1 = spx.BatchPlan(As, Ps, tuning=tun, stream=gstream)
            gAPs = q1.execute()
            q2 = spx.BatchPlan(PTs, gAPs, tuning=tun2, stream=gstream)
            q2.execute()
            gAPs = q1.capture()
            gGs = q2.capture()

            def replay():
                q1.replay()
                q2.replay()

            replay()
            gstream.synchronize()
            ok_g = closed_form_ok(gGs)
            t_g = time_steps(replay, 10, gstream.synchronize)
            replay()
            gstream.synchronize()
            ok_g = ok_g and closed_form_ok(gGs)
            q1.close()
            q2.close()
        del gAPs, gGs

        # fused P^T A P: with the aggregation S = P^T, P^T A P = S A S^T, one
        # contraction of the block-diagonal matrix of all instances with the
        # concatenated aggregation maps (A P is never formed)
        n64 = sizes.astype(np.int64)
        fo = np.concatenate([[0], np.cumsum(n64 ** 3)])
        co = np.concatenate([[0], np.cumsum((n64 // 2) ** 3)])
        zo = np.concatenate([[0], np.cumsum([L[int(n)].nnz for n in sizes])])
        dev = torch.device("cuda")
        bd_cp = torch.cat([L[int(n)].cp[:-1] + int(zo[i]) for i, n in enumerate(sizes)]
                          + [torch.tensor([int(zo[-1])], dtype=torch.int64, device=dev)])
        bd_ir = torch.cat([L[int(n)].ir + int(fo[i]) for i, n in enumerate(sizes)])
        bd_num = torch.cat([L[int(n)].num for n in sizes])
        Abd = spx.SpMat(int(fo[-1]), int(fo[-1]), bd_cp, bd_ir, bd_num)

        def agg_of(n):
            v = torch.arange(n ** 3, dtype=torch.int64, device=dev)
            h = n // 2
            return ((v % n) // 2 + h * (((v // n) % n) // 2) + h * h * (v // (n * n) // 2)).to(torch.int32)

        agg = torch.cat([agg_of(int(n)) + int(co[i]) for i, n in enumerate(sizes)])
        nct = int(co[-1])

        def fused():
            q = spx.ContractPlan(Abd, agg, nct, agg, nct)
            G = q.execute()
            q.close()
            return G

        G = fused()
        torch.cuda.synchronize()
        cp_h, ir_h, num_h = G.cp.cpu().numpy(), G.ir.cpu().numpy(), G.num.cpu().numpy()
        ok_f = True
        for i, n in enumerate(sizes):
            ref = W.laplacian7(int(n) // 2, dt)
            c0, c1 = int(co[i]), int(co[i + 1])
            sub_cp = cp_h[c0:c1 + 1] - cp_h[c0]
            sl = slice(int(cp_h[c0]), int(cp_h[c1]))
            ok_f &= bool(np.array_equal(sub_cp, ref.cp) and np.array_equal(ir_h[sl] - c0, ref.ir)
                         and np.array_equal(num_h[sl], 4 * ref.num))
        del G
        t_f = time_steps(fused, 3, torch.cuda.synchronize)
        fmults = int(zo[-1])
        del Abd, bd_cp, bd_ir, bd_num, agg
        out[name] = {"batched_ms": round(1e3 * t_b, 3), "plain_ms": round(1e3 * t_p, 3),
                     "speedup": round(t_p / t_b, 2), "mults": mults,
                     "batched_gflops": round(2 * mults / t_b / 1e9, 2), "closed_form_ok_all": ok,
                     "graph_replay_ms": round(1e3 * t_g, 3), "graph_replay_gflops": round(2 * mults / t_g / 1e9, 2),
                     "graph_replay_closed_form_ok_all": ok_g,
                     "fused_contraction_ms": round(1e3 * t_f, 3), "fused_mults": fmults,
                     "fused_closed_form_ok_all": ok_f,
                     "tuning": {"AP": tinfo["tuning"], "PtAP": tinfo2["tuning"]},
                     "tuning_cached": bool(tinfo["cached"] and tinfo2["cached"])}
        log(f"galerkin {name}: batched {1e3 * t_b:.1f} ms, fused contraction {1e3 * t_f:.1f} ms, "
            f"plain {1e3 * t_p:.1f} ms")
        del L, P, PT, As, Ps, PTs
        torch.cuda.empty_cache()
    return out


def serving(spx, torch, pool_size=256, n_req=5000, discard=500,
            fracs=(0.5, 0.6, 0.7, 0.8, 0.9, 1.0, 1.1, 1.15, 1.2, 1.22, 1.25, 1.28, 1.3, 1.35, 1.4, 1.5, 2.0, 3.0)):
    """Served request stream: plain per-request launches vs continuous
    batching, at offered loads relative to plain's saturation rate.  A pool
    of `pool_size` resident matrices (scales 10-18, about 28 per scale);
    each load point runs `n_req` Poisson arrivals and leaves the first
    `discard` out of the statistics."""
    from paper_1109_3739_amd import serve
    pool = serve.make_pool(pool_size, seed=5)
    store = serve.ResidentStore()
    scales = {}
    for key, (s, M) in enumerate(pool):
        store.add(key, M)
        scales[key] = s
    del pool
    # warm-up of both paths
    for mode in ("plain", "batched"):
        serve.Server(store, mode=mode).run(serve.make_requests(store, scales, 200, 1e6, seed=99))
    sat = serve.Server(store, mode="plain")
    reqs = sat.run(serve.make_requests(store, scales, n_req, 1e6, seed=7))
    plain_max = serve.latency_stats(reqs, skip=discard)["throughput_rps"]
    out = {"pool": f"{pool_size} matrices, scales 10-18, degree 2-16, half R-MAT / half ER",
           "requests_per_point": n_req, "discarded_per_point": discard, "lanes": 3,
           "plain_saturation_rps": plain_max, "points": []}
    for frac in fracs:
        qps = frac * plain_max
        row = {"qps": round(qps, 1), "frac": frac}
        for mode in ("plain", "batched"):
            srv = serve.Server(store, mode=mode)
            reqs = srv.run(serve.make_requests(store, scales, n_req, qps, seed=int(frac * 100)))
            st = serve.latency_stats(reqs, skip=discard)
            st["batches"] = srv.rounds
            st["max_busy_lanes"] = srv.max_busy_lanes
            row[mode] = st
        out["points"].append(row)
        log(f"serving qps={qps:.0f}: plain p99 {row['plain'].get('p99_ms')} ms "
            f"batched p99 {row['batched'].get('p99_ms')} ms")
    out["equal_p99"] = serve.equal_p99_summary(out["points"])
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--extra-only", choices=["latency", "stages", "tall", "index", "restriction", "galerkin",
                                             "serving"],
                    help="run only this group of the other workloads and print its figures")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=4.0, help="seconds per timed run of each CPU leg")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="first run one plain device-to-device copy of BYTES (reference for HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path, run it with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1109_3739_amd as spx
    import workloads as W

    spx.load()
    torch.cuda.set_device(0)
    sync = torch.cuda.synchronize
    gc.collect()
    gc.freeze()
    if args.calibrate_copy:
        x = torch.empty(args.calibrate_copy // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        sync()
        y.copy_(x)
        sync()
        del x, y
        torch.cuda.empty_cache()
    if args.extra_only == "galerkin":
        print(json.dumps({"galerkin": galerkin(spx, W, torch)}), flush=True)
        return
    if args.extra_only == "serving":
        print(json.dumps({"serving": serving(spx, torch)}), flush=True)
        return
    if args.extra_only:
        print(json.dumps({"extra": extra_workloads(spx, W, torch, only=args.extra_only)}), flush=True)
        return
    log("generating R-MAT scale 20")
    A = W.rmat(20, 8, seed=20)
    dA = spx.from_host(A)
    sync()
    gc.collect()
    gc.freeze()

    # warm-up (also sizes the output once)
    p = spx.GemmPlan(dA, dA)
    info = p.info()
    C = p.execute()
    p.close()
    sync()
    for i in range(args.warmup):
        p = spx.GemmPlan(dA, dA)
        p.execute(C)
        p.close()
    sync()
    log(f"warm-up done: mults={info['mults']} nnz(C)={info['nnz']}")

    phase = []

    def step():
        q = spx.GemmPlan(dA, dA, profile=True)
        q.execute(C)
        phase.append(q.times())
        q.close()

    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    sync()
    t_step = (time.perf_counter() - t0) / args.steps
    log(f"timed {args.steps} steps: {1e3 * t_step:.3f} ms/step")

    mults, nnz_c = info["mults"], info["nnz"]
    comp_bytes = 2 * csc_bytes(A.nnz, A.n) + csc_bytes(nnz_c, A.n)
    gflops = 2.0 * mults / t_step / 1e9
    gbs = comp_bytes / t_step / 1e9
    avg = {k: statistics.mean(ph[k] for ph in phase) for k in phase[0]}
    # dominant kernel: the launch over the row-range parts of the heavy
    # columns (it accumulates and writes most of C).  Algorithmic bytes per
    # launch: A and B read once, its share of C written once.
    multi_bytes = 2 * csc_bytes(A.nnz, A.n) + info["nnz_multi"] * 12
    info_wg = spx.default_tuning().part_threads
    multi_s = avg["numeric_multi_ms"] / 1e3
    achieved = multi_bytes / multi_s / 1e9
    roofline = {
        "bound": "hbm",
        "kernel": "k_numeric_parts<0,double> (multi-part launch)",
        "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic_from_profiles(f"void spx::k_numeric_parts_wg{info_wg}"),
        "algorithmic_bytes": int(multi_bytes),
        "avg_launch_ms": round(avg["numeric_multi_ms"], 4),
        "parts": int(info["multi_parts"]),
    }
    result = {
        "metric": METRIC,
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rmat20_AxA_plus_times_f64", "scale": 20, "edge_factor": 8,
                   "rmat": [0.57, 0.19, 0.19, 0.05], "seed": 20, "nnz_a": int(A.nnz), "mults": int(mults),
                   "nnz_c": int(nnz_c), "format": "csc int64 cp / int32 ir / f64"},
        "gbs": round(gbs, 2),
        "compulsory_bytes": int(comp_bytes),
        "phases_ms": {k: round(v, 4) for k, v in avg.items()},
        "roofline": roofline,
    }
    del C
    torch.cuda.empty_cache()
    if not args.no_extra:
        log("other workloads")
        result["extra"] = extra_workloads(spx, W, torch)
        log("batched galerkin")
        result["galerkin"] = galerkin(spx, W, torch)
        log("serving")
        result["serving"] = serving(spx, torch)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, sampled columns, all threads and one thread)")
        result["cpu_baseline"] = cpu_baseline(A, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
