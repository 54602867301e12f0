"""Request serving over the spx C ABI: continuous batching vs plain launches.

Matrices stay resident in HBM (:class:`ResidentStore`).  Requests are
SpGEMM products ``A*B`` of resident matrices or SpRef extractions
``A(I, J)``.  Two service disciplines run the same requests:

* ``plain``: first come, first served, one request at a time through the
  single-product entry points (``spx_spgemm_plan/exec``,
  ``spx_spref_plan/exec``) on one stream, synchronising after each.
* ``batched``: continuous batching over several device lanes.  A lane is a
  HIP stream with a host worker thread; it runs one batch at a time: the
  batch's products as one batch plan (one symbolic pass over all of them,
  persistent numeric launches), then its extractions.  Whenever a lane is
  idle and requests are queued, the dispatcher admits queued requests in
  arrival order into a new batch for that lane, as long as the free slots
  and the HBM budget allow, while the other lanes' batches are still on the
  device: requests that arrive while others run are admitted as soon as a
  lane frees up, and the batches of different lanes overlap on the GPU.  A
  completion event is recorded after each request's work (after the
  product batch for its products, after each extraction); the lane thread
  waits on these events in order and releases each request's slot and
  budget share as soon as its own event has fired.

The library's plan calls synchronise their stream to read back output
sizes; a lane thread blocks there while the dispatcher and the other lanes
go on (the foreign calls release Python's interpreter lock).

Admission uses upper bounds of the device memory each request takes while
in flight (:func:`estimate_bytes`): its output, bounded by the number of
multiplications (products) or of gathered entries times the largest
repetition of a row index (extractions), plus every scratch buffer the
plan may draw from the context's allocator.  The sum of the admitted
bounds never exceeds the budget, so neither does the memory actually drawn;
a request whose bound alone exceeds the budget is rejected with an error
status instead of waiting forever.

Latency of a request = completion time - arrival time (wall clock).
"""
from __future__ import annotations

import collections
import dataclasses
import queue as queue_mod
import threading
import time
from typing import List, Optional

import numpy as np

from . import BatchPlan, SpMat, from_host, spgemm, spref

F32_BYTES = 4
ARENA = 2 << 20        # small scratch buffers share blocks of this size
ALLOC_SLACK = 1 << 20  # rounding of the caching allocator, per request


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                 # "spgemm" or "spref"
    a: int                    # store id of A
    b: int = -1               # store id of B (spgemm)
    I: Optional[object] = None  # device int32 (spref)
    J: Optional[object] = None
    arrival: float = 0.0      # seconds after the start of the run
    start: float = -1.0
    done: float = -1.0
    status: str = "pending"   # pending / ok / rejected / failed
    est_bytes: int = 0
    result: Optional[SpMat] = None
    I_host: Optional[np.ndarray] = None
    J_host: Optional[np.ndarray] = None
    error: str = ""

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class ResidentStore:
    """Matrices kept on the device: FP32 values for products, int64 edge ids
    for extraction (sharing the pattern tensors)."""

    def __init__(self):
        self.f32 = {}
        self.i64 = {}
        self.host_meta = {}
        self.bytes = 0
        self._mc = {}
        self._irs = {}
        self.max_m = 0

    def add(self, key: int, M) -> None:
        import torch
        d = from_host(M, values=False)
        nnz = int(M.cp[-1])
        self.f32[key] = SpMat(d.m, d.n, d.cp, d.ir, torch.from_numpy(np.asarray(M.num, np.float32)).cuda())
        self.i64[key] = SpMat(d.m, d.n, d.cp, d.ir, torch.arange(nnz, dtype=torch.int64, device="cuda"))
        deg = np.diff(np.asarray(M.cp, dtype=np.int64))
        self.host_meta[key] = (M.m, M.n, deg)
        self.max_m = max(self.max_m, int(M.m))
        self._irs[key] = np.asarray(M.ir)
        self.bytes += d.cp.numel() * 8 + nnz * (4 + 4 + 8)

    def mults(self, a: int, b: int) -> int:
        """Multiplications of A*B (an upper bound on nnz(A*B)), cached."""
        key = (a, b)
        if key not in self._mc:
            self._mc[key] = int(self.host_meta[a][2][self._irs[b]].sum())
        return self._mc[key]


def _row_blocks(m: int, value_bytes: int, part_lds: int = 72 * 1024) -> int:
    """Row blocks of the SpGEMM plan for m rows (the largest power of two
    of rows, at most 2^14, whose dense block fits one part)."""
    rb = 14
    while rb > 6 and (1 << rb) * value_bytes + ((1 << rb) // 64) * 10 + 256 > part_lds:
        rb -= 1
    return max(1, -(-m // (1 << rb)))


def gemm_bytes(m: int, k: int, n: int, nnz_a: int, nnz_b: int, mults: int, value_bytes: int = F32_BYTES,
               bitmap_store_mb: int = 32768) -> int:
    """Upper bound of the device memory of C = A*B (A m x k, B k x n CSC,
    default tuning), alone or as one product of a batch whose left operands
    have at most m rows: the output (CSC, int64 pointers), the batch's
    concatenated copies of A and B, and every scratch buffer the plan may
    take (per-entry range data of B, per-column counts and offsets, the
    split table of A's long columns, row-block counts, the stored row
    bitmaps, part descriptors and the bucket lists)."""
    nblk = _row_blocks(m, value_bytes)
    heavy = min(n, mults // 1024 + 1)        # columns cut into row ranges
    counted = min(n, mults // 8192 + 1)      # bitmap-counted columns
    parts = min(max(mults, 1), n * nblk)     # every part holds at least one output
    out = (n + 1) * 8 + mults * (4 + value_bytes)
    concat = (4 + value_bytes) * (nnz_a + nnz_b) + 8 * (k + n + 2)
    scratch = (16 * nnz_b + 64 * (n + 1)
               + 8 * (k + 1) + 4 * (nnz_a // 33 + 1) * (nblk + 3)
               + 4 * heavy * nblk
               + min(counted * ((m + 63) // 64) * 8, bitmap_store_mb << 20)
               + 2 * 48 * parts
               + 4 * heavy * nblk + 16 * parts + 4 * mults
               + 64 * ((max(n, k) + 2047) // 2048 + 64))
    return out + concat + scratch + 2 * ARENA + ALLOC_SLACK


def spref_bytes(m: int, len_i: int, len_j: int, gathered: int, rep: int, value_bytes: int = 8) -> int:
    """Upper bound of the device memory of B = A(I, J): the output and the
    plan's scratch (row histogram and pointers, sorted positions of I, the
    per-column data of J)."""
    cap = 1024
    while cap < len_i:
        cap <<= 1
    out = (len_j + 1) * 8 + gathered * rep * (4 + value_bytes)
    scratch = 12 * (m + 1) + 4 * len_i + 8 * cap + 40 * (len_j + 1) + 64 * ((m + 2047) // 2048 + 64)
    return out + scratch + ARENA + ALLOC_SLACK


def estimate_bytes(store: ResidentStore, r: Request) -> int:
    """Upper bound of the HBM a request takes while in flight."""
    if r.kind == "spgemm":
        A, B = store.f32[r.a], store.f32[r.b]
        # in a batch the left operands are stacked to the tallest one's rows
        return gemm_bytes(max(A.m, store.max_m), A.n, B.n, A.nnz, B.nnz, store.mults(r.a, r.b))
    m = store.host_meta[r.a][0]
    deg = store.host_meta[r.a][2]
    Ih = r.I_host if r.I_host is not None else r.I.cpu().numpy()
    Jh = r.J_host if r.J_host is not None else r.J.cpu().numpy()
    gathered = int(deg[Jh].sum()) if Jh.size else 0
    rep = int(np.bincount(Ih).max()) if Ih.size else 0
    return spref_bytes(m, int(Ih.size), int(Jh.size), gathered, rep)


class _Lane:
    """A device lane: one HIP stream and one host worker thread."""

    def __init__(self, server: "Server", idx: int):
        import torch
        self.server, self.idx = server, idx
        self.stream = torch.cuda.Stream()
        self.inbox: "queue_mod.Queue" = queue_mod.Queue()
        self.busy = False
        self.thread = threading.Thread(target=self._loop, name=f"spx-lane-{idx}", daemon=True)
        self.thread.start()

    def _loop(self):
        import torch
        srv = self.server
        while True:
            batch = self.inbox.get()
            if batch is None:
                return
            events = []
            try:
                with torch.cuda.stream(self.stream):
                    events = srv._launch(batch, self.stream)
            except Exception as e:  # reported per request; the lane stays usable
                for r in batch:
                    r.status, r.error = "failed", str(e)[:200]
                events = [(batch, None)]
            for reqs, ev in events:
                if ev is not None:
                    ev.synchronize()
                td = srv.now()
                for r in reqs:
                    r.done = td
                    if r.status == "pending":
                        r.status = "ok"
                    if not srv.keep_results:
                        r.result = None
                srv.done_q.put((self.idx, reqs, False))
            srv.done_q.put((self.idx, [], True))


class Server:
    def __init__(self, store: ResidentStore, mode: str = "batched", budget_bytes: int = 64 << 30,
                 max_slots: int = 256, tuning=None, lanes: int = 3):
        import torch
        if mode not in ("plain", "batched"):
            raise ValueError("mode must be plain or batched")
        self.store, self.mode, self.budget, self.max_slots, self.tuning = store, mode, budget_bytes, max_slots, tuning
        self.stream = torch.cuda.Stream()
        self.nlanes = max(1, int(lanes))
        self.max_used = 0
        self.rounds = 0          # batches launched
        self.max_inflight = 0    # most requests in flight at once
        self.max_busy_lanes = 0  # most lanes busy at once
        self.keep_results = False
        self.done_q: "queue_mod.Queue" = queue_mod.Queue()
        self._t0 = 0.0

    def now(self) -> float:
        return time.perf_counter() - self._t0

    # ---- work of one request / one batch --------------------------------
    def _run_one(self, r: Request):
        s = self.store
        if r.kind == "spgemm":
            r.result = spgemm(s.f32[r.a], s.f32[r.b])
        else:
            r.result = spref(s.i64[r.a], r.I, r.J)

    def _launch(self, batch: List[Request], stream):
        """Enqueue a batch on `stream` (the current stream); returns the
        (requests, completion event) pairs in completion order."""
        import torch
        s = self.store
        gem = [r for r in batch if r.kind == "spgemm"]
        ref = [r for r in batch if r.kind == "spref"]
        events = []
        if len(gem) == 1:  # a lone product skips the batch set-up
            gem[0].result = spgemm(s.f32[gem[0].a], s.f32[gem[0].b])
        elif gem:
            plan = BatchPlan([s.f32[r.a] for r in gem], [s.f32[r.b] for r in gem], tuning=self.tuning,
                             stream=stream)
            try:
                outs = plan.execute()
            finally:
                plan.close()
            for r, c in zip(gem, outs):
                r.result = c
        if gem:
            ev = torch.cuda.Event()
            ev.record(stream)
            events.append((gem, ev))
        for r in ref:
            r.result = spref(s.i64[r.a], r.I, r.J)
            ev = torch.cuda.Event()
            ev.record(stream)
            events.append(([r], ev))
        return events

    # ---- request loops ---------------------------------------------------
    def run(self, requests: List[Request], keep_results: bool = False) -> List[Request]:
        """Serve `requests` (arrival times relative to the start).  The
        interpreter's cyclic garbage collector is paused meanwhile, as serving
        loops do: a full collection stops every thread for milliseconds and
        would land in the latency tail (reference counting still frees the
        requests' buffers as they complete)."""
        import gc
        import torch
        self.keep_results = keep_results
        for r in requests:
            r.est_bytes = estimate_bytes(self.store, r)
        torch.cuda.synchronize()
        was_enabled = gc.isenabled()
        gc.collect()
        gc.disable()
        try:
            self._t0 = time.perf_counter()
            if self.mode == "plain":
                self._run_plain(requests)
            else:
                self._run_batched(requests)
        finally:
            if was_enabled:
                gc.enable()
        return requests

    def _run_plain(self, requests: List[Request]):
        import torch
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue: collections.deque = collections.deque()
        with torch.cuda.stream(self.stream):
            while pending or queue:
                t = self.now()
                while pending and pending[0].arrival <= t:
                    queue.append(pending.popleft())
                if not queue:
                    wait = pending[0].arrival - self.now()
                    if wait > 0:
                        time.sleep(min(wait, 0.002))
                    continue
                r = queue.popleft()
                if r.est_bytes > self.budget:
                    r.status, r.done = "rejected", self.now()
                    continue
                r.start = self.now()
                try:
                    self._run_one(r)
                    self.stream.synchronize()
                    r.status = "ok"
                except Exception as e:  # reported on the request; the loop goes on
                    r.status, r.error, r.result = "failed", str(e)[:200], None
                r.done = self.now()
                self.max_used = max(self.max_used, r.est_bytes)
                self.max_inflight = max(self.max_inflight, 1)
                if not self.keep_results:
                    r.result = None

    def _run_batched(self, requests: List[Request]):
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue: collections.deque = collections.deque()
        lanes = [_Lane(self, i) for i in range(self.nlanes)]
        used, inflight = 0, 0
        stalled = False  # the last admission attempt found no budget or slot
        try:
            while pending or queue or inflight:
                # completions first: they free slots, budget and lanes; wait
                # for one unless a lane could take queued work right now
                try:
                    block = stalled or not queue or all(ln.busy for ln in lanes)
                    timeout = 0.0005
                    if pending:
                        timeout = max(0.0, min(timeout if inflight else 0.002, pending[0].arrival - self.now()))
                    elif not queue:
                        timeout = 0.005
                    if block and timeout > 0:
                        item = self.done_q.get(timeout=timeout)
                    else:
                        item = self.done_q.get_nowait()
                    stalled = False
                    while True:
                        li, reqs, idle = item
                        if idle:
                            lanes[li].busy = False
                        for r in reqs:
                            used -= r.est_bytes
                            inflight -= 1
                        item = self.done_q.get_nowait()
                except queue_mod.Empty:
                    pass
                t = self.now()
                while pending and pending[0].arrival <= t:
                    queue.append(pending.popleft())
                free = [ln for ln in lanes if not ln.busy]
                if not queue or not free:
                    continue
                batch = []
                while queue and inflight + len(batch) < self.max_slots:
                    r = queue[0]
                    if r.est_bytes > self.budget:
                        queue.popleft()
                        r.status, r.done = "rejected", self.now()
                        continue
                    if used + r.est_bytes > self.budget:
                        break
                    queue.popleft()
                    used += r.est_bytes
                    batch.append(r)
                if not batch:
                    stalled = bool(queue)
                    continue
                inflight += len(batch)
                self.max_used = max(self.max_used, used)
                self.max_inflight = max(self.max_inflight, inflight)
                ts = self.now()
                for r in batch:
                    r.start = ts
                # the admitted requests go to every idle lane: the heaviest
                # first, each to the lane with the least work so far (by the
                # requests' HBM estimates), keeping arrival order in a lane
                k = min(len(free), len(batch))
                parts: List[List[Request]] = [[] for _ in range(k)]
                load = [0] * k
                for r in sorted(batch, key=lambda r: -r.est_bytes):
                    i = load.index(min(load))
                    parts[i].append(r)
                    load[i] += r.est_bytes
                for lane, part in zip(free, parts):
                    part.sort(key=lambda r: r.arrival)
                    lane.busy = True
                    self.rounds += 1
                    lane.inbox.put(part)
                self.max_busy_lanes = max(self.max_busy_lanes, sum(ln.busy for ln in lanes))
        finally:
            for ln in lanes:
                ln.inbox.put(None)
            for ln in lanes:
                ln.thread.join()


def _best_within(pts: List[dict], target: float) -> dict:
    best = {}
    for mode in ("plain", "batched"):
        ok = [p[mode]["throughput_rps"] for p in pts if p[mode].get("p99_ms", 1e30) <= target]
        best[mode] = max(ok) if ok else None
    ratio = (best["batched"] / best["plain"]) if best.get("plain") and best.get("batched") else None
    return {"p99_target_ms": target, "plain_rps": best["plain"], "batched_rps": best["batched"],
            "batched_over_plain": round(ratio, 3) if ratio else None}


def equal_p99_summary(points: List[dict], frac: float = 0.8) -> dict:
    """Throughput of each mode at equal tail latency, for two p99 targets:
    the plain mode's p99 at the offered load closest to `frac` x its
    saturation (moderate load), and its p99 at the load where it reaches its
    highest throughput (saturation).  For each target and mode, the best
    throughput among the load points whose p99 stays within the target."""
    pts = sorted(points, key=lambda p: p["qps"])
    if not pts:
        return {}
    ref = min(pts, key=lambda p: abs(p.get("frac", 1.0) - frac))
    target = ref["plain"].get("p99_ms")
    if target is None:
        return {}
    out = _best_within(pts, target)
    sat = max(pts, key=lambda p: p["plain"].get("throughput_rps") or 0.0)
    out["saturation"] = _best_within(pts, sat["plain"]["p99_ms"])
    return out


def latency_stats(reqs: List[Request], skip: int = 0) -> dict:
    """p50 / p99 / mean latency and throughput of the completed requests,
    leaving out the first `skip` requests by arrival (warm-up)."""
    ordered = sorted(reqs, key=lambda r: r.arrival)[skip:]
    ok = [r for r in ordered if r.status == "ok"]
    if not ok:
        return {"completed": 0}
    lat = np.array([r.latency for r in ok])
    makespan = max(r.done for r in ok) - min(r.arrival for r in ok)
    return {
        "completed": len(ok),
        "rejected": sum(r.status == "rejected" for r in ordered),
        "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
        "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
        "mean_ms": round(1e3 * float(lat.mean()), 3),
        "throughput_rps": round(len(ok) / makespan, 2) if makespan > 0 else None,
    }


# ---- workload ------------------------------------------------------------------
def make_pool(count: int, seed: int, scales=range(10, 19), degrees=range(2, 17)):
    """`count` matrices (about evenly over the scales), half R-MAT, half
    Erdos-Renyi, degree uniform in `degrees`, each independently permuted
    (R-MAT) or uniform (ER); FP32 values uniform [0, 1)."""
    import workloads as W
    rng = np.random.default_rng(seed)
    scales = list(scales)
    pool = []
    for i in range(count):
        s = scales[i % len(scales)]
        d = int(rng.integers(min(degrees), max(degrees) + 1))
        sd = int(rng.integers(1 << 30))
        if (i // len(scales)) % 2 == 0:
            M = W.rmat(s, d, seed=sd, values="f32")
        else:
            M = W.erdos_renyi(1 << s, 1 << s, d, seed=sd, values="f32")
        pool.append((s, M))
    return pool


def make_requests(store: ResidentStore, pool_scales, n: int, qps: float, seed: int, spref_frac: float = 0.5):
    """Poisson arrivals at `qps`; (1 - spref_frac) FP32 products of two
    distinct pool matrices of one scale, spref_frac int64 extractions with
    len(I) = len(J) = n/16 and 10% repeated indices."""
    import torch
    import workloads as W
    rng = np.random.default_rng(seed)
    by_scale = collections.defaultdict(list)
    for key, s in pool_scales.items():
        by_scale[s].append(key)
    scales = sorted(by_scale)
    t = 0.0
    out = []
    for rid in range(n):
        t += rng.exponential(1.0 / qps)
        s = scales[int(rng.integers(len(scales)))]
        keys = by_scale[s]
        if rng.random() < spref_frac:
            a = keys[int(rng.integers(len(keys)))]
            m, nn, _ = store.host_meta[a]
            L = max(1, m // 16)
            Ih = W.index_vector(L, m, seed=int(rng.integers(1 << 30)))
            Jh = W.index_vector(L, nn, seed=int(rng.integers(1 << 30)))
            out.append(Request(rid, "spref", a, I=torch.from_numpy(Ih).cuda(), J=torch.from_numpy(Jh).cuda(),
                               arrival=t, I_host=Ih, J_host=Jh))
        else:
            i, j = rng.choice(len(keys), size=2, replace=len(keys) < 2)
            out.append(Request(rid, "spgemm", keys[i], keys[j], arrival=t))
    return out
