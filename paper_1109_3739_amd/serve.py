"""Request serving over the spx C ABI: continuous batching vs plain launches.

Matrices stay resident in HBM (:class:`ResidentStore`).  Requests are
SpGEMM products ``A*B`` of resident matrices or SpRef extractions
``A(I, J)``.  Two service disciplines run the same requests:

* ``plain``: first come, first served, one request at a time through the
  single-product entry points (``spx_spgemm_plan/exec``,
  ``spx_spref_plan/exec``), synchronising after each.
* ``batched``: continuous batching.  Whenever the device finishes a round,
  every request that has arrived in the meantime is admitted, as long as
  the free slots and the HBM budget (upper bounds of each request's output
  and scratch) allow; the admitted products run as one batch plan (one
  symbolic pass, one persistent numeric launch over all of them) on one
  stream while the admitted SpRef requests run on a second stream, so
  their work overlaps on the device.  Requests that arrive during a round
  join the next one.

Latency of a request = completion time - arrival time (wall clock).  The
admission control never lets the sum of admitted estimates exceed the
budget; a request whose estimate alone exceeds the budget is rejected with
an error status instead of waiting forever.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import List, Optional

import numpy as np

from . import BatchPlan, SpMat, from_host, spgemm, spref

F32_BYTES = 4


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
    status: str = "pending"   # pending / ok / rejected
    est_bytes: int = 0
    result: Optional[SpMat] = None

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

    def add(self, key: int, M) -> None:
        import torch
        d = from_host(M, values=False)
        nnz = int(M.cp[-1])
        self.f32[key] = SpMat(d.m, d.n, d.cp, d.ir, torch.from_numpy(np.asarray(M.num, np.float32)).cuda())
        self.i64[key] = SpMat(d.m, d.n, d.cp, d.ir, torch.arange(nnz, dtype=torch.int64, device="cuda"))
        deg = np.diff(M.cp)
        self.host_meta[key] = (M.m, M.n, deg)
        self.bytes += d.cp.numel() * 8 + nnz * (4 + 4 + 8)

    def mults(self, a: int, b: int) -> int:
        """Multiplications of A*B (an upper bound on nnz(A*B)), cached."""
        if not hasattr(self, "_mc"):
            self._mc, self._irs = {}, {}
        key = (a, b)
        if key not in self._mc:
            if b not in self._irs:
                self._irs[b] = self.f32[b].ir.cpu().numpy()
            da = self.host_meta[a][2]
            self._mc[key] = int(da[self._irs[b]].sum())
        return self._mc[key]


def estimate_bytes(store: ResidentStore, r: Request) -> int:
    """Upper bound of the HBM a request needs while in flight."""
    if r.kind == "spgemm":
        A, B = store.f32[r.a], store.f32[r.b]
        mults = store.mults(r.a, r.b)
        out = mults * (4 + F32_BYTES) + (B.n + 1) * 8
        scratch = B.nnz * 16 + B.n * 64 + A.n * 12 + (1 << 20)
        return out + scratch
    A = store.i64[r.a]
    lenI, lenJ = int(r.I.numel()), int(r.J.numel())
    deg = store.host_meta[r.a][2]
    gathered = int(deg[r.J.cpu().numpy()].sum()) if lenJ else 0
    # every gathered entry is copied once per occurrence of its row in I
    rep = int(np.bincount(r.I.cpu().numpy()).max()) if lenI else 0
    out = gathered * rep * 12 + (lenJ + 1) * 8
    scratch = (A.m + 1) * 12 + max(lenI, 4096) * 24 + lenJ * 48 + (1 << 20)
    return out + scratch


class Server:
    def __init__(self, store: ResidentStore, mode: str = "batched", budget_bytes: int = 64 << 30,
                 max_slots: int = 256, tuning=None):
        import torch
        if mode not in ("plain", "batched"):
            raise ValueError("mode must be plain or batched")
        self.store, self.mode, self.budget, self.max_slots, self.tuning = store, mode, budget_bytes, max_slots, tuning
        self.gemm_stream = torch.cuda.Stream()
        self.ref_stream = torch.cuda.Stream()
        self.max_used = 0
        self.rounds = 0

    # ---- one request / one round ---------------------------------------
    def _run_one(self, r: Request):
        s = self.store
        if r.kind == "spgemm":
            r.result = spgemm(s.f32[r.a], s.f32[r.b])
        else:
            r.result = spref(s.i64[r.a], r.I, r.J)

    def _run_round(self, reqs: List[Request]):
        import torch
        s = self.store
        gem = [r for r in reqs if r.kind == "spgemm"]
        ref = [r for r in reqs if r.kind == "spref"]
        # the batched products go first: their numeric launch is enqueued
        # before the extractions are planned, so the two overlap on the device
        if len(gem) == 1:  # a lone product skips the batch set-up
            with torch.cuda.stream(self.gemm_stream):
                gem[0].result = spgemm(s.f32[gem[0].a], s.f32[gem[0].b])
        elif gem:
            with torch.cuda.stream(self.gemm_stream):
                plan = BatchPlan([s.f32[r.a] for r in gem], [s.f32[r.b] for r in gem], tuning=self.tuning,
                                 stream=self.gemm_stream)
                outs = plan.execute()
                plan.close()
                for r, c in zip(gem, outs):
                    r.result = c
        with torch.cuda.stream(self.ref_stream):
            for r in ref:
                r.result = spref(s.i64[r.a], r.I, r.J)
        self.gemm_stream.synchronize()
        self.ref_stream.synchronize()
        self.rounds += 1

    # ---- request loop ----------------------------------------------------
    def run(self, requests: List[Request], keep_results: bool = False) -> List[Request]:
        import torch
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue: collections.deque = collections.deque()
        for r in pending:
            r.est_bytes = estimate_bytes(self.store, r)
        used = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        while pending or queue:
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            if not queue:
                wait = pending[0].arrival - now()
                if wait > 0:
                    time.sleep(min(wait, 0.002))
                continue
            if self.mode == "plain":
                r = queue.popleft()
                if r.est_bytes > self.budget:
                    r.status, r.done = "rejected", now()
                    continue
                r.start = now()
                self._run_one(r)
                torch.cuda.synchronize()
                r.done, r.status = now(), "ok"
                self.max_used = max(self.max_used, r.est_bytes)
                if not keep_results:
                    r.result = None
                continue
            batch = []
            while queue and len(batch) < self.max_slots:
                r = queue[0]
                if r.est_bytes > self.budget:
                    queue.popleft()
                    r.status, r.done = "rejected", now()
                    continue
                if used + r.est_bytes > self.budget:
                    break
                queue.popleft()
                used += r.est_bytes
                batch.append(r)
            if not batch:
                continue
            self.max_used = max(self.max_used, used)
            ts = now()
            for r in batch:
                r.start = ts
            self._run_round(batch)
            td = now()
            for r in batch:
                r.done, r.status = td, "ok"
                used -= r.est_bytes
                if not keep_results:
                    r.result = None
        return requests


def _best_within(pts: List[dict], target: float) -> dict:
    best = {}
    for mode in ("plain", "batched"):
        ok = [p[mode]["throughput_rps"] for p in pts if p[mode].get("p99_ms", 1e30) <= target]
        best[mode] = max(ok) if ok else None
    ratio = (best["batched"] / best["plain"]) if best.get("plain") and best.get("batched") else None
    return {"p99_target_ms": target, "plain_rps": best["plain"], "batched_rps": best["batched"],
            "batched_over_plain": round(ratio, 3) if ratio else None}


def equal_p99_summary(points: List[dict]) -> dict:
    """Throughput of each mode at equal tail latency, for two p99 targets:
    the plain mode's p99 at the lowest offered load above 0.6 x its
    saturation (moderate load), and its p99 at the load where it reaches
    its highest throughput (saturation).  For each target and mode, the best
    throughput among the load points whose p99 stays within the target."""
    pts = sorted(points, key=lambda p: p["qps"])
    target = None
    for p in pts:
        if p.get("frac", 1.0) >= 0.6:
            target = p["plain"]["p99_ms"]
            break
    if target is None:
        return {}
    out = _best_within(pts, target)
    sat = max(pts, key=lambda p: p["plain"].get("throughput_rps") or 0.0)
    out["saturation"] = _best_within(pts, sat["plain"]["p99_ms"])
    return out


def latency_stats(reqs: List[Request], t_first: float = 0.0) -> dict:
    ok = [r for r in reqs if r.status == "ok"]
    if not ok:
        return {"completed": 0}
    lat = np.array([r.latency for r in ok])
    makespan = max(r.done for r in ok) - min(r.arrival for r in ok)
    return {
        "completed": len(ok),
        "rejected": sum(r.status == "rejected" for r in reqs),
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
        if i % 2 == 0:
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
            I = torch.from_numpy(W.index_vector(L, m, seed=int(rng.integers(1 << 30)))).cuda()
            J = torch.from_numpy(W.index_vector(L, nn, seed=int(rng.integers(1 << 30)))).cuda()
            out.append(Request(rid, "spref", a, I=I, J=J, arrival=t))
        else:
            i, j = rng.choice(len(keys), size=2, replace=len(keys) < 2)
            out.append(Request(rid, "spgemm", keys[i], keys[j], arrival=t))
    return out
