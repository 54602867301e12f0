"""Autotuner for the SpGEMM bin thresholds, part sizes and workgroup sizes.

It times the real entry points (a batch plan + exec, or a single plan +
exec) for a list of candidate :class:`spx_tuning` settings on the caller's
workload and keeps the fastest.  Results are cached in a JSON file keyed by
a workload signature (operation, value type, product count, total products
and output size rounded to powers of two), so a later run with a workload of
the same shape reuses the choice without timing.

Cache file: ``$SPX_AUTOTUNE_CACHE`` or ``~/.cache/spx/autotune.json``.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Callable, Dict, List, Optional

from . import BatchPlan, GemmPlan, default_tuning

# candidate settings (fields of spx_tuning not listed keep their defaults)
CANDIDATES: List[Dict[str, int]] = [
    {},
    {"tiny_max": 32},
    {"single_part_max": 256, "single_threads": 256},
    {"single_part_max": 2048, "single_threads": 512},
    {"hash_count_max": 4096},
    {"part_lds_bytes": 144 * 1024, "part_threads": 1024},
    {"part_lds_bytes": 44 * 1024, "part_threads": 256},
    {"count_threads": 512},
]


def cache_path() -> str:
    return os.environ.get("SPX_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "spx",
                                                             "autotune.json"))


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except Exception:
        return {}


def _save_cache(c: dict) -> None:
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass


def make_tuning(overrides: Dict[str, int]):
    t = default_tuning()
    for k, v in overrides.items():
        setattr(t, k, int(v))
    return t


def signature(kind: str, val_t: int, count: int, mults: int, nnz: int) -> str:
    lg = lambda x: int(math.log2(max(1, x)))  # noqa: E731
    return f"{kind}:v{val_t}:n{lg(count)}:m{lg(mults)}:z{lg(nnz)}"


def _time(fn: Callable[[], None], reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune_batch(As, Bs, semiring: str = "plus_times", candidates: Optional[List[Dict[str, int]]] = None,
               reps: int = 2, use_cache: bool = True):
    """Best tuning for the batch (A_i, B_i); returns (spx_tuning, info dict)."""
    probe = BatchPlan(As, Bs, semiring)
    total_nnz = probe.nnz_total
    probe.close()
    sig = signature("batch", As[0].val_t, len(As), total_nnz, total_nnz)
    cache = _load_cache() if use_cache else {}
    if sig in cache:
        return make_tuning(cache[sig]["tuning"]), {"signature": sig, "cached": True, **cache[sig]}
    results = []
    for cand in candidates or CANDIDATES:
        t = make_tuning(cand)

        def run():
            p = BatchPlan(As, Bs, semiring, tuning=t)
            p.execute()
            p.close()

        try:
            results.append((_time(run, reps), cand))
        except Exception as e:  # a candidate the workload cannot use (e.g. LDS limits)
            results.append((float("inf"), {**cand, "error": str(e)[:80]}))
    best_t, best = min(results, key=lambda x: x[0])
    entry = {"tuning": {k: v for k, v in best.items() if k != "error"}, "seconds": best_t,
             "tried": [{"cand": c, "seconds": s} for s, c in results]}
    if use_cache:
        cache[sig] = entry
        _save_cache(cache)
    return make_tuning(entry["tuning"]), {"signature": sig, "cached": False, **entry}


def tune_single(A, B, semiring: str = "plus_times", candidates: Optional[List[Dict[str, int]]] = None,
                reps: int = 2, use_cache: bool = True):
    """Best tuning for one product A*B; returns (spx_tuning, info dict)."""
    p = GemmPlan(A, B, semiring)
    inf = p.info()
    C = p.execute()
    p.close()
    sig = signature("single", A.val_t, 1, inf["mults"], inf["nnz"])
    cache = _load_cache() if use_cache else {}
    if sig in cache:
        return make_tuning(cache[sig]["tuning"]), {"signature": sig, "cached": True, **cache[sig]}
    results = []
    for cand in candidates or CANDIDATES:
        t = make_tuning(cand)

        def run():
            q = GemmPlan(A, B, semiring, tuning=t)
            q.execute(C)
            q.close()

        try:
            results.append((_time(run, reps), cand))
        except Exception as e:
            results.append((float("inf"), {**cand, "error": str(e)[:80]}))
    best_t, best = min(results, key=lambda x: x[0])
    entry = {"tuning": {k: v for k, v in best.items() if k != "error"}, "seconds": best_t,
             "tried": [{"cand": c, "seconds": s} for s, c in results]}
    if use_cache:
        cache[sig] = entry
        _save_cache(cache)
    return make_tuning(entry["tuning"]), {"signature": sig, "cached": False, **entry}
