"""Host-side logic of the request loop (no GPU)."""
import numpy as np

from paper_1109_3739_amd.serve import Request, latency_stats


def test_latency_stats():
    reqs = [Request(i, "spgemm", 0, 1, arrival=0.01 * i) for i in range(100)]
    for i, r in enumerate(reqs):
        r.done = r.arrival + 0.001 * (i + 1)
        r.status = "ok"
    reqs[5].status = "rejected"
    st = latency_stats(reqs)
    assert st["completed"] == 99 and st["rejected"] == 1
    lat = np.array([r.latency for r in reqs if r.status == "ok"])
    assert abs(st["p50_ms"] - 1e3 * np.percentile(lat, 50)) < 1e-6
    assert abs(st["p99_ms"] - 1e3 * np.percentile(lat, 99)) < 1e-6


def test_equal_p99_summary():
    from paper_1109_3739_amd.serve import equal_p99_summary
    pts = [
        {"qps": 100, "frac": 0.5, "plain": {"p99_ms": 2.0, "throughput_rps": 100}, "batched": {"p99_ms": 3.0, "throughput_rps": 100}},
        {"qps": 160, "frac": 0.8, "plain": {"p99_ms": 5.0, "throughput_rps": 160}, "batched": {"p99_ms": 4.0, "throughput_rps": 160}},
        {"qps": 400, "frac": 2.0, "plain": {"p99_ms": 90.0, "throughput_rps": 200}, "batched": {"p99_ms": 4.5, "throughput_rps": 390}},
    ]
    s = equal_p99_summary(pts)
    assert s["p99_target_ms"] == 5.0 and s["plain_rps"] == 160 and s["batched_rps"] == 390
    # plain saturates at 200 rps with p99 90 ms; batched serves 390 within it
    sat = s["saturation"]
    assert sat["p99_target_ms"] == 90.0 and sat["plain_rps"] == 200 and sat["batched_rps"] == 390
    assert sat["batched_over_plain"] == 1.95
