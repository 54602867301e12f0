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
