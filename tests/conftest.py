import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def spx():
    """The HIP library binding (GPU tests only)."""
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_1109_3739_amd as spx_mod
    spx_mod.load()  # raises if the HIP library is missing
    return spx_mod


def read_golden(name):
    """Parse a tests/golden/*.txt fixture: '# ...' comments, 'KEY v1 v2 ...' lines."""
    out, rows = {}, []
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0][0].isalpha():
                out[parts[0]] = parts[1:]
            else:
                rows.append(parts)
    if rows:
        out["_rows"] = rows
    return out
