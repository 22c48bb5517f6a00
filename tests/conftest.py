import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def load_exact_small():
    """Cases of tests/golden/exact_small.txt as (name, d, e, exact ascending eigenvalues)."""
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", "exact_small.txt")
    with open(path) as f:
        rows = [ln.rstrip("\n") for ln in f if not ln.startswith("#")]
    out = []
    for k in range(0, len(rows), 4):
        name, n = rows[k].split()
        vals = [np.array([float(x) for x in r.split()], dtype=np.float64) for r in rows[k + 1:k + 4]]
        assert len(vals[0]) == int(n) and len(vals[1]) == max(int(n) - 1, 0) and len(vals[2]) == int(n), name
        out.append((name, vals[0], vals[1], vals[2]))
    return out
