import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def golden_path(name):
    return os.path.join(ROOT, "tests", "golden", name)


def read_golden_table(name):
    rows = []
    with open(golden_path(name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([float(x) for x in line.split()])
    return rows


def read_golden_kv(name):
    out = {}
    with open(golden_path(name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            out[k] = float(v)
    return out


def dense_kernel(kernel):
    """A kernel dict as the oracle takes it: dense (d, R, N) factor arrays and
    no weights (a rank's weight multiplies its mode-1 column, which gives the
    same C^(d) = sum_r w_r prod_m U_m)."""
    import numpy as np
    out = {}
    for d, v in kernel.items():
        w = None
        if isinstance(v, dict):
            w, v = v.get("weight"), v["U"]
        U = np.array([np.asarray(x, dtype=np.float64) for x in v])
        if w is not None:
            U[0] = U[0] * np.asarray(w, dtype=np.float64)[:, None]
        out[d] = U
    return out


def unweighted_modes(kernel):
    """The factor arrays of a kernel dict without its weights (what the plan's
    integer tables depend on)."""
    import numpy as np
    return {d: np.array([np.asarray(x, dtype=np.float64) for x in (v["U"] if isinstance(v, dict) else v)])
            for d, v in kernel.items()}
