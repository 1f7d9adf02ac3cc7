import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for p in (ROOT, os.path.join(ROOT, "oracle")):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds")


def relerr(a, ref):
    """Normwise relative error ||a - ref|| / ||ref|| in float64."""
    import numpy as np
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.linalg.norm(ref)
    num = np.linalg.norm(a - ref)
    return num / den if den > 0 else num


def maxerr(a, ref):
    """Max-scaled element-wise error max|a - ref| / max|ref| in float64."""
    import numpy as np
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.max(np.abs(ref)) if ref.size else 0.0
    num = np.max(np.abs(a - ref)) if ref.size else 0.0
    return num / den if den > 0 else num


def check(label, err, tol, floor=None, factor=3.0, literal=False):
    """Assert err <= gate and print the error reached, the gate and the floor.

    The gate is the tolerance itself (no floor given, or literal=True: the
    floor is then only printed), or max(tol, factor x floor), the floor being
    the error of the oracle's rounding model on the same inputs."""
    gate = tol if (floor is None or literal) else max(tol, factor * floor)
    fl = "" if floor is None else f" floor {floor:.3e}"
    print(f"[parity] {label}: err {err:.3e} gate {gate:.1e}{fl}", flush=True)
    assert err <= gate, f"{label}: error {err:.3e} above gate {gate:.3e}{fl}"
