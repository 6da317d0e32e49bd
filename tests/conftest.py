import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    oracle.lib()
    yield


def pytest_terminal_summary(terminalreporter):
    """Tolerance report of the GPU parity checks: how many comparisons were made, and which
    passed only because of an absolute floor (error above the relative bar alone)."""
    try:
        from gpu_util import FLOOR_LOG
    except Exception:
        return
    if not FLOOR_LOG:
        return
    tr = terminalreporter
    need = [x for x in FLOOR_LOG if x[3] > 1.0]
    worst = max(FLOOR_LOG, key=lambda x: x[2])
    tr.write_line(f"tolerance report: {len(FLOOR_LOG)} floating-point comparisons, worst ratio with floors "
                  f"{worst[2]:.3f} ({worst[0]} {worst[1]}); {len(need)} pass only through a floor")
    by = {}
    for t, k, wf, wo in need:
        key = (t, k)
        by[key] = max(by.get(key, 0.0), wo)
    for (t, k), wo in sorted(by.items(), key=lambda kv: -kv[1])[:40]:
        tr.write_line(f"  floor needed: {t} [{k}] relative-only ratio {wo:.2f}")
