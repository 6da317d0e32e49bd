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
    need = [x for x in FLOOR_LOG if x[3] > 1.0 or x[4] > 0]
    worst = max(FLOOR_LOG, key=lambda x: x[2])
    tr.write_line(f"tolerance report: {len(FLOOR_LOG)} floating-point comparisons, worst ratio with floors "
                  f"{worst[2]:.3f} ({worst[0]} {worst[1]}); {len(need)} pass only through a floor")
    by = {}
    for t, k, wf, wo, nz in need:
        key = (t, k)
        o_wo, o_nz = by.get(key, (0.0, 0))
        by[key] = (max(o_wo, wo), o_nz + nz)
    # kinds summarised over tests: how far past the relative bar alone, and how many
    # differences sit on a reference that underflows to zero
    kinds = {}
    for (t, k), (wo, nz) in by.items():
        n, w, z = kinds.get(k, (0, 0.0, 0))
        kinds[k] = (n + 1, max(w, wo), z + nz)
    for k, (n, w, z) in sorted(kinds.items()):
        tr.write_line(f"  [{k}] {n} tests need the floor: worst relative-only ratio {w:.2f}, "
                      f"{z} elements on a zero reference")
    for (t, k), (wo, nz) in sorted(by.items(), key=lambda kv: -kv[1][0])[:20]:
        tr.write_line(f"  floor needed: {t} [{k}] relative-only ratio {wo:.2f}, zero-reference elements {nz}")
