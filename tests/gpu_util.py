"""Helpers for the GPU parity tests: tolerances and tensor plumbing."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

# Tolerances (floating point parity, FP32 library vs FP64 oracle on identical inputs):
#  objective U:       |U - U_ref| <= 1e-5 U_ref + 1e-6 sum(w)       (relative, floor near SAT)
#  per-constraint:    |u - u_ref| <= 1e-5 u_ref + 1e-7
#  gradient (vector): ||g - g_ref||_2 <= 1e-5 ||g_ref||_2 + 1e-6 ||S||_2, S_i = sum_c |dU_c/dv_i|
#                     (an FP32 sum of mixed-sign terms is accurate relative to the sum of
#                     magnitudes; the floor is ~8 ulps of it and matters only under cancellation)
#  gradient (coord):  |g_i - g_ref_i| <= 1e-5 * sum_c |dU_c/dv_i| + 4e-7 * max_i sum_c |dU_c/dv_i|
REL = 1e-5

# Every floating-point comparison records its worst error ratio with its floor and without
# it (the relative part alone); the session summary lists the cases that pass only through
# the floor (see conftest.py).
FLOOR_LOG = []


def _record(kind, err, rel_tol, floor):
    """Log (test, kind, worst ratio with the floor, worst ratio of the relative bar alone,
    elements whose reference is (numerically) zero and that differ from it)."""
    import os
    err = np.atleast_1d(np.asarray(err, np.float64))
    rel_tol = np.broadcast_to(np.asarray(rel_tol, np.float64), err.shape)
    floor = np.broadcast_to(np.asarray(floor, np.float64), err.shape)
    with_floor = float(np.max(err / (rel_tol + floor + 1e-300))) if err.size else 0.0
    # the relative bar alone is meaningless where the reference underflows to (almost) zero:
    # those elements are counted apart
    zero_ref = rel_tol <= 1e-30 * np.maximum(floor, 1e-300)
    rel = ~zero_ref & (err > 0)
    without = float(np.max(err[rel] / rel_tol[rel])) if rel.any() else 0.0
    n_zero = int(np.count_nonzero(zero_ref & (err > 0)))
    FLOOR_LOG.append((os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0], kind, with_floor, without, n_zero))


def dev():
    return torch.device("cuda", 0)


def T(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), device=dev(), dtype=dtype)


def assert_objective(U, U_ref, wsum):
    U = np.asarray(U, np.float64)
    err = np.abs(U - U_ref)
    tol = REL * np.abs(U_ref) + 1e-6 * np.asarray(wsum)
    _record("objective", err, REL * np.abs(U_ref), 1e-6 * np.asarray(wsum))
    assert np.all(err <= tol), f"objective: max err {err.max():.3e}, worst ratio {(err / tol).max():.3f}"


def assert_unsat(u, u_ref):
    u = np.asarray(u, np.float64)
    err = np.abs(u - u_ref)
    tol = REL * np.abs(u_ref) + 1e-7
    _record("unsat", err, REL * np.abs(u_ref), 1e-7)
    assert np.all(err <= tol), f"unsat: max err {err.max():.3e}, worst ratio {(err / tol).max():.3f}"


def assert_gradient(g, g_ref, absg, name="grad"):
    g = np.asarray(g, np.float64)
    for r in range(g.shape[0]):
        nrm = np.linalg.norm(g_ref[r])
        floor = 1e-6 * np.linalg.norm(absg[r]) if absg is not None else 0.0
        e = np.linalg.norm(g[r] - g_ref[r])
        _record(name + " (norm)", e, REL * nrm, floor + 1e-12)
        assert e <= REL * nrm + floor + 1e-12, f"{name}[{r}]: ||err|| {e:.3e} vs ||ref|| {nrm:.3e}, floor {floor:.3e}"
        if absg is not None and absg.shape[1] > 0:
            tol = REL * absg[r] + 4e-7 * absg[r].max() + 1e-30
            err = np.abs(g[r] - g_ref[r])
            _record(name + " (coord)", err, REL * absg[r], 4e-7 * absg[r].max() + 1e-30)
            assert np.all(err <= tol), f"{name}[{r}]: coord err ratio {(err / tol).max():.3f}"
