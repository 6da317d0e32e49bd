"""GPU test of the allocation-free solver entry point (fsmt_solve_batched_noalloc): two calls
in a row through the C ABI, the second on a smaller input, each against fsmt_solve_batched
on identical inputs (persistent schedule on both sides)."""
import ctypes as ct

import numpy as np
import pytest

import workloads as W

from gpu_util import torch

pytestmark = pytest.mark.gpu
fsmt = pytest.importorskip("paper_2603_22877_amd")
from paper_2603_22877_amd import _abi  # noqa: E402
from paper_2603_22877_amd import solver as S  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cfg(p, levels, steps, cluster=0):
    kap = S.kappa_schedule(p.meta["mean_duration"], levels)
    return S.SolveConfig(kappas=kap, steps_per_level=steps, eta_a=0.5, eta_b=5.0, eps=0.0, stop_on_sat=0,
                         schedule=1, cluster=cluster)


def _run_pair(p, R, levels, steps, seed):
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, R, 77, seed)
    ref = S.BatchState(h, a0, b0)
    got = S.BatchState(h, a0, b0)
    opts, keep = _cfg(p, levels, steps).abi()
    fsmt.fsmt_solve_batched([h], opts, [ref.abi()])
    fsmt.fsmt_solve_batched_noalloc([h], opts, [got.abi()])
    fsmt.fsmt_solve_status([ref.abi(), got.abi()])
    del keep
    return h, ref, got


def _assert_same(ref, got, n_cons):
    # integer work bit-exact; the relaxed point within FP32 rounding of the two runs (their
    # LDS float atomics may add in different orders)
    for k in ("level_done", "steps_done", "n_unsat", "verdict", "sat_bits"):
        np.testing.assert_array_equal(getattr(got, k).cpu().numpy(), getattr(ref, k).cpu().numpy(), err_msg=k)
    for k in ("a", "b"):
        x, y = getattr(got, k).cpu().numpy(), getattr(ref, k).cpu().numpy()
        np.testing.assert_allclose(x, y, rtol=1e-5, atol=1e-5 * (1 + np.abs(y).max()), err_msg=k)
    np.testing.assert_allclose(got.obj.cpu().numpy(), ref.obj.cpu().numpy(), rtol=1e-5, atol=1e-6 * n_cons)
    np.testing.assert_allclose(got.w.cpu().numpy(), ref.w.cpu().numpy(), rtol=2e-5)
    np.testing.assert_allclose(got.hist.cpu().numpy(), ref.hist.cpu().numpy(), rtol=0, atol=0)


def test_noalloc_matches_allocating_call_twice():
    # first call: scheduling 200 x 10, 8 restarts (clusters of workgroups use the partial
    # gradient buffers of the scratch)
    p2 = W.make_workload("scheduling_200x10")
    print("noalloc call 1: scheduling 200 x 10, R=8, 2 levels x 5 steps", flush=True)
    h2, ref, got = _run_pair(p2, 8, 2, 5, 0)
    _assert_same(ref, got, p2.n_cons)
    # second call, smaller input: scheduling 10 x 2, 3 restarts, 3 levels
    p1 = W.make_workload("scheduling_10x2")
    print("noalloc call 2: scheduling 10 x 2, R=3, 3 levels x 20 steps", flush=True)
    h1, ref, got = _run_pair(p1, 3, 3, 20, 1)
    _assert_same(ref, got, p1.n_cons)
    h1.free()
    h2.free()


def test_noalloc_rejects_what_it_cannot_run():
    p = W.make_workload("scheduling_200x10")
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, 4, 77, 2)
    st = S.BatchState(h, a0, b0)
    opts, keep = _cfg(p, 1, 1).abi()
    opts.schedule = 2   # the grid schedule allocates; the allocation-free call refuses it
    with pytest.raises(fsmt.FsmtError) as e:
        fsmt.fsmt_solve_batched_noalloc([h], opts, [st.abi()])
    assert e.value.code == _abi.FSMT_EUNSUPPORTED
    # a call whose cluster partials exceed the scratch: 320 restarts x 2 workgroups x 2
    # buffers x (n + m + 1) floats is past FSMT_NOALLOC_SCRATCH_BYTES
    R = 320
    need = R * 2 * 2 * (p.n_bool + p.n_real + 1) * 4
    assert need > (8 << 20)
    a0, b0 = W.initial_points(p, R, 77, 3)
    big = S.BatchState(h, a0, b0)
    opts, keep2 = _cfg(p, 1, 1, cluster=2).abi()
    with pytest.raises(fsmt.FsmtError) as e:
        fsmt.fsmt_solve_batched_noalloc([h], opts, [big.abi()])
    # refused before launching: either the scratch bound or, on a device that cannot hold
    # all 640 workgroups at once, the co-residency of the clusters
    assert e.value.code in (_abi.FSMT_ELIMIT, _abi.FSMT_EUNSUPPORTED), str(e.value)
    if e.value.code == _abi.FSMT_ELIMIT:
        assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert int(big.level_done.max()) == 0 and int(big.steps_done.max()) == 0
    del keep, keep2
    h.free()
