"""GPU parity on the large workloads where the full oracle is too slow: sampled gradient
coordinates (every constraint that touches a variable gives its exact partial derivative),
fused solver steps on the uneven batch and on the paper-scale placement instance, and the
projection's edge cases (a zero coefficient in a half-space, a half-space that misses the
box)."""
import numpy as np
import pytest

import oracle
import workloads as W

from gpu_util import T, assert_objective, dev, torch

pytestmark = pytest.mark.gpu
fsmt = pytest.importorskip("paper_2603_22877_amd")
from paper_2603_22877_amd import solver as S  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def touching(p, boolean=(), real=()):
    """Constraints whose support contains one of the given Boolean or real variables."""
    lit_id = p.con_lit >> 1
    con_of_lit = np.repeat(np.arange(p.n_cons), np.diff(p.con_ptr))
    hit = np.zeros(p.n_cons, bool)
    if len(boolean):
        hit[con_of_lit[np.isin(lit_id, boolean)]] = True
    if len(real):
        atom_of_nnz = np.repeat(np.arange(len(p.atom_rhs)), np.diff(p.atom_ptr))
        atoms = np.unique(atom_of_nnz[np.isin(p.atom_var, real)])
        hit[con_of_lit[np.isin(lit_id, p.n_bool + atoms)]] = True
    return np.nonzero(hit)[0].astype(np.int32)


def assert_sampled_gradient(op, p, a, b, kap, ga, gb, bools, reals, w=None):
    """ga, gb at the given coordinates against the oracle's partial derivatives over the
    constraints that touch them (the others contribute nothing), coordinate bar of Q12."""
    sel = touching(p, bools, reals)
    o = oracle.objective(op, a, b, kap, w=w, sel=sel, per_constraint=False)
    for r in range(a.shape[0]):
        # coordinate bar: 1e-5 S_i + 4e-7 max S, the max taken over the sampled coordinates
        # of the block (a lower bound of the maximum over all of them)
        fa = 4e-7 * (o["absg_a"][r, bools].max() if len(bools) else 0.0)
        fb = 4e-7 * (o["absg_b"][r, reals].max() if len(reals) else 0.0)
        for i in bools:
            ref, s = o["grad_a"][r, i], o["absg_a"][r, i]
            assert abs(ga[r, i] - ref) <= 1e-5 * s + fa + 1e-12, ("a", r, i, ga[r, i], ref, s)
        for j in reals:
            ref, s = o["grad_b"][r, j], o["absg_b"][r, j]
            assert abs(gb[r, j] - ref) <= 1e-5 * s + fb + 1e-12, ("b", r, j, gb[r, j], ref, s)
    return o


def _pick(p, rng, nb, nr):
    bools = rng.choice(p.n_bool, min(nb, p.n_bool), replace=False) if p.n_bool else np.zeros(0, int)
    reals = rng.choice(p.n_real, min(nr, p.n_real), replace=False)
    return np.sort(bools), np.sort(reals)


def test_uneven_batch_sampled_gradients():
    """Uneven batch: cop_backward of every instance (16 restarts, row-major), sampled Boolean
    and real coordinates of each against the oracle."""
    probs = W.uneven_batch()
    rng = np.random.default_rng(41)
    R = 16
    for i, p in enumerate(probs):
        op = oracle.OracleProblem(p)
        h = fsmt.xbdd_compile(p)
        a, b = W.initial_points(p, R, 4, i)
        kap = 0.5 / p.meta.get("mean_duration", p.meta.get("mean_side", 1.0))
        ga = torch.zeros(R, p.n_bool, device=dev())
        gb = torch.zeros(R, p.n_real, device=dev())
        obj = torch.zeros(R, device=dev())
        fsmt.cop_backward(h, T(a), T(b), kap, T(np.ones(p.n_cons)), obj, ga, gb)
        torch.cuda.synchronize()
        bools, reals = _pick(p, rng, 3, 3)
        print(f"uneven batch instance {i} {p.meta['family']} C={p.n_cons}: booleans {bools.tolist()} "
              f"reals {reals.tolist()}", flush=True)
        assert_sampled_gradient(op, p, a, b, kap, ga.cpu().numpy(), gb.cpu().numpy(), bools, reals)
        h.free()


def test_one_restart_gradient_both_paths():
    """cop_backward at one restart on the uneven batch's instances: those whose n + m fits
    the per-workgroup LDS gradient take that path, the larger ones the device-atomic path;
    sampled coordinates of both against the oracle, and the objective."""
    probs = W.uneven_batch()
    picks = [i for i, p in enumerate(probs) if p.n_bool + p.n_real <= 8192][:3]
    picks += [i for i, p in enumerate(probs) if p.n_bool + p.n_real > 8192][:2]
    rng = np.random.default_rng(43)
    for i in picks:
        p = probs[i]
        op = oracle.OracleProblem(p)
        h = fsmt.xbdd_compile(p)
        a, b = W.initial_points(p, 1, 4, 100 + i)
        kap = 0.5 / p.meta.get("mean_duration", p.meta.get("mean_side", 1.0))
        ga = torch.zeros(1, p.n_bool, device=dev())
        gb = torch.zeros(1, p.n_real, device=dev())
        obj = torch.zeros(1, device=dev())
        fsmt.cop_backward(h, T(a), T(b), kap, T(np.ones(p.n_cons)), obj, ga, gb)
        torch.cuda.synchronize()
        bools, reals = _pick(p, rng, 4, 4)
        print(f"one restart, instance {i} {p.meta['family']} n+m={p.n_bool + p.n_real} C={p.n_cons}", flush=True)
        assert_sampled_gradient(op, p, a, b, kap, ga.cpu().numpy(), gb.cpu().numpy(), bools, reals)
        o = oracle.objective(op, a, b, kap, grad=False, per_constraint=False)
        assert_objective(obj.cpu().numpy(), o["U"], float(p.n_cons))
        h.free()


def test_uneven_batch_fused_step_sampled_instances():
    """One fused step of the whole uneven batch (persistent and grid schedules in one call):
    on the smaller instances of each family, the step against the oracle's projected step
    from its FP64 gradient, the objective at the start point, and the exact check at the
    GPU's post-step point."""
    probs = W.uneven_batch()
    R = 16
    hs = [fsmt.xbdd_compile(p) for p in probs]
    init = [W.initial_points(p, R, 44, i) for i, p in enumerate(probs)]
    states = [S.BatchState(h, a, b) for h, (a, b) in zip(hs, init)]
    ell = min(p.meta.get("mean_duration", p.meta.get("mean_side", 1.0)) for p in probs)
    kap, eta_a, eta_b = 0.5 / ell, 0.5, 5.0
    cfg = S.SolveConfig(kappas=[kap], steps_per_level=1, eta_a=eta_a, eta_b=eta_b, eps=0.0, stop_on_sat=0)
    S.solve_batched(hs, states, cfg)
    S.check_batched(states)
    fams = {}
    for i, p in enumerate(probs):
        fams.setdefault(p.meta["family"], []).append(i)
    picked = []
    for fam, ids in fams.items():
        ids = sorted(ids, key=lambda i: probs[i].n_cons)
        picked += ids[:2]
    for i in picked:
        p, (a0, b0), st = probs[i], init[i], states[i]
        print(f"uneven batch fused step: instance {i} {p.meta['family']} C={p.n_cons}", flush=True)
        o = oracle.objective(p, a0, b0, kap, per_constraint=False)
        ref = oracle.pgd(p, a0, b0, o["grad_a"].astype(np.float32), o["grad_b"].astype(np.float32), eta_a, eta_b)
        a1, b1 = st.a.cpu().numpy(), st.b.cpu().numpy()
        for r in range(R):
            tol_a = eta_a * (1e-5 * o["absg_a"][r] + 4e-7 * o["absg_a"][r].max()) + 3e-7 * (1 + np.abs(ref["a"][r]))
            assert np.all(np.abs(a1[r] - ref["a"][r]) <= tol_a), np.abs(a1[r] - ref["a"][r]).max()
            tol_b = eta_b * (1e-5 * o["absg_b"][r] + 4e-7 * o["absg_b"][r].max()) + 2e-6 * (1 + np.abs(ref["b"][r]))
            assert np.all(np.abs(b1[r] - ref["b"][r]) <= tol_b), np.abs(b1[r] - ref["b"][r]).max()
        assert_objective(st.obj.cpu().numpy(), o["U"], p.n_cons)
        ch = oracle.check(p, a1, b1)
        np.testing.assert_array_equal(st.sat_bits.cpu().numpy().view(np.uint32), ch["sat_bits"])
        np.testing.assert_array_equal(st.n_unsat.cpu().numpy(), ch["n_unsat"])
    for h in hs:
        h.free()


@pytest.mark.parametrize("R", [1, 16])
def test_placement1200_per_call_sampled(R):
    """Paper-scale placement per call (cop_backward), where the large-instance gradient
    paths run: at one restart the gradient summed per workgroup in LDS and added from one
    row per CU, at 16 the restart-contiguous stage. Sampled rectangles (rotation bit and
    both coordinates) against the oracle's partial derivatives, and a second call with
    FSMT_ACCUMULATE doubling them."""
    p = W.make_workload("placement_1200")
    op = oracle.OracleProblem(p)
    h = fsmt.xbdd_compile(p)
    a, b = W.initial_points(p, R, 5, 11)
    kap = 1.0 / p.meta["mean_side"]
    ga = torch.zeros(R, p.n_bool, device=dev())
    gb = torch.zeros(R, p.n_real, device=dev())
    obj = torch.zeros(R, device=dev())
    wt = T(np.ones(p.n_cons))
    fsmt.cop_backward(h, T(a), T(b), kap, wt, obj, ga, gb)
    torch.cuda.synchronize()
    rng = np.random.default_rng(47)
    rects = np.sort(rng.choice(p.n_bool, 4, replace=False))
    print(f"placement 1200 per call R={R}: rectangles {rects.tolist()}", flush=True)
    g1a, g1b, o1 = ga.cpu().numpy().copy(), gb.cpu().numpy().copy(), obj.cpu().numpy().copy()
    assert_sampled_gradient(op, p, a, b, kap, g1a, g1b, rects, np.concatenate([rects, p.n_bool + rects]))
    fsmt.cop_backward(h, T(a), T(b), kap, wt, obj, ga, gb, flags=fsmt.FSMT_ACCUMULATE)
    torch.cuda.synchronize()
    for two, one in ((ga.cpu().numpy(), g1a), (gb.cpu().numpy(), g1b), (obj.cpu().numpy(), o1)):
        d = np.abs(two - 2 * one).max()
        assert d <= 1e-5 * max(np.abs(one).max(), 1e-30), d
    h.free()


def test_placement1200_fused_step_sampled():
    """Paper-scale placement, 16 restarts, one fused step in the benchmark's launch
    configuration: the step at sampled rectangles (rotation bit and both coordinates)
    against the projected step of the oracle's partial derivatives, and the exact check of
    the post-step point over all 721,800 constraints."""
    p = W.make_workload("placement_1200")
    op = oracle.OracleProblem(p)
    R = 16
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, R, 5, 3)
    kap, eta_a, eta_b = 1.0 / p.meta["mean_side"], 0.5, 5.0
    st = S.BatchState(h, a0, b0)
    cfg = S.SolveConfig(kappas=[kap], steps_per_level=1, eta_a=eta_a, eta_b=eta_b, eps=0.0, stop_on_sat=0)
    S.solve_batched([h], [st], cfg)
    S.check_batched([st])
    a1, b1 = st.a.cpu().numpy(), st.b.cpu().numpy()
    N = p.meta["n_rect"]
    rng = np.random.default_rng(5)
    rects = np.sort(rng.choice(N, 4, replace=False))
    reals = np.concatenate([rects, N + rects])
    sel = touching(p, rects, reals)
    o = oracle.objective(op, a0, b0, kap, sel=sel, per_constraint=False)
    lo, hi = p.real_lo, p.real_hi
    for r in range(R):
        fa, fb = 4e-7 * o["absg_a"][r, rects].max(), 4e-7 * o["absg_b"][r, reals].max()
        for i in rects:
            ref = np.clip(float(a0[r, i]) - eta_a * o["grad_a"][r, i], -1.0, 1.0)
            tol = eta_a * (1e-5 * o["absg_a"][r, i] + fa) + 3e-7 * (1 + abs(ref))
            assert abs(a1[r, i] - ref) <= tol, ("a", r, i, a1[r, i], ref)
        for j in reals:
            ref = np.clip(float(b0[r, j]) - eta_b * o["grad_b"][r, j], lo[j], hi[j])
            tol = eta_b * (1e-5 * o["absg_b"][r, j] + fb) + 3e-7 * (1 + abs(ref))
            assert abs(b1[r, j] - ref) <= tol, ("b", r, j, b1[r, j], ref)
    ch = oracle.check(op, a1, b1)
    np.testing.assert_array_equal(st.sat_bits.cpu().numpy().view(np.uint32), ch["sat_bits"])
    np.testing.assert_array_equal(st.n_unsat.cpu().numpy(), ch["n_unsat"])
    h.free()


def test_paper_placement_64x8_sampled_gradients():
    """The paper's placement encoding at 64 macros x 8 layers (410,304 constraints): sampled
    macro / layer bits and coordinates against the oracle's partial derivatives."""
    from workloads.paper_suite import make_paper_placement
    p = make_paper_placement(64, 8, W.seed_seq(9, 64, 8, 0))
    op = oracle.OracleProblem(p)
    h = fsmt.xbdd_compile(p)
    R, kap = 2, 10.0
    a, b = W.initial_points(p, R, 14, 2)
    a[0], b[0] = 0.8 * p.cert_x, p.cert_y
    ga = torch.zeros(R, p.n_bool, device=dev())
    gb = torch.zeros(R, p.n_real, device=dev())
    obj = torch.zeros(R, device=dev())
    fsmt.cop_backward(h, T(a), T(b), kap, T(np.ones(p.n_cons)), obj, ga, gb)
    torch.cuda.synchronize()
    bools, reals = _pick(p, np.random.default_rng(64), 3, 3)
    print(f"paper placement 64x8: booleans {bools.tolist()} reals {reals.tolist()}", flush=True)
    assert_sampled_gradient(op, p, a, b, kap, ga.cpu().numpy(), gb.cpu().numpy(), bools, reals)
    h.free()


def _halfspace_instance(rows, box=(0.0, 10.0), n_real=6):
    from workloads.format import KIND_CLAUSE, OP_LE, Builder, lit
    bld = Builder(1, n_real, real_lo=np.full(n_real, box[0]), real_hi=np.full(n_real, box[1]))
    for vars_, coefs, rhs in rows:
        bld.add(KIND_CLAUSE, [lit(bld.atom(vars_, coefs, OP_LE, rhs))])
    bld.add(KIND_CLAUSE, [lit(0)])
    return bld.build()


def test_separable_projection_zero_coefficient_matches_oracle():
    """Closed-form projection onto half-spaces on disjoint variables, one with a zero
    coefficient (its variable is only clipped), against the oracle's FP64 Dykstra."""
    p = _halfspace_instance([([0, 1], [1.0, 1.0], 3.0), ([2, 3], [2.0, 0.0], 4.0), ([4, 5], [1.0, -2.0], -1.0)])
    h = fsmt.xbdd_compile(p)
    info = fsmt.xbdd_info(h)
    assert info["n_halfspaces"] == 3 and info["hs_separable"] == 1
    R = 64
    rng = np.random.default_rng(8)
    a = rng.uniform(-1, 1, (R, 1)).astype(np.float32)
    b = rng.uniform(0, 10, (R, 6)).astype(np.float32)
    gb = rng.normal(scale=4.0, size=(R, 6)).astype(np.float32)
    ga = np.zeros_like(a)
    ta, tb = T(a), T(b)
    fsmt.pgd_step(h, ta, tb, T(ga), T(gb), 0.5, 1.0, torch.zeros(R, device=dev()))
    torch.cuda.synchronize()
    ref = oracle.pgd(p, a, b, ga, gb, 0.5, 1.0, unit_proj=True)
    err = np.abs(tb.cpu().numpy() - ref["b"]) / np.maximum(1.0, np.abs(ref["b"]))
    print(f"separable projection with a zero coefficient: max rel err {err.max():.2e}", flush=True)
    assert err.max() <= 2e-6
    h.free()


def test_separable_projection_empty_intersection_takes_least_excess():
    """A half-space that misses the box (y4 + 2 y5 <= -5 with y in [0, 10]^2) has no
    projection (Prop. "qp" assumes D non-empty); the reading is the box point of least
    excess: each of its variables at the bound that minimizes its term (here both at 0). The
    other half-space is projected as usual."""
    p = _halfspace_instance([([0, 1], [1.0, 1.0], 3.0), ([4, 5], [1.0, 2.0], -5.0)])
    h = fsmt.xbdd_compile(p)
    assert fsmt.xbdd_info(h)["hs_separable"] == 1
    R = 32
    rng = np.random.default_rng(9)
    a = rng.uniform(-1, 1, (R, 1)).astype(np.float32)
    b = rng.uniform(0, 10, (R, 6)).astype(np.float32)
    gb = rng.normal(scale=4.0, size=(R, 6)).astype(np.float32)
    tb = T(b)
    fsmt.pgd_step(h, T(a), tb, T(np.zeros_like(a)), T(gb), 0.5, 1.0, torch.zeros(R, device=dev()))
    torch.cuda.synchronize()
    nb = tb.cpu().numpy()
    assert np.all(nb[:, 4] == 0.0) and np.all(nb[:, 5] == 0.0)
    y = np.clip(b - gb, 0.0, 10.0)
    np.testing.assert_array_equal(nb[:, [2, 3]], y[:, [2, 3]])   # untouched variables: clipped only
    viol = nb[:, 0] + nb[:, 1] - 3.0
    assert np.all(viol <= 1e-5)
    h.free()
