"""GPU tests of the fused batched solver, the plain per-call driver and the autograd wrapper."""
import numpy as np
import pytest

import oracle
import workloads as W

from gpu_util import T, assert_gradient, assert_objective, dev, torch

pytestmark = pytest.mark.gpu
fsmt = pytest.importorskip("paper_2603_22877_amd")
from paper_2603_22877_amd import solver as S  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bits_of(st):
    return st.sat_bits.cpu().numpy().view(np.uint32)


def _one_step(p, R, kap, eta_a, eta_b, seed, schedule=0, messages=0):
    h = fsmt.xbdd_compile(p, messages=messages)
    a0, b0 = W.initial_points(p, R, 50, seed)
    st = S.BatchState(h, a0, b0)
    cfg = S.SolveConfig(kappas=[kap], steps_per_level=1, eta_a=eta_a, eta_b=eta_b, eps=0.0, stop_on_sat=0,
                        schedule=schedule)
    S.solve_batched([h], [st], cfg)
    torch.cuda.synchronize()
    return h, a0, b0, st


def _assert_step(p, a0, b0, st, kap, eta_a, eta_b):
    o = oracle.objective(p, a0, b0, kap, per_constraint=False)
    ref = oracle.pgd(p, a0, b0, o["grad_a"].astype(np.float32), o["grad_b"].astype(np.float32), eta_a, eta_b)
    a1, b1 = st.a.cpu().numpy(), st.b.cpu().numpy()
    for r in range(a0.shape[0]):
        tol_a = eta_a * (1e-5 * o["absg_a"][r] + 4e-7 * o["absg_a"][r].max()) + 3e-7 * (1 + np.abs(ref["a"][r]))
        assert np.all(np.abs(a1[r] - ref["a"][r]) <= tol_a), np.abs(a1[r] - ref["a"][r]).max()
        tol_b = eta_b * (1e-5 * o["absg_b"][r] + 4e-7 * o["absg_b"][r].max()) + 2e-6 * (1 + np.abs(ref["b"][r]))
        assert np.all(np.abs(b1[r] - ref["b"][r]) <= tol_b), np.abs(b1[r] - ref["b"][r]).max()
    # the objective reported is U at the point where the step started
    assert_objective(st.obj.cpu().numpy(), o["U"], p.n_cons)
    # check and ERWA at the GPU's own post-step point: bit-exact / FP32 rounding only
    ch = oracle.check(p, a1, b1)
    np.testing.assert_array_equal(_bits_of(st), ch["sat_bits"])
    np.testing.assert_array_equal(st.n_unsat.cpu().numpy(), ch["n_unsat"])
    np.testing.assert_array_equal(st.verdict.cpu().numpy(), ch["verdict"])
    hh, ww = np.zeros((a0.shape[0], p.n_cons)), np.ones((a0.shape[0], p.n_cons))
    oracle.erwa(ch["sat_bits"], p.n_cons, 1, hh, ww)
    np.testing.assert_allclose(st.w.cpu().numpy(), ww, rtol=2e-6)
    np.testing.assert_array_equal(st.hist.cpu().numpy(), hh)
    assert np.all(st.level_done.cpu().numpy() == 1) and np.all(st.steps_done.cpu().numpy() == 1)


@pytest.mark.parametrize("schedule", [1, 2])
@pytest.mark.parametrize("name,R,kap,eta_b", [("scheduling_10x2", 4, 0.05, 5.0), ("scheduling_200x10", 8, 0.1, 5.0),
                                              ("placement_150", 4, 0.2, 8.0)])
@pytest.mark.parametrize("messages", [0, 2])   # closed forms / generic node-by-node passes
def test_fused_step_matches_oracle(name, R, kap, eta_b, schedule, messages):
    print(f"fused step {name} R={R} schedule {schedule} messages {messages}", flush=True)
    p = W.make_workload(name)
    h, a0, b0, st = _one_step(p, R, kap, 0.5, eta_b, W.STREAM[name], schedule, messages)
    _assert_step(p, a0, b0, st, kap, 0.5, eta_b)


def test_fused_step_random_formulas():
    for seed in range(3):
        p = W.make_random_formula(3000 + seed, n_cons=120, max_len=5)
        h, a0, b0, st = _one_step(p, 5, 0.7, 0.3, 0.4, seed)
        _assert_step(p, a0, b0, st, 0.7, 0.3, 0.4)


@pytest.mark.parametrize("kind,R", [("hybrid", 3), ("hybrid", 12), ("mixed", 5)])
def test_fused_step_big_diagrams(kind, R):
    """Instances with big diagrams go to the grid schedule, where the level-synchronous
    kernel adds their gradient: one fused step matches the oracle (random hybrid: all
    constraints big; mixed: short constraints one lane each, long ones level by level)."""
    from workloads.format import KIND_AND, KIND_CARD_GE, KIND_CARD_LE, KIND_CLAUSE, KIND_NAE, KIND_XOR
    if kind == "hybrid":
        p = W.make_random_hybrid(100)
    else:
        p = W.make_random_formula(4100, n_bool=16, n_real=5, n_atoms=16, n_cons=80, max_len=32,
                                  allow_repeats=False,
                                  kinds=(KIND_CLAUSE, KIND_AND, KIND_XOR, KIND_NAE, KIND_CARD_LE, KIND_CARD_GE))
    print(f"fused step {kind} R={R}", flush=True)
    h, a0, b0, st = _one_step(p, R, 0.6, 0.3, 0.4, 7)
    assert fsmt.xbdd_info(h)["n_big"] > 0
    _assert_step(p, a0, b0, st, 0.6, 0.3, 0.4)


def _paper_instance(fam, A, B, k=0):
    from workloads.paper_suite import make_paper_placement, make_paper_scheduling
    if fam == "sched":
        return make_paper_scheduling(A, B, W.seed_seq(8, A, B, k))
    return make_paper_placement(A, B, W.seed_seq(9, A, B, k))


@pytest.mark.parametrize("fam,A,B,schedule", [("sched", 16, 2, 1), ("sched", 16, 2, 2), ("sched", 32, 3, 2),
                                              ("sched", 64, 2, 1), ("sched", 64, 2, 2), ("place", 4, 4, 1),
                                              ("place", 4, 4, 2), ("place", 32, 8, 1), ("place", 32, 8, 2)])
def test_fused_step_paper_suite(fam, A, B, schedule):
    """One fused step on the paper's encodings (unit-atom projection: precedences, routing
    adjacency and module bounds are projected onto)."""
    p = _paper_instance(fam, A, B)
    ell = p.meta.get("mean_duration", p.meta.get("mean_side"))
    kap, eta_b = 2.0 / ell, 0.2 * ell * ell
    print(f"fused step paper {fam} {A}x{B} schedule {schedule}", flush=True)
    R = 1 if p.n_cons > 50000 else 4            # the oracle takes ~30 s per restart at 32 x 8
    h, a0, b0, st = _one_step(p, R, kap, 0.5, eta_b, A * 10 + B, schedule)
    _assert_step(p, a0, b0, st, kap, 0.5, eta_b)


def test_multi_instance_batch_equals_single():
    probs = [W.make_workload("scheduling_10x2"), W.make_random_formula(3100, n_cons=60), W.make_fig2_toy(), W.make_workload("scheduling_200x10")]
    Rs = [3, 5, 2, 4]
    hs = [fsmt.xbdd_compile(p) for p in probs]
    init = [W.initial_points(p, R, 60, i) for i, (p, R) in enumerate(zip(probs, Rs))]
    # one workgroup per restart in both runs (the automatic cluster size depends on the batch)
    cfg = S.SolveConfig(kappas=[0.3, 0.6], steps_per_level=3, eta_a=0.4, eta_b=1.0, eps=0.0, stop_on_sat=0,
                        cluster=1)
    batch = [S.BatchState(h, a, b) for h, (a, b) in zip(hs, init)]
    S.solve_batched(hs, batch, cfg)
    for h, (a, b), bs in zip(hs, init, batch):
        single = S.BatchState(h, a, b)
        S.solve_batched([h], [single], cfg)
        torch.cuda.synchronize()
        np.testing.assert_allclose(bs.a.cpu().numpy(), single.a.cpu().numpy(), rtol=0, atol=1e-5)
        np.testing.assert_allclose(bs.b.cpu().numpy(), single.b.cpu().numpy(), rtol=1e-5, atol=1e-5)
        np.testing.assert_array_equal(bs.level_done.cpu().numpy(), single.level_done.cpu().numpy())


def test_levels_replay_erwa_and_check():
    """Level by level (one call per level, resuming): the check bits equal the oracle's at the
    GPU point, and the weights equal the oracle's ERWA update of the previous weights."""
    p = W.make_workload("scheduling_200x10")
    R = 8
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, R, 2, 3)
    st = S.BatchState(h, a0, b0)
    kappas = S.kappa_schedule(p.meta["mean_duration"], 6)
    hh = np.zeros((R, p.n_cons))
    for t in range(1, 4):
        w_prev = st.w.cpu().numpy().astype(np.float64)
        cfg = S.SolveConfig(kappas=kappas[:t], steps_per_level=5, eta_a=0.5, eta_b=5.0, eps=0.0, stop_on_sat=0)
        S.solve_batched([h], [st], cfg)
        torch.cuda.synchronize()
        a1, b1 = st.a.cpu().numpy(), st.b.cpu().numpy()
        ch = oracle.check(p, a1, b1)
        np.testing.assert_array_equal(_bits_of(st), ch["sat_bits"])
        ww = w_prev.copy()
        oracle.erwa(ch["sat_bits"], p.n_cons, t, hh, ww)
        np.testing.assert_allclose(st.w.cpu().numpy(), ww, rtol=2e-5)
        np.testing.assert_allclose(st.hist.cpu().numpy(), hh, rtol=1e-6)
        assert np.all(st.level_done.cpu().numpy() == t)
        assert np.all(st.steps_done.cpu().numpy() == 5 * t)


@pytest.mark.parametrize("name,R", [("scheduling_10x2", 16), ("scheduling_200x10", 64)])
def test_batched_solver_reaches_sat(name, R):
    p = W.make_workload(name)
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, R, W.STREAM[name], 0)
    st = S.BatchState(h, a0, b0)
    scfg = S.SolveConfig(kappas=S.kappa_schedule(p.meta["mean_duration"], 40), steps_per_level=100,
                         eta_a=0.5, eta_b=5.0, eps=1e-2, stop_on_sat=2)
    S.solve_batched([h], [st], scfg)
    torch.cuda.synchronize()
    ver = st.verdict.cpu().numpy()
    assert ver.max() == 1, st.n_unsat.cpu().numpy()
    r = int(np.argmax(ver))
    ch = oracle.check(p, st.a.cpu().numpy()[r:r + 1], st.b.cpu().numpy()[r:r + 1])
    assert ch["verdict"][0] == 1


def test_plain_solver_reaches_sat_scheduling10x2():
    p = W.make_workload("scheduling_10x2")
    h = fsmt.xbdd_compile(p)
    plain = S.PlainSolver(h, R=1)
    cfg = S.SolveConfig(kappas=S.kappa_schedule(p.meta["mean_duration"], 40), steps_per_level=100,
                        eta_a=0.5, eta_b=5.0, eps=1e-2)
    found = False
    for seed in range(4):
        a0, b0 = W.initial_points(p, 1, 1, 100 + seed)
        res = plain.run(a0, b0, cfg)
        if res["verdict"] == 1:
            ch = oracle.check(p, res["a"].cpu().numpy(), res["b"].cpu().numpy())
            assert ch["verdict"][0] == 1
            found = True
            break
    assert found


def test_autograd_function_matches_reverse_sweep():
    p = W.make_workload("placement_150")
    R = 4
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, R, 3, 7)
    a = T(a0).requires_grad_(True)
    b = T(b0).requires_grad_(True)
    w = T(np.ones(p.n_cons))
    U = S.cop_objective(a, b, h, 0.2, w)
    gout = torch.tensor([1.0, 2.0, -0.5, 3.0], device=dev())
    U.backward(gout)
    o = oracle.objective(p, a0, b0, 0.2, per_constraint=False)
    assert_objective(U.detach().cpu().numpy(), o["U"], p.n_cons)
    g = gout.cpu().numpy()[:, None]
    # the gradient bar of every reverse-sweep test, on the output-weighted rows
    assert_gradient(a.grad.cpu().numpy(), g * o["grad_a"], np.abs(g) * o["absg_a"], "autograd grad_a")
    assert_gradient(b.grad.cpu().numpy(), g * o["grad_b"], np.abs(g) * o["absg_b"], "autograd grad_b")
    with torch.no_grad():
        U2 = S.cop_objective(a, b, h, 0.2, w)
    # forward-only and forward + reverse calls sum the same per-constraint values in a
    # different order (float atomics over ~180 wave partials): the objective tolerance
    assert_objective(U2.cpu().numpy(), U.detach().cpu().numpy().astype(np.float64), p.n_cons)


def test_solver_rejects_bad_options():
    p = W.make_workload("scheduling_10x2")
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, 2, 1, 0)
    st = S.BatchState(h, a0, b0)
    with pytest.raises(fsmt.FsmtError):
        S.solve_batched([h], [st], S.SolveConfig(kappas=[0.1] * 200))
    with pytest.raises(fsmt.FsmtError):
        S.solve_batched([h], [st], S.SolveConfig(kappas=[0.1], eta_a=0.0))
    with pytest.raises(fsmt.FsmtError):
        S.solve_batched([h], [st], S.SolveConfig(kappas=[-1.0]))
    assert int(st.level_done.max()) == 0
    # big diagrams run in the grid schedule only: the persistent one refuses them
    hb = fsmt.xbdd_compile(W.make_random_hybrid(100))
    ab, bb = W.initial_points(W.make_random_hybrid(100), 2, 6, 0)
    stb = S.BatchState(hb, ab, bb)
    with pytest.raises(fsmt.FsmtError) as e:
        S.solve_batched([hb], [stb], S.SolveConfig(kappas=[0.1], schedule=1))
    assert e.value.code == fsmt._abi.FSMT_EUNSUPPORTED
    assert int(stb.level_done.max()) == 0


def test_plain_solver_on_big_diagrams_descends():
    """The per-call path (level kernel + PGD) lowers the objective of a random hybrid
    instance whose diagrams are all big."""
    p = W.make_random_hybrid(200)
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, 1, 6, 1)
    ps = S.PlainSolver(h, R=1)
    a = torch.as_tensor(a0, device=dev()); b = torch.as_tensor(b0, device=dev())
    w = torch.ones(p.n_cons, device=dev())
    obj0 = torch.zeros(1, device=dev())
    fsmt.cop_forward(h, a, b, 0.5, w, obj0)
    out = ps.run(a0, b0, S.SolveConfig(kappas=[0.5] * 3, steps_per_level=50, eta_a=0.2, eta_b=0.5, eps=0.0,
                                        stop_on_sat=0))
    obj1 = torch.zeros(1, device=dev())
    fsmt.cop_forward(h, out["a"], out["b"], 0.5, w, obj1)
    torch.cuda.synchronize()
    print(f"random hybrid 200: U {float(obj0[0]):.4f} -> {float(obj1[0]):.4f}", flush=True)
    assert float(obj1[0]) < float(obj0[0])


def _run(h, a, b, cfg):
    st = S.BatchState(h, a, b)
    S.solve_batched([h], [st], cfg)
    torch.cuda.synchronize()
    return st


@pytest.mark.parametrize("name,R", [("scheduling_10x2", 8), ("scheduling_200x10", 16), ("placement_150", 4)])
def test_grid_and_persistent_schedules_agree(name, R):
    """Both schedules run the same algorithm: over 3 levels x 4 steps (no early exit) the
    states agree to FP32 accumulation-order noise and the bookkeeping is identical."""
    p = W.make_workload(name)
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, R, 70, W.STREAM[name])
    kap = S.kappa_schedule(p.meta.get("mean_duration", p.meta.get("mean_side", 1.0)), 3)
    res = []
    for sched in (1, 2):
        cfg = S.SolveConfig(kappas=kap, steps_per_level=4, eta_a=0.5, eta_b=2.0, eps=0.0, stop_on_sat=0,
                            schedule=sched)
        res.append(_run(h, a0, b0, cfg))
    A, B = res
    np.testing.assert_allclose(A.a.cpu().numpy(), B.a.cpu().numpy(), rtol=0, atol=2e-4)
    np.testing.assert_allclose(A.b.cpu().numpy(), B.b.cpu().numpy(), rtol=2e-4, atol=2e-4)
    for k in ("level_done", "steps_done"):
        np.testing.assert_array_equal(getattr(A, k).cpu().numpy(), getattr(B, k).cpu().numpy())
    assert np.all(A.steps_done.cpu().numpy() == 12)


@pytest.mark.parametrize("schedule", [1, 2])
def test_levels_end_early_at_eps(schedule):
    """With kappa = 0 the b-gradient vanishes and the Booleans saturate at the box, so the
    gradient map falls below eps and every level ends before its step cap."""
    p = W.make_workload("scheduling_10x2")
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, 8, 1, 12)
    cfg = S.SolveConfig(kappas=[0.0, 0.0], steps_per_level=100, eta_a=0.5, eta_b=5.0, eps=1e-2, stop_on_sat=0,
                        schedule=schedule)
    st = _run(h, a0, b0, cfg)
    assert np.all(st.level_done.cpu().numpy() == 2)
    assert st.steps_done.cpu().numpy().max() < 200


def test_grid_schedule_reaches_sat_and_stops():
    p = W.make_workload("scheduling_200x10")
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, 16, 2, 11)
    cfg = S.SolveConfig(kappas=S.kappa_schedule(p.meta["mean_duration"], 40), steps_per_level=100, eta_a=0.5,
                        eta_b=5.0, eps=1e-2, stop_on_sat=2, schedule=2)
    st = _run(h, a0, b0, cfg)
    ver = st.verdict.cpu().numpy()
    assert ver.max() == 1
    levels = st.level_done.cpu().numpy()
    assert levels.max() - levels.min() <= 1          # the others stopped at the next level boundary
    r = int(np.argmax(ver))
    assert oracle.check(p, st.a.cpu().numpy()[r:r + 1], st.b.cpu().numpy()[r:r + 1])["verdict"][0] == 1


def test_uneven_batch_mixes_schedules():
    """The uneven batch (48 instances, 16 restarts each): large scheduling instances go to the grid
    schedule, small ones to the persistent one, in one call; per-instance bookkeeping and
    check bits are verified against the oracle on a sample of instances."""
    print("uneven batch", flush=True)
    probs = W.uneven_batch()
    R = 16
    hs = [fsmt.xbdd_compile(p) for p in probs]
    states = [S.BatchState(h, *W.initial_points(p, R, 4, i)) for i, (h, p) in enumerate(zip(hs, probs))]
    cfg = S.SolveConfig(kappas=[0.05, 0.1], steps_per_level=3, eta_a=0.5, eta_b=2.0, eps=0.0, stop_on_sat=0)
    S.solve_batched(hs, states, cfg)
    torch.cuda.synchronize()
    for st in states:
        assert np.all(st.level_done.cpu().numpy() == 2) and np.all(st.steps_done.cpu().numpy() == 6)
    rng = np.random.default_rng(0)
    big = int(np.argmax([p.n_cons for p in probs]))
    for i in sorted(set(rng.choice(len(probs), 4, replace=False).tolist() + [big])):
        p, st = probs[i], states[i]
        ch = oracle.check(p, st.a.cpu().numpy(), st.b.cpu().numpy())
        np.testing.assert_array_equal(_bits_of(st), ch["sat_bits"])
        np.testing.assert_array_equal(st.n_unsat.cpu().numpy(), ch["n_unsat"])


@pytest.mark.parametrize("cluster", [2, 4])
def test_cluster_split_step_matches_oracle(cluster):
    """Several workgroups per restart (partials summed in rank order): one step still
    matches the oracle, and every rank applies the same update."""
    p = W.make_workload("scheduling_200x10")
    R = 8
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, R, 50, 2)
    st = S.BatchState(h, a0, b0)
    cfg = S.SolveConfig(kappas=[0.1], steps_per_level=1, eta_a=0.5, eta_b=5.0, eps=0.0, stop_on_sat=0,
                        schedule=1, cluster=cluster)
    S.solve_batched([h], [st], cfg)
    torch.cuda.synchronize()
    _assert_step(p, a0, b0, st, 0.1, 0.5, 5.0)


def test_cluster_split_agrees_with_single_workgroup_over_levels():
    p = W.make_workload("scheduling_200x10")
    R = 16
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, R, 71, 0)
    kap = S.kappa_schedule(p.meta["mean_duration"], 3)
    res = []
    for cl in (1, 4):
        cfg = S.SolveConfig(kappas=kap, steps_per_level=5, eta_a=0.5, eta_b=5.0, eps=0.0, stop_on_sat=0,
                            schedule=1, cluster=cl)
        res.append(_run(h, a0, b0, cfg))
    A, B = res
    np.testing.assert_allclose(A.a.cpu().numpy(), B.a.cpu().numpy(), rtol=0, atol=2e-4)
    np.testing.assert_allclose(A.b.cpu().numpy(), B.b.cpu().numpy(), rtol=2e-4, atol=2e-4)
    np.testing.assert_array_equal(A.level_done.cpu().numpy(), B.level_done.cpu().numpy())
    np.testing.assert_array_equal(A.steps_done.cpu().numpy(), B.steps_done.cpu().numpy())
    assert B.verdict.cpu().numpy().min() >= 0        # no barrier abort


def test_unsat_instance_returns_unknown():
    """A planted contradiction (x and not x) beside satisfiable constraints: the fused solver
    runs every level and reports no SAT, the plain path too, and the PAR-2 harness scores the
    instance at twice its limit after restarting from new seeds."""
    from workloads.format import KIND_CLAUSE, Builder, lit
    from paper_2603_22877_amd import par2 as P2
    b = Builder(n_bool=3, n_real=2, real_lo=[-1.0, -1.0], real_hi=[1.0, 1.0])
    y0 = b.atom([0, 1], [1.0, -1.0], 0, 0.25)
    b.add(KIND_CLAUSE, [lit(0)])
    b.add(KIND_CLAUSE, [lit(0, neg=True)])
    b.add(KIND_CLAUSE, [lit(1), lit(y0)])
    b.add(KIND_CLAUSE, [lit(2, neg=True), lit(y0, neg=True)])
    p = b.build()
    h = fsmt.xbdd_compile(p)
    R, levels = 8, 4
    cfg = S.SolveConfig(kappas=S.kappa_schedule(0.5, levels), steps_per_level=20, eta_a=0.5, eta_b=0.1,
                        eps=1e-2, stop_on_sat=2)
    st = S.BatchState(h, *W.initial_points(p, R, 70, 0))
    S.solve_batched([h], [st], cfg)
    torch.cuda.synchronize()
    assert np.all(st.verdict.cpu().numpy() == 0)
    assert np.all(st.level_done.cpu().numpy() == levels)
    assert np.all(st.n_unsat.cpu().numpy() >= 1)
    out = S.PlainSolver(h, R=1).run(*W.initial_points(p, 1, 70, 1), cfg)
    assert out["verdict"] == 0 and out["level"] == levels
    r = P2.run_instance(p, cfg, 4, 0.3, lambda q, R_, att: W.initial_points(q, R_, 71, att), name="unsat")
    assert not r.solved and r.attempts >= 1 and r.best_unsat >= 1
    assert r.score(0.3) == 0.6 and P2.par2([r], 0.3) == 0.6
