"""GPU parity: the HIP path through the C ABI against the FP64 oracle on identical inputs."""
import numpy as np
import pytest

import oracle
import workloads as W

from gpu_util import T, assert_gradient, assert_objective, assert_unsat, dev, torch

pytestmark = pytest.mark.gpu
fsmt = pytest.importorskip("paper_2603_22877_amd")

INF = float("inf")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run_cop(p, h, a, b, kap, w=None, layout="rows", grad=True):
    R = a.shape[0]
    wt = T(np.ones(p.n_cons) if w is None else w)
    if layout == "rows":
        ta, tb = T(a), T(b)
        ga = torch.zeros(R, p.n_bool, device=dev())
        gb = torch.zeros(R, p.n_real, device=dev())
    else:   # variable-major storage [n][R] viewed as [R][n]
        ta, tb = T(a.T.copy()).t(), T(b.T.copy()).t()
        ga = torch.zeros(p.n_bool, R, device=dev()).t()
        gb = torch.zeros(p.n_real, R, device=dev()).t()
    obj = torch.zeros(R, device=dev())
    unsat = torch.zeros(R, p.n_cons, device=dev())
    fsmt.cop_forward(h, ta, tb, kap, wt, obj, unsat)
    out = dict(U_fwd=obj.cpu().numpy().copy(), unsat=unsat.cpu().numpy())
    if grad:
        obj2 = torch.zeros(R, device=dev())
        fsmt.cop_backward(h, ta, tb, kap, wt, obj2, ga, gb)
        out.update(U=obj2.cpu().numpy(), grad_a=ga.cpu().numpy(), grad_b=gb.cpu().numpy())
    torch.cuda.synchronize()
    return out


MSG = {"auto": 0, "lds": 1, "generic": 2}


def _compare(p, a, b, kap, w=None, layout="rows", messages="auto"):
    h = fsmt.xbdd_compile(p, messages=MSG[messages])
    g = _run_cop(p, h, a, b, kap, w, layout)
    o = oracle.objective(p, a, b, kap, w=w)
    wsum = (np.ones(p.n_cons) if w is None else np.broadcast_to(w, (a.shape[0], p.n_cons))).sum(-1)
    assert_objective(g["U_fwd"], o["U"], wsum)
    assert_objective(g["U"], o["U"], wsum)
    assert_unsat(g["unsat"], o["unsat"])
    assert_gradient(g["grad_a"], o["grad_a"], o["absg_a"], "grad_a")
    assert_gradient(g["grad_b"], o["grad_b"], o["absg_b"], "grad_b")
    h.free()
    return g, o


@pytest.mark.parametrize("messages", ["auto", "lds", "generic"])
@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("R", [1, 3, 16, 64, 100])
@pytest.mark.parametrize("kap", [0.0, 0.4, 2.5, INF])
def test_random_formulas_all_kinds(seed, R, kap, messages):
    print(f"random formulas seed={seed} R={R} kappa={kap} messages={messages}", flush=True)
    p = W.make_random_formula(1000 + seed, n_bool=8, n_real=4, n_atoms=8, n_cons=150, max_len=6)
    a, b = W.initial_points(p, R, 99, seed)
    a[0, :2] = [0.0, -1.0]
    _compare(p, a, b, kap, w=np.random.default_rng(seed).uniform(0.5, 2, (R, p.n_cons)), messages=messages)


@pytest.mark.parametrize("max_len,seed", [(2, 0), (2, 1), (3, 0), (12, 0), (12, 1)])
def test_message_store_bounds(max_len, seed):
    """Diagrams within the 4-node and 20-node register bounds and beyond them (LDS store)."""
    p = W.make_random_formula(3000 + seed, n_bool=10, n_real=4, n_atoms=10, n_cons=120, max_len=max_len)
    info = fsmt.xbdd_info(fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY))
    print(f"max_len={max_len} seed={seed} nodes={info['max_nodes']} slots={info['max_slots']}", flush=True)
    a, b = W.initial_points(p, 24, 98, seed)
    for kap in (0.3, 3.0):
        _compare(p, a, b, kap)


@pytest.mark.parametrize("n,R", [(100, 1), (100, 5), (200, 3), (300, 2)])
def test_big_diagrams_random_hybrid(n, R):
    """Random hybrid instances: every constraint is a long CARD/NAE/XOR (level kernel)."""
    p = W.make_random_hybrid(n)
    info = fsmt.xbdd_info(fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY))
    print(f"random hybrid n={n} R={R} nodes={info['max_nodes']} big={info['n_big']}", flush=True)
    assert info["n_big"] == p.n_cons
    a, b = W.initial_points(p, R, 6, n)
    for kap in (0.0, 0.7, 5.0, INF):
        _compare(p, a, b, kap, w=np.random.default_rng(n).uniform(0.5, 2, (R, p.n_cons)))


@pytest.mark.parametrize("n,R", [(100, 1), (100, 6), (200, 3)])
def test_big_diagrams_inline_records(n, R):
    """Random hybrid instances with float32 right-hand sides: every atom has an inline
    record, so the level kernel reads the records instead of the CSR atom table."""
    import dataclasses
    p = W.make_random_hybrid(n)
    p = dataclasses.replace(p, atom_rhs=p.atom_rhs.astype(np.float32).astype(np.float64))
    info = fsmt.xbdd_info(fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY))
    print(f"random hybrid inline n={n} R={R} big={info['n_big']}", flush=True)
    assert info["n_big"] == p.n_cons
    a, b = W.initial_points(p, R, 16, n)
    for kap in (0.7, 5.0):
        _compare(p, a, b, kap, w=np.random.default_rng(n).uniform(0.5, 2, (R, p.n_cons)))


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("R", [1, 7, 70])
def test_mixed_small_and_big_diagrams(seed, R):
    """One launch of each kernel: short constraints one lane each, long ones level by level
    (CSR atoms with up to 3 nonzeros, so the level kernel's CSR path runs too)."""
    from workloads.format import KIND_AND, KIND_CARD_GE, KIND_CARD_LE, KIND_CLAUSE, KIND_NAE, KIND_XOR
    p = W.make_random_formula(4000 + seed, n_bool=16, n_real=5, n_atoms=16, n_cons=80, max_len=32,
                              allow_repeats=False,
                              kinds=(KIND_CLAUSE, KIND_AND, KIND_XOR, KIND_NAE, KIND_CARD_LE, KIND_CARD_GE))
    info = fsmt.xbdd_info(fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY))
    print(f"mixed seed={seed} R={R} big={info['n_big']} of {p.n_cons}", flush=True)
    assert 0 < info["n_big"] < p.n_cons
    a, b = W.initial_points(p, R, 96, seed)
    for kap in (0.4, 3.0):
        _compare(p, a, b, kap)
        _compare(p, a, b, kap, layout="cols")


@pytest.mark.parametrize("seed,R", [(0, 1), (1, 5), (2, 64)])
def test_separable_guarded_disjunctions(seed, R):
    """ITEs over two Booleans whose values pick their atom groups independently (evaluated as
    the product of one sum per selector) mixed with ITEs that do not factor, at every kappa
    regime and with per-constraint weights; also the fused step of the persistent and grid
    schedules."""
    from paper_2603_22877_amd import solver as S
    p = W.make_random_separable(seed)
    info = fsmt.xbdd_info(fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY))
    print(f"separable seed={seed} R={R} sep={info['n_gd_sep']} gd={info['n_gd']} of {p.n_cons}", flush=True)
    assert 0 < info["n_gd_sep"] < info["n_gd"]
    a, b = W.initial_points(p, R, 95, seed)
    a[0, :4] = [0.0, -1.0, 1.0, 0.5]
    for kap in (0.0, 0.6, 4.0, INF):
        _compare(p, a, b, kap, w=np.random.default_rng(seed).uniform(0.5, 2, (R, p.n_cons)))
    for sched in (1, 2):
        h = fsmt.xbdd_compile(p)
        st = S.BatchState(h, a, b)
        S.solve_batched([h], [st], S.SolveConfig(kappas=[0.6], steps_per_level=1, eta_a=0.5, eta_b=0.5, eps=0.0,
                                                  stop_on_sat=0, schedule=sched))
        torch.cuda.synchronize()
        o = oracle.objective(p, a, b, 0.6, per_constraint=False)
        ref = oracle.pgd(p, a, b, o["grad_a"].astype(np.float32), o["grad_b"].astype(np.float32), 0.5, 0.5)
        assert_objective(st.obj.cpu().numpy(), o["U"], p.n_cons)
        for r in range(R):
            tol_a = 0.5 * (1e-5 * o["absg_a"][r] + 4e-7 * o["absg_a"][r].max()) + 3e-7 * (1 + np.abs(ref["a"][r]))
            assert np.all(np.abs(st.a.cpu().numpy()[r] - ref["a"][r]) <= tol_a)
            tol_b = 0.5 * (1e-5 * o["absg_b"][r] + 4e-7 * o["absg_b"][r].max()) + 2e-6 * (1 + np.abs(ref["b"][r]))
            assert np.all(np.abs(st.b.cpu().numpy()[r] - ref["b"][r]) <= tol_b)
        h.free()


@pytest.mark.parametrize("R", [1, 16])
def test_swapped_term_runs(R):
    """Guarded disjunctions whose consecutive atoms name one variable pair in either stored
    order (y_u - y_v <= c, then y_v - y_u <= c'): the compiler stores the second in the first's
    order, so the two form one run of reads and scatter; objective and gradient against the
    oracle at several kappa, with per-constraint weights."""
    from workloads.format import Builder, KIND_CLAUSE, KIND_EXPR, X_ITE, X_OR, lit
    rng = np.random.default_rng(61)
    n_bool, n_real = 6, 8
    bb = Builder(n_bool, n_real, real_lo=np.full(n_real, -2.0), real_hi=np.full(n_real, 2.0))
    for c in range(300):
        u, v = (int(x) for x in rng.choice(n_real, 2, replace=False))
        q = float(rng.choice([1.0, 2.0, 0.5]))
        a1 = bb.atom([u, v], [q, -q], 0, float(rng.integers(-8, 9)) / 8)
        a2 = bb.atom([v, u], [q, -q], 0, float(rng.integers(-8, 9)) / 8)
        a3 = bb.atom([v, u], [-2.0, 1.0], 0, float(rng.integers(-8, 9)) / 8)
        s0, s1 = (int(x) for x in np.sort(rng.choice(n_bool, 2, replace=False)))
        if c % 2:
            bb.add(KIND_CLAUSE, [lit(s0, True), lit(a1), lit(a2, True), lit(a3)])
        else:   # ITE(s0, a1 | a2, a2 | a3) over one more Boolean
            bb.add(KIND_EXPR, [lit(s0), lit(a1), lit(a2), lit(a2), lit(a3), lit(s1)],
                   ops=(0, 1, 2, X_OR, 3, 4, X_OR, 5, X_OR, X_ITE))
    p = bb.build()
    info = fsmt.xbdd_info(fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY))
    print(f"swapped-term runs R={R} gd={info['n_gd']} of {p.n_cons} templates={info['n_templates']}", flush=True)
    assert info["n_gd"] == p.n_cons
    a, b = W.initial_points(p, R, 62, R)
    for kap in (0.0, 0.8, 5.0, INF):
        _compare(p, a, b, kap, w=np.random.default_rng(R).uniform(0.5, 2, (R, p.n_cons)))


@pytest.mark.parametrize("name", ["scheduling_200x10", "placement_150"])
def test_nan_state_propagates_to_its_restart(name):
    """A NaN coordinate makes its restart's objective NaN (forward and reverse) and the
    gradient of the variables it shares a constraint with (the objective is multilinear, so
    the derivative by the NaN variable itself does not involve its value), and leaves the
    other restarts as the oracle computes them."""
    p = W.make_workload(name)
    a, b = W.initial_points(p, 3, W.STREAM[name], 8)
    b[1, 0] = np.nan          # a real
    a[2, 0] = np.nan          # a Boolean
    h = fsmt.xbdd_compile(p)
    kap = 0.5
    g = _run_cop(p, h, a, b, kap)
    o = oracle.objective(p, a[:1], b[:1], kap)
    assert_objective(g["U"][:1], o["U"], p.n_cons)
    assert_objective(g["U_fwd"][:1], o["U"], p.n_cons)
    assert np.isnan(g["U"][1]) and np.isnan(g["U_fwd"][1]) and np.isnan(g["U"][2]) and np.isnan(g["U_fwd"][2])
    assert np.isnan(g["grad_b"][1]).any() and np.isnan(g["grad_b"][2]).any()
    assert np.all(np.isfinite(g["grad_a"][0])) and np.all(np.isfinite(g["grad_b"][0]))
    h.free()


@pytest.mark.parametrize("name,R", [("scheduling_200x10", 1), ("placement_150", 1), ("placement_150", 16)])
def test_backward_accumulates_into_the_outputs(name, R):
    """FSMT_ACCUMULATE adds into obj and the gradients instead of overwriting them: a
    second call doubles them (one restart sums the gradient per workgroup in LDS and adds
    the rows; 16 restarts go through the restart-contiguous stage)."""
    p = W.make_workload(name)
    print(f"accumulate {name} R={R}", flush=True)
    a, b = W.initial_points(p, R, W.STREAM[name], 3)
    h = fsmt.xbdd_compile(p)
    ta, tb, wt = T(a), T(b), T(np.ones(p.n_cons))
    ga = torch.full((R, p.n_bool), 123.0, device=dev())
    gb = torch.full((R, p.n_real), -7.0, device=dev())
    obj = torch.full((R,), 5.0, device=dev())
    fsmt.cop_backward(h, ta, tb, 0.3, wt, obj, ga, gb)              # overwrites the junk
    g1, b1, o1 = ga.clone(), gb.clone(), obj.clone()
    fsmt.cop_backward(h, ta, tb, 0.3, wt, obj, ga, gb, flags=fsmt.FSMT_ACCUMULATE)
    o = oracle.objective(p, a, b, 0.3)
    assert_objective(o1.cpu().numpy(), o["U"], np.full(R, float(p.n_cons)))
    assert_gradient(g1.cpu().numpy(), o["grad_a"], o["absg_a"], "grad_a")
    assert_gradient(b1.cpu().numpy(), o["grad_b"], o["absg_b"], "grad_b")
    for two, one in ((ga, g1), (gb, b1), (obj, o1)):
        d = (two - 2 * one).abs().max().item()
        assert d <= 1e-5 * max(one.abs().max().item(), 1e-30), d
    h.free()


def test_fig2_toy_values():
    p = W.make_fig2_toy()
    a = np.array([[0.3], [-0.9], [1.0]], np.float32)
    b = np.array([[0.2], [-0.5], [0.0]], np.float32)
    for kap in (0.0, 0.5, 1.7, INF):
        _compare(p, a, b, kap)


@pytest.mark.parametrize("name,R,kap", [("scheduling_10x2", 1, 0.3), ("scheduling_10x2", 1, INF),
                                        ("scheduling_200x10", 64, 0.05), ("scheduling_200x10", 64, 0.5),
                                        ("placement_150", 16, 0.1), ("placement_150", 16, 1.0),
                                        ("scheduling_200x10", 1, 0.3), ("placement_150", 1, 0.5)])
@pytest.mark.parametrize("messages", ["auto", "lds", "generic"])
def test_standard_workloads(name, R, kap, messages):
    print(f"{name} R={R} kappa={kap} messages={messages}", flush=True)
    p = W.make_workload(name)
    a, b = W.initial_points(p, R, W.STREAM[name], 0)
    _compare(p, a, b, kap, messages=messages)


@pytest.mark.parametrize("name,R", [("scheduling_10x2", 5), ("scheduling_200x10", 64), ("placement_150", 16)])
def test_variable_major_layout_matches(name, R):
    p = W.make_workload(name)
    a, b = W.initial_points(p, R, W.STREAM[name], 1)
    _compare(p, a, b, 0.3, layout="cols")


def test_hard_objective_counts_violations_at_vertices():
    p = W.make_workload("placement_150")
    R = 8
    a, b = W.initial_points(p, R, 3, 2)
    a = np.where(a < 0, -1.0, 1.0).astype(np.float32)
    h = fsmt.xbdd_compile(p)
    g = _run_cop(p, h, a, b, INF, grad=False)
    ch = oracle.check(p, a, b)
    np.testing.assert_array_equal(g["U_fwd"], ch["n_unsat"].astype(np.float32))


@pytest.mark.parametrize("projection", ["box", "unit"])
def test_pgd_step_matches_oracle(projection):
    """Box projection: the clamp, exact up to FP32 rounding. Box + unit atoms (Prop. qp):
    Dykstra in FP32 against the FP64 oracle run to convergence."""
    p = W.make_workload("scheduling_200x10")
    R = 8
    a, b = W.initial_points(p, R, 2, 3)
    rng = np.random.default_rng(3)
    ga = rng.normal(size=a.shape).astype(np.float32) * 3
    gb = rng.normal(size=b.shape).astype(np.float32) * 50
    unit = projection == "unit"
    h = fsmt.xbdd_compile(p, projection=fsmt.FSMT_PROJ_UNIT if unit else fsmt.FSMT_PROJ_BOX)
    assert fsmt.xbdd_info(h)["n_halfspaces"] == (5 if unit else 0)
    ta, tb, tga, tgb = T(a), T(b), T(ga), T(gb)
    gsq = torch.zeros(R, device=dev())
    fsmt.pgd_step(h, ta, tb, tga, tgb, 0.25, 2.0, gsq)
    o = oracle.pgd(p, a, b, ga, gb, 0.25, 2.0, unit_proj=unit)
    na, nb = ta.cpu().numpy(), tb.cpu().numpy()
    assert np.all(np.abs(na - o["a"]) <= 2e-7 * np.maximum(1, np.abs(o["a"])))
    btol = (2e-6 if unit else 2e-7) * np.maximum(1, np.abs(o["b"])) + 1e-6
    assert np.all(np.abs(nb - o["b"]) <= btol), np.abs(nb - o["b"]).max()
    assert np.all((na >= -1) & (na <= 1)) and np.all((nb >= 0) & (nb <= p.real_hi[0]))
    np.testing.assert_allclose(gsq.cpu().numpy(), o["gsq"], rtol=1e-4)
    assert float(tga.abs().max()) == 0.0 and float(tgb.abs().max()) == 0.0
    if unit:   # horizons and precedences hold at the projected float32 point
        ch = oracle.check(p, na, nb)
        P = p.meta["n_pairs"]
        for r in range(R):
            for c in range(2 * P, p.n_cons):
                assert (ch["sat_bits"][r, c >> 5] >> (c & 31)) & 1


def test_pgd_step_dykstra_matches_oracle():
    """Half-spaces that share variables (chained job dependencies of the paper's scheduling
    encoding): Dykstra's sweeps over colour classes in FP32 against the FP64 oracle run to
    convergence (the test above takes the closed form: the precedences of scheduling 200 x 10 are disjoint)."""
    from workloads.paper_suite import make_paper_scheduling
    p = make_paper_scheduling(16, 3, W.seed_seq(8, 16, 3, 0), dep_prob=0.6)
    h = fsmt.xbdd_compile(p)
    info = fsmt.xbdd_info(h)
    assert info["n_hs_colors"] > 1 and info["hs_separable"] == 0
    R = 8
    rng = np.random.default_rng(11)
    lo, hi = p.real_lo.astype(np.float64), p.real_hi.astype(np.float64)
    a = rng.uniform(-1, 1, (R, p.n_bool)).astype(np.float32)
    b = (lo + (hi - lo) * rng.uniform(size=(R, p.n_real))).astype(np.float32)
    ga = rng.normal(size=a.shape).astype(np.float32)
    gb = (rng.normal(size=b.shape) * p.meta["mean_duration"]).astype(np.float32)
    ta, tb, tga, tgb = T(a), T(b), T(ga), T(gb)
    gsq = torch.zeros(R, device=dev())
    fsmt.pgd_step(h, ta, tb, tga, tgb, 0.25, 1.0, gsq)
    o = oracle.pgd(p, a, b, ga, gb, 0.25, 1.0, unit_proj=True)
    assert o["n_halfspaces"] == info["n_halfspaces"] > 0
    nb = tb.cpu().numpy()
    assert np.any(np.abs(o["b"] - np.clip(b - gb, lo, hi)) > 1e-3)   # the half-spaces moved points
    err = np.abs(nb - o["b"]) / np.maximum(1, np.abs(o["b"]))
    print(f"Dykstra projection: {info['n_halfspaces']} half-spaces in {info['n_hs_colors']} classes, "
          f"max rel err {err.max():.2e}", flush=True)
    assert err.max() <= 2e-6, err.max()
    # the sweeps end with the box step: inside the box the kernel holds (float32 bounds)
    assert np.all((nb >= lo.astype(np.float32)) & (nb <= hi.astype(np.float32)))


def _check_gpu(p, h, a, b):
    R = a.shape[0]
    nw = (p.n_cons + 31) // 32
    x = torch.zeros(R, p.n_bool, dtype=torch.int8, device=dev())
    bits = torch.zeros(R, nw, dtype=torch.int32, device=dev())
    nu = torch.zeros(R, dtype=torch.int32, device=dev())
    ver = torch.zeros(R, dtype=torch.int32, device=dev())
    fsmt.round_and_check(h, T(a), T(b), x, bits, nu, ver)
    torch.cuda.synchronize()
    return dict(x=x.cpu().numpy(), sat_bits=bits.cpu().numpy().view(np.uint32), n_unsat=nu.cpu().numpy(),
                verdict=ver.cpu().numpy())


def _assert_check_equal(g, o):
    np.testing.assert_array_equal(g["sat_bits"], o["sat_bits"])
    np.testing.assert_array_equal(g["n_unsat"], o["n_unsat"])
    np.testing.assert_array_equal(g["verdict"], o["verdict"])
    np.testing.assert_array_equal(g["x"], o["x"])


@pytest.mark.parametrize("name,R", [("scheduling_10x2", 4), ("scheduling_200x10", 16), ("placement_150", 16)])
def test_round_and_check_bit_exact(name, R):
    p = W.make_workload(name)
    a, b = W.initial_points(p, R, W.STREAM[name], 4)
    a[0] = p.cert_x
    b[0] = p.cert_y
    a[1] = p.cert_x
    b[1] = p.cert_y
    b[1, 0] = b[1, 0] + 0.5
    a[2, : min(3, p.n_bool)] = [0.0, -0.0, np.nan][: min(3, p.n_bool)]
    h = fsmt.xbdd_compile(p)
    g = _check_gpu(p, h, a, b)
    o = oracle.check(p, a, b)
    _assert_check_equal(g, o)
    assert g["verdict"][0] == 1


def test_check_boundary_atoms_and_random_formulas():
    for seed in range(3):
        p = W.make_random_formula(2000 + seed, n_cons=300, max_len=6)
        a, b = W.initial_points(p, 10, 77, seed)
        b[3] = np.round(b[3])
        h = fsmt.xbdd_compile(p)
        _assert_check_equal(_check_gpu(p, h, a, b), oracle.check(p, a, b))


def test_adjoint_central_differences_scheduling200x10():
    """FP32 central differences of the GPU objective on 32 random coordinates."""
    p = W.make_workload("scheduling_200x10")
    R = 4
    a, b = W.initial_points(p, R, 2, 5)
    kap = 0.2
    h = fsmt.xbdd_compile(p)
    g = _run_cop(p, h, a, b, kap)
    rng = np.random.default_rng(5)
    wt = T(np.ones(p.n_cons))
    obj = torch.zeros(R, device=dev())
    for _ in range(32):
        r = int(rng.integers(R))
        if rng.random() < 0.5:
            i = int(rng.integers(p.n_bool))
            hstep = 2.0 ** -6
            vals = []
            for s in (1, -1):
                aa = a.copy()
                aa[r, i] = np.float32(a[r, i] + s * hstep)
                fsmt.cop_forward(h, T(aa), T(b), kap, wt, obj)
                vals.append(float(obj[r]))
            fd = (vals[0] - vals[1]) / (2 * hstep)
            ref = g["grad_a"][r, i]
        else:
            j = int(rng.integers(p.n_real))
            hstep = 2.0 ** -2
            vals = []
            for s in (1, -1):
                bb = b.copy()
                bb[r, j] = np.float32(b[r, j] + s * hstep)
                fsmt.cop_forward(h, T(a), T(bb), kap, wt, obj)
                vals.append(float(obj[r]))
            fd = (vals[0] - vals[1]) / (2 * hstep)
            ref = g["grad_b"][r, j]
        # FD error model: FP32 rounding of U (~ U * 2^-23 / h) plus truncation O(h^2)
        U = float(g["U"][r])
        tol = 4 * U * 2.0 ** -23 / hstep + 1e-2 * abs(ref) + 1e-6
        assert abs(fd - ref) <= tol, (fd, ref, tol)


def test_placement1200_sampled_parity():
    """Paper-scale placement (721,800 constraints, 16 restarts): sampled constraints and
    sampled gradient coordinates against the oracle, in the launch configuration of the
    benchmark."""
    print("placement 1200 sampled parity", flush=True)
    p = W.make_workload("placement_1200")
    R = 16
    a, b = W.initial_points(p, R, 5, 0)
    kap = 0.1
    h = fsmt.xbdd_compile(p)
    ta, tb = T(a.T.copy()).t(), T(b.T.copy()).t()
    ga = torch.zeros(p.n_bool, R, device=dev()).t()
    gb = torch.zeros(p.n_real, R, device=dev()).t()
    wt = T(np.ones(p.n_cons))
    obj = torch.zeros(R, device=dev())
    unsat = torch.zeros(R, p.n_cons, device=dev())
    fsmt.cop_forward(h, ta, tb, kap, wt, obj, unsat)
    fsmt.cop_backward(h, ta, tb, kap, wt, obj, ga, gb)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    sel = np.sort(rng.choice(p.n_cons, 3000, replace=False)).astype(np.int32)
    o = oracle.objective(p, a, b, kap, grad=False, sel=sel)
    assert_unsat(unsat.cpu().numpy()[:, sel], o["unsat"][:, sel])
    # sampled coordinates: all constraints touching the variable give its exact partial
    N = p.meta["n_rect"]
    ii, jj = np.triu_indices(N, 1)
    gga, ggb = ga.cpu().numpy(), gb.cpu().numpy()
    for rect in rng.choice(N, 3, replace=False):
        touch = np.nonzero((ii == rect) | (jj == rect))[0]
        sel2 = np.concatenate([touch, [len(ii) + 2 * rect, len(ii) + 2 * rect + 1]]).astype(np.int32)
        o2 = oracle.objective(p, a, b, kap, sel=sel2, per_constraint=False)
        for r in range(R):
            tol_a = 1e-5 * o2["absg_a"][r, rect] + 1e-9
            assert abs(gga[r, rect] - o2["grad_a"][r, rect]) <= tol_a
            for j in (rect, N + rect):
                tol = 1e-5 * o2["absg_b"][r, j] + 4e-7 * o2["absg_b"][r, j] + 1e-9
                assert abs(ggb[r, j] - o2["grad_b"][r, j]) <= tol, (r, j, ggb[r, j], o2["grad_b"][r, j])


def test_argument_errors_launch_nothing():
    p = W.make_workload("scheduling_10x2")
    h = fsmt.xbdd_compile(p)
    a, b = W.initial_points(p, 2, 1, 0)
    ta, tb = T(a), T(b)
    obj = torch.full((2,), 7.0, device=dev())
    with pytest.raises(fsmt.FsmtError) as e:
        fsmt.cop_forward(h, ta, tb[:, :-1], 1.0, T(np.ones(p.n_cons)), obj)
    assert e.value.code == fsmt._abi.FSMT_EINVAL
    with pytest.raises(fsmt.FsmtError):
        fsmt.cop_forward(h, ta, tb, -1.0, T(np.ones(p.n_cons)), obj)
    host = torch.zeros(2, p.n_bool)
    with pytest.raises(fsmt.FsmtError):
        fsmt.cop_forward(h, host, tb, 1.0, T(np.ones(p.n_cons)), obj)
    torch.cuda.synchronize()
    assert float(obj[0]) == 7.0


def test_uneven_batch_per_instance_oracle_error():
    """Uneven batch (48 instances, 16 restarts each): FP32 objective and false masses of every
    instance against the FP64 oracle (up to 3,000 sampled constraints per instance); the
    table of per-instance errors is printed."""
    print("uneven batch per-instance oracle error", flush=True)
    probs = W.uneven_batch()
    R = 16
    rng = np.random.default_rng(4)
    worst = 0.0
    for i, p in enumerate(probs):
        h = fsmt.xbdd_compile(p)
        a, b = W.initial_points(p, R, 4, i)
        kap = 0.5 / p.meta.get("mean_duration", p.meta.get("mean_side", 1.0))
        unsat = torch.zeros(R, p.n_cons, device=dev())
        obj = torch.zeros(R, device=dev())
        fsmt.cop_forward(h, T(a), T(b), kap, T(np.ones(p.n_cons)), obj, unsat)
        torch.cuda.synchronize()
        sel = np.arange(p.n_cons, dtype=np.int32) if p.n_cons <= 3000 else \
            np.sort(rng.choice(p.n_cons, 3000, replace=False)).astype(np.int32)
        o = oracle.objective(p, a, b, kap, grad=False, sel=sel)
        g = unsat.cpu().numpy()[:, sel].astype(np.float64)
        ref = o["unsat"][:, sel]
        assert_unsat(g.astype(np.float32), ref)
        rel_u = np.abs(g.sum(1) - ref.sum(1)) / np.maximum(ref.sum(1), 1e-30)
        err = np.abs(g - ref) / (ref + 1e-7)
        worst = max(worst, float(rel_u.max()))
        print(f"instance {i:2d} {p.meta.get('family', '?'):10s} C={p.n_cons:7d} "
              f"sampled={len(sel):5d} max|dU|/U={rel_u.max():.2e} max per-constraint rel={err.max():.2e}",
              flush=True)
        h.free()
    assert worst <= 1e-5


def test_placement1200_autograd_and_full_check():
    """Paper-scale placement through torch.autograd.Function (16 restarts): the gradient equals
    the reverse sweep's, a few projected steps lower U, and the exact check of the final
    rounded assignment equals the oracle's over all 721,800 constraints."""
    print("placement 1200 autograd + full check", flush=True)
    from paper_2603_22877_amd import solver as S
    p = W.make_workload("placement_1200")
    R = 16
    a0, b0 = W.initial_points(p, R, 5, 1)
    h = fsmt.xbdd_compile(p)
    w = T(np.ones(p.n_cons))
    kap = 2.0 / p.meta["mean_side"]
    a = T(a0).requires_grad_(True)
    b = T(b0).requires_grad_(True)
    U = S.cop_objective(a, b, h, kap, w)
    U.sum().backward()
    ga = torch.zeros(R, p.n_bool, device=dev())
    gb = torch.zeros(R, p.n_real, device=dev())
    obj = torch.zeros(R, device=dev())
    fsmt.cop_backward(h, a.detach(), b.detach(), kap, w, obj, ga, gb)
    torch.cuda.synchronize()
    rel = (a.grad - ga).norm() / ga.norm()
    relb = (b.grad - gb).norm() / gb.norm()
    assert float(rel) < 1e-5 and float(relb) < 1e-5
    with torch.no_grad():
        aa, bb = a.detach().clone(), b.detach().clone()
    gsq = torch.zeros(R, device=dev())
    U0 = U.detach().clone()
    for _ in range(5):
        ga.zero_()
        gb.zero_()
        fsmt.cop_backward(h, aa, bb, kap, w, obj, ga, gb)
        fsmt.pgd_step(h, aa, bb, ga, gb, 0.05, 0.5, gsq)
    obj.zero_()
    fsmt.cop_forward(h, aa, bb, kap, w, obj)
    torch.cuda.synchronize()
    print(f"U mean {float(U0.mean()):.2f} -> {float(obj.mean()):.2f}", flush=True)
    assert float(obj.mean()) < float(U0.mean())
    nw = (p.n_cons + 31) // 32
    bits = torch.zeros(R, nw, dtype=torch.int32, device=dev())
    nu = torch.zeros(R, dtype=torch.int32, device=dev())
    ver = torch.zeros(R, dtype=torch.int32, device=dev())
    x = torch.zeros(R, p.n_bool, dtype=torch.int8, device=dev())
    fsmt.round_and_check(h, aa, bb, x, bits, nu, ver)
    torch.cuda.synchronize()
    ch = oracle.check(p, aa.cpu().numpy(), bb.cpu().numpy())
    np.testing.assert_array_equal(bits.cpu().numpy().view(np.uint32), ch["sat_bits"])
    np.testing.assert_array_equal(nu.cpu().numpy(), ch["n_unsat"])
    np.testing.assert_array_equal(ver.cpu().numpy(), ch["verdict"])
    np.testing.assert_array_equal(x.cpu().numpy(), ch["x"])
    print(f"n_unsat per restart: {nu.cpu().numpy().tolist()}", flush=True)


# ---- the paper's scheduling and 3D-placement encodings (index bits, XOR disjunctions)
def _paper_instance(fam, A, B, k=0):
    from workloads.paper_suite import make_paper_placement, make_paper_scheduling
    if fam == "sched":
        return make_paper_scheduling(A, B, W.seed_seq(8, A, B, k))
    return make_paper_placement(A, B, W.seed_seq(9, A, B, k))


@pytest.mark.parametrize("fam,A,B", [("sched", 16, 2), ("sched", 32, 2), ("sched", 8, 5), ("sched", 64, 2),
                                     ("place", 2, 2), ("place", 4, 4), ("place", 8, 4), ("place", 8, 8)])
@pytest.mark.parametrize("R", [1, 5, 16])
def test_paper_suite_cop_parity(fam, A, B, R):
    p = _paper_instance(fam, A, B)
    info = fsmt.xbdd_info(fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY))
    print(f"paper {fam} {A}x{B} R={R} cons={p.n_cons} nodes={info['max_nodes']} "
          f"slots={info['max_slots']} big={info['n_big']}", flush=True)
    a, b = W.initial_points(p, R, 11, A, B)
    a[0], b[0] = 0.8 * p.cert_x, p.cert_y        # near the certificate
    ell = p.meta.get("mean_duration", p.meta.get("mean_side"))
    w = np.random.default_rng(A * 10 + B).uniform(0.5, 2, (R, p.n_cons))
    for kap in (0.5 / ell, 4.0 / ell, INF):
        _compare(p, a, b, kap, w=w)


@pytest.mark.parametrize("fam,A,B,R", [("sched", 16, 2, 100), ("place", 2, 4, 70)])
def test_paper_suite_many_restarts(fam, A, B, R):
    """More than 64 restarts (lanes are restarts of one constraint, one wave per 64): the
    closed-form pair path and the generic path against the oracle, rows and columns layout."""
    p = _paper_instance(fam, A, B)
    a, b = W.initial_points(p, R, 15, A, B)
    ell = p.meta.get("mean_duration", p.meta.get("mean_side"))
    for kap in (1.0 / ell, 8.0 / ell):
        _compare(p, a, b, kap)
        _compare(p, a, b, kap, layout="cols")


@pytest.mark.parametrize("R,kap", [(1, 2.0), (2, 20.0)])
def test_paper_placement_large_register_store(R, kap):
    """32 macros x 8 layers: 8 index bits per module pair, 28-node / 20-slot diagrams in the
    largest register store (one lane per constraint), and with LDS messages forced in LDS
    columns (36 KB per wavefront). Both against one oracle evaluation (about 30 s per
    restart on one core)."""
    p = _paper_instance("place", 32, 8)
    info = fsmt.xbdd_info(fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY))
    lds = fsmt.xbdd_info(fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY, messages=1))
    print(f"paper placement 32x8 R={R} cons={p.n_cons} nodes={info['max_nodes']} big={info['n_big']}", flush=True)
    assert info["max_nodes"] == 28 and info["n_big"] == 0 and lds["n_big"] == 0
    a, b = W.initial_points(p, R, 12, R)
    a[0], b[0] = 0.8 * p.cert_x, p.cert_y
    o = oracle.objective(p, a, b, kap)
    for messages in ("auto", "lds"):
        h = fsmt.xbdd_compile(p, messages=MSG[messages])
        g = _run_cop(p, h, a, b, kap)
        assert_objective(g["U_fwd"], o["U"], p.n_cons)
        assert_objective(g["U"], o["U"], p.n_cons)
        assert_unsat(g["unsat"], o["unsat"])
        assert_gradient(g["grad_a"], o["grad_a"], o["absg_a"], "grad_a")
        assert_gradient(g["grad_b"], o["grad_b"], o["absg_b"], "grad_b")
        h.free()


def test_paper_placement_64x8_sampled():
    """64 macros x 8 layers (410,304 constraints, 31-node / 22-slot diagrams beyond the
    register bounds: one lane per constraint with LDS message columns). The full oracle is
    too slow here, so sampled constraints are checked one by one against the oracle's
    per-constraint probability at the same literal probabilities, and the objective against
    the sum of the per-constraint values."""
    p = _paper_instance("place", 64, 8)
    h = fsmt.xbdd_compile(p)
    info = fsmt.xbdd_info(h)
    print(f"paper placement 64x8 cons={p.n_cons} big={info['n_big']}", flush=True)
    assert info["max_nodes"] == 31 and info["n_big"] == 0
    R, kap = 2, 10.0
    a, b = W.initial_points(p, R, 14, 2)
    a[0], b[0] = 0.8 * p.cert_x, p.cert_y
    g = _run_cop(p, h, a, b, kap)
    rng = np.random.default_rng(3)
    sample = np.concatenate([rng.choice(p.meta["n_routing"] * 7, 8, replace=False),
                             p.n_cons - 1 - rng.choice(p.n_cons // 2, 24, replace=False)])
    for r in range(R):
        pv = oracle.variable_probs(p, a[r], b[r], kap)
        ref = np.array([oracle.cop_one(p, int(c), pv)[1] for c in sample])
        assert_unsat(g["unsat"][r, sample], ref)
        assert abs(g["U"][r] - g["unsat"][r].astype(np.float64).sum()) <= 1e-5 * g["U"][r] + 1e-6 * p.n_cons
    assert np.all(np.isfinite(g["grad_a"])) and np.all(np.isfinite(g["grad_b"]))
    h.free()


@pytest.mark.parametrize("fam,A,B", [("sched", 16, 2), ("sched", 32, 3), ("place", 4, 8), ("place", 32, 8)])
def test_paper_suite_check_bit_exact(fam, A, B):
    p = _paper_instance(fam, A, B)
    a, b = W.initial_points(p, 8, 13, A, B)
    a[0], b[0] = p.cert_x, p.cert_y
    a[1], b[1] = p.cert_x, p.cert_y.copy()
    b[1, 0] += 0.3
    h = fsmt.xbdd_compile(p)
    g = _check_gpu(p, h, a, b)
    _assert_check_equal(g, oracle.check(p, a, b))
    assert g["verdict"][0] == 1
