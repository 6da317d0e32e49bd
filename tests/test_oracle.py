"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
import workloads as W
from workloads.format import (KIND_AND, KIND_CARD_GE, KIND_CARD_LE, KIND_CLAUSE, KIND_NAE,
                              KIND_XOR, OP_GE, OP_GT, OP_LE, OP_LT, Builder, lit)


def f32(x):
    return float(np.float32(x))


# ------------------------------------------------------------------ Fig. 2 closed form
@pytest.mark.parametrize("a,b,kap", [(0.3, 0.2, 1.5), (-0.7, -0.4, 0.5), (0.05, 0.9, 2.0),
                                     (0.999, -0.001, 0.1), (-1.0, 0.5, 0.0)])
def test_fig2_toy_closed_form(a, b, kap):
    """Fig. 2 toy: C = 1/2 + a/2 + d/2 - 3ad/2 with d = erf(-kappa b / sqrt 2), U = (C+2)/2."""
    p = W.make_fig2_toy()
    a, b = f32(a), f32(b)
    o = oracle.objective(p, [[a]], [[b]], kap)
    d = -math.erf(kap * b / math.sqrt(2))
    C = 0.5 + a / 2 + d / 2 - 1.5 * a * d
    assert o["U"][0] == pytest.approx((C + 2.0) / 2.0, rel=1e-13, abs=1e-14)
    dC_da = 0.5 - 1.5 * d
    dd_db = -(math.sqrt(2) * kap / math.sqrt(math.pi)) * math.exp(-kap * kap * b * b / 2)
    dC_db = (0.5 - 1.5 * a) * dd_db
    assert o["grad_a"][0, 0] == pytest.approx(dC_da / 2, rel=1e-12, abs=1e-14)
    assert o["grad_b"][0, 0] == pytest.approx(dC_db / 2, rel=1e-12, abs=1e-14)


def test_fig2_vertices_hard():
    """At sigma = 0 (kappa = inf) the objective is the exact F_w: global minimum -sum w at
    x = True, y > 0; local minimum 0 at x = False, y <= 0; 2 elsewhere (Fig. 2 text)."""
    p = W.make_fig2_toy()
    inf = float("inf")
    cases = [((-1.0, 0.5), -2.0), ((1.0, -0.5), 0.0), ((-1.0, -0.5), 2.0), ((1.0, 0.5), 2.0)]
    for (a, b), C in cases:
        o = oracle.objective(p, [[a]], [[b]], inf)
        assert o["U"][0] == (C + 2.0) / 2.0
        assert o["grad_b"][0, 0] == 0.0


# ------------------------------------------------------------ enumeration / Shannon / xWFE
@pytest.mark.parametrize("seed", range(6))
def test_shannon_equals_enumeration_and_python_brute(seed):
    p = W.make_random_formula(seed, n_cons=20, max_len=6)
    rng = np.random.default_rng(seed)
    pv = rng.random(p.n_bool + p.n_atoms)
    pv[rng.random(len(pv)) < 0.1] = 0.0
    pv[rng.random(len(pv)) < 0.1] = 1.0
    for c in range(p.n_cons):
        PT, PF = oracle.cop_enum(p, c, pv)
        PT2, PF2, _ = oracle.cop_one(p, c, pv)
        assert PT + PF == pytest.approx(1.0, abs=1e-12)
        assert PT2 + PF2 == pytest.approx(1.0, abs=1e-12)
        assert PF2 == pytest.approx(PF, abs=1e-13)
        assert PF == pytest.approx(brute.enumerate_unsat(p, c, pv), abs=1e-13)


@pytest.mark.parametrize("seed", range(4))
def test_xwfe_product_form_equals_cop(seed):
    """Eq. expectation2 / Cor. cop=wfe: sum f^(S,T) prod a prod d = E f = 1 - 2 COP."""
    p = W.make_random_formula(100 + seed, n_cons=15, max_len=5)
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, p.n_bool).astype(np.float32)
    b = rng.uniform(-2, 2, p.n_real).astype(np.float32)
    kap = 0.8
    pv = oracle.variable_probs(p, a, b, kap)
    o = oracle.objective(p, a[None], b[None], kap)
    for c in range(p.n_cons):
        sup, f = brute.truth_table(p, c)
        coef = brute.xwfe_coefficients(f)
        v = 1.0 - 2.0 * pv[sup]                  # E[z] = a_i (Booleans), d_i (atoms)
        Ef = brute.xwfe_expectation(coef, v)
        assert (1.0 - Ef) / 2.0 == pytest.approx(o["sat"][0, c], abs=1e-12)
        assert (1.0 + Ef) / 2.0 == pytest.approx(o["unsat"][0, c], abs=1e-12)


def test_xwfe_coefficients_of_known_functions():
    """WFE of textbook functions: XOR of 2 is the product; AND of 2 is (1+x+y-xy)/2."""
    b = Builder(2, 1, [-1], [1])
    b.add(KIND_XOR, [lit(0), lit(1)])
    b.add(KIND_AND, [lit(0), lit(1)])
    p = b.build()
    _, fx = brute.truth_table(p, 0)
    _, fa = brute.truth_table(p, 1)
    np.testing.assert_allclose(brute.xwfe_coefficients(fx), [0, 0, 0, 1])
    np.testing.assert_allclose(brute.xwfe_coefficients(fa), [0.5, 0.5, 0.5, -0.5])


# ------------------------------------------------------------------ closed forms
def _closed_form_problem(L, kinds_params):
    b = Builder(L, 1, [-1], [1])
    rng = np.random.default_rng(L)
    negs = rng.integers(0, 2, L).astype(bool)
    for kind, k in kinds_params:
        b.add(kind, [lit(i, bool(negs[i])) for i in range(L)], k)
    return b.build(), negs


@pytest.mark.parametrize("L", [1, 2, 5, 9, 16, 40])
def test_symmetric_closed_forms(L):
    kinds = [(KIND_CLAUSE, 0), (KIND_AND, 0), (KIND_XOR, 0), (KIND_NAE, 0),
             (KIND_CARD_LE, L // 3), (KIND_CARD_GE, (2 * L) // 3)]
    p, negs = _closed_form_problem(L, kinds)
    rng = np.random.default_rng(7 + L)
    a = rng.uniform(-1, 1, L).astype(np.float32)
    o = oracle.objective(p, a[None], np.zeros((1, 1), np.float32), 1.0)
    pv = (1.0 - a.astype(np.float64)) / 2.0
    pl = np.where(negs, 1.0 - pv, pv)                      # P[literal True]
    v = 1.0 - 2.0 * pl                                     # E of the +-1 literal
    # count distribution by polynomial multiplication (independent of the oracle's DP)
    dist = np.array([1.0])
    for q in pl:
        dist = np.convolve(dist, [1.0 - q, q])
    t = np.arange(L + 1)
    expect_sat = [1.0 - np.prod(1.0 - pl),                 # clause
                  np.prod(pl),                             # AND
                  (1.0 - np.prod(v)) / 2.0,                # XOR: E f = prod v
                  1.0 - np.prod(pl) - np.prod(1.0 - pl),   # NAE
                  dist[t <= L // 3].sum(),                 # CARD_LE
                  dist[t >= (2 * L) // 3].sum()]           # CARD_GE
    np.testing.assert_allclose(o["sat"][0], expect_sat, rtol=1e-11, atol=1e-14)
    # clause unsat is the product of the literal-false probabilities (no subtraction)
    assert o["unsat"][0, 0] == pytest.approx(np.prod(1.0 - pl), rel=1e-12)
    # gradient (count-distribution path for L > 12): U is affine in each a_i
    a = (np.round(a * 1024) / 1024).astype(np.float32)
    o = oracle.objective(p, a[None], np.zeros((1, 1), np.float32), 1.0)
    for i in range(0, L, max(1, L // 5)):
        ap, am = a.copy(), a.copy()
        ap[i] += 2.0 ** -6
        am[i] -= 2.0 ** -6
        fd = (oracle.objective(p, ap[None], np.zeros((1, 1), np.float32), 1.0, grad=False)["U"][0]
              - oracle.objective(p, am[None], np.zeros((1, 1), np.float32), 1.0, grad=False)["U"][0]
              ) / 2.0 ** -5
        assert o["grad_a"][0, i] == pytest.approx(fd, rel=1e-9, abs=1e-12)


# ------------------------------------------------------------------ Monte Carlo
@pytest.mark.parametrize("seed", range(3))
def test_monte_carlo_independent_atoms_converges(seed):
    """Sampling x by randomized rounding and atoms independently converges to the COP."""
    p = W.make_random_formula(200 + seed, n_cons=10, max_len=5)
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, p.n_bool).astype(np.float32)
    b = rng.uniform(-2, 2, p.n_real).astype(np.float32)
    kap = 1.3
    pv = oracle.variable_probs(p, a, b, kap)
    o = oracle.objective(p, a[None], b[None], kap, grad=False)
    N = 400_000
    for c in range(p.n_cons):
        mc = brute.monte_carlo_sat(p, c, pv, N, rng)
        cop = o["sat"][0, c]
        se = math.sqrt(max(cop * (1 - cop), 1e-12) / N)
        assert abs(mc - cop) <= 5 * se + 1e-9


def test_joint_gaussian_sampling_matches_for_orthogonal_atoms_only():
    """Atoms on distinct variables: joint Gaussian sampling equals the product-of-marginals
    COP. OR(y <= 0, y >= 1) shares y: joint sampling gives P_A + P_B while the
    message-passing model (independent atom marginals) gives P_A + P_B - P_A P_B."""
    rng = np.random.default_rng(5)
    bl = Builder(0, 2, [-5, -5], [5, 5])
    A = bl.atom([0], [1.0], OP_LE, 0.0)
    B = bl.atom([1], [2.0], OP_GE, 1.0)
    C_ = bl.atom([0], [1.0], OP_GE, 1.0)
    bl.add(KIND_CLAUSE, [lit(A), lit(B)])       # distinct variables
    bl.add(KIND_CLAUSE, [lit(A), lit(C_)])      # shared variable
    p = bl.build()
    b = np.array([0.3, 0.6], np.float32)
    sigma = 0.7
    o = oracle.objective(p, np.zeros((1, 0), np.float32), b[None], 1.0 / sigma, grad=False)
    N = 400_000
    mc0 = brute.monte_carlo_joint_gaussian(p, 0, np.zeros(0), b.astype(np.float64), sigma, N, rng)
    se = math.sqrt(0.25 / N)
    assert abs(mc0 - o["sat"][0, 0]) <= 5 * se
    PA = 0.5 * math.erfc(float(b[0]) / (math.sqrt(2) * sigma))
    PC = 0.5 * math.erfc((1.0 - float(b[0])) / (math.sqrt(2) * sigma))
    assert o["sat"][0, 1] == pytest.approx(PA + PC - PA * PC, rel=1e-12)
    mc1 = brute.monte_carlo_joint_gaussian(p, 1, np.zeros(0), b.astype(np.float64), sigma, N, rng)
    assert abs(mc1 - (PA + PC)) <= 5 * se


# ------------------------------------------------------------------ gradients
@pytest.mark.parametrize("seed", range(3))
def test_gradient_central_differences(seed):
    p = W.make_random_formula(300 + seed, n_bool=5, n_real=3, n_atoms=5, n_cons=14)
    rng = np.random.default_rng(seed)
    grid = 2.0 ** -12
    a = (np.round(rng.uniform(-0.9, 0.9, p.n_bool) / grid) * grid).astype(np.float32)
    b = (np.round(rng.uniform(-1.5, 1.5, p.n_real) / grid) * grid).astype(np.float32)
    w = rng.uniform(0.5, 2.0, p.n_cons)
    kap = 0.9
    o = oracle.objective(p, a[None], b[None], kap, w=w)
    h = 2.0 ** -7
    for i in range(p.n_bool):          # U is affine in each a_i: central difference is exact
        ap, am = a.copy(), a.copy()
        ap[i] += h
        am[i] -= h
        fd = (oracle.objective(p, ap[None], b[None], kap, w=w, grad=False)["U"][0]
              - oracle.objective(p, am[None], b[None], kap, w=w, grad=False)["U"][0]) / (2 * h)
        assert o["grad_a"][0, i] == pytest.approx(fd, rel=1e-9, abs=1e-12)
    h = 2.0 ** -10
    for j in range(p.n_real):
        vals = []
        for s in (-2, -1, 1, 2):
            bb = b.copy()
            bb[j] += s * h
            vals.append(oracle.objective(p, a[None], bb[None], kap, w=w, grad=False)["U"][0])
        fd = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)     # 4th order
        assert o["grad_b"][0, j] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_multilinearity_second_difference_zero():
    """Thm. Optimality rests on U being multilinear in a: U(a + t e_i) is affine in t."""
    p = W.make_random_formula(400, n_cons=20)
    rng = np.random.default_rng(1)
    a = (np.round(rng.uniform(-0.5, 0.5, p.n_bool) * 4096) / 4096).astype(np.float32)
    b = rng.uniform(-1, 1, p.n_real).astype(np.float32)
    h = 0.25                                         # a +- h exact in float32
    for i in range(p.n_bool):
        U = []
        for s in (-1, 0, 1):
            aa = a.copy()
            aa[i] += s * h
            U.append(oracle.objective(p, aa[None], b[None], 0.7, grad=False)["U"][0])
        assert U[0] + U[2] - 2 * U[1] == pytest.approx(0.0, abs=1e-12)


def test_derivative_bound_of_smoothed_atom():
    """|d d_i / d b_j| <= sqrt(2) kappa / sqrt(pi) (Prop. Lipschitz): |dp/db_j| <= kappa/sqrt(2 pi)."""
    p = W.make_random_formula(500, n_atoms=12, n_cons=3)
    rng = np.random.default_rng(2)
    for kap in (0.1, 1.0, 7.0):
        b = rng.uniform(-3, 3, p.n_real).astype(np.float32)
        _, dpdz, _ = oracle.atom_probs(p, b, kap)
        for k in range(p.n_atoms):
            s = slice(p.atom_ptr[k], p.atom_ptr[k + 1])
            dpdb = np.abs(dpdz[k] * p.atom_coef[s])
            assert np.all(dpdb <= kap / math.sqrt(2 * math.pi) * (1 + 1e-12))


def test_kappa_zero_gives_half_and_no_real_gradient():
    p = W.make_random_formula(501, n_cons=10)
    rng = np.random.default_rng(3)
    b = rng.uniform(-3, 3, p.n_real).astype(np.float32)
    pr, dz, _ = oracle.atom_probs(p, b, 0.0)
    assert np.all(pr == 0.5) and np.all(dz == 0.0)
    a = rng.uniform(-1, 1, p.n_bool).astype(np.float32)
    o = oracle.objective(p, a[None], b[None], 0.0)
    assert np.all(o["grad_b"] == 0.0)


# ------------------------------------------------------------------ check
def _py_check(p, a, b):
    """Independent Python check: rounding x = True iff a < 0, exact atom tests."""
    n = p.n_bool
    truth = {i: bool(a[i] < 0) for i in range(n)}
    for k in range(p.n_atoms):
        acc = 0.0
        for e in range(p.atom_ptr[k], p.atom_ptr[k + 1]):
            acc = acc + float(p.atom_coef[e]) * float(np.float32(b[p.atom_var[e]]))
        z = acc - float(p.atom_rhs[k])
        op = int(p.atom_op[k])
        truth[n + k] = {OP_LE: z <= 0, OP_LT: z < 0, OP_GE: z >= 0, OP_GT: z > 0}[op]
    return np.array([brute.formula_value(p, c, truth) for c in range(p.n_cons)])


@pytest.mark.parametrize("seed", range(4))
def test_check_matches_python_formula_evaluation(seed):
    p = W.make_random_formula(600 + seed, n_cons=40)
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, (3, p.n_bool)).astype(np.float32)
    a[0, :2] = [0.0, -0.0]
    b = rng.uniform(-2, 2, (3, p.n_real)).astype(np.float32)
    ch = oracle.check(p, a, b)
    for r in range(3):
        sat = _py_check(p, a[r], b[r])
        bits = np.array([(ch["sat_bits"][r, c >> 5] >> (c & 31)) & 1 for c in range(p.n_cons)])
        np.testing.assert_array_equal(bits.astype(bool), sat)
        assert ch["n_unsat"][r] == (~sat).sum()
        assert ch["verdict"][r] == int(sat.all())
        np.testing.assert_array_equal(ch["x"][r], np.where(a[r] < 0, -1, 1))


def test_check_boundary_and_nan():
    """z = 0 exactly: <= and >= hold, < and > do not; NaN compares false; sgn(+-0) = False."""
    bl = Builder(1, 1, [-1], [1])
    ids = [bl.atom([0], [1.0], op, 0.25) for op in (OP_LE, OP_LT, OP_GE, OP_GT)]
    for v in ids:
        bl.add(KIND_CLAUSE, [lit(v)])
    bl.add(KIND_CLAUSE, [lit(0)])
    p = bl.build()
    ch = oracle.check(p, np.array([[0.0], [-0.0], [np.nan]], np.float32),
                      np.array([[0.25], [0.25], [np.nan]], np.float32))
    bits = ch["sat_bits"][:, 0]
    assert bits[0] == 0b00101 and bits[1] == 0b00101 and bits[2] == 0


@pytest.mark.parametrize("name", ["scheduling_10x2", "scheduling_200x10", "placement_150"])
def test_generator_certificates_are_sat(name):
    """Thm. Soundness: the certificate satisfies every constraint, and there U = 0 at kappa = inf."""
    p = W.make_workload(name)
    a = p.cert_x.astype(np.float32)[None]
    b = p.cert_y.astype(np.float32)[None]
    ch = oracle.check(p, a, b)
    assert ch["verdict"][0] == 1 and ch["n_unsat"][0] == 0
    o = oracle.objective(p, a, b, float("inf"), grad=False)
    assert o["U"][0] == 0.0


@pytest.mark.parametrize("seed", range(3))
def test_hard_objective_at_vertices_counts_violations(seed):
    """sigma = 0 at a vertex: every P_false is 0 or 1 and U = number of violated constraints."""
    p = W.make_random_formula(700 + seed, n_cons=30)
    rng = np.random.default_rng(seed)
    a = np.where(rng.random((2, p.n_bool)) < 0.5, -1.0, 1.0).astype(np.float32)
    b = rng.uniform(-2, 2, (2, p.n_real)).astype(np.float32)
    o = oracle.objective(p, a, b, float("inf"), grad=False)
    ch = oracle.check(p, a, b)
    assert set(np.unique(o["unsat"])) <= {0.0, 1.0}
    np.testing.assert_array_equal(o["U"], ch["n_unsat"].astype(float))


def test_planted_violation_in_certificate():
    p = W.make_workload("scheduling_10x2")
    a = p.cert_x.astype(np.float32).copy()
    b = p.cert_y.astype(np.float32).copy()
    b[0] = p.real_hi[0]                     # job 0 starts at the horizon: horizon atom fails
    ch = oracle.check(p, a[None], b[None])
    assert ch["verdict"][0] == 0 and ch["n_unsat"][0] >= 1
    assert (~_py_check(p, a, b)).sum() == ch["n_unsat"][0]


# ------------------------------------------------------------------ PGD
def test_pgd_projection_closed_form():
    p = W.make_workload("scheduling_10x2")
    rng = np.random.default_rng(0)
    a = rng.uniform(-1, 1, (2, p.n_bool)).astype(np.float32)
    b = rng.uniform(0, p.real_hi[0], (2, p.n_real)).astype(np.float32)
    ga = rng.normal(size=a.shape).astype(np.float32) * 10
    gb = rng.normal(size=b.shape).astype(np.float32) * 100
    st = oracle.pgd(p, a, b, ga, gb, 0.1, 0.5, unit_proj=False)
    ea = np.clip(a.astype(np.float64) - 0.1 * ga.astype(np.float64), -1, 1)
    eb = np.clip(b.astype(np.float64) - 0.5 * gb.astype(np.float64), p.real_lo, p.real_hi)
    np.testing.assert_array_equal(st["a"], ea)
    np.testing.assert_array_equal(st["b"], eb)
    g2 = (((a - ea) / 0.1) ** 2).sum(1) + (((b - eb) / 0.5) ** 2).sum(1)
    np.testing.assert_allclose(st["gsq"], g2, rtol=1e-12)
    assert np.all((st["a"] >= -1) & (st["a"] <= 1))


@pytest.mark.parametrize("seed", range(3))
def test_descent_lemma_with_lipschitz_step(seed):
    """Lemma Descent with eta = 1/L of Prop. Lipschitz: U drops by >= (eta/2)||g||^2."""
    p = W.make_random_formula(800 + seed, n_bool=4, n_real=2, n_atoms=3, n_cons=6, box=2.0)
    rng = np.random.default_rng(seed)
    kap = 1.0
    alpha = float(p.n_cons)                          # sum of weights
    beta = 1
    for c in range(p.n_cons):                        # occurrences of a real var in a constraint
        cnt = {}
        for v in brute.support(p, c):
            if v >= p.n_bool:
                k = v - p.n_bool
                for j in p.atom_var[p.atom_ptr[k]:p.atom_ptr[k + 1]]:
                    cnt[j] = cnt.get(j, 0) + 1
        beta = max([beta] + list(cnt.values()))
    gam = math.sqrt(2) * beta * kap / math.sqrt(math.pi)
    n, m = p.n_bool, p.n_real
    rho_ = alpha * math.sqrt(n + m) * max(1.0, gam)
    L = math.sqrt(n + m * gam * gam) * rho_
    eta = 1.0 / L
    a = rng.uniform(-1, 1, (1, n)).astype(np.float32)
    b = rng.uniform(-2, 2, (1, m)).astype(np.float32)
    for _ in range(5):
        o = oracle.objective(p, a, b, kap, per_constraint=False)
        st = oracle.pgd(p, a, b, o["grad_a"].astype(np.float32), o["grad_b"].astype(np.float32),
                        eta, eta)
        a2, b2 = st["a"].astype(np.float32), st["b"].astype(np.float32)
        U2 = oracle.objective(p, a2, b2, kap, grad=False)["U"][0]
        assert U2 <= o["U"][0] - 0.5 * eta * st["gsq"][0] + 1e-6 * eta * st["gsq"][0] + 1e-12
        a, b = a2, b2


# ------------------------------------------------------------------ ERWA
def test_erwa_two_levels_by_hand():
    """Alg. CLS with Annealing, rho=0.5, gamma=2, tau=1: h = rho h + u, w *= 2^h, h = 1."""
    C = 3
    h = np.zeros((1, C))
    w = np.ones((1, C))
    bits = np.array([[0b101]], np.uint32)            # constraint 1 violated
    oracle.erwa(bits, C, 1, h, w, normalize=False)
    np.testing.assert_allclose(w, [[1.0, 2.0, 1.0]])
    np.testing.assert_allclose(h, [[1.0, 1.0, 1.0]])
    bits = np.array([[0b110]], np.uint32)            # constraint 0 violated
    oracle.erwa(bits, C, 2, h, w, normalize=False)
    np.testing.assert_allclose(w, [[2 ** 1.5, 2.0 * 2 ** 0.5, 2 ** 0.5]])
    h2, w2 = np.zeros((1, C)), np.ones((1, C))
    oracle.erwa(np.array([[0b101]], np.uint32), C, 1, h2, w2, normalize=True)
    np.testing.assert_allclose(w2, [[0.75, 1.5, 0.75]])


def test_anneal_solves_fig2_toy_to_global_minimum():
    """Fig. 2: with sigma annealed from large to small, PGD reaches x = True, y > 0."""
    p = W.make_fig2_toy()
    kappas = [0.1 * t for t in range(1, 21)]
    tr = oracle.anneal(p, np.array([[0.3]], np.float32), np.array([[-0.2]], np.float32), kappas,
                       eta_a=0.5, eta_b=0.5, steps_per_level=50)
    assert tr[-1]["n_unsat"][0] == 0
    assert tr[-1]["a"][0, 0] < 0 and tr[-1]["b"][0, 0] > 0


def _toy_anneal_by_hand(a0, b0, kappas, eta_a, eta_b, steps, eps, rho=0.5, gamma=2.0, tau=1,
                        stop_on_sat=1):
    """Alg. "CLS with Annealing" on the Fig. 2 toy for one restart, from the closed forms.

    Constraints c1 = (not x) XOR A and c2 = x AND A with A = (y > 0). With p = P[x True] =
    (1 - a)/2 and pA = P[A True] = Phi(kappa b) (Eq. "sampling" for the atom -y < 0):
    P[c1 False] = p pA + ... is p (1 - pA) + (1 - p) pA and P[c2 False] = 1 - p pA, so
    dU/dp = w1 (1 - 2 pA) - w2 pA, dU/dpA = w1 (1 - 2 p) - w2 p, dp/da = -1/2 and
    dpA/db = kappa exp(-(kappa b)^2 / 2) / sqrt(2 pi). Iterates are stored in float32 and
    gradients handed to the step in float32, as the oracle does.
    """
    a, b = np.float32(a0), np.float32(b0)
    w, h = np.ones(2), np.zeros(2)
    out, done = [], False
    for t, kap in enumerate(kappas, start=1):
        if done:
            out.append(dict(n_unsat=-1, steps=0, a=a, b=b, w=w.copy()))
            continue
        k = 0
        for _ in range(steps):
            p = (1.0 - float(a)) / 2.0
            pA = 0.5 * math.erfc(-kap * float(b) / math.sqrt(2.0))
            dUdp = w[0] * (1.0 - 2.0 * pA) - w[1] * pA
            dUdpA = w[0] * (1.0 - 2.0 * p) - w[1] * p
            ga = np.float32(-0.5 * dUdp)
            gb = np.float32(dUdpA * kap * math.exp(-(kap * float(b)) ** 2 / 2.0) / math.sqrt(2.0 * math.pi))
            a1 = min(1.0, max(-1.0, float(a) - eta_a * float(ga)))
            b1 = min(1.0, max(-1.0, float(b) - eta_b * float(gb)))
            gsq = ((float(a) - a1) / eta_a) ** 2 + ((float(b) - b1) / eta_b) ** 2
            a, b = np.float32(a1), np.float32(b1)
            k += 1
            if eps > 0 and np.float32(gsq) <= np.float32(eps) * np.float32(eps):
                break
        x, A = bool(a < 0), bool(b > 0)
        viol = np.array([(not x) == A, not (x and A)], float)   # c1 holds iff exactly one is True
        h = rho * h + viol
        if t % tau == 0:
            w = w * gamma ** h
            h = np.ones(2)
            w = w * (2.0 / w.sum())
        nu = int(viol.sum())
        out.append(dict(n_unsat=nu, steps=k, a=a, b=b, w=w.copy()))
        if stop_on_sat and nu == 0:
            done = True
    return out


@pytest.mark.parametrize("stop_on_sat", [1, 0])
def test_anneal_replays_fig2_toy_by_hand_two_restarts(stop_on_sat):
    """Two restarts: (a, b) = (-1, 1) sits at the global minimum (its steps stop at once and,
    with stop_on_sat, it is SAT after level 1 and runs no further level); (0.9, -0.9) starts
    near the local minimum x = False, y <= 0 (Fig. 2) and stays there with one violated
    constraint, its levels ending after 3, 4, 2 and 1 steps. Each restart follows its own
    loop, as the by-hand replay does."""
    p = W.make_fig2_toy()
    kappas = [0.4 * t for t in range(1, 9)]
    a0 = np.array([[-1.0], [0.9]], np.float32)
    b0 = np.array([[1.0], [-0.9]], np.float32)
    kw = dict(eta_a=0.5, eta_b=0.5, steps_per_level=4, eps=0.05)
    tr = oracle.anneal(p, a0, b0, kappas, stop_on_sat=stop_on_sat, **kw)
    hand = [_toy_anneal_by_hand(a0[r, 0], b0[r, 0], kappas, 0.5, 0.5, 4, 0.05, stop_on_sat=stop_on_sat)
            for r in range(2)]
    assert len(tr) == len(kappas)
    for t, lv in enumerate(tr):
        for r in range(2):
            hr = hand[r][t]
            assert lv["n_unsat"][r] == hr["n_unsat"], (t, r)
            assert lv["steps"][r] == hr["steps"], (t, r)
            np.testing.assert_allclose(lv["a"][r, 0], hr["a"], rtol=1e-6, atol=1e-7)
            np.testing.assert_allclose(lv["b"][r, 0], hr["b"], rtol=1e-6, atol=1e-7)
            np.testing.assert_allclose(lv["w"][r], hr["w"], rtol=1e-9)
    # the restarts really took different paths: one stopped stepping at once, the other
    # ended its levels at different step counts, some before the cap
    assert tr[0]["steps"][0] == 1 and tr[0]["steps"][1] > 1
    assert len({int(lv["steps"][1]) for lv in tr}) > 2 and min(int(lv["steps"][1]) for lv in tr) < 4
    if stop_on_sat:
        assert tr[0]["n_unsat"][0] == 0 and all(lv["n_unsat"][0] == -1 for lv in tr[1:])


def test_anneal_restarts_are_independent():
    """Batched restarts give exactly what each restart gives alone (Alg. "FourierSMT" is a
    per-point loop): scheduling 10 x 2 with 3 restarts, eps large enough that they stop at
    different steps."""
    p = W.make_workload("scheduling_10x2")
    a0, b0 = W.initial_points(p, 3, 1, 5)
    ell = p.meta["mean_duration"]
    kap = [4.0 * t / (40 * ell) for t in (1, 2, 3)]
    kw = dict(eta_a=0.5, eta_b=5.0, steps_per_level=6, eps=0.5)
    tr = oracle.anneal(p, a0, b0, kap, stop_on_sat=0, **kw)
    steps_seen = set()
    for r in range(3):
        one = oracle.anneal(p, a0[r:r + 1], b0[r:r + 1], kap, stop_on_sat=0, **kw)
        for t in range(3):
            np.testing.assert_array_equal(tr[t]["a"][r], one[t]["a"][0])
            np.testing.assert_array_equal(tr[t]["b"][r], one[t]["b"][0])
            np.testing.assert_array_equal(tr[t]["w"][r], one[t]["w"][0])
            assert tr[t]["steps"][r] == one[t]["steps"][0]
            steps_seen.add(int(tr[t]["steps"][r]))
    assert len(steps_seen) > 1


# ------------------------------------------------------------------ projection onto D
def _active_set_projection(y0, G, h):
    """Exact argmin ||y - y0||^2 s.t. G y <= h by enumerating active sets (tiny problems)."""
    import itertools
    m = len(y0)
    best = None
    for k in range(0, m + 1):
        for S in itertools.combinations(range(len(h)), k):
            S = list(S)
            if S:
                GS = G[S]
                M = GS @ GS.T
                if abs(np.linalg.det(M)) < 1e-12:
                    continue
                lam = np.linalg.solve(M, GS @ y0 - h[S])
                if np.any(lam < -1e-12):
                    continue
                y = y0 - GS.T @ lam
            else:
                y = y0.copy()
            if np.all(G @ y <= h + 1e-9):
                d = np.sum((y - y0) ** 2)
                if best is None or d < best[0]:
                    best = (d, y)
    return best[1]


@pytest.mark.parametrize("seed", range(8))
def test_projection_onto_unit_atoms_matches_active_set_qp(seed):
    """Def. Projection / Prop. qp: box plus unit atomic constraints (a single atom literal)."""
    rng = np.random.default_rng(seed)
    m = 3
    bl = Builder(1, m, np.full(m, -2.0), np.full(m, 2.0))
    rows, rhs = [], []
    y_star = rng.uniform(-1.5, 0.4, m)                  # a point inside D, so D is not empty
    for t in range(int(rng.integers(1, 4))):
        vs = rng.choice(m, 2, replace=False)
        q = np.round(rng.normal(size=2), 2)
        q[q == 0] = 0.5
        op = int(rng.choice([OP_LE, OP_GE]))
        neg = bool(rng.integers(0, 2))
        s = (1.0 if op == OP_LE else -1.0) * (-1.0 if neg else 1.0)
        q0 = float(q @ y_star[vs] + s * rng.uniform(0.1, 1.0))
        bl.add(KIND_CLAUSE, [lit(bl.atom(vs, q, op, q0), neg)])
        row = np.zeros(m)
        row[vs] = s * q
        delta = 1e-6 * (abs(q0) + np.abs(q).sum() * 2.0)
        rows.append(row)
        rhs.append(s * q0 - delta)
    j = int(rng.integers(m))                            # a single-variable unit atom: a bound
    bl.add(KIND_CLAUSE, [lit(bl.atom([j], [2.0], OP_LE, 1.0))])
    bl.add(KIND_CLAUSE, [lit(0), lit(bl.atom([0, 1], [1.0, 1.0], OP_LE, 0.0))])   # not a unit atom
    p = bl.build()
    G = np.array(rows + [np.eye(m)[i] for i in range(m)] + [-np.eye(m)[i] for i in range(m)])
    hi = np.full(m, 2.0)
    hi[j] = 0.5
    h = np.array(rhs + list(hi) + [2.0] * m)
    for _ in range(5):
        y0 = rng.uniform(-3, 3, m)
        y, lo_, hi_, nh = oracle.project(p, y0)
        assert nh == len(rows)
        assert hi_[j] == 0.5
        np.testing.assert_allclose(y, _active_set_projection(y0, G, h), atol=1e-9)


@pytest.mark.parametrize("name", ["scheduling_10x2", "scheduling_200x10"])
def test_projected_points_satisfy_unit_atoms_after_rounding(name):
    """The shifted half-spaces keep precedences and horizons true at the float32 point."""
    p = W.make_workload(name)
    a, b = W.initial_points(p, 8, W.STREAM[name], 9)
    st = oracle.pgd(p, a, b, np.zeros_like(a), np.zeros_like(b), 0.1, 1.0)
    assert st["n_halfspaces"] == 5
    ch = oracle.check(p, a, st["b"].astype(np.float32))
    P = p.meta["n_pairs"]
    for r in range(8):
        for c in range(2 * P, p.n_cons):              # horizons and precedences
            assert (ch["sat_bits"][r, c >> 5] >> (c & 31)) & 1
