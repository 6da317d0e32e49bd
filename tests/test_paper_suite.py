"""The paper's scheduling and 3D-placement encodings (Methods): generators, oracle and compiler.

CPU only. The encodings are checked against the formulas as the Methods state them (a
direct Python evaluation per constraint), the oracle's probability of a pair constraint
against its closed form, and the compiled diagrams against their closed-form sizes.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from workloads.format import KIND_CLAUSE, KIND_EXPR, KIND_XOR, OP_GE, OP_LE
from workloads.paper_suite import make_paper_placement, make_paper_scheduling

fsmt = pytest.importorskip("paper_2603_22877_amd")


def sched(nw, r, k=0, **kw):
    return make_paper_scheduling(nw, r, W.seed_seq(8, nw, r, k), **kw)


def place(nm, nl, k=0):
    return make_paper_placement(nm, nl, W.seed_seq(9, nm, nl, k))


def _atom(p, aid):
    """(vars, coefs, op, rhs) of the atom with variable id ``aid``."""
    k = aid - p.n_bool
    s, e = p.atom_ptr[k], p.atom_ptr[k + 1]
    return list(p.atom_var[s:e]), list(p.atom_coef[s:e]), int(p.atom_op[k]), float(p.atom_rhs[k])


def _lits(p, c):
    return p.con_lit[p.con_ptr[c]:p.con_ptr[c + 1]]


@pytest.mark.parametrize("nw,r", [(16, 2), (16, 5), (32, 3), (64, 2)])
def test_scheduling_certificate_holds(nw, r):
    p = sched(nw, r)
    ch = oracle.check(p, p.cert_x[None], p.cert_y[None])
    assert ch["n_unsat"][0] == 0 and ch["verdict"][0] == 1
    assert p.n_bool == nw * r * int(np.log2(nw)) and p.n_real == nw * r
    assert p.meta["n_pairs"] == nw * r * (nw * r - 1) // 2
    assert p.n_cons == p.meta["n_deps"] + p.meta["n_pairs"] + nw * r * nw


@pytest.mark.parametrize("nm,nl", [(2, 2), (4, 8), (16, 4), (8, 2)])
def test_placement_certificate_holds(nm, nl):
    p = place(nm, nl)
    ch = oracle.check(p, p.cert_x[None], p.cert_y[None])
    assert ch["n_unsat"][0] == 0 and ch["verdict"][0] == 1
    N = nm * (2 + 3 * nl // 2)
    assert p.meta["n_modules"] == N and p.n_real == 2 * N


def test_certificate_perturbations_violate():
    """Moving one job onto another's worker and start, or one module onto another, breaks it."""
    p = sched(16, 2)
    L, nj = p.meta["n_bits"], p.meta["n_jobs"]
    x, y = p.cert_x.copy().reshape(L, nj), p.cert_y.copy()
    x[:, 1], y[1] = x[:, 0], y[0]
    assert oracle.check(p, x.reshape(1, -1), y[None])["n_unsat"][0] > 0
    q = place(4, 4)
    N = q.meta["n_modules"]
    xb, yy = q.cert_x.copy().reshape(-1, N), q.cert_y.copy()
    xb[:, 1], yy[1], yy[N + 1] = xb[:, 0], yy[0], yy[N]     # small process 1 onto large process 0
    assert oracle.check(q, xb.reshape(1, -1), yy[None])["n_unsat"][0] > 0


def test_scheduling_constraints_are_the_methods_formulas():
    """Every constraint of a small instance, evaluated by the oracle on random truth values,
    equals the Methods formula evaluated here from the instance parameters."""
    p = sched(4, 2, dep_prob=0.6)
    L, nj, nw, T = p.meta["n_bits"], p.meta["n_jobs"], p.meta["n_workers"], p.meta["cutoff"]
    nd, P = p.meta["n_deps"], p.meta["n_pairs"]
    rng = np.random.default_rng(5)
    jj, kk = np.triu_indices(nj, 1)
    for c in range(p.n_cons):
        lits = _lits(p, c)
        ids = lits >> 1
        if c < nd:
            assert p.con_kind[c] == KIND_CLAUSE and len(lits) == 1 and lits[0] & 1 == 0
            v, co, op, rhs = _atom(p, ids[0])
            assert op == OP_GE and co == [1.0, -1.0] and len(v) == 2
            continue
        assert p.con_kind[c] == KIND_EXPR
        if c < nd + P:
            q = c - nd
            j, k = jj[q], kk[q]
            A, B = ids[-2], ids[-1]
            vA, cA, oA, rA = _atom(p, A)
            vB, cB, oB, rB = _atom(p, B)
            assert (oA, oB) == (OP_GE, OP_GE) and vA == [j, k] and vB == [k, j]
            assert cA == [1.0, -1.0] and cB == [1.0, -1.0] and rA > 0 and rB > 0
        else:
            q = c - nd - P
            j, w = q // nw, q % nw
        for _ in range(24):
            truth = rng.integers(0, 2, p.n_bool + p.n_atoms).astype(np.int8)
            bits = truth[:p.n_bool].reshape(L, nj)
            if c < nd + P:
                want = bool(np.any(bits[:, j] != bits[:, k])) or bool(truth[A]) or bool(truth[B])
            else:
                index = int(sum(int(bits[i, j]) << i for i in range(L)))
                C, D = ids[-2], ids[-1]
                vC, _, oC, rC = _atom(p, C)
                vD, _, oD, rD = _atom(p, D)
                assert vC == [j] and vD == [j] and oC == OP_GE and oD == OP_LE and rD - rC < T
                want = index != w or (bool(truth[C]) and bool(truth[D]))
            assert oracle.eval_formula(p, c, truth) == int(want), (c, truth)


def test_scheduling_feasibility_windows():
    """Feasibility atoms of job j and worker w are y_j >= d_w and y_j <= d_w + T - t_j."""
    p = sched(8, 2)
    nj, nw, T = p.meta["n_jobs"], p.meta["n_workers"], p.meta["cutoff"]
    nd, P = p.meta["n_deps"], p.meta["n_pairs"]
    jj, kk = np.triu_indices(nj, 1)
    t = np.zeros(nj)
    for q in range(P):                           # t_k from the pair atoms A: y_j - y_k >= t_k
        t[kk[q]] = _atom(p, _lits(p, nd + q)[-2] >> 1)[3]
        t[jj[q]] = _atom(p, _lits(p, nd + q)[-1] >> 1)[3]
    for q in range(nj * nw):
        j, w = q // nw, q % nw
        lits = _lits(p, nd + P + q)
        dw = _atom(p, lits[-2] >> 1)[3]
        assert _atom(p, lits[-1] >> 1)[3] == pytest.approx(dw + T - t[j], abs=4e-7)


@pytest.mark.parametrize("make", [lambda: sched(16, 3), lambda: place(4, 8)])
def test_constants_are_float32(make):
    """Atom coefficients and right-hand sides are float32 values (exact device records)."""
    p = make()
    for x in (p.atom_coef, p.atom_rhs):
        np.testing.assert_array_equal(x.astype(np.float32).astype(np.float64), x)


def test_placement_constraints_are_the_methods_formulas():
    p = place(2, 4)
    N, Lm, Ll = p.meta["n_modules"], p.meta["n_macro_bits"], p.meta["n_layer_bits"]
    rng = np.random.default_rng(6)
    kinds = {}
    for c in range(p.n_cons):
        kinds.setdefault(int(p.con_kind[c]), 0)
        kinds[int(p.con_kind[c])] += 1
        lits = _lits(p, c)
        ids = lits >> 1
        for _ in range(16):
            truth = rng.integers(0, 2, p.n_bool + p.n_atoms).astype(np.int8)
            if p.con_kind[c] == KIND_XOR:           # macro bit equality of an associated pair
                assert len(lits) == 2 and lits[0] & 1 == 0 and lits[1] & 1 == 1
                want = truth[ids[0]] == truth[ids[1]]
            elif p.con_kind[c] == KIND_CLAUSE:
                want = bool(truth[ids[0]]) != bool(lits[0] & 1)
            else:
                nb = Lm + Ll
                pairs = ids[:2 * nb].reshape(nb, 2)
                # the two modules' bits for every index bit: same bit position, modules j < j'
                assert np.all(pairs[:, 0] % N == pairs[0, 0] % N) and np.all(pairs[:, 1] % N == pairs[0, 1] % N)
                assert np.all(pairs[:, 0] // N == np.arange(nb)) and np.all(pairs[:, 1] // N == np.arange(nb))
                want = bool(np.any(truth[pairs[:, 0]] != truth[pairs[:, 1]])) or bool(np.any(truth[ids[2 * nb:]]))
            assert oracle.eval_formula(p, c, truth) == int(want)
    P = N * (N - 1) // 2
    assert kinds[KIND_EXPR] == P
    assert kinds[KIND_XOR] == Lm * p.meta["n_routing"]
    assert kinds[KIND_CLAUSE] == 4 * p.meta["n_routing"] + 4 * N


def test_pair_constraint_probability_closed_form():
    """P[pair constraint False] = prod_i P[bits i equal] * (1 - p_A) * (1 - p_B), by the
    independence of the rounded variables (randomized rounding); the oracle's per-constraint
    value and its enumeration both equal it."""
    p = sched(16, 2)
    L, nd = p.meta["n_bits"], p.meta["n_deps"]
    rng = np.random.default_rng(7)
    for c in (nd, nd + 17, nd + 200):
        ids = _lits(p, c) >> 1
        pv = np.full(p.n_bool + p.n_atoms, 0.5)
        pv[ids] = rng.uniform(0.05, 0.95, ids.shape[0])
        bits = ids[:2 * L].reshape(L, 2)
        eq = np.prod(pv[bits[:, 0]] * pv[bits[:, 1]] + (1 - pv[bits[:, 0]]) * (1 - pv[bits[:, 1]]))
        want = eq * (1 - pv[ids[-2]]) * (1 - pv[ids[-1]])
        PT, PF, dF = oracle.cop_one(p, c, pv)
        assert PF == pytest.approx(want, rel=1e-12) and PT == pytest.approx(1 - want, rel=1e-12)
        assert oracle.cop_enum(p, c, pv)[1] == pytest.approx(want, rel=1e-12)
        # dP_false/dp_A = -eq (1 - p_B)
        assert dF[int(ids[-2])] == pytest.approx(-eq * (1 - pv[ids[-1]]), rel=1e-12)


@pytest.mark.parametrize("nw", [2, 16, 256])
def test_scheduling_diagram_sizes(nw):
    """Interleaved bit order: OR_i (x_ij XOR x_ij') OR A OR B has 3 L + 2 decision nodes;
    the feasibility constraint of one worker is a chain of L + 2 nodes."""
    L = int(np.log2(nw))
    p = sched(nw, 2, dep_prob=0.0) if nw <= 16 else _sched_pairs_only(nw)
    h = fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY)
    d = fsmt.xbdd_export_diagram(h, 0)
    assert (d["n_nodes"], d["n_slots"], d["n_bslots"]) == (3 * L + 2, 2 * L + 2, 2 * L)
    if nw <= 16:
        f = fsmt.xbdd_export_diagram(h, p.meta["n_pairs"])
        assert (f["n_nodes"], f["n_slots"], f["n_bslots"]) == (L + 2, L + 2, L)
    assert fsmt.xbdd_info(h)["n_big"] == 0


def _sched_pairs_only(nw):
    return make_paper_scheduling(nw, 1, W.seed_seq(8, nw, 1, 0), dep_prob=0.0, feasibility=False)


@pytest.mark.parametrize("nm,nl", [(2, 2), (8, 4), (64, 8)])
def test_placement_diagram_sizes(nm, nl):
    """Non-overlap: 3 (Lm + Ll) nodes for the index bits and 4 for the separation atoms."""
    nb = int(np.log2(nm)) + int(np.log2(nl))
    p = place(nm, nl)
    h = fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY)
    c = int(np.nonzero(p.con_kind == KIND_EXPR)[0][0])
    d = fsmt.xbdd_export_diagram(h, c)
    assert (d["n_nodes"], d["n_slots"], d["n_bslots"]) == (3 * nb + 4, 2 * nb + 4, 2 * nb)


def test_big_diagram_threshold():
    """One lane per constraint up to 40 KB of LDS message columns per wavefront
    ((2 (nodes + 2) + 4 slots) x 64 lanes x 4 bytes), in registers or LDS: the 28-node
    placement pair diagrams either way, and clauses of up to 26 distinct atoms (n nodes,
    n slots); a clause of 27 atoms (41.5 KB) is big (level kernel)."""
    from workloads.format import BlockBuilder
    host = fsmt.FSMT_HOST_ONLY
    p = place(32, 8)
    for messages in (0, 1):
        assert fsmt.xbdd_info(fsmt.xbdd_compile(p, device=host, messages=messages))["n_big"] == 0
    rng = np.random.default_rng(9)
    for L, big in ((26, False), (27, True)):
        bb = BlockBuilder(0, 6, -1.0, 1.0)
        ids = bb.atoms(rng.integers(0, 6, (40, 2)), [1.0, -1.0], OP_LE, np.float32(0.25))
        bb.constraints(KIND_CLAUSE, 2 * np.stack([rng.choice(ids, L, replace=False) for _ in range(3)]))
        info = fsmt.xbdd_info(fsmt.xbdd_compile(bb.build(), device=host))
        assert info["max_nodes"] == L and info["n_big"] == (3 if big else 0)


@pytest.mark.parametrize("make", [lambda: place(16, 4), lambda: sched(32, 3, dep_prob=0.6)])
def test_halfspace_colour_classes(make):
    """Half-spaces (two-variable unit atoms: routing adjacency, dependencies) are split into
    colour classes whose members share no variable; greedy colouring uses at least the
    largest variable degree and at most one more than the largest conflict count."""
    from collections import Counter
    p = make()
    hs = []
    for c in range(p.n_cons):
        lits = _lits(p, c)
        if p.con_kind[c] == KIND_CLAUSE and len(lits) == 1 and (lits[0] >> 1) >= p.n_bool:
            v = _atom(p, lits[0] >> 1)[0]
            if len(v) > 1:
                hs.append(v)
    deg = Counter(j for v in hs for j in v)
    info = fsmt.xbdd_info(fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY))
    assert info["n_halfspaces"] == len(hs) > 0
    lo = max(deg.values())
    hi = 1 + max(sum(deg[j] - 1 for j in v) for v in hs)
    assert lo <= info["n_hs_colors"] <= hi
    # half-spaces that share a variable are projected onto by Dykstra's sweeps
    assert lo > 1 and info["hs_separable"] == 0


def test_separable_halfspaces_flag():
    """The closed-form projection is chosen exactly when no two half-spaces share a
    variable (one colour class) and each has at most 4 distinct variables."""
    p = W.make_workload("scheduling_200x10")      # 5 precedences on distinct jobs among 200
    info = fsmt.xbdd_info(fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY))
    assert info["n_halfspaces"] == 5 and info["n_hs_colors"] == 1 and info["hs_separable"] == 1
    box = fsmt.xbdd_info(fsmt.xbdd_compile(p, device=fsmt.FSMT_HOST_ONLY, projection=fsmt.FSMT_PROJ_BOX))
    assert box["n_halfspaces"] == 0 and box["hs_separable"] == 0


def test_par2_scoring():
    """PAR-2: the wall time when solved within the limit, twice the limit otherwise."""
    from paper_2603_22877_amd.par2 import InstanceResult, par2
    rs = [InstanceResult("a", True, 1.5, 0.1, 1, 3, 0, 10), InstanceResult("b", False, 20.0, 0.1, 4, 80, 2, 10),
          InstanceResult("c", True, 25.0, 0.1, 9, 5, 0, 10)]
    assert [r.score(20.0) for r in rs] == [1.5, 40.0, 40.0]
    assert par2(rs, 20.0) == pytest.approx(81.5 / 3)
    assert par2([], 20.0) == 0.0


def test_pair_disjunctions_are_recognized():
    """Non-overlap constraints of both encodings, OR_i (x_2i XOR x_2i+1) OR atoms, are marked
    for the closed-form sweep; the same program with a negated literal, a different
    connective, or other workloads are not."""
    import dataclasses
    host = fsmt.FSMT_HOST_ONLY
    p = sched(16, 2)
    assert fsmt.xbdd_info(fsmt.xbdd_compile(p, device=host))["n_pair"] == p.meta["n_pairs"]
    q = place(4, 4)
    assert fsmt.xbdd_info(fsmt.xbdd_compile(q, device=host))["n_pair"] == q.meta["n_pairs"]
    for name in ("scheduling_200x10", "placement_150"):
        assert fsmt.xbdd_info(fsmt.xbdd_compile(W.make_workload(name), device=host))["n_pair"] == 0
    nd = p.meta["n_deps"]
    lit = p.con_lit.copy()
    lit[p.con_ptr[nd]] |= 1                      # negate the first literal of the first pair
    assert fsmt.xbdd_info(fsmt.xbdd_compile(dataclasses.replace(p, con_lit=lit), device=host))["n_pair"] == \
        p.meta["n_pairs"] - 1
    ops = p.expr_ops.copy()
    ops[p.expr_ptr[nd] + 2] = -1                 # XOR -> AND in the first pair constraint
    assert fsmt.xbdd_info(fsmt.xbdd_compile(dataclasses.replace(p, expr_ops=ops), device=host))["n_pair"] == \
        p.meta["n_pairs"] - 1
