"""The standard workloads, random formulas for tests, and seeded initial points.

Each standard workload is drawn from ``numpy.random.SeedSequence([stream, instance_seed])``
with the workload's fixed stream key (``STREAM``); initial points of restart r use
``SeedSequence([*keys, 1000 + r])`` with the caller's keys.

* ``scheduling_10x2``: scheduling, 10 jobs on 2 machines, 1 restart (the plain path)
* ``scheduling_200x10``: scheduling, 200 jobs on 10 machines, 64 restarts (batched fused path)
* ``placement_150``: placement, 150 rectangles, 256 restarts
* ``uneven_batch``: 24 scheduling instances (J ~ logU[50, 1500], M ~ U{4..16}) and 24
  placement instances (N ~ logU[50, 400]), shuffled, 16 restarts each
* ``placement_1200``: placement, 1200 rectangles (721,800 constraints), 16 restarts
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from .format import (KIND_AND, KIND_CARD_GE, KIND_CARD_LE, KIND_CLAUSE, KIND_EXPR, KIND_NAE,
                     KIND_XOR, OP_EQ, X_AND, X_ITE, X_NOT, X_OR, X_XOR, Builder, Problem, lit)
from .placement import make_placement
from .scheduling import make_scheduling

# seed stream of each standard workload (first key of its SeedSequence) and its restarts
STREAM = {"scheduling_10x2": 1, "scheduling_200x10": 2, "placement_150": 3, "uneven_batch": 4, "placement_1200": 5}
RESTARTS = {"scheduling_10x2": 1, "scheduling_200x10": 64, "placement_150": 256, "uneven_batch": 16,
            "placement_1200": 16}


def seed_seq(*keys: int) -> np.random.SeedSequence:
    return np.random.SeedSequence([int(k) for k in keys])


_SINGLE = {
    "scheduling_10x2": lambda ss: make_scheduling(10, 2, ss),
    "scheduling_200x10": lambda ss: make_scheduling(200, 10, ss),
    "placement_150": lambda ss: make_placement(150, ss),
    "placement_1200": lambda ss: make_placement(1200, ss),
}


def make_workload(name: str, instance_seed: int = 0) -> Problem:
    """Instance ``instance_seed`` of the single-instance standard workload ``name``."""
    if name not in _SINGLE:
        raise ValueError(f"{name!r} is not a single-instance workload (the batch is uneven_batch())")
    p = _SINGLE[name](seed_seq(STREAM[name], instance_seed))
    p.meta.update(workload=name, instance_seed=instance_seed)
    return p


def uneven_batch_sizes(instance_seed: int = 0) -> List[Tuple[str, int, int]]:
    """(family, size, machines) for the 48 instances of the uneven batch, shuffled."""
    rng = np.random.Generator(np.random.PCG64(seed_seq(STREAM["uneven_batch"], instance_seed)))
    out = []
    for _ in range(24):
        J = int(round(math.exp(rng.uniform(math.log(50), math.log(1500)))))
        M = int(rng.integers(4, 17))
        out.append(("scheduling", J, M))
    for _ in range(24):
        N = int(round(math.exp(rng.uniform(math.log(50), math.log(400)))))
        out.append(("placement", N, 0))
    order = rng.permutation(48)
    return [out[i] for i in order]


def uneven_batch(instance_seed: int = 0, max_instances: int = 48) -> List[Problem]:
    probs = []
    for k, (fam, size, M) in enumerate(uneven_batch_sizes(instance_seed)[:max_instances]):
        ss = seed_seq(STREAM["uneven_batch"], instance_seed, k)
        p = make_scheduling(size, M, ss) if fam == "scheduling" else make_placement(size, ss)
        p.meta.update(workload="uneven_batch", instance_seed=instance_seed, batch_index=k)
        probs.append(p)
    return probs


def initial_points(p: Problem, n_restarts: int, *keys: int) -> Tuple[np.ndarray, np.ndarray]:
    """a ~ U[-1,1]^n and b ~ U[lo,hi]^m per restart, float32, shapes [R][n] and [R][m]."""
    a = np.empty((n_restarts, p.n_bool), np.float32)
    b = np.empty((n_restarts, p.n_real), np.float32)
    lo = np.where(np.isfinite(p.real_lo), p.real_lo, -1.0)
    hi = np.where(np.isfinite(p.real_hi), p.real_hi, 1.0)
    for r in range(n_restarts):
        rng = np.random.Generator(np.random.PCG64(seed_seq(*keys, 1000 + r)))
        a[r] = rng.uniform(-1.0, 1.0, p.n_bool)
        b[r] = rng.uniform(lo, hi)
    return a, b


# --------------------------------------------------------------------------------------
# random formulas (test inputs)
# --------------------------------------------------------------------------------------
def _random_expr(rng, n_lits: int, depth: int) -> list:
    """Random postfix program over literal slots 0..n_lits-1 using every connective."""
    if depth == 0 or rng.random() < 0.25:
        return [int(rng.integers(0, n_lits))]
    op = rng.choice(["and", "or", "xor", "not", "ite"])
    if op == "not":
        return _random_expr(rng, n_lits, depth - 1) + [X_NOT]
    if op == "ite":
        return (_random_expr(rng, n_lits, depth - 1) + _random_expr(rng, n_lits, depth - 1)
                + _random_expr(rng, n_lits, depth - 1) + [X_ITE])
    code = {"and": X_AND, "or": X_OR, "xor": X_XOR}[op]
    return _random_expr(rng, n_lits, depth - 1) + _random_expr(rng, n_lits, depth - 1) + [code]


def make_random_formula(seed: int, n_bool: int = 6, n_real: int = 3, n_atoms: int = 5,
                        n_cons: int = 12, max_len: int = 5, allow_repeats: bool = True,
                        kinds=(KIND_CLAUSE, KIND_AND, KIND_XOR, KIND_NAE, KIND_CARD_LE,
                               KIND_CARD_GE, KIND_EXPR), box: float = 3.0,
                        ops=(0, 1, 2, 3)) -> Problem:
    """Random constraints of every kind over Booleans and random LRA atoms.

    Atoms have 1..3 nonzero Gaussian coefficients, a Gaussian right-hand side and a random
    comparison from ``ops``. Literals are negated with probability 1/2. With
    ``allow_repeats`` a variable may occur several times in one constraint.
    """
    rng = np.random.Generator(np.random.PCG64(seed_seq(7777, seed)))
    b = Builder(n_bool, n_real, real_lo=np.full(n_real, -box), real_hi=np.full(n_real, box))
    atom_ids = []
    for _ in range(n_atoms):
        k = int(rng.integers(1, min(3, n_real) + 1))
        vs = rng.choice(n_real, k, replace=False)
        cs = np.round(rng.normal(size=k), 3)
        cs[cs == 0] = 0.5
        op = int(rng.choice(ops))
        atom_ids.append(b.atom(vs, cs, op, float(np.round(rng.normal(), 3))))
    pool = list(range(n_bool)) + atom_ids
    for _ in range(n_cons):
        kind = int(rng.choice(kinds))
        L = int(rng.integers(1, max_len + 1))
        if allow_repeats:
            vs = rng.choice(pool, L, replace=True)
        else:
            vs = rng.choice(pool, min(L, len(pool)), replace=False)
        lits = [lit(int(v), bool(rng.integers(0, 2))) for v in vs]
        param, ops_ = 0, ()
        if kind in (KIND_CARD_LE, KIND_CARD_GE):
            param = int(rng.integers(0, len(lits) + 1))
        if kind == KIND_EXPR:
            ops_ = _random_expr(rng, len(lits), 4)
        b.add(kind, lits, param, ops_)
    return b.build(meta=dict(family="random", seed=seed))


def make_random_hybrid(n: int, seed_keys=(6, 0), card_len=None, xor_len: int = 50) -> Problem:
    """Random hybrid benchmark shape (Methods, "Random Hybrid Constraints").

    n Booleans, n reals, n LRA atoms; n/5 cardinality, n/5 not-all-equal and n/50 parity
    constraints of lengths min(50, n/5), min(50, n/5) and 50 over literals drawn from the
    Booleans and atoms with random polarity. The paper leaves the atom form, the
    cardinality bound and the polarities unspecified; here atoms are
    ``y_u - y_v <= c`` with c ~ N(0, 1), the bound is k = floor(len/2) (at most), and literals are
    negated with probability 1/2.
    """
    rng = np.random.Generator(np.random.PCG64(seed_seq(*seed_keys, n)))
    L = card_len or min(50, n // 5)
    b = Builder(n, n, real_lo=np.full(n, -3.0), real_hi=np.full(n, 3.0))
    atoms = []
    for _ in range(n):
        u, v = rng.choice(n, 2, replace=False)
        atoms.append(b.atom([u, v], [1.0, -1.0], 0, float(np.round(rng.normal(), 3))))
    pool = np.asarray(list(range(n)) + atoms)
    for kind, cnt, ln in ((KIND_CARD_LE, n // 5, L), (KIND_NAE, n // 5, L),
                          (KIND_XOR, max(1, n // 50), min(xor_len, len(pool)))):
        for _ in range(cnt):
            vs = rng.choice(pool, ln, replace=False)
            lits = [lit(int(v), bool(rng.integers(0, 2))) for v in vs]
            b.add(kind, lits, ln // 2 if kind == KIND_CARD_LE else 0)
    return b.build(meta=dict(family="random_hybrid", n=n))


def make_random_separable(seed: int, n_bool: int = 12, n_real: int = 6, n_cons: int = 240) -> Problem:
    """ITEs over two Booleans u < v of disjunctions of atoms (test inputs):
    ITE(u, ITE(v, A1 | B1, A1 | B0), ITE(v, A0 | B1, A0 | B0)) with A0, A1, B0, B1 disjoint
    groups of one or two atoms, so u picks the A group and v the B group independently; a
    quarter of the constraints instead mix the groups (ITE(u, ITE(v, A1 | B1, A0 | B1),
    ITE(v, A0 | B0, A1 | B0))), which no choice of groups factors. Three shapes (group sizes,
    literal polarities, atom coefficients) recur, with random variables and right-hand sides
    that are multiples of 1/8, so constraints share templates."""
    from .format import KIND_EXPR as _EXPR
    rng = np.random.Generator(np.random.PCG64(seed_seq(7788, seed)))
    b = Builder(n_bool, n_real, real_lo=np.full(n_real, -3.0), real_hi=np.full(n_real, 3.0))
    shapes = [((2, 2, 2, 2), ((1.0, -1.0), (1.0, -1.0), (1.0, -1.0), (1.0, -1.0), (1.0, -1.0), (1.0, -1.0),
                              (1.0, -1.0), (1.0, -1.0)), (0, 1, 0, 0, 1, 0, 0, 0)),
              ((1, 2, 2, 1), ((2.0,), (1.0, -0.5), (1.0, 1.0), (-1.0,), (1.0, -1.0), (0.5,)), (1, 0, 0, 1, 0, 0)),
              ((1, 1, 1, 1), ((1.0,), (-1.0,), (1.0, -1.0), (1.0, 2.0)), (0, 0, 1, 0))]
    for c in range(n_cons):
        sizes, forms, negs = shapes[c % len(shapes)]
        u, v = (int(x) for x in np.sort(rng.choice(n_bool, 2, replace=False)))
        atoms = []
        for cf in forms:
            vs = rng.choice(n_real, len(cf), replace=False)
            atoms.append(b.atom(vs, list(cf), 0, float(rng.integers(-16, 17)) / 8.0))
        groups, k = [], 0
        for sz in sizes:
            groups.append(list(range(k, k + sz)))
            k += sz
        lits = [lit(u), lit(v)] + [lit(a, bool(nb)) for a, nb in zip(atoms, negs)]

        def disj(g1, g2):
            ids = [2 + j for j in g1 + g2]
            prog = [ids[0]]
            for j in ids[1:]:
                prog += [j, X_OR]
            return prog
        A0, A1, B0, B1 = groups
        if c % 4 == 3:   # mixed: not a product of two independent choices
            prog = ([0, 1] + disj(A1, B1) + disj(A0, B1) + [X_ITE] + [1] + disj(A0, B0) + disj(A1, B0)
                    + [X_ITE, X_ITE])
        else:
            prog = ([0, 1] + disj(A1, B1) + disj(A1, B0) + [X_ITE] + [1] + disj(A0, B1) + disj(A0, B0)
                    + [X_ITE, X_ITE])
        b.add(_EXPR, lits, 0, prog)
    return b.build(meta=dict(family="random_separable", seed=seed))


__all__ = ["STREAM", "RESTARTS", "make_workload", "uneven_batch", "uneven_batch_sizes", "initial_points",
           "make_random_formula", "make_random_hybrid", "make_random_separable", "seed_seq", "OP_EQ"]
