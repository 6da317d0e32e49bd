"""Brute-force pins for tiny constraints (TEST INFRASTRUCTURE ONLY; pure Python / numpy).

* ``truth_table``: the +-1 value of a constraint's formula on all 2^k assignments of its
  distinct variables (-1 = True, Cor. "xWFE"), by a direct Python evaluation of the formula.
* ``xwfe_coefficients``: the extended Walsh-Fourier coefficients f^(S,T) =
  E_z[f(z) prod_{i in S u T} z_i] (Thm. "WFE", Cor. "xWFE"), by a fast Walsh-Hadamard
  transform of the truth table.
* ``xwfe_expectation``: the product form sum_{S,T} f^(S,T) prod a_i prod d_i
  (Eq. "expectation2", Thm. "expectation").
* ``monte_carlo_sat``: the fraction of sampled assignments that satisfy the formula, with
  Booleans drawn by randomized rounding (Eq. "rounding") and each atom's truth drawn
  independently with its smoothed probability (the product-of-marginals model of the
  message-passing algorithm, Alg. "Forward Traversal of XBDDs").
* ``monte_carlo_joint_gaussian``: atoms decided by one shared Gaussian sample
  y ~ N(b, sigma^2 I) (Eq. "sampling" applied jointly).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from workloads.format import (KIND_AND, KIND_CARD_GE, KIND_CARD_LE, KIND_CLAUSE, KIND_EXPR,
                              KIND_NAE, KIND_XOR, OP_GE, OP_GT, OP_LE, OP_LT, X_AND, X_FALSE,
                              X_ITE, X_NOT, X_OR, X_TRUE, X_XOR)


def support(prob, c):
    lits = prob.con_lit[prob.con_ptr[c]:prob.con_ptr[c + 1]]
    return sorted(set(int(l) >> 1 for l in lits))


def formula_value(prob, c, truth: dict) -> bool:
    """Truth of constraint c given {var id: bool}."""
    lits = [int(l) for l in prob.con_lit[prob.con_ptr[c]:prob.con_ptr[c + 1]]]
    vals = [truth[l >> 1] != bool(l & 1) for l in lits]
    kind = int(prob.con_kind[c])
    k = int(prob.con_param[c])
    t = sum(vals)
    if kind == KIND_CLAUSE:
        return any(vals)
    if kind == KIND_AND:
        return all(vals)
    if kind == KIND_XOR:
        return t % 2 == 1
    if kind == KIND_NAE:
        return 0 < t < len(vals)
    if kind == KIND_CARD_LE:
        return t <= k
    if kind == KIND_CARD_GE:
        return t >= k
    assert kind == KIND_EXPR
    st = []
    for op in prob.expr_ops[prob.expr_ptr[c]:prob.expr_ptr[c + 1]]:
        op = int(op)
        if op >= 0:
            st.append(vals[op])
        elif op == X_TRUE:
            st.append(True)
        elif op == X_FALSE:
            st.append(False)
        elif op == X_NOT:
            st.append(not st.pop())
        elif op == X_ITE:
            e, th, cd = st.pop(), st.pop(), st.pop()
            st.append(th if cd else e)
        else:
            y, x = st.pop(), st.pop()
            st.append({X_AND: x and y, X_OR: x or y, X_XOR: x != y}[op])
    assert len(st) == 1
    return st[0]


def truth_table(prob, c):
    """(support ids, f values +-1 over all assignments; bit s of the index = var s True)."""
    sup = support(prob, c)
    k = len(sup)
    f = np.empty(1 << k)
    for m in range(1 << k):
        truth = {v: bool((m >> s) & 1) for s, v in enumerate(sup)}
        f[m] = -1.0 if formula_value(prob, c, truth) else 1.0
    return sup, f


def xwfe_coefficients(f: np.ndarray) -> np.ndarray:
    """f^(U) for every subset U (bitmask), with z_i = -1 when variable i is True."""
    k = int(round(math.log2(len(f))))
    # index bit s = 1 means variable s True, i.e. z_s = -1; chi_U(z) = prod_{s in U} z_s
    c = f.astype(np.float64).copy()
    h = 1
    while h < len(c):
        for i in range(0, len(c), 2 * h):
            x, y = c[i:i + h].copy(), c[i + h:i + 2 * h].copy()
            c[i:i + h], c[i + h:i + 2 * h] = x + y, x - y
        h *= 2
    return c / (1 << k)


def xwfe_expectation(coef: np.ndarray, v: np.ndarray) -> float:
    """sum_U f^(U) prod_{s in U} v_s with v_s = E[z_s] (a_i for Booleans, d_i for atoms)."""
    tot = 0.0
    for U in range(len(coef)):
        prod = 1.0
        for s in range(len(v)):
            if (U >> s) & 1:
                prod *= v[s]
        tot += coef[U] * prod
    return tot


def monte_carlo_sat(prob, c, pvar: np.ndarray, n_samples: int, rng) -> float:
    sup, f = truth_table(prob, c)
    bits = (rng.random((n_samples, len(sup))) < pvar[sup][None, :]).astype(np.int64)
    idx = (bits << np.arange(len(sup))[None, :]).sum(1)
    return float((f[idx] < 0).mean())


def monte_carlo_joint_gaussian(prob, c, a, b, sigma, n_samples, rng) -> float:
    """Satisfaction frequency when all atoms read one shared y ~ N(b, sigma^2 I)."""
    sup = support(prob, c)
    n = prob.n_bool
    y = b[None, :] + sigma * rng.standard_normal((n_samples, len(b)))
    cols = []
    for v in sup:
        if v < n:
            cols.append(rng.random(n_samples) < (1.0 - a[v]) / 2.0)
        else:
            k = v - n
            s = slice(prob.atom_ptr[k], prob.atom_ptr[k + 1])
            z = y[:, prob.atom_var[s]] @ prob.atom_coef[s] - prob.atom_rhs[k]
            op = int(prob.atom_op[k])
            cols.append({OP_LE: z <= 0, OP_LT: z < 0, OP_GE: z >= 0, OP_GT: z > 0}[op])
    sup_, f = truth_table(prob, c)
    bits = np.stack(cols, 1).astype(np.int64)
    idx = (bits << np.arange(len(sup))[None, :]).sum(1)
    return float((f[idx] < 0).mean())


def enumerate_unsat(prob, c, pvar) -> float:
    """P[constraint false] by summing assignment probabilities (pure Python)."""
    sup, f = truth_table(prob, c)
    tot = 0.0
    for m, val in enumerate(f):
        pr = 1.0
        for s, v in enumerate(sup):
            pr *= pvar[v] if (m >> s) & 1 else 1.0 - pvar[v]
        if val > 0:
            tot += pr
    return tot


__all__ = ["support", "formula_value", "truth_table", "xwfe_coefficients", "xwfe_expectation",
           "monte_carlo_sat", "monte_carlo_joint_gaussian", "enumerate_unsat", "itertools"]
