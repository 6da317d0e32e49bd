"""Problem encoding shared by every consumer (the library binding, the oracle, tests, bench).

This module fixes the *input format* only: how an SMT(LRA) formula, a conjunction of
constraints over Booleans and linear real-arithmetic atoms (paper, "Satisfiability Modulo
Theories" section, and the atom / indicator definitions of the "Walsh-Fourier Expansions"
section), is laid out as flat arrays. It contains none of the method's arithmetic.

Truth convention (paper, Supplementary Note 1, Cor. xWFE): -1 means True, +1 means False.

Arrays (all numpy, CSR-style):

* atoms: ``atom_ptr[n_atoms+1]`` (int64) into ``atom_var`` (int32 real-variable ids) and
  ``atom_coef`` (float64 q_ij); ``atom_rhs[n_atoms]`` (float64 q_i0); ``atom_op[n_atoms]``
  (int8, one of ``OP_*``). Atom i reads ``sum_j q_ij y_j  (op)  q_i0``.
* constraints: ``con_kind[C]`` (int32, one of ``KIND_*``); ``con_ptr[C+1]`` (int64) into
  ``con_lit`` (int32 literals, ``2*id + neg``; ``id < n_bool`` is a Boolean, otherwise atom
  ``id - n_bool``); ``con_param[C]`` (int32, k for the cardinality kinds);
  ``expr_ptr[C+1]`` (int64) into ``expr_ops`` (int32 postfix program, EXPR kind only).
* box of the real variables: ``real_lo[m]``, ``real_hi[m]`` (float64).

EXPR programs: an op ``v >= 0`` pushes literal number ``v`` of the constraint's literal
list; negative ops are the connectives below. ITE pops ``else``, ``then``, ``cond``
(pushed in the order cond, then, else).
"""
from __future__ import annotations

import dataclasses
import io
from typing import Any, Dict, Optional

import numpy as np

# atom comparison operators
OP_LE, OP_LT, OP_GE, OP_GT, OP_EQ = 0, 1, 2, 3, 4

# constraint kinds
KIND_CLAUSE, KIND_AND, KIND_XOR, KIND_NAE, KIND_CARD_LE, KIND_CARD_GE, KIND_EXPR = range(7)
KIND_NAMES = ["CLAUSE", "AND", "XOR", "NAE", "CARD_LE", "CARD_GE", "EXPR"]

# EXPR connectives
X_AND, X_OR, X_XOR, X_NOT, X_ITE, X_TRUE, X_FALSE = -1, -2, -3, -4, -5, -6, -7


def lit(var_id: int, neg: bool = False) -> int:
    """Literal code for variable ``var_id`` (Boolean id, or ``n_bool + atom id``)."""
    return 2 * int(var_id) + (1 if neg else 0)


@dataclasses.dataclass
class Problem:
    n_bool: int
    n_real: int
    atom_ptr: np.ndarray
    atom_var: np.ndarray
    atom_coef: np.ndarray
    atom_rhs: np.ndarray
    atom_op: np.ndarray
    con_kind: np.ndarray
    con_ptr: np.ndarray
    con_lit: np.ndarray
    con_param: np.ndarray
    expr_ptr: np.ndarray
    expr_ops: np.ndarray
    real_lo: np.ndarray
    real_hi: np.ndarray
    meta: Dict[str, Any] = dataclasses.field(default_factory=dict)
    # satisfying certificate from the generator (x in {-1,+1}^n, y in R^m) or None
    cert_x: Optional[np.ndarray] = None
    cert_y: Optional[np.ndarray] = None

    @property
    def n_atoms(self) -> int:
        return int(self.atom_rhs.shape[0])

    @property
    def n_cons(self) -> int:
        return int(self.con_kind.shape[0])

    def arrays(self) -> Dict[str, np.ndarray]:
        return {f.name: getattr(self, f.name) for f in dataclasses.fields(self)
                if isinstance(getattr(self, f.name), np.ndarray)}

    def validate(self) -> None:
        n_var = self.n_bool + self.n_atoms
        assert self.atom_ptr.dtype == np.int64 and self.con_ptr.dtype == np.int64
        assert self.atom_ptr[0] == 0 and self.atom_ptr[-1] == self.atom_var.shape[0]
        assert self.con_ptr[0] == 0 and self.con_ptr[-1] == self.con_lit.shape[0]
        assert self.expr_ptr[0] == 0 and self.expr_ptr[-1] == self.expr_ops.shape[0]
        assert np.all(np.diff(self.atom_ptr) >= 1), "every atom needs a real variable"
        assert np.all((self.atom_var >= 0) & (self.atom_var < self.n_real))
        assert np.all((self.con_lit >= 0) & ((self.con_lit >> 1) < n_var))
        assert np.all(self.real_lo <= self.real_hi)


def save_npz(p: Problem, path_or_buf) -> None:
    extra = {"n_bool": np.int64(p.n_bool), "n_real": np.int64(p.n_real)}
    if p.cert_x is not None:
        extra["cert_x"] = p.cert_x
        extra["cert_y"] = p.cert_y
    np.savez_compressed(path_or_buf, **p.arrays(), **extra,
                        meta=np.frombuffer(repr(p.meta).encode(), dtype=np.uint8))


def load_npz(path_or_buf) -> Problem:
    import ast
    z = np.load(path_or_buf, allow_pickle=False)
    kw = {k: z[k] for k in z.files if k not in ("n_bool", "n_real", "meta", "cert_x", "cert_y")}
    meta = ast.literal_eval(bytes(z["meta"]).decode()) if "meta" in z.files else {}
    return Problem(n_bool=int(z["n_bool"]), n_real=int(z["n_real"]), meta=meta,
                   cert_x=z["cert_x"] if "cert_x" in z.files else None,
                   cert_y=z["cert_y"] if "cert_y" in z.files else None, **kw)


class Builder:
    """Incremental construction of a :class:`Problem` (atoms interned by content)."""

    def __init__(self, n_bool: int, n_real: int, real_lo, real_hi):
        self.n_bool = n_bool
        self.n_real = n_real
        self.real_lo = np.asarray(real_lo, dtype=np.float64).reshape(n_real)
        self.real_hi = np.asarray(real_hi, dtype=np.float64).reshape(n_real)
        self._atoms: list = []          # (vars tuple, coefs tuple, rhs, op)
        self._atom_index: dict = {}
        self._cons: list = []           # (kind, lits, param, ops)

    def atom(self, vars_, coefs, op: int, rhs: float) -> int:
        """Intern atom ``sum coefs*y[vars] op rhs``; returns its variable id n_bool+k."""
        key = (tuple(int(v) for v in vars_), tuple(float(c) for c in coefs), int(op), float(rhs))
        k = self._atom_index.get(key)
        if k is None:
            k = len(self._atoms)
            self._atoms.append(key)
            self._atom_index[key] = k
        return self.n_bool + k

    def add(self, kind: int, lits, param: int = 0, ops=()) -> int:
        self._cons.append((int(kind), [int(x) for x in lits], int(param), [int(o) for o in ops]))
        return len(self._cons) - 1

    def build(self, meta=None) -> Problem:
        a_ptr = [0]
        a_var, a_coef, a_rhs, a_op = [], [], [], []
        for vars_, coefs, op, rhs in self._atoms:
            a_var.extend(vars_)
            a_coef.extend(coefs)
            a_ptr.append(len(a_var))
            a_rhs.append(rhs)
            a_op.append(op)
        c_ptr, e_ptr = [0], [0]
        c_lit, c_kind, c_param, e_ops = [], [], [], []
        for kind, lits, param, ops in self._cons:
            c_kind.append(kind)
            c_lit.extend(lits)
            c_ptr.append(len(c_lit))
            c_param.append(param)
            e_ops.extend(ops)
            e_ptr.append(len(e_ops))
        p = Problem(
            n_bool=self.n_bool, n_real=self.n_real,
            atom_ptr=np.asarray(a_ptr, np.int64), atom_var=np.asarray(a_var, np.int32),
            atom_coef=np.asarray(a_coef, np.float64), atom_rhs=np.asarray(a_rhs, np.float64),
            atom_op=np.asarray(a_op, np.int8),
            con_kind=np.asarray(c_kind, np.int32), con_ptr=np.asarray(c_ptr, np.int64),
            con_lit=np.asarray(c_lit, np.int32), con_param=np.asarray(c_param, np.int32),
            expr_ptr=np.asarray(e_ptr, np.int64), expr_ops=np.asarray(e_ops, np.int32),
            real_lo=self.real_lo, real_hi=self.real_hi, meta=dict(meta or {}))
        p.validate()
        return p


class BlockBuilder:
    """Vectorized construction of a :class:`Problem` from blocks of equally shaped rows.

    ``atoms`` appends K atoms with the same number of terms and comparison; ``constraints``
    appends K constraints of one kind with the same literal count and EXPR program. Atoms
    are not interned (the caller makes them distinct).
    """

    def __init__(self, n_bool: int, n_real: int, real_lo, real_hi):
        self.n_bool = n_bool
        self.n_real = n_real
        self.real_lo = np.broadcast_to(np.asarray(real_lo, np.float64), (n_real,)).copy()
        self.real_hi = np.broadcast_to(np.asarray(real_hi, np.float64), (n_real,)).copy()
        self._atoms: list = []
        self._n_atoms = 0
        self._cons: list = []

    def atoms(self, vars_, coefs, op: int, rhs) -> np.ndarray:
        """K atoms ``sum_t coefs[k,t] * y[vars[k,t]]  op  rhs[k]``; returns their variable ids."""
        v = np.asarray(vars_, np.int32)
        if v.ndim == 1:
            v = v[:, None]
        K = v.shape[0]
        c = np.broadcast_to(np.asarray(coefs, np.float64), v.shape).copy()
        r = np.broadcast_to(np.asarray(rhs, np.float64), (K,)).copy()
        self._atoms.append((v, c, int(op), r))
        ids = self.n_bool + self._n_atoms + np.arange(K, dtype=np.int64)
        self._n_atoms += K
        return ids

    def constraints(self, kind: int, lits, param: int = 0, program=()) -> None:
        """K constraints of ``kind`` with literal rows ``lits[k]`` (codes from :func:`lit`)."""
        L = np.asarray(lits, np.int64)
        if L.ndim == 1:
            L = L[:, None]
        self._cons.append((int(kind), L.astype(np.int32), int(param),
                           np.asarray(program, np.int32)))

    def build(self, meta=None) -> Problem:
        atom_ptr = np.zeros(self._n_atoms + 1, np.int64)
        if self._atoms:
            np.cumsum(np.concatenate([np.full(v.shape[0], v.shape[1]) for v, _, _, _ in self._atoms]),
                      out=atom_ptr[1:])
        cat = (lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt))
        atom_var = cat([v.reshape(-1) for v, _, _, _ in self._atoms], np.int32)
        atom_coef = cat([c.reshape(-1) for _, c, _, _ in self._atoms], np.float64)
        atom_rhs = cat([r for _, _, _, r in self._atoms], np.float64)
        atom_op = cat([np.full(v.shape[0], op) for v, _, op, _ in self._atoms], np.int8)
        C = sum(L.shape[0] for _, L, _, _ in self._cons)
        con_ptr = np.zeros(C + 1, np.int64)
        expr_ptr = np.zeros(C + 1, np.int64)
        if C:
            np.cumsum(np.concatenate([np.full(L.shape[0], L.shape[1]) for _, L, _, _ in self._cons]),
                      out=con_ptr[1:])
            np.cumsum(np.concatenate([np.full(L.shape[0], len(pg)) for _, L, _, pg in self._cons]),
                      out=expr_ptr[1:])
        p = Problem(
            n_bool=self.n_bool, n_real=self.n_real, atom_ptr=atom_ptr, atom_var=atom_var,
            atom_coef=atom_coef, atom_rhs=atom_rhs, atom_op=atom_op,
            con_kind=cat([np.full(L.shape[0], k) for k, L, _, _ in self._cons], np.int32),
            con_ptr=con_ptr,
            con_lit=cat([L.reshape(-1) for _, L, _, _ in self._cons], np.int32),
            con_param=cat([np.full(L.shape[0], pa) for _, L, pa, _ in self._cons], np.int32),
            expr_ptr=expr_ptr,
            expr_ops=cat([np.tile(pg, L.shape[0]) for _, L, _, pg in self._cons], np.int32),
            real_lo=self.real_lo, real_hi=self.real_hi, meta=dict(meta or {}))
        p.validate()
        return p
