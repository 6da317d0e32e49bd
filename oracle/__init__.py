"""FP64 reference oracle (TEST INFRASTRUCTURE ONLY).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark use this
package; the library never imports it. The arithmetic lives in ``fsmt_oracle.c`` (plain C,
FP64, compiled with gcc, no FMA contraction) and, for the tiny brute-force pins, in
``brute.py`` (pure Python / numpy). Paper references are given per function in the C file.

The annealing driver ``anneal`` (Alg. "CLS with Annealing") has no printed trace in the
paper; it is pinned by a by-hand replay of the Fig. 2 toy (closed-form gradients, two
restarts that stop at different steps) and, against the library, level by level.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fsmt_oracle.c")
_LIB = os.path.join(_HERE, "libfsmt_oracle.so")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _OProblem(ct.Structure):
    _fields_ = [("n_bool", ct.c_int32), ("n_real", ct.c_int32), ("n_atoms", ct.c_int32),
                ("n_cons", ct.c_int32)] + [(k, ct.c_void_p) for k in (
                    "atom_ptr", "atom_var", "atom_coef", "atom_rhs", "atom_op", "con_kind",
                    "con_ptr", "con_lit", "con_param", "expr_ptr", "expr_ops")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ct.CDLL(_LIB)
        vp, i32, dbl = ct.c_void_p, ct.c_int, ct.c_double
        L.oracle_objective.argtypes = [vp, i32, vp, vp, dbl, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32]
        L.oracle_check.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.oracle_pgd.argtypes = [vp, i32, vp, vp, vp, vp, dbl, dbl, vp, vp, i32, vp, vp, vp]
        L.oracle_project.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp]
        L.oracle_erwa.argtypes = [i32, i32, vp, i32, dbl, dbl, i32, i32, vp, vp]
        L.oracle_erwa.restype = None
        L.oracle_cop_enum.argtypes = [vp, i32, vp, vp, vp]
        L.oracle_cop_one.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.oracle_eval_formula.argtypes = [vp, i32, vp]
        L.oracle_atom_probs.argtypes = [vp, vp, dbl, vp, vp, vp]
        _lib = L
    return _lib


def _p(x: Optional[np.ndarray]):
    return None if x is None else x.ctypes.data


class OracleProblem:
    """Contiguous copies of a :class:`workloads.Problem` plus the C view of them."""

    def __init__(self, prob):
        self.prob = prob
        self.n, self.m, self.C = prob.n_bool, prob.n_real, prob.n_cons
        self.A = prob.n_atoms
        self._keep = {}
        s = _OProblem()
        s.n_bool, s.n_real, s.n_atoms, s.n_cons = self.n, self.m, self.A, self.C
        for name, dt in (("atom_ptr", np.int64), ("atom_var", np.int32), ("atom_coef", np.float64),
                         ("atom_rhs", np.float64), ("atom_op", np.int8), ("con_kind", np.int32),
                         ("con_ptr", np.int64), ("con_lit", np.int32), ("con_param", np.int32),
                         ("expr_ptr", np.int64), ("expr_ops", np.int32)):
            arr = np.ascontiguousarray(getattr(prob, name), dtype=dt)
            if arr.size == 0:
                arr = np.zeros(1, dt)
            self._keep[name] = arr
            setattr(s, name, arr.ctypes.data)
        self.s = s
        self.lo = np.ascontiguousarray(prob.real_lo, np.float64)
        self.hi = np.ascontiguousarray(prob.real_hi, np.float64)

    @property
    def ref(self):
        return ct.byref(self.s)


def _as(prob) -> OracleProblem:
    return prob if isinstance(prob, OracleProblem) else OracleProblem(prob)


def _f32(x, shape):
    x = np.asarray(x, np.float32)
    if shape[0] == -1 and shape[1] == 0:          # no variables of this kind: keep R
        shape = (x.shape[0] if x.ndim == 2 else 1, 0)
    return np.ascontiguousarray(x.reshape(shape))


def objective(prob, a, b, kappa: float, w=None, grad: bool = True, per_constraint: bool = True,
              sel=None):
    """U[R], unsat/sat [R][C], grad_a [R][n], grad_b [R][m], |contribution| sums (FP64)."""
    op = _as(prob)
    a = _f32(a, (-1, op.n))
    R = a.shape[0]
    b = _f32(b, (R, op.m))
    wv = None if w is None else np.ascontiguousarray(np.broadcast_to(
        np.asarray(w, np.float64), (R, op.C)))
    out = dict(U=np.zeros(R))
    if per_constraint:
        out["unsat"] = np.full((R, op.C), np.nan)
        out["sat"] = np.full((R, op.C), np.nan)
    if grad:
        for k, d in (("grad_a", op.n), ("grad_b", op.m), ("absg_a", op.n), ("absg_b", op.m)):
            out[k] = np.zeros((R, d))
    selv = None if sel is None else np.ascontiguousarray(sel, np.int32)
    rc = lib().oracle_objective(
        op.ref, R, _p(a), _p(b), float(kappa), _p(wv), _p(out["U"]), _p(out.get("unsat")),
        _p(out.get("sat")), _p(out.get("grad_a")), _p(out.get("grad_b")), _p(out.get("absg_a")),
        _p(out.get("absg_b")), _p(selv), 0 if selv is None else len(selv))
    if rc != 0:
        raise ValueError(f"oracle_objective failed ({rc})")
    return out


def check(prob, a, b):
    """Rounded x [R][n] (int8 +-1), sat_bits [R][ceil(C/32)], n_unsat [R], verdict [R]."""
    op = _as(prob)
    a = _f32(a, (-1, op.n))
    R = a.shape[0]
    b = _f32(b, (R, op.m))
    nw = (op.C + 31) // 32
    x = np.zeros((R, op.n), np.int8)
    bits = np.zeros((R, max(nw, 1)), np.uint32)
    nu = np.zeros(R, np.int32)
    ver = np.zeros(R, np.int32)
    rc = lib().oracle_check(op.ref, R, _p(a), _p(b), _p(x), _p(bits), _p(nu), _p(ver))
    if rc != 0:
        raise ValueError(f"oracle_check failed ({rc})")
    return dict(x=x, sat_bits=bits[:, :nw], n_unsat=nu, verdict=ver)


def pgd(prob, a, b, ga, gb, eta_a: float, eta_b: float, unit_proj: bool = True):
    """Projected step (clamp a; project b onto the box and, with unit_proj, the unit atoms)."""
    op = _as(prob)
    a = _f32(a, (-1, op.n))
    R = a.shape[0]
    b, ga, gb = _f32(b, (R, op.m)), _f32(ga, (R, op.n)), _f32(gb, (R, op.m))
    ao, bo, gsq = np.zeros((R, op.n)), np.zeros((R, op.m)), np.zeros(R)
    nh = lib().oracle_pgd(op.ref, R, _p(a), _p(b), _p(ga), _p(gb), float(eta_a), float(eta_b),
                          _p(op.lo), _p(op.hi), int(bool(unit_proj)), _p(ao), _p(bo), _p(gsq))
    return dict(a=ao, b=bo, gsq=gsq, n_halfspaces=nh)


def project(prob, y, unit_proj: bool = True):
    """Euclidean projection of one real point onto the feasible set D; returns (y, lo, hi)."""
    op = _as(prob)
    yi = np.ascontiguousarray(np.asarray(y, np.float64).reshape(op.m))
    yo, lo, hi = np.zeros(op.m), np.zeros(op.m), np.zeros(op.m)
    nh = lib().oracle_project(op.ref, _p(yi), _p(op.lo), _p(op.hi), int(bool(unit_proj)), _p(yo),
                              _p(lo), _p(hi))
    return yo, lo, hi, nh


def erwa(sat_bits, n_cons: int, t: int, h, w, rho=0.5, gamma=2.0, tau=1, normalize=True):
    """In-place ERWA update of h, w ([R][C] float64) from the satisfied-constraint bits."""
    bits = np.ascontiguousarray(sat_bits, np.uint32)
    R = bits.shape[0]
    assert h.dtype == np.float64 and w.dtype == np.float64 and h.flags.c_contiguous
    lib().oracle_erwa(R, n_cons, _p(bits), int(t), float(rho), float(gamma), int(tau),
                      int(normalize), _p(h), _p(w))
    return h, w


def cop_enum(prob, c: int, pvar):
    op = _as(prob)
    pv = np.ascontiguousarray(pvar, np.float64)
    PT, PF = ct.c_double(), ct.c_double()
    rc = lib().oracle_cop_enum(op.ref, int(c), _p(pv), ct.byref(PT), ct.byref(PF))
    if rc != 0:
        raise ValueError(f"oracle_cop_enum failed ({rc})")
    return PT.value, PF.value


def cop_one(prob, c: int, pvar):
    """(P_true, P_false, {var id: dP_false/dp}) of constraint c at variable probabilities."""
    op = _as(prob)
    pv = np.ascontiguousarray(pvar, np.float64)
    PT, PF, k = ct.c_double(), ct.c_double(), ct.c_int()
    dF = np.zeros(64)
    ids = np.zeros(64, np.int32)
    rc = lib().oracle_cop_one(op.ref, int(c), _p(pv), ct.byref(PT), ct.byref(PF), _p(dF),
                              _p(ids), ct.byref(k))
    if rc != 0:
        raise ValueError(f"oracle_cop_one failed ({rc})")
    return PT.value, PF.value, dict(zip(ids[:k.value].tolist(), dF[:k.value].tolist()))


def eval_formula(prob, c: int, truth) -> int:
    op = _as(prob)
    t = np.ascontiguousarray(truth, np.int8)
    return int(lib().oracle_eval_formula(op.ref, int(c), _p(t)))


def atom_probs(prob, b, kappa: float):
    op = _as(prob)
    bb = _f32(b, (op.m,))
    p, d, z = np.zeros(op.A), np.zeros(op.A), np.zeros(op.A)
    rc = lib().oracle_atom_probs(op.ref, _p(bb), float(kappa), _p(p), _p(d), _p(z))
    if rc != 0:
        raise ValueError(f"oracle_atom_probs failed ({rc})")
    return p, d, z


def variable_probs(prob, a, b, kappa: float) -> np.ndarray:
    """P[variable True] by variable id (Booleans, then atoms) at one point."""
    p_atoms, _, _ = atom_probs(prob, b, kappa)
    return np.concatenate([(1.0 - np.asarray(a, np.float32).astype(np.float64)) / 2.0, p_atoms])


def anneal_level(prob, a, b, w, h, kappa: float, t: int, eta_a, eta_b, steps_per_level: int,
                 eps: float = 1e-2, rho=0.5, gamma=2.0, tau=1, normalize=True, unit_proj=True,
                 active=None):
    """One annealing level t (1-based) of Alg. "CLS with Annealing" for each restart r with
    active[r] (all when None), every restart on its own:

    * ProjGradDesc at kappa (Alg. "FourierSMT"): projected-gradient steps on U
      (Eq. "pg1"/"pg2"), at most ``steps_per_level``; the loop's test is taken on the
      gradient map of the step just made, so a restart stops once a step had
      ||g||^2 <= eps^2 (Eq. "critical"; eps <= 0: never) while the others go on. Iterates
      are stored in float32 between steps, as the library stores them.
    * rounding x = sgn(a), exact check, ERWA update of h and w (float64 rows of [R][C]).

    a, b (float32 [R][n], [R][m]), w, h are updated in place for the active rows only.
    The stop test compares the step's ||g||^2, rounded to float32, with eps^2 in float32:
    the library takes that decision in float32, and a decision must be taken in the same
    precision on both sides.
    Returns dict(n_unsat [R] (-1 for inactive rows), verdict [R], steps [R], sat_bits,
    gsq [R] (||g||^2 of each restart's last step, float64)).
    """
    op = _as(prob)
    R = a.shape[0]
    act = np.ones(R, bool) if active is None else np.asarray(active, bool).copy()
    steps = np.zeros(R, np.int64)
    last_gsq = np.full(R, np.nan)
    eps2 = np.float32(eps) * np.float32(eps)
    stepping = act.copy()
    for _ in range(steps_per_level):
        idx = np.nonzero(stepping)[0]
        if idx.size == 0:
            break
        o = objective(op, a[idx], b[idx], kappa, w=w[idx], per_constraint=False)
        st = pgd(op, a[idx], b[idx], o["grad_a"].astype(np.float32), o["grad_b"].astype(np.float32),
                 eta_a, eta_b, unit_proj)
        a[idx] = st["a"].astype(np.float32)
        b[idx] = st["b"].astype(np.float32)
        steps[idx] += 1
        last_gsq[idx] = st["gsq"]
        if eps > 0:
            stepping[idx[st["gsq"].astype(np.float32) <= eps2]] = False
    n_unsat = np.full(R, -1, np.int64)
    verdict = np.zeros(R, np.int32)
    nw = (op.C + 31) // 32
    bits = np.zeros((R, nw), np.uint32)
    idx = np.nonzero(act)[0]
    if idx.size:
        ch = check(op, a[idx], b[idx])
        hh, ww = h[idx].copy(), w[idx].copy()
        erwa(ch["sat_bits"], op.C, t, hh, ww, rho, gamma, tau, normalize)
        h[idx], w[idx] = hh, ww
        n_unsat[idx] = ch["n_unsat"]
        verdict[idx] = ch["verdict"]
        bits[idx] = ch["sat_bits"]
    return dict(n_unsat=n_unsat, verdict=verdict, steps=steps, sat_bits=bits, gsq=last_gsq)


def anneal(prob, a0, b0, kappas, eta_a, eta_b, steps_per_level: int, eps: float = 1e-2,
           rho=0.5, gamma=2.0, tau=1, normalize=True, w0=None, unit_proj=True, stop_on_sat: int = 1):
    """Alg. "CLS with Annealing" literally, with the PGD of Alg. "FourierSMT" inside, for R
    independent restarts (the rows of a0, b0), each running its own loop.

    h starts at 0 and w at w0 (1 by default). Per level t = 1..T (kappa_t): ``anneal_level``.
    With stop_on_sat = 1 a restart whose check passes is SAT and runs no further level
    (returns SAT); with 0 every restart runs every level (fixed work). Returns the per-level
    trace: n_unsat per restart (-1 once a restart has stopped), the iterates and weights after
    the level, and the steps each restart took. Parity unpinned by the paper (no printed
    trace); pinned by a by-hand replay of the Fig. 2 toy and level-by-level GPU replays.
    """
    op = _as(prob)
    a = _f32(a0, (-1, op.n)).copy()
    R = a.shape[0]
    b = _f32(b0, (R, op.m)).copy()
    w = np.ones((R, op.C)) if w0 is None else np.array(np.broadcast_to(w0, (R, op.C)), np.float64)
    h = np.zeros((R, op.C))
    trace = []
    done = np.zeros(R, bool)
    for t, kap in enumerate(kappas, start=1):
        act = ~done if stop_on_sat else np.ones(R, bool)
        lv = anneal_level(op, a, b, w, h, kap, t, eta_a, eta_b, steps_per_level, eps, rho, gamma,
                          tau, normalize, unit_proj, active=act)
        if stop_on_sat:
            done |= lv["verdict"] == 1
        trace.append(dict(level=t, kappa=kap, n_unsat=lv["n_unsat"].copy(), steps=lv["steps"].copy(),
                          verdict=lv["verdict"].copy(), a=a.copy(), b=b.copy(), w=w.copy(), h=h.copy()))
        if stop_on_sat and np.all(done):
            break
    return trace
