"""Seeded generator: 2D rectangle placement with rotation bits.

Workload (stands in for the paper's placement suite, Methods, "3D Placement"; the paper's
instances are not public): N axis-aligned rectangles with integer sides w_i, h_i ~ U{1..20}
in a W x W square, W = ceil(sqrt(sum(w*h) / 0.6)) (60 % area fill). Real variables x_i
(ids 0..N-1) and y_i (ids N..2N-1) in the box [0, W]; Boolean r_i (True = rotated, sides
swapped).

* Non-overlap, one EXPR constraint per pair i<j:
  ITE(r_i, ITE(r_j, OR4(TT), OR4(TF)), ITE(r_j, OR4(FT), OR4(FF))), where each OR4 is the
  disjunction "i left of j, j left of i, i below j, j below i" with the rotated or unrotated
  sides. The literal list of a pair constraint is
  [r_i, r_j, X1w, X1h, X2w, X2h, Y1h, Y1w, Y2h, Y2w] with
  X1v: x_i - x_j <= -v,  X2v: x_j - x_i <= -v,  Y1v: y_i - y_j <= -v,  Y2v: y_j - y_i <= -v.
  A square rectangle (w = h) makes two of its atoms identical; they are interned once.
* Feasibility, two EXPR constraints per rectangle:
  ITE(r_i, x_i <= W - h_i, x_i <= W - w_i) and ITE(r_i, y_i <= W - w_i, y_i <= W - h_i).

A shelf packing (largest side horizontal, shelves by decreasing height) must fit, otherwise
the instance is redrawn; the packing is stored as the SAT certificate.
"""
from __future__ import annotations

import math

import numpy as np

from .format import KIND_EXPR, OP_LE, X_ITE, X_OR, Problem

# postfix program over literal slots [r_i, r_j, X1w, X1h, X2w, X2h, Y1h, Y1w, Y2h, Y2w]
_R_I, _R_J, _X1W, _X1H, _X2W, _X2H, _Y1H, _Y1W, _Y2H, _Y2W = range(10)


def _or4(a, b, c, d):
    return [a, b, X_OR, c, X_OR, d, X_OR]


PAIR_PROGRAM = np.asarray(
    [_R_I, _R_J] + _or4(_X1H, _X2H, _Y1W, _Y2W) + _or4(_X1H, _X2W, _Y1W, _Y2H) + [X_ITE]
    + [_R_J] + _or4(_X1W, _X2H, _Y1H, _Y2W) + _or4(_X1W, _X2W, _Y1H, _Y2H) + [X_ITE]
    + [X_ITE], np.int32)
# feasibility: literals [r_i, A_rot, A_unrot]
FEAS_PROGRAM = np.asarray([0, 1, 2, X_ITE], np.int32)


def _shelf_pack(w, h, W):
    """Shelf packing with the longer side horizontal; returns (x, y, rot) or None."""
    rot = h > w                         # rotate so that the stored height is the short side
    ww = np.where(rot, h, w)
    hh = np.where(rot, w, h)
    order = np.argsort(-hh, kind="stable")
    x = np.zeros(len(w))
    y = np.zeros(len(w))
    cx, cy, shelf_h = 0.0, 0.0, 0.0
    for i in order:
        if cx + ww[i] > W:
            cy += shelf_h
            cx, shelf_h = 0.0, 0.0
        if shelf_h == 0.0:
            shelf_h = float(hh[i])
        x[i], y[i] = cx, cy
        cx += ww[i]
    if cy + shelf_h > W:
        return None
    return x, y, rot


def make_placement(n_rect: int, seed_seq, fill: float = 0.6, max_side: int = 20,
                   max_tries: int = 1000) -> Problem:
    rng = np.random.Generator(np.random.PCG64(seed_seq))
    for attempt in range(max_tries):
        w = rng.integers(1, max_side + 1, n_rect).astype(np.float64)
        h = rng.integers(1, max_side + 1, n_rect).astype(np.float64)
        W = float(math.ceil(math.sqrt(float((w * h).sum()) / fill)))
        packed = _shelf_pack(w, h, W)
        if packed is not None:
            break
    else:
        raise RuntimeError("no packable placement instance found")
    px, py, prot = packed
    N = n_rect
    sq = (w == h)

    # ---- pair atoms (vectorized) ----
    ii, jj = np.triu_indices(N, 1)
    P = ii.shape[0]
    sq_i, sq_j = sq[ii], sq[jj]
    # per pair atom slots in allocation order: X1w,[X1h],X2w,[X2h],Y1h,[Y1w],Y2h,[Y2w]
    present = np.stack([np.ones(P, bool), ~sq_i, np.ones(P, bool), ~sq_j,
                        np.ones(P, bool), ~sq_i, np.ones(P, bool), ~sq_j], axis=1)
    cnt = present.sum(1)
    base = np.zeros(P + 1, np.int64)
    np.cumsum(cnt, out=base[1:])
    n_pair_atoms = int(base[-1])
    rank = np.cumsum(present, axis=1) - 1                      # position among present
    slot_atom = base[:-1, None] + rank                          # atom index per slot
    # duplicated slots reuse their partner: X1h->X1w, X2h->X2w, Y1w->Y1h, Y2w->Y2h
    for dup, src in ((1, 0), (3, 2), (5, 4), (7, 6)):
        slot_atom[:, dup] = np.where(present[:, dup], slot_atom[:, dup], slot_atom[:, src])
    # atom contents per slot: (first var, second var, coef first, coef second, rhs)
    xi, xj, yi, yj = ii, jj, N + ii, N + jj
    slot_vars = [(xi, xj), (xi, xj), (xi, xj), (xi, xj), (yi, yj), (yi, yj), (yi, yj), (yi, yj)]
    slot_coef = [(1., -1.), (1., -1.), (-1., 1.), (-1., 1.), (1., -1.), (1., -1.), (-1., 1.), (-1., 1.)]
    slot_rhs = [-w[ii], -h[ii], -w[jj], -h[jj], -h[ii], -w[ii], -h[jj], -w[jj]]

    # ---- feasibility atoms ----
    # per rect: XR: x <= W - h (rotated), XU: x <= W - w, YR: y <= W - w, YU: y <= W - h
    f_present = np.stack([np.ones(N, bool), ~sq, np.ones(N, bool), ~sq], axis=1)
    f_cnt = f_present.sum(1)
    f_base = np.zeros(N + 1, np.int64)
    np.cumsum(f_cnt, out=f_base[1:])
    f_rank = np.cumsum(f_present, axis=1) - 1
    f_slot_atom = n_pair_atoms + f_base[:-1, None] + f_rank
    for dup, src in ((1, 0), (3, 2)):
        f_slot_atom[:, dup] = np.where(f_present[:, dup], f_slot_atom[:, dup], f_slot_atom[:, src])
    n_atoms = n_pair_atoms + int(f_base[-1])

    atom_rhs = np.empty(n_atoms, np.float64)
    nnz = np.concatenate([np.full(n_pair_atoms, 2), np.full(int(f_base[-1]), 1)])
    atom_ptr = np.zeros(n_atoms + 1, np.int64)
    np.cumsum(nnz, out=atom_ptr[1:])
    atom_var = np.empty(int(atom_ptr[-1]), np.int32)
    atom_coef = np.empty(int(atom_ptr[-1]), np.float64)
    for s in range(8):
        sel = present[:, s]
        k = slot_atom[sel, s]
        atom_var[2 * k] = slot_vars[s][0][sel]
        atom_var[2 * k + 1] = slot_vars[s][1][sel]
        atom_coef[2 * k] = slot_coef[s][0]
        atom_coef[2 * k + 1] = slot_coef[s][1]
        atom_rhs[k] = slot_rhs[s][sel]
    off = 2 * n_pair_atoms
    f_vars = [np.arange(N), np.arange(N), N + np.arange(N), N + np.arange(N)]
    f_rhs = [W - h, W - w, W - w, W - h]
    for s in range(4):
        sel = f_present[:, s]
        k = f_slot_atom[sel, s]
        atom_var[off + (k - n_pair_atoms)] = f_vars[s][sel]
        atom_coef[off + (k - n_pair_atoms)] = 1.0
        atom_rhs[k] = f_rhs[s][sel]
    atom_op = np.full(n_atoms, OP_LE, np.int8)

    # ---- constraints ----
    n_bool = N
    C = P + 2 * N
    con_kind = np.full(C, KIND_EXPR, np.int32)
    con_ptr = np.zeros(C + 1, np.int64)
    con_ptr[1:P + 1] = 10 * np.arange(1, P + 1)
    con_ptr[P + 1:] = 10 * P + 3 * np.arange(1, 2 * N + 1)
    con_lit = np.empty(int(con_ptr[-1]), np.int32)
    pl = con_lit[:10 * P].reshape(P, 10)
    pl[:, 0] = 2 * ii
    pl[:, 1] = 2 * jj
    for s in range(8):
        pl[:, 2 + s] = 2 * (n_bool + slot_atom[:, s])
    fl = con_lit[10 * P:].reshape(N, 2, 3)
    fl[:, :, 0] = 2 * np.arange(N)[:, None]
    fl[:, 0, 1] = 2 * (n_bool + f_slot_atom[:, 0])
    fl[:, 0, 2] = 2 * (n_bool + f_slot_atom[:, 1])
    fl[:, 1, 1] = 2 * (n_bool + f_slot_atom[:, 2])
    fl[:, 1, 2] = 2 * (n_bool + f_slot_atom[:, 3])
    con_param = np.zeros(C, np.int32)
    lp, lf = len(PAIR_PROGRAM), len(FEAS_PROGRAM)
    expr_ptr = np.zeros(C + 1, np.int64)
    expr_ptr[1:P + 1] = lp * np.arange(1, P + 1)
    expr_ptr[P + 1:] = lp * P + lf * np.arange(1, 2 * N + 1)
    expr_ops = np.concatenate([np.tile(PAIR_PROGRAM, P), np.tile(FEAS_PROGRAM, 2 * N)]).astype(np.int32)

    cert_x = np.where(prot, -1.0, 1.0)
    cert_y = np.concatenate([px, py])
    prob = Problem(
        n_bool=n_bool, n_real=2 * N, atom_ptr=atom_ptr, atom_var=atom_var,
        atom_coef=atom_coef, atom_rhs=atom_rhs, atom_op=atom_op, con_kind=con_kind,
        con_ptr=con_ptr, con_lit=con_lit, con_param=con_param, expr_ptr=expr_ptr,
        expr_ops=expr_ops, real_lo=np.zeros(2 * N), real_hi=np.full(2 * N, W),
        meta=dict(family="placement", n_rect=N, width=W, n_pairs=P, attempts=attempt + 1,
                  mean_side=float((w.mean() + h.mean()) / 2)),
        cert_x=cert_x, cert_y=cert_y)
    prob.validate()
    return prob
