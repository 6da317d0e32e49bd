"""Seeded generators for the paper's own scheduling and 3D-placement encodings.

Both follow the Methods sections "Scheduling with Continuous Time" and "3D Placement": the
discrete choices (worker, macro, layer) are index variables written in binary with one
Boolean per bit, and "two modules use the same resource" is the negation of a disjunction
of bitwise XORs. The paper's instances are not public; these generators draw instances of
the same shape from the distributions the paper states and fill in what it leaves open
(listed per generator).

Boolean ids are bit-major (bit i of item j has id ``i * n_items + j``), so the sorted
support of a pair constraint interleaves the two items' bits (x_0j, x_0j', x_1j, x_1j',
...). The diagram of "some bit differs, or an atom holds" is then a chain of three nodes
per bit followed by the atoms, instead of a tree over all bits of the first item.

Every constant of an instance (durations, start offsets, sizes and the right-hand sides
built from them) is a float32 value, so the device keeps atoms as exact float32 records.

Truth convention of the package: a Boolean's value -1 is True, so bit value 1 is a = -1.
"""
from __future__ import annotations

import math

import numpy as np

from .format import (KIND_CLAUSE, KIND_EXPR, KIND_XOR, OP_GE, OP_LE, X_AND, X_OR, X_XOR,
                     BlockBuilder, Problem)


def _log2(n: int, name: str) -> int:
    L = int(round(math.log2(n))) if n > 0 else -1
    if n < 2 or (1 << L) != n:
        raise ValueError(f"{name}={n} must be a power of two >= 2")
    return L


def _bits_lit(var_ids, neg=None):
    """Literal codes for Boolean ids (``neg`` selects the negated literal)."""
    v = np.asarray(var_ids, np.int64)
    return 2 * v + (0 if neg is None else np.asarray(neg, np.int64))


def index_differs_program(n_bits: int, n_tail: int, tail_and: bool = False):
    """Postfix program: OR over bits of XOR(lit 2i, lit 2i+1), then the tail literals.

    The tail literals 2*n_bits .. 2*n_bits+n_tail-1 are ORed to the result, or, with
    ``tail_and``, ANDed together first.
    """
    prog = [0, 1, X_XOR]
    for i in range(1, n_bits):
        prog += [2 * i, 2 * i + 1, X_XOR, X_OR]
    t0 = 2 * n_bits
    if tail_and:
        prog += [t0] + sum(([t0 + k, X_AND] for k in range(1, n_tail)), []) + [X_OR]
    else:
        prog += sum(([t0 + k, X_OR] for k in range(n_tail)), [])
    return prog


def _f32(x):
    """Round instance constants to float32 values (kept as float64 arrays)."""
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def _bits_of(values, n_bits: int) -> np.ndarray:
    """[len(values), n_bits] 0/1 array of the binary digits (bit 0 first)."""
    v = np.asarray(values, np.int64)
    return (v[:, None] >> np.arange(n_bits)[None, :]) & 1


def make_paper_scheduling(n_workers: int, ratio: int, seed_seq, dep_prob: float = 0.25,
                          feasibility: bool = True, gap: float = 1e-3) -> Problem:
    """Continuous-time scheduling of n_j = ratio * n_w jobs on n_w workers.

    Variables: bits x_{i,j} of the worker index of job j (i < log2 n_w), start times y_j.
    Parameters drawn as the paper states: worker start d_w ~ U(0,1), run time t_j ~ U(0,1),
    cutoff d_w + T with T from a greedy list schedule (so a solution exists).

    Constraints:

    * dependency j' -> j: y_j - y_j' >= t_j' (one-literal clause);
    * non-overlap, every pair j < j': some worker bit differs, or y_j - y_j' >= t_j', or
      y_j' - y_j >= t_j (one EXPR constraint);
    * feasibility, every job j and worker w: the worker index of j is not w, or
      (y_j >= d_w and y_j <= d_w + T - t_j) (one EXPR constraint).

    Choices the paper leaves open: the dependency graph (a random order of the jobs; each
    job after the first gets one predecessor, uniform among the earlier jobs, with
    probability ``dep_prob``); the greedy heuristic (jobs in that order, each on the worker
    where it finishes first, T the longest resulting window; the schedule leaves ``gap``
    before and after every job, so that the stored certificate holds with that margin after
    rounding to float32); the feasibility clause is read
    per worker, with the two bounds joined by AND (the paper prints it for one worker
    symbolically with an OR between the bounds, which would hold for any y_j). Start times
    are boxed to the hull of the job's windows, [min_w d_w, max_w d_w + T - t_j]: bounds the
    feasibility constraints imply, so the solutions are unchanged, while a start far beyond
    every window (where the smoothed atoms have no gradient left) is cut off.
    """
    L = _log2(n_workers, "n_workers")
    if ratio < 1:
        raise ValueError("ratio must be >= 1")
    rng = np.random.Generator(np.random.PCG64(seed_seq))
    nw, nj = n_workers, ratio * n_workers
    d = _f32(rng.uniform(0.0, 1.0, nw))
    t = _f32(rng.uniform(0.0, 1.0, nj))
    order = rng.permutation(nj)
    deps = []                                   # (pred, succ)
    for k in range(1, nj):
        if rng.random() < dep_prob:
            deps.append((int(order[rng.integers(0, k)]), int(order[k])))
    preds = [[] for _ in range(nj)]
    for p, s in deps:
        preds[s].append(p)
    free = d + gap
    y = np.zeros(nj)
    worker = np.zeros(nj, np.int64)
    for j in order:
        ready = max((y[p] + t[p] + gap for p in preds[j]), default=0.0)
        start = np.maximum(free, ready)
        w = int(np.argmin(start + t[j]))
        worker[j], y[j] = w, start[w]
        free[w] = start[w] + t[j] + gap
    T = float(np.max(free - d))
    # start-time box: the hull of the job's windows over all workers, which the feasibility
    # constraints imply (whatever its worker, job j starts in [min_w d_w, max_w d_w + T - t_j])
    y_lo = np.full(nj, float(d.min()))
    y_hi = float(d.max()) + T - t

    xid = lambda i, j: i * nj + np.asarray(j, np.int64)  # noqa: E731
    bb = BlockBuilder(L * nj, nj, y_lo, y_hi)
    if deps:
        dp = np.asarray(deps, np.int64)
        a = bb.atoms(np.stack([dp[:, 1], dp[:, 0]], 1), [1.0, -1.0], OP_GE, t[dp[:, 0]])
        bb.constraints(KIND_CLAUSE, _bits_lit(a)[:, None])
    jj, kk = np.triu_indices(nj, 1)
    A = bb.atoms(np.stack([jj, kk], 1), [1.0, -1.0], OP_GE, t[kk])
    B = bb.atoms(np.stack([kk, jj], 1), [1.0, -1.0], OP_GE, t[jj])
    lits = [_bits_lit(np.stack([xid(i, jj), xid(i, kk)], 1)) for i in range(L)]
    lits = np.concatenate(lits + [_bits_lit(A)[:, None], _bits_lit(B)[:, None]], 1)
    bb.constraints(KIND_EXPR, lits, program=index_differs_program(L, 2))
    n_feas = 0
    if feasibility:
        fj = np.repeat(np.arange(nj), nw)
        fw = np.tile(np.arange(nw), nj)
        C = bb.atoms(fj, [1.0], OP_GE, d[fw])
        D = bb.atoms(fj, [1.0], OP_LE, _f32(d[fw] + T - t[fj]))
        wb = _bits_of(fw, L)
        # "bit i of job j differs from bit i of w": x_ij if w's bit is 0, not x_ij if it is 1
        blits = np.stack([_bits_lit(xid(i, fj), wb[:, i]) for i in range(L)], 1)
        lits = np.concatenate([blits, _bits_lit(C)[:, None], _bits_lit(D)[:, None]], 1)
        prog = [0] + sum(([i, X_OR] for i in range(1, L)), []) + [L, L + 1, X_AND, X_OR]
        bb.constraints(KIND_EXPR, lits, program=prog)
        n_feas = nj * nw
    p = bb.build(meta=dict(family="paper_scheduling", n_workers=nw, ratio=ratio, n_jobs=nj,
                           n_bits=L, cutoff=T, n_deps=len(deps), n_pairs=int(jj.shape[0]),
                           n_feasibility=n_feas, mean_duration=float(t.mean())))
    xb = _bits_of(worker, L)                    # [nj, L]
    p.cert_x = np.where(xb.T.reshape(-1) == 1, -1.0, 1.0)
    p.cert_y = y
    return p


# module kinds of the placement suite, in id order
PLACEMENT_KINDS = ("large_process", "small_process", "large_memory", "small_memory")


def make_paper_placement(n_macros: int, n_layers: int, seed_seq) -> Problem:
    """3D placement of n_m (2 + 1.5 n_l) modules into n_m unit macros with n_l layers.

    Modules (ids in this order): n_m large processes 0.4 x 0.4, n_m n_l small processes
    0.2 x 0.2, n_m large memories 0.1 x 0.1, n_m n_l / 2 small memories 0.1 x 0.05 whose
    orientation (long side along x or along y) is drawn per module with probability 1/2.
    Variables: bits m_{i,j} of the macro index and l_{i,j} of the layer index of module j,
    coordinates x_j, y_j in [0, 1].

    Constraints:

    * routing, per associated pair (j, j') and macro bit i: m_{i,j} = m_{i,j'} (a two-literal
      parity constraint), and the four unit atoms x_j - x_j' <= w_j', x_j' - x_j <= w_j,
      y_j - y_j' <= h_j', y_j' - y_j <= h_j (the footprints touch or intersect);
    * non-overlap, every pair j < j': some macro bit differs, or some layer bit differs, or
      x_j - x_j' >= w_j', or x_j' - x_j >= w_j, or y_j - y_j' >= h_j', or y_j' - y_j >= h_j;
    * feasibility, per module: x_j >= 0, x_j <= 1 - w_j, y_j >= 0, y_j <= 1 - h_j.

    Reading of the association: large process k with large memory k, and small memory k with
    small processes 2k and 2k+1 (there are half as many small memories as small processes,
    so each memory serves two processes). The paper's h_j and d_j are both the height.
    """
    Lm = _log2(n_macros, "n_macros")
    Ll = _log2(n_layers, "n_layers")
    rng = np.random.Generator(np.random.PCG64(seed_seq))
    nm, nl = n_macros, n_layers
    n_lp, n_sp, n_lm, n_sm = nm, nm * nl, nm, nm * nl // 2
    N = n_lp + n_sp + n_lm + n_sm
    o_sp, o_lm, o_sm = n_lp, n_lp + n_sp, n_lp + n_sp + n_lm
    w = np.concatenate([np.full(n_lp, 0.4), np.full(n_sp, 0.2), np.full(n_lm, 0.1), np.zeros(n_sm)])
    h = w.copy()
    along_x = rng.random(n_sm) < 0.5
    w[o_sm:] = np.where(along_x, 0.1, 0.05)
    h[o_sm:] = np.where(along_x, 0.05, 0.1)
    w, h = _f32(w), _f32(h)

    mid = lambda i, j: i * N + np.asarray(j, np.int64)            # noqa: E731
    lid = lambda i, j: (Lm + i) * N + np.asarray(j, np.int64)     # noqa: E731
    X = lambda j: np.asarray(j, np.int64)                         # noqa: E731
    Y = lambda j: N + np.asarray(j, np.int64)                     # noqa: E731
    bb = BlockBuilder((Lm + Ll) * N, 2 * N, 0.0, 1.0)

    # routing pairs
    k = np.arange(n_sm)
    ra = np.concatenate([np.arange(n_lp), o_sm + k, o_sm + k])
    rb = np.concatenate([o_lm + np.arange(n_lm), o_sp + 2 * k, o_sp + 2 * k + 1])
    for i in range(Lm):
        bb.constraints(KIND_XOR, np.stack([_bits_lit(mid(i, ra)), _bits_lit(mid(i, rb), 1)], 1))
    for V, size in ((X, w), (Y, h)):
        a1 = bb.atoms(np.stack([V(ra), V(rb)], 1), [1.0, -1.0], OP_LE, size[rb])
        a2 = bb.atoms(np.stack([V(rb), V(ra)], 1), [1.0, -1.0], OP_LE, size[ra])
        bb.constraints(KIND_CLAUSE, _bits_lit(a1)[:, None])
        bb.constraints(KIND_CLAUSE, _bits_lit(a2)[:, None])

    # non-overlap
    jj, kk = np.triu_indices(N, 1)
    tails = []
    for V, size in ((X, w), (Y, h)):
        tails.append(bb.atoms(np.stack([V(jj), V(kk)], 1), [1.0, -1.0], OP_GE, size[kk]))
        tails.append(bb.atoms(np.stack([V(kk), V(jj)], 1), [1.0, -1.0], OP_GE, size[jj]))
    bits = ([np.stack([mid(i, jj), mid(i, kk)], 1) for i in range(Lm)]
            + [np.stack([lid(i, jj), lid(i, kk)], 1) for i in range(Ll)])
    lits = np.concatenate([_bits_lit(b) for b in bits] + [_bits_lit(a)[:, None] for a in tails], 1)
    bb.constraints(KIND_EXPR, lits, program=index_differs_program(Lm + Ll, 4))

    # feasibility
    j = np.arange(N)
    for V, size in ((X, w), (Y, h)):
        bb.constraints(KIND_CLAUSE, _bits_lit(bb.atoms(V(j), [1.0], OP_GE, 0.0))[:, None])
        bb.constraints(KIND_CLAUSE, _bits_lit(bb.atoms(V(j), [1.0], OP_LE, _f32(1.0 - size)))[:, None])

    p = bb.build(meta=dict(family="paper_placement", n_macros=nm, n_layers=nl, n_modules=N,
                           n_macro_bits=Lm, n_layer_bits=Ll, n_pairs=int(jj.shape[0]),
                           n_routing=int(ra.shape[0]), mean_side=float((w + h).mean() / 2)))
    p.cert_x, p.cert_y = _placement_certificate(nm, nl, Lm, Ll, w, h, (o_sp, o_lm, o_sm))
    return p


def _placement_certificate(nm, nl, Lm, Ll, w, h, offs):
    """A placement with margins: every macro holds the same layout.

    Layer 0: the large process at (0.05, 0.05); the small processes of the macro in rows
    u = 0 .. n_l/2 - 1 at x = 0.5 and x = 0.71, y = 0.02 + 0.22 u. Layer 1: the large memory
    at (0.1, 0.1) over the large process, and small memory u at (0.68, y_u + 0.05), which
    reaches into both small processes of row u.
    """
    o_sp, o_lm, o_sm = offs
    N = w.shape[0]
    macro = np.zeros(N, np.int64)
    layer = np.zeros(N, np.int64)
    x = np.zeros(N)
    y = np.zeros(N)
    for m in range(nm):
        x[m], y[m] = 0.05, 0.05
        macro[o_lm + m], layer[o_lm + m] = m, 1
        x[o_lm + m], y[o_lm + m] = 0.1, 0.1
        macro[m] = m
        for u in range(nl // 2):
            yu = 0.02 + 0.22 * u
            for s, xs in ((2 * u, 0.5), (2 * u + 1, 0.71)):
                jdx = o_sp + m * nl + s
                macro[jdx], x[jdx], y[jdx] = m, xs, yu
            q = o_sm + m * (nl // 2) + u
            macro[q], layer[q], x[q], y[q] = m, 1, 0.68, yu + 0.05
    mb = _bits_of(macro, Lm).T.reshape(-1) if Lm else np.zeros(0)
    lb = _bits_of(layer, Ll).T.reshape(-1) if Ll else np.zeros(0)
    cert_x = np.where(np.concatenate([mb, lb]) == 1, -1.0, 1.0)
    return cert_x, np.concatenate([x, y])


def paper_scheduling_grid(workers=(16, 32, 64, 128, 256), ratios=(2, 3, 4, 5), per_cell: int = 10):
    """(n_w, r, instance) triples of the paper's scheduling suite (10 per cell)."""
    return [(nw, r, s) for nw in workers for r in ratios for s in range(per_cell)]


def paper_placement_grid(macros=(2, 4, 8, 16, 32, 64), layers=(2, 4, 8), per_cell: int = 10):
    """(n_m, n_l, instance) triples of the paper's placement suite (10 per cell)."""
    return [(nm, nl, s) for nm in macros for nl in layers for s in range(per_cell)]


__all__ = ["make_paper_scheduling", "make_paper_placement", "index_differs_program",
           "paper_scheduling_grid", "paper_placement_grid", "PLACEMENT_KINDS"]
