"""Seeded generator: job-shop scheduling with continuous start times.

Workload (stands in for the paper's continuous-time scheduling suite, Methods,
"Scheduling with Continuous Time"; the paper's instances are not public):

* J jobs, each pre-assigned uniformly at random to one of M machines; integer durations
  d_j ~ U{1..10}; horizon H = sum(d)/2 + 10; real start times s_j in the box [0, H].
* For every same-machine pair j<k a Boolean o_jk (True = j runs before k) and two clauses
  (not o_jk  or  s_j - s_k <= -d_j) and (o_jk  or  s_k - s_j <= -d_k).
* Horizon atoms s_j <= H - d_j (unit clauses).
* ``n_prec`` precedence atoms s_a - s_b <= -d_a with (a, b) ordered by a random
  permutation, so the precedence graph is acyclic (unit clauses).

An instance is accepted only if a precedence-aware greedy list schedule fits in H (like the
paper's greedy time budgets); the greedy schedule is stored as the SAT certificate.
"""
from __future__ import annotations

import numpy as np

from .format import KIND_CLAUSE, OP_LE, Problem


def make_scheduling(n_jobs: int, n_machines: int, seed_seq, n_prec: int = 5,
                    max_tries: int = 1000) -> Problem:
    rng = np.random.Generator(np.random.PCG64(seed_seq))
    for attempt in range(max_tries):
        mach = rng.integers(0, n_machines, n_jobs)
        d = rng.integers(1, 11, n_jobs).astype(np.float64)
        H = float(d.sum()) / 2.0 + 10.0
        perm = rng.permutation(n_jobs)
        # precedence pairs: positions i<k in the permutation (distinct pairs)
        prec = []
        seen = set()
        while len(prec) < min(n_prec, n_jobs * (n_jobs - 1) // 2):
            i, k = sorted(rng.choice(n_jobs, 2, replace=False).tolist())
            if (i, k) in seen:
                continue
            seen.add((i, k))
            prec.append((int(perm[i]), int(perm[k])))
        # greedy list schedule in permutation order (a topological order of precedences)
        preds = [[] for _ in range(n_jobs)]
        for a, b in prec:
            preds[b].append(a)
        free = np.zeros(n_machines)
        s = np.zeros(n_jobs)
        for j in perm:
            t = free[mach[j]]
            for a in preds[j]:
                t = max(t, s[a] + d[a])
            s[j] = t
            free[mach[j]] = t + d[j]
        if np.all(s + d <= H):
            break
    else:
        raise RuntimeError("no feasible scheduling instance found")

    # same-machine pairs, machine-major, j<k
    pj, pk = [], []
    for mm in range(n_machines):
        jobs = np.nonzero(mach == mm)[0]
        if len(jobs) < 2:
            continue
        jj, kk = np.triu_indices(len(jobs), 1)
        pj.append(jobs[jj])
        pk.append(jobs[kk])
    pj = np.concatenate(pj) if pj else np.zeros(0, np.int64)
    pk = np.concatenate(pk) if pk else np.zeros(0, np.int64)
    P = int(pj.shape[0])
    n_bool = P
    n_prec_eff = len(prec)
    n_atoms = 2 * P + n_jobs + n_prec_eff

    # atoms: pair p -> 2p: s_j - s_k <= -d_j ; 2p+1: -s_j + s_k <= -d_k
    atom_var = np.empty(2 * (2 * P) + n_jobs + 2 * n_prec_eff, np.int32)
    atom_coef = np.empty_like(atom_var, dtype=np.float64)
    atom_rhs = np.empty(n_atoms, np.float64)
    nnz = np.concatenate([np.full(2 * P, 2), np.full(n_jobs, 1), np.full(n_prec_eff, 2)])
    atom_ptr = np.zeros(n_atoms + 1, np.int64)
    np.cumsum(nnz, out=atom_ptr[1:])
    q = 0
    atom_var[0:4 * P:4] = pj
    atom_var[1:4 * P:4] = pk
    atom_var[2:4 * P:4] = pj
    atom_var[3:4 * P:4] = pk
    atom_coef[0:4 * P:4] = 1.0
    atom_coef[1:4 * P:4] = -1.0
    atom_coef[2:4 * P:4] = -1.0
    atom_coef[3:4 * P:4] = 1.0
    atom_rhs[0:2 * P:2] = -d[pj]
    atom_rhs[1:2 * P:2] = -d[pk]
    q = 4 * P
    atom_var[q:q + n_jobs] = np.arange(n_jobs)
    atom_coef[q:q + n_jobs] = 1.0
    atom_rhs[2 * P:2 * P + n_jobs] = H - d
    q += n_jobs
    for t, (a, b) in enumerate(prec):
        atom_var[q + 2 * t] = a
        atom_var[q + 2 * t + 1] = b
        atom_coef[q + 2 * t] = 1.0
        atom_coef[q + 2 * t + 1] = -1.0
        atom_rhs[2 * P + n_jobs + t] = -d[a]
    atom_op = np.full(n_atoms, OP_LE, np.int8)

    # constraints: per pair (not o or A1), (o or A2); then horizons; then precedences
    C = 2 * P + n_jobs + n_prec_eff
    con_kind = np.full(C, KIND_CLAUSE, np.int32)
    lens = np.concatenate([np.full(2 * P, 2), np.full(n_jobs + n_prec_eff, 1)])
    con_ptr = np.zeros(C + 1, np.int64)
    np.cumsum(lens, out=con_ptr[1:])
    con_lit = np.empty(int(con_ptr[-1]), np.int32)
    p = np.arange(P)
    atom_id = lambda k: n_bool + k  # noqa: E731
    con_lit[0:4 * P:4] = 2 * p + 1                    # not o_p
    con_lit[1:4 * P:4] = 2 * atom_id(2 * p)           # A1
    con_lit[2:4 * P:4] = 2 * p                        # o_p
    con_lit[3:4 * P:4] = 2 * atom_id(2 * p + 1)       # A2
    rest = np.arange(2 * P, n_atoms)
    con_lit[4 * P:] = 2 * atom_id(rest)
    con_param = np.zeros(C, np.int32)
    expr_ptr = np.zeros(C + 1, np.int64)

    cert_x = np.where(s[pj] < s[pk], -1.0, 1.0).astype(np.float64)   # -1 = True = j first
    prob = Problem(
        n_bool=n_bool, n_real=n_jobs, atom_ptr=atom_ptr, atom_var=atom_var,
        atom_coef=atom_coef, atom_rhs=atom_rhs, atom_op=atom_op, con_kind=con_kind,
        con_ptr=con_ptr, con_lit=con_lit, con_param=con_param, expr_ptr=expr_ptr,
        expr_ops=np.zeros(0, np.int32), real_lo=np.zeros(n_jobs), real_hi=np.full(n_jobs, H),
        meta=dict(family="scheduling", n_jobs=n_jobs, n_machines=n_machines, horizon=H,
                  n_pairs=P, n_prec=n_prec_eff, attempts=attempt + 1,
                  mean_duration=float(d.mean())),
        cert_x=cert_x, cert_y=s.copy())
    prob.validate()
    return prob
