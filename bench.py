#!/usr/bin/env python3
"""Benchmark of the FourierSMT hot path on one MI355X.

Workload: job-shop scheduling, 200 jobs on 10 machines (~2,000 order Booleans, ~4,100
constraints), 64 restarts, seeded synthetic instance (the paper's instances are not public).
A step is one pass of the whole hot path over the batch: literal probabilities, forward
and reverse sweep with gradient scatter (one kernel), the projected-gradient step, and the
rounding + exact check. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3       # MI355X vector FP32 (published)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kappa", type=float, default=0.05)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-mode", action="store_true",
                    help="few launches plus a 256 MiB copy kernel, for counter collection")
    return ap.parse_args()


def algorithmic_cost(p, stats):
    """Per-launch algorithmic work of the forward + reverse sweep."""
    nnz = np.diff(p.atom_ptr)
    n_bool_lits = n_atom_lits = 0
    for c in range(p.n_cons):
        ids = np.unique(p.con_lit[p.con_ptr[c]:p.con_ptr[c + 1]] >> 1)
        n_bool_lits += int((ids < p.n_bool).sum())
        n_atom_lits += int((ids >= p.n_bool).sum())
    atom_nnz_per_con = float(nnz.sum())
    return dict(total_nodes=int(stats["total_nodes"]), bool_slots=n_bool_lits, atom_slots=n_atom_lits,
                atom_nnz=atom_nnz_per_con, table_bytes=int(stats["table_bytes"]))


def flops_per_step(cost, R):
    # forward 4 flops/node (two multiply-adds), reverse 6 flops/node (p*bh + q*bl: 3,
    # (bh - bl) and the multiply-add into the slot sensitivity: 3);
    # Boolean slot: p, 1-p, gradient (-1/2 w G): 6; atom slot: z (2 per nnz + 1), u (1),
    # erfc (25, rational approximation), exp (10), dp/dz (2), p and 1-p (2),
    # gradient (2 + 2 per nnz)
    per = (10 * cost["total_nodes"] + 6 * cost["bool_slots"]
           + (1 + 1 + 25 + 10 + 2 + 2 + 2) * cost["atom_slots"] + 4 * cost["atom_nnz"])
    return float(per) * R


def bytes_per_step(cost, p, R):
    # compiled tables streamed once per launch + per restart state: read a, b; gradient
    # read-modify-write and the projected step (read a, b, grads; write a, b, zero grads)
    S = 4 * (p.n_bool + p.n_real)
    return float(cost["table_bytes"]) + R * S * 6


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_2603_22877_amd as fsmt
    import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    p = W.make_config(2)
    R = W.RESTARTS[2]
    a0, b0 = W.initial_points(p, R, 2, 0)
    h = fsmt.xbdd_compile(p)
    stats = fsmt.xbdd_info(h)
    cost = algorithmic_cost(p, stats)
    st = torch.cuda.Stream(device=dev)
    # variable-major state [n][R] viewed as [R][n]: lanes = restarts read consecutive words
    a = torch.as_tensor(a0.T.copy(), device=dev).t()
    b = torch.as_tensor(b0.T.copy(), device=dev).t()
    ga = torch.zeros(p.n_bool, R, device=dev).t()
    gb = torch.zeros(p.n_real, R, device=dev).t()
    w = torch.ones(p.n_cons, device=dev)
    obj = torch.zeros(R, device=dev)
    gsq = torch.zeros(R, device=dev)
    nw = (p.n_cons + 31) // 32
    x = torch.zeros(R, p.n_bool, dtype=torch.int8, device=dev)
    bits = torch.zeros(R, nw, dtype=torch.int32, device=dev)
    nu = torch.zeros(R, dtype=torch.int32, device=dev)
    ver = torch.zeros(R, dtype=torch.int32, device=dev)
    eta_a, eta_b = 0.05, 1.0
    kap = args.kappa

    def step(ev=None):
        obj.zero_()
        if ev is not None:
            ev[0].record(st)
        fsmt.cop_backward(h, a, b, kap, w, obj, ga, gb, flags=fsmt.FSMT_ACCUMULATE, stream=st)
        if ev is not None:
            ev[1].record(st)
        fsmt.pgd_step(h, a, b, ga, gb, eta_a, eta_b, gsq, stream=st)
        fsmt.round_and_check(h, a, b, x, bits, nu, ver, stream=st)

    if args.pmc_mode:
        src = torch.empty(64 * 1024 * 1024, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)                       # calibration: 256 MiB read + 256 MiB written
        for _ in range(5):
            step()
        torch.cuda.synchronize()
        print(json.dumps({"pmc_mode": True, "copy_bytes": src.numel() * 4}))
        return

    with torch.cuda.stream(st):
        for _ in range(args.warmup):
            step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(st):
        for k in range(args.steps):
            step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    kern_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    evals = p.n_cons * R * args.steps
    value = evals / dt

    fl = flops_per_step(cost, R)
    by = bytes_per_step(cost, p, R)
    achieved_tf = fl / (kern_ms * 1e-3) / 1e12
    achieved_gbs = by / (kern_ms * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic_sched200.json")
    if os.path.exists(tfile):
        try:
            traffic = json.load(open(tfile)).get("bytes_per_launch")
        except Exception:
            traffic = None

    out = {
        "metric": "constraint-evals/s (fwd+bwd) and time-to-SAT, batched fused vs plain, 1 GPU",
        "value": value, "unit": "constraint-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "scheduling 200 jobs / 10 machines, 64 restarts",
                   "n_cons": p.n_cons, "n_bool": p.n_bool, "n_real": p.n_real, "restarts": R,
                   "kappa": kap, "path": "per-call kernels (cop_backward, pgd_step, round_and_check)"},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tf / PEAK_FP32_TFLOPS,
                     "traffic": traffic, "kernel": "cop_kernel<true>", "kernel_ms": kern_ms,
                     "hbm_achieved_gbs": achieved_gbs, "hbm_frac": achieved_gbs / PEAK_HBM_GBS},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, a0, b0, kap)
    print(json.dumps(out))


def cpu_baseline(p, a0, b0, kap):
    """The FP64 oracle, single-threaded, on a sample of the same workload (~10 s)."""
    import oracle
    op = oracle.OracleProblem(p)
    R = a0.shape[0]
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < 10.0:
        r = done % R
        oracle.objective(op, a0[r:r + 1], b0[r:r + 1], kap, per_constraint=False)
        done += 1
    dt = time.perf_counter() - t0
    return {"value": p.n_cons * done / dt, "unit": "constraint-evals/s", "cores": 1, "kind": "oracle",
            "sample": f"objective + gradient of all {p.n_cons} constraints at {done} restart points "
                      f"(cycling over the 64), FP64, one thread, ~10 s"}


if __name__ == "__main__":
    main()
