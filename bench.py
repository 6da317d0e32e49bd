#!/usr/bin/env python3
"""Benchmark of the FourierSMT hot path on one MI355X.

Workload of the main line: placement of 1,200 rectangles with rotation bits (721,800
constraints: 719,400 pairwise non-overlap ITEs over eight separation atoms and 2,400
feasibility ITEs; 1,200 Booleans, 2,400 reals), 16 restarts, seeded synthetic instance (the
paper's instances are not public; the generator is in workloads/placement.py). This is the
size of the paper's scale claim (about 700,000 constraints).

* value: constraint-evals/s of the fused batched solver. A step is one annealing level:
  100 PGD iterations, each the literal probabilities, forward + reverse sweep with the
  gradient scatter, objective, and the projected step, followed by the rounding + exact
  check and the ERWA weight update. One constraint-eval = one (constraint, restart)
  forward + backward; evals per step = C x R x 100. Inputs are resident on the device
  before the timed region; no early exit (eps = 0, no stop on SAT) so the work is fixed.
* roofline: the solver kernel's duration from HIP events on its stream (the launch is the
  kernel: one persistent launch per call); algorithmic bytes per PGD iteration T + R S
  (compiled tables once per pass over the restarts, plus each restart's state) and
  modelled FLOPs per constraint-eval (flops_per_pass), against the HBM peak and the FP32
  FMA issue rate without packed math; `bound` names the larger fraction. `traffic` is the
  measured HBM bytes (FETCH_SIZE + WRITE_SIZE, calibrated) of the committed rocprofv3
  summary, per iteration, times the launch's iterations.
* time_to_sat: solver wall time until a SAT verdict on job-shop scheduling 200 jobs x 10
  machines (from each solve launch to the host reading the verdict; initial points drawn
  and uploaded outside the clock), batched fused (64 restarts in one launch) against the
  plain per-call path (one restart at a time, separate launches per step), same
  hyperparameters, median and PAR-2 over instance seeds; time_to_sat_index_encoding: the
  same comparison on the paper's scheduling encoding (16 workers x 32 jobs), where a single
  restart rarely reaches SAT.
* other_workloads: fixed-work rates of the same solver on scheduling 200 x 10 (64 restarts)
  and the uneven batch of 48 instances (16 restarts each, 2.0M constraints).
* cpu_baseline: the FP64 oracle on a bounded sample of the main workload (~10 s, one
  thread); cpu_baseline_all_cores: the same on up to 16 host threads.
* paper_protocol: the paper's gradient-timing protocol (Supplementary Note "Gradient
  Computation Time"): random hybrid instances with n Booleans, n reals and n atoms, 100
  annealing parameters x 100 points, one cop_backward call (objective + gradient) per
  parameter; reported next to the paper's L40S figure as context (other hardware, other
  instances of the same shape); also on the scheduling instance above.

Other modes (each prints its own JSON line instead of the main one):

* --suite scheduling|placement: PAR-2 of the fused solver on the paper's own encodings
  (Booleanized worker / macro / layer indices, XOR disjunctions; workloads/paper_suite.py).
* --scale-mode: fixed-work fused-solver throughput at the largest sizes of those suites.
* --configs-mode: fixed-work rates on placement 150 x 256 restarts and time-to-SAT there.
* --pmc-mode, --percall-mode: short runs for hardware-counter collection.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-tts]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
# MI355X vector FP32: 157.3 TFLOP/s published with packed FP32; the library is built without
# packed FP32, so its issue rate is 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz
PEAK_FP32_TFLOPS = 78.6
STEPS_PER_LEVEL = 100
ETA_A, ETA_B, EPS = 0.5, 5.0, 1e-2
LEVELS = 40


def log(msg: str) -> None:
    """A progress line on stderr (the JSON result goes to stdout)."""
    print(f"# {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed annealing levels (<= 128)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tts", action="store_true", help="skip the time-to-SAT comparison")
    ap.add_argument("--no-protocol", action="store_true", help="skip the paper's gradient-timing protocol")
    ap.add_argument("--no-other", action="store_true", help="skip the rates on the other workloads")
    ap.add_argument("--tts-seeds", type=int, default=10)
    ap.add_argument("--tts-cap", type=float, default=30.0, help="time limit per instance (s)")
    ap.add_argument("--percall-mode", action="store_true",
                    help="profiling aid: per-call forward + reverse sweeps on placement with 1,200 "
                         "rectangles (1 and 16 restarts) after a calibration copy")
    ap.add_argument("--pmc-mode", action="store_true",
                    help="one short solver launch plus a 256 MiB copy, for counter collection")
    ap.add_argument("--suite", choices=["scheduling", "placement"],
                    help="PAR-2 of the fused solver on the paper's own encodings (index bits, XOR "
                         "disjunctions) instead of the default line")
    ap.add_argument("--cells", default=None,
                    help="suite cells, e.g. 16x2,16x3 (n_w x ratio, or n_m x n_l)")
    ap.add_argument("--per-cell", type=int, default=3, help="instances per cell (the paper has 10)")
    ap.add_argument("--limit", type=float, default=30.0, help="PAR-2 time limit per instance (s)")
    ap.add_argument("--suite-restarts", type=int, default=0,
                    help="restarts per attempt (0: 64, fewer for instances past 125k constraints)")
    ap.add_argument("--configs-mode", action="store_true",
                    help="fixed-work fused-solver throughput on placement 150 x 256 restarts and "
                         "time-to-SAT on placement 150")
    ap.add_argument("--scale-mode", action="store_true",
                    help="fixed-work solver throughput on the paper's largest encodings "
                         "(scheduling 256 workers x 5, placement 64 macros x 8 layers)")
    return ap.parse_args()


def algorithmic_cost(p, stats):
    """Slots, atoms and nodes of the instance (per constraint-eval work model)."""
    nnz = np.diff(p.atom_ptr)
    n_bool = n_atom = nnz_used = 0
    for c in range(p.n_cons):
        ids = np.unique(p.con_lit[p.con_ptr[c]:p.con_ptr[c + 1]] >> 1)
        n_bool += int((ids < p.n_bool).sum())
        atoms = ids[ids >= p.n_bool] - p.n_bool
        n_atom += len(atoms)
        nnz_used += int(nnz[atoms].sum())
    # the table stream of the method, independent of this library's layout: per constraint a
    # 16-byte header, 8 bytes per decision node, 4 per support variable, and per atom 8 per
    # nonzero plus 8
    model = (16 * p.n_cons + 8 * int(stats["total_nodes"]) + 4 * (n_bool + n_atom)
             + 8 * nnz_used + 8 * n_atom)
    return dict(total_nodes=int(stats["total_nodes"]), bool_slots=n_bool, atom_slots=n_atom,
                atom_nnz=nnz_used, table_bytes=int(stats["table_bytes"]), table_model_bytes=int(model))


def flops_per_pass(cost, R):
    """FP32-equivalent operations of one forward + reverse sweep over all constraints.

    forward 4/node (two multiply-adds), reverse 6/node; Boolean slot 6 (p, 1-p, gradient);
    atom slot: z 2/nnz + 1, u 1, erfc 25, exp 10, dp/dz 2, p and 1-p 2, gradient 2 + 2/nnz.
    """
    per = (10 * cost["total_nodes"] + 6 * cost["bool_slots"]
           + 43 * cost["atom_slots"] + 4 * cost["atom_nnz"])
    return float(per) * R


def bytes_per_pass(cost, p, R):
    """T + R S: the method's table stream (``table_model_bytes``) read once per pass over the
    restarts, plus per restart a, b read, gradient written and read, projected state
    written, and one weight per constraint read."""
    return float(cost["table_model_bytes"]) + R * (4 * (p.n_bool + p.n_real) * 5 + 4 * p.n_cons)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                                   "(restarts and instances shard across GPUs without exchange)"}))
        sys.exit(2)
    import torch

    import paper_2603_22877_amd as fsmt
    from paper_2603_22877_amd import solver as S
    import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.suite:
        print(json.dumps(paper_suite(args, S)))
        return
    if args.scale_mode:
        print(json.dumps(paper_scale(args, fsmt, S)))
        return
    if args.configs_mode:
        print(json.dumps(other_configs(args, fsmt, S)))
        return
    log("compiling placement 1200 rectangles")
    p = W.make_workload("placement_1200")
    R = W.RESTARTS["placement_1200"]
    ell = p.meta["mean_side"]
    t0 = time.perf_counter()
    h = fsmt.xbdd_compile(p)
    compile_s = time.perf_counter() - t0
    stats = fsmt.xbdd_info(h)
    cost = algorithmic_cost(p, stats)
    st = torch.cuda.Stream(device=dev)
    a0, b0 = W.initial_points(p, R, 5, 0)
    levels = max(1, min(args.steps, 128))
    kappas = S.kappa_schedule(ell, max(LEVELS, levels, 2))

    plan = None

    def fixed_cfg(n_levels, steps=STEPS_PER_LEVEL):
        c = S.SolveConfig(kappas=kappas[:n_levels], steps_per_level=steps, eta_a=ETA_A,
                          eta_b=ETA_B, eps=0.0, stop_on_sat=0)
        return plan.apply(c) if plan is not None else c

    if args.pmc_mode or args.percall_mode:
        # calibration: one element-wise shader kernel reading 256 MiB and writing 256 MiB
        src = torch.ones(64 * 1024 * 1024, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
    if args.percall_mode:
        percall_placement(fsmt, W, st)
        print(json.dumps({"percall_mode": True, "copy_bytes": src.numel() * 4}))
        return
    if args.pmc_mode:
        # one launch of one level of PMC_STEPS PGD iterations (and its check), under the plan
        # the main line's autotuner cached (the model's plan when there is none)
        from paper_2603_22877_amd import autotune as AT
        plan = AT.cached_plan([h], [(a0, b0)], fixed_cfg(levels))
        state = S.BatchState(h, a0, b0)
        S.solve_batched([h], [state], fixed_cfg(1, PMC_STEPS), stream=st)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_mode": True, "copy_bytes": src.numel() * 4, "pgd_steps": PMC_STEPS}))
        return

    # the solver plan (schedule, cluster size) measured by the autotuner, outside the clock
    from paper_2603_22877_amd import autotune as AT
    t0 = time.perf_counter()
    plan = AT.tune([h], [(a0, b0)], fixed_cfg(levels), stream=st, log=log)
    tune_s = time.perf_counter() - t0
    log(f"autotuned plan: {plan.label} (cluster {plan.cluster}) in {tune_s:.1f} s")

    # the K timed steps (annealing levels) are one fused launch; each of the W warmup runs is
    # an identical launch on a throwaway state, so every launch of this kernel carries the
    # same work (the profiler's per-launch average is the timed launch's duration)
    for _ in range(args.warmup):
        warm = S.BatchState(h, a0, b0)
        S.solve_batched([h], [warm], fixed_cfg(levels), stream=st)
    torch.cuda.synchronize()
    state = S.BatchState(h, a0, b0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    S.solve_batched([h], [state], fixed_cfg(levels), stream=st)
    e1.record(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_s = e0.elapsed_time(e1) * 1e-3                 # the launch
    pgd_steps = int(state.steps_done.cpu().numpy().min())
    assert pgd_steps == levels * STEPS_PER_LEVEL
    evals = p.n_cons * R * pgd_steps
    value = evals / dt
    log(f"timed launch: {levels} levels, {value:.3e} constraint-evals/s")

    out = {
        "metric": "constraint-evals/s (fwd+bwd) and time-to-SAT, batched fused vs plain, 1 GPU",
        "value": value, "unit": "constraint-evals/s", "n_gpus": 1, "steps": levels,
        "warmup": args.warmup, "ms_per_step": dt / levels * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "placement of 1,200 rectangles with rotation bits (721,800 constraints), "
                               "16 restarts (fused batched solver; step = one annealing level of 100 PGD "
                               "iterations + check + ERWA)",
                   "n_cons": p.n_cons, "n_bool": p.n_bool, "n_real": p.n_real, "restarts": R,
                   "pgd_steps_timed": pgd_steps, "compile_s": compile_s,
                   "table_bytes": stats["table_bytes"], "closed_form_constraints": stats["n_gd"],
                   "plan": {"label": plan.label, "cluster": plan.cluster, "inst_schedule": plan.inst_schedule,
                            "candidates_ms_per_level": {k: v / 1e3 for k, v in plan.candidates.items()},
                            "tune_s": tune_s, "cached": plan.cached}},
        "roofline": roofline(p, cost, R, pgd_steps, kern_s, "solve_wg_kernel",
                             "solve_wg_kernel_placement1200.md"),
    }
    h.free()
    if not args.no_tts:
        out["time_to_sat"] = time_to_sat(args, fsmt, S, W, st)
        log("time-to-SAT on scheduling 200 x 10 done")
        out["time_to_sat_index_encoding"] = time_to_sat_hard(args, fsmt, S, W, st)
        log("time-to-SAT on the index encoding done")
    if not args.no_other:
        out["other_workloads"] = {
            "scheduling 200 x 10, 64 restarts": _fixed_work(fsmt, S, [W.make_workload("scheduling_200x10")], 64, (2, 0), steps=100),
            "uneven batch, 48 instances x 16 restarts": _fixed_work(fsmt, S, W.uneven_batch(), 16, (4, 0)),
            "uneven batch, 48 instances x 16 restarts, autotuned plan":
                _fixed_work(fsmt, S, W.uneven_batch(), 16, (4, 0), tuned=True),
        }
        log("other workloads done")
    if not args.no_protocol:
        out["paper_protocol"] = paper_protocol(fsmt, W, st)
        log("gradient-timing protocol done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, a0, b0, kappas[0])
        out["cpu_baseline_all_cores"] = cpu_baseline(p, a0, b0, kappas[0], threads=min(16, os.cpu_count() or 1))
        log("CPU baselines done")
    print(json.dumps(out))


PMC_STEPS = 20   # PGD iterations of the --pmc-mode launch


def roofline(p, cost, R, pgd_steps, kern_s, kernel, profile_name):
    """Roofline of the solver launch: modelled FLOPs and algorithmic bytes per launch over the
    launch's duration (HIP events on its stream), and the measured HBM bytes per PGD
    iteration from the committed rocprofv3 summary."""
    fl = flops_per_pass(cost, R) * pgd_steps
    by = bytes_per_pass(cost, p, R) * pgd_steps
    ach_tf = fl / kern_s / 1e12
    ach_gbs = by / kern_s / 1e9
    f_alu, f_hbm = ach_tf / PEAK_FP32_TFLOPS, ach_gbs / PEAK_HBM_GBS
    traffic = None
    tfile = os.path.join(ROOT, "profiles", profile_name)
    if os.path.exists(tfile):
        for line in open(tfile):
            if line.startswith("hbm_bytes_per_pgd_step:"):
                traffic = float(line.split(":")[1]) * pgd_steps
    if f_alu >= f_hbm:
        head = {"bound": "alu", "achieved": ach_tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": f_alu}
    else:
        head = {"bound": "hbm", "achieved": ach_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": f_hbm}
    return {**head, "traffic": traffic, "kernel": kernel, "kernel_ms": kern_s * 1e3,
            "flop_per_launch": fl, "bytes_per_launch": by, "alu_achieved_tflops": ach_tf, "alu_frac": f_alu,
            "hbm_achieved_gbs": ach_gbs, "hbm_frac": f_hbm,
            "traffic_gbs": traffic / kern_s / 1e9 if traffic else None}


def percall_placement(fsmt, W, st):
    """cop_backward on the paper-scale placement instance (721,800 constraints): 3 calls at
    1 restart (the tables stream from HBM) and 3 at 16 restarts."""
    import torch
    dev = torch.device("cuda", 0)
    p = W.make_workload("placement_1200")
    h = fsmt.xbdd_compile(p)
    for R in (1, 16):
        a0, b0 = W.initial_points(p, R, 5, 0)
        a, b = torch.as_tensor(a0, device=dev), torch.as_tensor(b0, device=dev)
        ga, gb = torch.zeros_like(a), torch.zeros_like(b)
        w = torch.ones(p.n_cons, device=dev)
        obj = torch.zeros(R, device=dev)
        for _ in range(3):
            fsmt.cop_backward(h, a, b, 0.1, w, obj, ga, gb, stream=st)
        torch.cuda.synchronize()
    h.free()


def time_to_sat(args, fsmt, S, W, st):
    """Batched fused vs plain per-call time-to-SAT on scheduling 200x10 instance seeds."""
    import torch
    res = {"batched_s": [], "plain_s": [], "plain_restarts": [], "batched_level": []}
    cap = args.tts_cap
    for seed in range(args.tts_seeds):
        p = W.make_workload("scheduling_200x10", seed)
        h = fsmt.xbdd_compile(p)
        kap = S.kappa_schedule(p.meta["mean_duration"], LEVELS)
        cfg = S.SolveConfig(kappas=kap, steps_per_level=STEPS_PER_LEVEL, eta_a=ETA_A, eta_b=ETA_B,
                            eps=EPS, stop_on_sat=2)
        # batched: 64 restarts per launch; relaunch with fresh seeds until SAT or cap. The
        # clock runs from each solve launch to the host reading the verdict (the initial
        # points are drawn and uploaded outside it)
        elapsed, tb, batch_round = 0.0, None, 0
        while elapsed < cap:
            a0, b0 = W.initial_points(p, 64, 2, seed, 100 + batch_round)
            state = S.BatchState(h, a0, b0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.solve_batched([h], [state], cfg, stream=st)
            torch.cuda.synchronize()          # the solver runs on its own stream
            ver = state.verdict.cpu().numpy()
            elapsed += time.perf_counter() - t0
            if ver.max() == 1:
                tb = elapsed
                res["batched_level"].append(int(state.level_done.cpu().numpy()[ver == 1].min()))
                break
            batch_round += 1
        res["batched_s"].append(tb)
        # plain: one restart at a time with new seeds (its host loop uploads the point)
        plain = S.PlainSolver(h, R=1)
        elapsed, tp, r = 0.0, None, 0
        while elapsed < cap:
            a0, b0 = W.initial_points(p, 1, 2, seed, 100 + r)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = plain.run(a0, b0, cfg, stream=st)
            torch.cuda.synchronize()
            elapsed += time.perf_counter() - t0
            if out["verdict"] == 1:
                tp = elapsed
                break
            r += 1
        res["plain_s"].append(tp)
        res["plain_restarts"].append(r + 1)
        log(f"time-to-SAT seed {seed}: batched {tb}, plain {tp}")

    def par2(ts):
        return float(np.mean([t if t is not None else 2 * cap for t in ts]))

    def med(ts):
        return float(statistics.median([t if t is not None else 2 * cap for t in ts]))

    return {"instances": args.tts_seeds, "cap_s": cap,
            "batched_median_s": med(res["batched_s"]), "plain_median_s": med(res["plain_s"]),
            "batched_par2_s": par2(res["batched_s"]), "plain_par2_s": par2(res["plain_s"]),
            "speedup_median": med(res["plain_s"]) / med(res["batched_s"]),
            "batched_solved": sum(t is not None for t in res["batched_s"]),
            "plain_solved": sum(t is not None for t in res["plain_s"]),
            "per_instance": res,
            "hyperparameters": {"levels": LEVELS, "kappa": "4 t / (40 mean duration)",
                                "steps_per_level": STEPS_PER_LEVEL, "eta_a": ETA_A, "eta_b": ETA_B,
                                "eps": EPS, "rho": 0.5, "gamma": 2.0, "tau": 1}}


def time_to_sat_hard(args, fsmt, S, W, st, cap=5.0, instances=10):
    """Batched (64 restarts per fused launch) vs plain (one restart at a time, per-call
    launches) time-to-SAT on the paper's scheduling encoding, 16 workers x 32 jobs, where a
    single restart often fails (instance seeds 0-9, a limit of 5 s per path and instance)."""
    import torch
    from workloads.paper_suite import make_paper_scheduling
    res = {"batched_s": [], "plain_s": [], "batched_restarts": [], "plain_restarts": []}
    for k in range(instances):
        p = make_paper_scheduling(16, 2, W.seed_seq(8, 16, 2, k))
        h = fsmt.xbdd_compile(p)
        cfg = _suite_cfg(S, p)
        # solver time only, as above: launches to the verdict, points drawn outside the clock
        elapsed, tb, att = 0.0, None, 0
        while elapsed < cap:
            state = S.BatchState(h, *W.initial_points(p, 64, 55, 16, 2, k, att))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.solve_batched([h], [state], cfg, stream=st)
            torch.cuda.synchronize()          # the solver runs on its own stream
            ver = state.verdict.cpu().numpy()
            elapsed += time.perf_counter() - t0
            att += 1
            if ver.max() == 1:
                tb = elapsed
                break
        res["batched_s"].append(tb)
        res["batched_restarts"].append(64 * att)
        plain = S.PlainSolver(h, R=1)
        elapsed, tp, r = 0.0, None, 0
        while elapsed < cap:
            a0, b0 = W.initial_points(p, 1, 56, 16, 2, k, r)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = plain.run(a0, b0, cfg, stream=st)
            torch.cuda.synchronize()
            elapsed += time.perf_counter() - t0
            r += 1
            if out["verdict"] == 1:
                tp = elapsed
                break
        res["plain_s"].append(tp)
        res["plain_restarts"].append(r)
        log(f"time-to-SAT index encoding instance {k}: batched {tb}, plain {tp}")
        h.free()
    sc = lambda ts: [t if t is not None else 2 * cap for t in ts]  # noqa: E731
    return {"workload": f"paper's scheduling encoding, 16 workers x 32 jobs (instances 0-{instances - 1})",
            "cap_s": cap, "batched_par2_s": float(np.mean(sc(res["batched_s"]))),
            "plain_par2_s": float(np.mean(sc(res["plain_s"]))),
            "batched_median_s": float(statistics.median(sc(res["batched_s"]))),
            "plain_median_s": float(statistics.median(sc(res["plain_s"]))),
            "batched_solved": sum(t is not None for t in res["batched_s"]),
            "plain_solved": sum(t is not None for t in res["plain_s"]), "per_instance": res,
            "hyperparameters": SUITE_HP}


# mean GPU ms per gradient call reported by the paper for its random hybrid instances
# (NVIDIA L40S; Supplementary Table "gradient-time", group means over the 10 instances)
PAPER_L40S_MS = {100: 12.702, 500: 12.603, 1000: 12.653}


def paper_protocol(fsmt, W, st, ns=(100, 500, 1000)):
    """Gradient timing: 100 kappa values (0.00 .. 0.99) x 100 points, one call per kappa."""
    import torch
    dev = torch.device("cuda", 0)
    rows = {}
    for n in ns:
        p = W.make_random_hybrid(n)
        h = fsmt.xbdd_compile(p)
        a0, b0 = W.initial_points(p, 100, 6, n)
        a = torch.as_tensor(a0, device=dev)
        b = torch.as_tensor(b0, device=dev)
        ga, gb = torch.zeros_like(a), torch.zeros_like(b)
        w = torch.ones(p.n_cons, device=dev)
        obj = torch.zeros(100, device=dev)
        kaps = [0.01 * t for t in range(100)]
        for k in kaps[:3]:
            fsmt.cop_backward(h, a, b, k, w, obj, ga, gb, stream=st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in kaps:
            fsmt.cop_backward(h, a, b, k, w, obj, ga, gb, stream=st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        info = fsmt.xbdd_info(h)
        rows[str(n)] = {"n_cons": p.n_cons, "max_nodes": info["max_nodes"], "ms_per_call_100_points": dt * 10,
                        "us_per_point": dt / 10000 * 1e6, "paper_L40S_ms_per_gradient": PAPER_L40S_MS.get(n)}
    # the same protocol on the benchmark's scheduling instance (200 jobs on 10 machines)
    p = W.make_workload("scheduling_200x10")
    h = fsmt.xbdd_compile(p)
    a0, b0 = W.initial_points(p, 100, 2, 7)
    a, b = torch.as_tensor(a0, device=dev), torch.as_tensor(b0, device=dev)
    ga, gb = torch.zeros_like(a), torch.zeros_like(b)
    w = torch.ones(p.n_cons, device=dev)
    obj = torch.zeros(100, device=dev)
    ell = p.meta["mean_duration"]
    kaps = [0.01 * t / ell for t in range(100)]
    for k in kaps[:3]:
        fsmt.cop_backward(h, a, b, k, w, obj, ga, gb, stream=st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in kaps:
        fsmt.cop_backward(h, a, b, k, w, obj, ga, gb, stream=st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rows["scheduling 200x10"] = {"n_cons": p.n_cons, "max_nodes": fsmt.xbdd_info(h)["max_nodes"],
                                 "ms_per_call_100_points": dt * 10, "us_per_point": dt / 10000 * 1e6,
                                 "paper_L40S_ms_per_gradient": None}
    return {"workload": "random hybrid (n Booleans, n reals, n atoms; n/5 CARD and NAE of length "
                        "min(50, n/5), n/50 XOR of length 50), 100 kappa x 100 points, FP32; and the "
                        "scheduling instance of the main line (kappa 0 .. 0.99 / mean duration)",
            "per_n": rows,
            "note": "the paper does not say whether its figure is per point or per 100-point call; "
                    "its hardware and instances differ (context, not a target)"}


# hyperparameters of the paper-encoding runs: eta_b scales with the square of the length
# scale ell (mean duration or mean module side) and the last level reaches kappa = 40 / ell
SUITE_HP = {"levels": 80, "kmax": 40.0, "steps_per_level": 100, "eta_a": 0.5, "eta_b_per_ell2": 0.05,
            "eps": 1e-2, "rho": 0.5, "gamma": 2.0, "tau": 1}
SUITE_CELLS = {"scheduling": "16x2,16x3,16x4,16x5", "placement": "2x2,4x4,8x4,8x8,16x8"}


def suite_restarts(n_cons):
    """Restarts per attempt: 64, and 16 for instances past 125k constraints, where a PGD
    step over 64 restarts costs tens of milliseconds and the annealing levels, not the
    restarts, run out within the limit."""
    return 64 if n_cons <= 125000 else 16


def _paper_make(suite, A, B, k):
    import workloads as W
    from workloads.paper_suite import make_paper_placement, make_paper_scheduling
    if suite == "scheduling":
        return make_paper_scheduling(A, B, W.seed_seq(8, A, B, k))
    return make_paper_placement(A, B, W.seed_seq(9, A, B, k))


def _suite_cfg(S, p, **over):
    hp = dict(SUITE_HP, **over)
    ell = p.meta.get("mean_duration", p.meta.get("mean_side"))
    return S.SolveConfig(kappas=S.kappa_schedule(ell, hp["levels"], hp["kmax"]),
                         steps_per_level=hp["steps_per_level"], eta_a=hp["eta_a"],
                         eta_b=hp["eta_b_per_ell2"] * ell * ell, eps=hp["eps"], rho=hp["rho"],
                         gamma=hp["gamma"], tau=hp["tau"], stop_on_sat=2)


def paper_suite(args, S):
    """PAR-2 over cells of the paper's scheduling or placement suite (fresh instances)."""
    import workloads as W
    from paper_2603_22877_amd import par2 as P2
    cells = [tuple(int(v) for v in c.split("x")) for c in (args.cells or SUITE_CELLS[args.suite]).split(",")]
    limit = args.limit
    rows, results = {}, []
    for A, B in cells:
        res = []
        for k in range(args.per_cell):
            p = _paper_make(args.suite, A, B, k)
            init = (lambda q, R_, att, A=A, B=B, k=k: W.initial_points(q, R_, 55, A, B, k, att))
            R = args.suite_restarts or suite_restarts(p.n_cons)
            r = P2.run_instance(p, _suite_cfg(S, p), R, limit, init, name=f"{A}x{B}#{k}")
            print(f"# {args.suite} {r.name} cons={p.n_cons} R={R} solved={r.solved} s={r.seconds:.3f} "
                  f"attempts={r.attempts} levels={r.levels} best_unsat={r.best_unsat}", file=sys.stderr, flush=True)
            res.append(r)
        results += res
        rows[f"{A}x{B}"] = {"n_cons": int(p.n_cons), "solved": sum(r.solved for r in res), "instances": len(res),
                            "par2_s": P2.par2(res, limit),
                            "median_s": float(statistics.median([r.score(limit) for r in res])),
                            "compile_s_max": max(r.compile_s for r in res),
                            "best_unsat": [r.best_unsat for r in res], "restarts": R}
    return {"metric": "PAR-2 (s) of the fused annealing solver", "suite": args.suite,
            "value": P2.par2(results, limit), "unit": "s", "higher_is_better": False,
            "time_limit_s": limit, "solved": sum(r.solved for r in results), "instances": len(results),
            "restarts": args.suite_restarts or "64, or 16 past 125k constraints (per cell)", "cells": rows,
            "hyperparameters": SUITE_HP, "n_gpus": 1, "data": "synthetic",
            "note": "wall time per instance includes diagram compilation and upload; the paper's "
                    "limit is 1000 s on its own instances and hardware"}


def _fixed_work(fsmt, S, probs, R, keys, levels=1, steps=20, tuned=False):
    """One warm-up and one timed fused call of ``levels`` x ``steps`` PGD iterations (with
    ``tuned``, under the autotuner's plan, measured outside the clock)."""
    import torch
    import workloads as W
    hs = [fsmt.xbdd_compile(p) for p in probs]
    init = [W.initial_points(p, R, *keys, i) for i, p in enumerate(probs)]
    ell = [p.meta.get("mean_duration", p.meta.get("mean_side", 1.0)) for p in probs]
    cfg = S.SolveConfig(kappas=S.kappa_schedule(min(ell), levels), steps_per_level=steps, eta_a=ETA_A,
                        eta_b=ETA_B, eps=0.0, stop_on_sat=0)
    plan = None
    if tuned:
        from paper_2603_22877_amd import autotune as AT
        plan = AT.tune(hs, init, dataclasses.replace(cfg, steps_per_level=STEPS_PER_LEVEL))
        cfg = plan.apply(cfg)
    for _ in range(2):
        states = [S.BatchState(h, a, b) for h, (a, b) in zip(hs, init)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.solve_batched(hs, states, cfg)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    it = levels * steps
    evals = sum(p.n_cons for p in probs) * R * it
    for h in hs:
        h.free()
    out = {"instances": len(probs), "n_cons_total": int(sum(p.n_cons for p in probs)), "restarts": R,
           "pgd_steps": it, "ms_per_pgd_step": dt / it * 1e3, "constraint_evals_per_s": evals / dt,
           "includes": "one fused call: sweeps, projections, one check + ERWA"}
    if plan is not None:
        out["plan"] = {"label": plan.label, "cluster": plan.cluster,
                       "persistent_instances": sum(1 for v in plan.inst_schedule if v == 1),
                       "grid_instances": sum(1 for v in plan.inst_schedule if v == 2)}
    return out


# Placement time-to-SAT: the suite's sigma schedule sharpens too fast for dense packings (a
# deep overlap's smoothed gradient vanishes once kappa * depth >> 1), so these runs end at a
# gentler final kappa of 7 / (mean side) over 120 levels, run every level's 100 steps
# (eps = 0) and grow ERWA weights by 1.5
PLACE_HP = dict(SUITE_HP, levels=120, kmax=7.0, eps=0.0, gamma=1.5)


def placement_tts(fsmt, S, fill: float, seeds: int, cap: float) -> dict:
    """PAR-2 time to SAT on placement with 150 rectangles (compile and upload included),
    256 restarts per attempt, fresh initial points per attempt until SAT or the cap."""
    import workloads as W
    from workloads import placement as PL
    from paper_2603_22877_amd import par2 as P2
    res = []
    for seed in range(seeds):
        p = W.make_workload("placement_150", seed) if fill == 0.6 else PL.make_placement(150, W.seed_seq(3, seed), fill=fill)
        cfg = _suite_cfg(S, p, **{k: PLACE_HP[k] for k in ("levels", "kmax", "eps", "gamma")})
        r = P2.run_instance(p, cfg, 256, cap, lambda q, R, att, seed=seed: W.initial_points(q, R, 3, seed, 100 + att),
                            name=f"placement150 fill {fill} #{seed}")
        res.append(r)
        log(f"placement 150 fill {fill} seed {seed}: solved {r.solved} in {r.seconds:.2f} s, best {r.best_unsat}")
    sc = [r.score(cap) for r in res]
    return {"instances": seeds, "solved": sum(r.solved for r in res), "cap_s": cap, "fill": fill,
            "median_s": float(statistics.median(sc)), "par2_s": P2.par2(res, cap),
            "per_instance_s": [round(r.seconds, 3) if r.solved else None for r in res],
            "best_violations_unsolved": [int(r.best_unsat) for r in res if not r.solved],
            "attempts": [int(r.attempts) for r in res], "hyperparameters": PLACE_HP}


def other_configs(args, fsmt, S):
    """Rates of the fused solver on placement 150, and time-to-SAT there (the generator's 60 %
    area fill and, where the method solves, 50 %)."""
    import workloads as W
    out = {"placement 150 x 256 restarts": _fixed_work(fsmt, S, [W.make_workload("placement_150")], 256, (3, 0))}
    cap = min(args.tts_cap, 20.0)
    out["time_to_sat placement 150 (60% fill), 256 restarts"] = placement_tts(fsmt, S, 0.6, 10, cap)
    out["time_to_sat placement 150 at 50% fill, 256 restarts"] = placement_tts(fsmt, S, 0.5, 10, cap)
    return {"configs_mode": True, **out}


def paper_scale(args, fsmt, S):
    """Fixed-work fused-solver throughput on the largest encodings of the paper's suites."""
    import torch
    import workloads as W
    out = {}
    for suite, A, B in (("scheduling", 256, 5), ("placement", 64, 8)):
        p = _paper_make(suite, A, B, 0)
        t0 = time.perf_counter()
        h = fsmt.xbdd_compile(p)
        comp = time.perf_counter() - t0
        info = fsmt.xbdd_info(h)
        R = 16
        a0, b0 = W.initial_points(p, R, 57, A, B)
        cfg = _suite_cfg(S, p, eps=0.0, levels=1, steps_per_level=20)
        cfg.stop_on_sat = 0
        warm = S.BatchState(h, a0, b0)
        S.solve_batched([h], [warm], cfg)
        torch.cuda.synchronize()
        st = S.BatchState(h, a0, b0)
        t0 = time.perf_counter()
        S.solve_batched([h], [st], cfg)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        steps = int(st.steps_done.cpu().numpy().min())
        out[f"{suite} {A}x{B}"] = {"n_cons": p.n_cons, "n_bool": p.n_bool, "n_real": p.n_real,
                                   "max_nodes": info["max_nodes"], "n_big": info["n_big"], "restarts": R,
                                   "compile_s": comp, "pgd_steps": steps, "ms_per_pgd_step": dt / steps * 1e3,
                                   "constraint_evals_per_s": p.n_cons * R * steps / dt}
        h.free()
    return {"scale_mode": True, "per_instance": out}


def cpu_baseline(p, a0, b0, kap, threads: int = 1):
    """The FP64 oracle on a sample of the same workload (~10 s): one restart point per call,
    cycling over the restarts, on ``threads`` threads (the oracle's C calls release the
    interpreter lock and keep no shared state)."""
    import threading
    import oracle
    op = oracle.OracleProblem(p)
    R = a0.shape[0]
    counts = [0] * threads
    t0 = time.perf_counter()

    def work(i):
        while time.perf_counter() - t0 < 10.0:
            r = (counts[i] * threads + i) % R
            oracle.objective(op, a0[r:r + 1], b0[r:r + 1], kap, per_constraint=False)
            counts[i] += 1

    ts = [threading.Thread(target=work, args=(i,)) for i in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    dt = time.perf_counter() - t0
    done = sum(counts)
    return {"value": p.n_cons * done / dt, "unit": "constraint-evals/s", "cores": threads, "kind": "oracle",
            "sample": f"objective + gradient of all {p.n_cons} constraints at {done} restart points "
                      f"(cycling over the {R}), FP64, {threads} thread{'s' if threads > 1 else ''}, ~10 s"}


if __name__ == "__main__":
    main()
