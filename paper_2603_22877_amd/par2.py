"""PAR-2 harness: wall time to SAT of the fused annealing solver over a suite of instances.

The paper ranks solvers by PAR-2 (Results, the scheduling and placement comparisons): an
instance scores its wall time when it is solved within the time limit and twice the limit
otherwise, and a suite scores the mean. Here an instance's clock starts before its diagrams
are compiled and stops when a fused solver call returns with a restart whose exact check
passed (Thm. "Soundness": the rounded point satisfies every constraint). The solver runs in
chunks of annealing levels (a call resumes at each restart's ``level_done``), so the limit
is checked between chunks; a schedule that ends without SAT starts over from new initial
points while time is left.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional, Sequence

import numpy as np

from . import xbdd_compile
from .solver import BatchState, SolveConfig, check_batched, solve_batched


@dataclasses.dataclass
class InstanceResult:
    name: str
    solved: bool
    seconds: float              # wall time to SAT, or the time spent when unsolved
    compile_s: float
    attempts: int               # schedules started (fresh initial points each)
    levels: int                 # levels run by the winning restart (or the last attempt)
    best_unsat: int             # fewest violated constraints seen at a level boundary
    n_cons: int
    a: Optional[np.ndarray] = None   # SAT restart's point (float32), when solved
    b: Optional[np.ndarray] = None

    def score(self, time_limit: float) -> float:
        return self.seconds if self.solved and self.seconds <= time_limit else 2.0 * time_limit


def run_instance(problem, cfg: SolveConfig, restarts: int, time_limit: float,
                 init_points: Callable[[object, int, int], tuple], name: str = "",
                 chunk_levels: int = 5, projection: int = 0, stream=None) -> InstanceResult:
    """Solve one instance under the PAR-2 protocol.

    ``init_points(problem, restarts, attempt)`` returns float32 arrays a0 [R][n_bool] and
    b0 [R][n_real] for attempt number ``attempt``. ``cfg.stop_on_sat`` should be 2 so that
    the other restarts stop at the next level boundary once one is SAT.
    """
    import torch
    t0 = time.perf_counter()
    h = xbdd_compile(problem, projection=projection)
    compile_s = time.perf_counter() - t0
    kap = list(cfg.kappas)
    best, attempts, levels = np.iinfo(np.int32).max, 0, 0
    while True:
        a0, b0 = init_points(problem, restarts, attempts)
        st = BatchState(h, a0, b0)
        attempts += 1
        for end in range(chunk_levels, len(kap) + chunk_levels, chunk_levels):
            # every restart has finished the previous chunk's levels (or stopped)
            sub = dataclasses.replace(cfg, kappas=kap[:min(end, len(kap))], level_begin=end - chunk_levels)
            solve_batched([h], [st], sub, stream=stream)
            check_batched([st], stream=stream)      # waits; raises if the call gave up early
            ver = st.verdict.cpu().numpy()
            nu = st.n_unsat.cpu().numpy()
            if np.any(nu >= 0):
                best = min(best, int(nu[nu >= 0].min()))
            elapsed = time.perf_counter() - t0
            if ver.max() == 1:
                r = int(np.nonzero(ver == 1)[0][0])
                levels = int(st.level_done[r].item())
                res = InstanceResult(name, True, elapsed, compile_s, attempts, levels, 0,
                                     problem.n_cons, st.a[r].cpu().numpy(), st.b[r].cpu().numpy())
                h.free()
                return res
            if elapsed >= time_limit:
                levels = int(st.level_done.max().item())
                h.free()
                return InstanceResult(name, False, elapsed, compile_s, attempts, levels, best,
                                      problem.n_cons)
        torch.cuda.synchronize()


def par2(results: Sequence[InstanceResult], time_limit: float) -> float:
    """Mean PAR-2 score of a suite."""
    return float(np.mean([r.score(time_limit) for r in results])) if results else 0.0


def run_suite(problems: Sequence[tuple], cfg_for: Callable[[object], SolveConfig], restarts: int,
              time_limit: float, init_points, log=None, **kw) -> List[InstanceResult]:
    """``problems``: (name, factory) pairs; the factory builds the instance (not timed)."""
    out = []
    for name, make in problems:
        p = make()
        r = run_instance(p, cfg_for(p), restarts, time_limit, init_points, name=name, **kw)
        out.append(r)
        if log:
            log(r)
    return out


__all__ = ["InstanceResult", "run_instance", "run_suite", "par2"]
