"""The two-constraint example of the paper's Fig. 2 ("Optimization trajectories ...").

Constraints (not x) XOR (y > 0) and x AND (y > 0), one Boolean x and one real y in [-1, 1].
The global minimum is at x = True with y > 0; a local minimum sits at x = False, y <= 0.
"""
from __future__ import annotations

from .format import KIND_AND, KIND_XOR, OP_GT, Builder, Problem, lit


def make_fig2_toy() -> Problem:
    b = Builder(n_bool=1, n_real=1, real_lo=[-1.0], real_hi=[1.0])
    a = b.atom([0], [1.0], OP_GT, 0.0)          # y > 0
    b.add(KIND_XOR, [lit(0, neg=True), lit(a)])
    b.add(KIND_AND, [lit(0), lit(a)])
    p = b.build(meta=dict(family="fig2_toy"))
    p.cert_x = __import__("numpy").array([-1.0])
    p.cert_y = __import__("numpy").array([0.5])
    return p
