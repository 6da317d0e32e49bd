"""Seeded synthetic workloads: the only module shared by the library's tests and the oracle.

It builds problem instances and initial points; it computes nothing of the method itself.
"""
from .format import *  # noqa: F401,F403
from .format import Builder, Problem, load_npz, save_npz, lit  # noqa: F401
from .standard import (RESTARTS, STREAM, initial_points, make_random_formula,  # noqa: F401
                       make_random_hybrid, make_random_separable, make_workload, seed_seq, uneven_batch,
                       uneven_batch_sizes)
from .placement import make_placement  # noqa: F401
from .scheduling import make_scheduling  # noqa: F401
from .toy import make_fig2_toy  # noqa: F401
