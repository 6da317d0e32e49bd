"""Seeded synthetic workloads: the only module shared by the library's tests and the oracle.

It builds problem instances and initial points; it computes nothing of the method itself.
"""
from .format import *  # noqa: F401,F403
from .format import Builder, Problem, load_npz, save_npz, lit  # noqa: F401
from .configs import (RESTARTS, config4_sizes, initial_points, make_batch_config4,  # noqa: F401
                      make_config, make_random_formula, make_random_hybrid, seed_seq)
from .placement import make_placement  # noqa: F401
from .scheduling import make_scheduling  # noqa: F401
from .toy import make_fig2_toy  # noqa: F401
