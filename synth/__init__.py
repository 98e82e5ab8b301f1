"""Seeded synthetic least-squares problems (inputs only; none of the solver's arithmetic)."""
from .problems import (Problem, ProblemSpec, make_problem_cpu, make_problem_gpu, integer_problem,
                       sub_seeds, CONFIGS)

__all__ = ["Problem", "ProblemSpec", "make_problem_cpu", "make_problem_gpu", "integer_problem",
           "sub_seeds", "CONFIGS"]
