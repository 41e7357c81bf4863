"""Seeded synthetic shallow-water 4D-Var problems (inputs only).

This module draws every random quantity of a twin experiment on the sphere
(Sec. 7 of the paper: a truth snapshot, a perturbed background, and
observations sampled from the truth trajectory plus noise) and fixes the
space-time partition edges.  It holds none of the assimilation arithmetic:
the truth trajectory is produced by a caller-supplied model run, so the same
inputs serve both the CPU reference and the GPU library.
"""
from .problems import (CONFIGS, Problem, make_problem, make_spec, finish_spec,
                       composition, DEFAULT_CONSTANTS)

__all__ = ["CONFIGS", "Problem", "make_problem", "make_spec", "finish_spec",
           "composition", "DEFAULT_CONSTANTS"]
