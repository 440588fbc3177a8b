"""Seeded synthetic inputs for the LT-AC G0W0 hot path.

This package only draws random numbers and lays them out as the inputs of
the method (orbital energies and RI three-index tensors).  It contains none
of the method's arithmetic, so both the CPU oracle and the GPU path may
import it.
"""
from .configs import CONFIGS, Config, batched_configs, get_config
from .problem import Problem, make_problem

__all__ = ["CONFIGS", "Config", "Problem", "batched_configs", "get_config",
           "make_problem"]
