"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

Nothing in this package computes any part of the phase-field method.
"""
from .configs import (CONFIGS, GLASS, H_GRID, L0, V_PULL, Problem, config0, config1, config2,
                      config3, config4, config4_draws, plate_problem, small_plate)
from .meshes import grid_nodes, grid_triangles, plate_mesh, rng

__all__ = ["CONFIGS", "GLASS", "H_GRID", "L0", "V_PULL", "Problem", "config0", "config1", "config2",
           "config3", "config4", "config4_draws", "plate_problem", "small_plate", "grid_nodes",
           "grid_triangles", "plate_mesh", "rng"]
