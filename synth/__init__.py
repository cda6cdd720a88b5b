"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package draws island geometries, densities, right-hand sides and sphere
target points.  It holds none of the solver's arithmetic: no kernel, no
projection derivatives, no quadrature, no expansion.  The only formula in it
besides sampling is the closed-form boundary data of the paper's examples
(Section 6, eq. exact_bcs), which both sides receive as an input.
"""
from .islands import (IslandSet, cap_island, star_islands, config_islands,
                      batch_geometries, deep_tree_islands, CONFIGS)
from .data import (exact_harmonic, paper_data_coeffs, random_data_coeffs,
                   sphere_targets, random_vector, near_curve_targets,
                   point_vortices)

__all__ = ["IslandSet", "cap_island", "star_islands", "config_islands",
           "batch_geometries", "deep_tree_islands", "CONFIGS", "exact_harmonic",
           "paper_data_coeffs", "random_data_coeffs", "sphere_targets",
           "random_vector", "near_curve_targets", "point_vortices"]
