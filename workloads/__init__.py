"""Seeded synthetic problem generators shared by the oracle, the tests and the benchmark.

This package only describes problems: node coordinates, Q1 or Q2 hexahedra, the
subdomain of each element, materials, fibre directions, Dirichlet data, body
forces and pressure faces.  It contains none of the solver's arithmetic
(no element integrals, no tearing, no factorisation), so that the CPU oracle
and the GPU path can both consume its output without sharing any method code.
"""
from .meshes import (Mesh, cube_mesh, random_box_cube, tube_mesh, box_partition, partial_dirichlet_cube,
                     kelvin_displacement, config_mesh, CONFIGS, request_mesh, request_stream)

__all__ = ["Mesh", "cube_mesh", "random_box_cube", "tube_mesh", "box_partition", "partial_dirichlet_cube",
           "kelvin_displacement", "config_mesh", "CONFIGS", "request_mesh", "request_stream"]
