"""Seeded synthetic inputs (geometry, boundary data, random vectors).

Shared by the CPU oracle and the GPU path; holds none of the solver's
arithmetic.
"""
from .geometry import (CONFIGS, Geometry, batch_member, build_geometry,
                       make_geometry, place_pores, rounded_rectangle)
from .rhs import (poiseuille_rhs, random_vector, shear_rhs,
                  stokeslet_rotlet_data, stokeslet_rotlet_field,
                  stokeslet_rotlet_rhs)
