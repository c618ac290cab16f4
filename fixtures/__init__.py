"""Seeded synthetic inputs shared by the oracle and the GPU library (no method arithmetic)."""
from .meshgen import (Mesh, Workload, BatchProblem, box, ogrid, random_unique,  # noqa: F401
                      sine_field, unit_cube, periodic_box_deformed,
                      cylinder_ogrid, batch_problems, batch_mesh, ROTATIONS)
