"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

Holds meshes, bases, EQ sets and evaluation points only; none of the
method's arithmetic lives here.
"""
from .mesh import Mesh, structured_mesh  # noqa: F401
from .inputs import (Workload, BatchWorkload, tiny_burgers, spacetime_burgers, euler_p2, euler_batch, with_eq,  # noqa: F401
                     orthonormal_columns, inflow_elements, eq_set_with_inflow)
