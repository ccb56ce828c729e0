"""Seeded synthetic inputs shared by the tests, the bench and the oracle.

This package only *generates* inputs: triangulated squares with element
labels, published quadrature tables and the workload recipes.  It holds none
of the assembly arithmetic, so the GPU library and the CPU oracle can both be
fed from it without sharing any of the method's code.
"""
from .meshes import Mesh, square_mesh, batched_meshes, boundary_triangles_to_layer  # noqa: F401
from .rules import Rule, gauss7, paper7, centroid1, collapsed  # noqa: F401
from .workloads import WORKLOADS, workload  # noqa: F401
