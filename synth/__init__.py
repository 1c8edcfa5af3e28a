"""Seeded synthetic inputs (meshes, query sets, workloads).

This module generates inputs only.  It holds none of the point-to-mesh
arithmetic, so both the product path and the test oracle may draw from it.
"""
from . import configs, mesh, noise, queries  # noqa: F401
