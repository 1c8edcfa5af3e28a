"""MI355X-native P2M point-to-mesh distance queries.

Host precompute (KD tree, Voronoi cells, convexity-filtered flooding
interception table) and hand-written gfx950 HIP query / backward / batched
kernels behind the C interface in include/p2m.h; this package is its thin
Python binding.
"""
from .api import (EDGE, FACE, NONE, NONFINITE, OUT_OF_DOMAIN, TABLE_ALL_PAIRS, TABLE_EVERYTHING, TABLE_FLOODING_DEVICE,
                  TABLE_FLOODING, VERTEX, Batch, Mesh, P2MError, p2m_distance, precompute_many, prim_id,
                  prim_type)

__all__ = ["Mesh", "Batch", "precompute_many", "p2m_distance", "P2MError", "prim_type", "prim_id", "VERTEX", "EDGE", "FACE", "NONE",
           "OUT_OF_DOMAIN", "NONFINITE", "TABLE_FLOODING", "TABLE_ALL_PAIRS", "TABLE_EVERYTHING",
           "TABLE_FLOODING_DEVICE"]
