"""ctypes loader for libp2m.so (the C interface in include/p2m.h).

The library must have been built (``__graft_entry__.build()`` or
``python paper_2308_16084_amd/build.py``); a missing library is an error,
never a silent fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libp2m.so")

P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32
INT = ctypes.c_int


class BuildOpts(ctypes.Structure):
    _fields_ = [("domain_lo", ctypes.c_double * 3), ("domain_hi", ctypes.c_double * 3),
                ("use_default_domain", INT), ("num_threads", INT), ("margin_rel", ctypes.c_double),
                ("table_mode", INT), ("device_visit_cap", INT)]


class BuildStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("t_validate", "t_kdt", "t_delaunay", "t_cells", "t_flood",
                                               "t_pack")] + \
               [(n, I64) for n in ("nv", "ne", "nf", "delaunay_edges", "tets", "exact_predicates",
                                   "flood_tests", "flood_hits", "quick_rejects", "skipped_clips",
                                   "nnz_edges", "nnz_faces", "max_list")] + \
               [("avg_list", ctypes.c_double)] + \
               [(n, ctypes.c_double) for n in ("t_dev_upload", "t_dev_kernel", "t_dev_download")] + \
               [("device_redo", I64), ("device_cells_back", I64)] + \
               [(n, ctypes.c_double) for n in ("avg_edges", "avg_faces", "avg_list_volw", "avg_edges_volw",
                                               "avg_faces_volw")] + \
               [("max_edges", I64), ("max_faces", I64), ("flood_visits", I64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class QueryOpts(ctypes.Structure):
    _fields_ = [("sort_queries", INT), ("block_size", INT), ("profile", INT), ("traversal", INT),
                ("lds_levels", INT), ("reserved", INT * 3)]


_SIGS = {
    "p2m_mesh_create": (INT, [P, I64, P, I64, P]),
    "p2m_mesh_destroy": (None, [P]),
    "p2m_mesh_counts": (INT, [P, P, P, P]),
    "p2m_mesh_edges": (INT, [P, P, P]),
    "p2m_precompute": (INT, [P, P, P]),
    "p2m_mesh_table": (INT, [P, P, P, P]),
    "p2m_mesh_table_boxes": (INT, [P, P]),
    "p2m_mesh_create_mixed": (INT, [P, I64, P, I64, P, I64, P]),
    "p2m_mesh_neighbors": (INT, [P, P, P, P]),
    "p2m_mesh_kdtree": (INT, [P, P, P]),
    "p2m_save": (INT, [P, ctypes.c_char_p]),
    "p2m_load": (INT, [ctypes.c_char_p, P]),
    "p2m_query_host": (INT, [P, P, I64, P, P, P, P, INT, P]),
    "p2m_last_error": (ctypes.c_char_p, []),
    "p2m_upload": (INT, [P, INT, P, P]),
    "p2m_query": (INT, [P, P, I64, P, P, P, P, P, P, P, P]),
    "p2m_query_noalloc": (INT, [P, P, I64, P, P, P, P, P, P, P, P]),
    "p2m_query_profile": (INT, [P, P, P, P]),
    "p2m_nearest_vertex": (INT, [P, P, I64, P, P, INT, P]),
    "p2m_order_queries": (INT, [P, P, I64, P, P, P]),
    "p2m_query_backward": (INT, [P, P, I64, P, P, P, P, P, P, P, P]),
    "p2m_batch_create": (INT, [P, I32, INT, P, P]),
    "p2m_batch_destroy": (None, [P]),
    "p2m_batch_query": (INT, [P, P, P, P, P, P, P, P]),
    "p2m_batch_query_eager": (INT, [P, P, P, P, P, P, P, P]),
    "p2m_batch_order_queries": (INT, [P, P, P, P, P, P]),
    "p2m_batch_set_shape": (INT, [P, INT, INT, INT]),
    "p2m_batch_get_shape": (INT, [P, P, P, P]),
    "p2m_batch_set_lds_levels": (INT, [P, INT]),
    "p2m_batch_get_lds_levels": (INT, [P, P]),
    "p2m_batch_set_schedule": (INT, [P, INT]),
    "p2m_batch_get_schedule": (INT, [P, P]),
    "p2m_batch_autotune": (INT, [P, P, P, P, P, P, P, P, P, P]),
}

STATUS = {0: "P2M_OK", -1: "P2M_ERR_ARG", -2: "P2M_ERR_MESH", -3: "P2M_ERR_STATE", -4: "P2M_ERR_OOM",
          -5: "P2M_ERR_HIP", -6: "P2M_ERR_INTERNAL", -7: "P2M_ERR_IO"}


class P2MError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != 0:
        msg = lib().p2m_last_error()
        raise P2MError(status, msg.decode() if msg else "")


def exported_symbols() -> list[str]:
    return list(_SIGS)
