"""TEST ORACLE -- test infrastructure only.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product library never links, loads
or calls it, and it imports nothing from the product package.

Contents
  p2m_oracle.c    FP64 brute force over every vertex, open edge and open face
                  (problem statement, Sec. 4.1; gated tests of Algorithm A.2),
                  plus an independent clamped point-triangle formulation.
  numpy_ref.py    a NumPy twin of the same definition for tiny meshes.
  morton.py       the definition of the query ordering (bit-interleaved
                  quantised coordinates, stable sort).
  grad.py         gradient of the distance from the oracle's closest
                  primitive (the paper is silent on derivatives).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libp2m_oracle.so")
SRC_PATH = os.path.join(_HERE, "p2m_oracle.c")

VERTEX, EDGE, FACE, NONE = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP over queries)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def load(path: str):
    """Load an oracle library build (the default one, or a test's own build)."""
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    L.p2mo_edges.restype = i64
    L.p2mo_edges.argtypes = [i64, P, i64, P]
    L.p2mo_query.restype = None
    L.p2mo_query.argtypes = [P, i64, P, i64, P, i64, P, i64, P, P, P, P, P]
    L.p2mo_near_set.restype = i64
    L.p2mo_near_set.argtypes = [P, i64, P, i64, P, i64, P, ctypes.c_double, ctypes.c_double, P, P, i64]
    L.p2mo_dist_clamped.restype = None
    L.p2mo_dist_clamped.argtypes = [P, i64, P, i64, P, i64, P]
    L.p2mo_point_to_primitive.restype = ctypes.c_double
    L.p2mo_point_to_primitive.argtypes = [P, P, P, ctypes.c_int32, i64, P]
    L.p2mo_num_threads.restype = ctypes.c_int
    L.p2mo_set_threads.argtypes = [ctypes.c_int]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        _lib = load(LIB_PATH)
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleMesh:
    """A mesh promoted exactly to FP64, with its canonical edge list."""

    def __init__(self, V, F, library=None, promote: bool = True, segments=None):
        """promote=True rounds V to float32 first (the product's input type)
        and widens exactly; promote=False takes float64 coordinates as given.
        segments: extra free segments (vertex pairs) of a mixed primitive set
        (Sec. 5.5); the edges are then the distinct pairs of the face sides
        and the segments, in lexicographic (min, max) order."""
        self._L = library if library is not None else lib()
        self._promote = promote
        self.V = np.ascontiguousarray(self._widen(V))
        self.F = np.ascontiguousarray(np.asarray(F, dtype=np.int32).reshape(-1, 3))
        self.nv = self.V.shape[0]
        self.nf = self.F.shape[0]
        L = self._L
        ne = L.p2mo_edges(self.nv, _p(self.F), self.nf, None) if self.nf else 0
        E = np.zeros((ne, 2), dtype=np.int32)
        if ne:
            L.p2mo_edges(self.nv, _p(self.F), self.nf, _p(E))
        if segments is not None:
            S = np.sort(np.asarray(segments, dtype=np.int32).reshape(-1, 2), axis=1)
            E = np.unique(np.concatenate([E, S]), axis=0).astype(np.int32)
        self.E = np.ascontiguousarray(E)
        self.ne = self.E.shape[0]
        lo, hi = self.V.min(0), self.V.max(0)
        self.diag = float(np.linalg.norm(hi - lo))

    def _widen(self, X):
        if self._promote:
            return np.asarray(X, dtype=np.float32).astype(np.float64)
        return np.asarray(X, dtype=np.float64)

    def query(self, Q):
        """Brute-force answer for each query: dict of type, id, closest, dist, runner_up."""
        Q = np.ascontiguousarray(self._widen(Q).reshape(-1, 3))
        n = Q.shape[0]
        t = np.zeros(n, np.int32)
        i = np.zeros(n, np.int64)
        c = np.zeros((n, 3), np.float64)
        d = np.zeros(n, np.float64)
        r = np.zeros(n, np.float64)
        self._L.p2mo_query(_p(self.V), self.nv, _p(self.F), self.nf, _p(self.E), self.ne,
                         _p(Q), n, _p(t), _p(i), _p(c), _p(d), _p(r))
        return {"type": t, "id": i, "closest": c, "dist": d, "runner_up": r}

    def near_set(self, q, dstar: float, tol: float, cap: int = 4096):
        """(type, id) pairs whose tolerance-relaxed distance is <= dstar + tol."""
        q = np.ascontiguousarray(self._widen(q).reshape(3))
        ts = np.zeros(cap, np.int32)
        ids = np.zeros(cap, np.int64)
        n = self._L.p2mo_near_set(_p(self.V), self.nv, _p(self.F), self.nf, _p(self.E), self.ne,
                                _p(q), float(dstar), float(tol), _p(ts), _p(ids), cap)
        n = min(n, cap)
        return set(zip(ts[:n].tolist(), ids[:n].tolist()))

    def dist_clamped(self, Q):
        """Independent formulation: min over closed triangles of the clamped distance."""
        Q = np.ascontiguousarray(self._widen(Q).reshape(-1, 3))
        d = np.zeros(Q.shape[0], np.float64)
        self._L.p2mo_dist_clamped(_p(self.V), self.nv, _p(self.F), self.nf, _p(Q), Q.shape[0], _p(d))
        return d

    def point_to_primitive(self, ptype: int, pid: int, x) -> float:
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3))
        return float(self._L.p2mo_point_to_primitive(_p(self.V), _p(self.F), _p(self.E),
                                                   int(ptype), int(pid), _p(x)))


def num_threads() -> int:
    return int(lib().p2mo_num_threads())


def set_threads(n: int) -> None:
    lib().p2mo_set_threads(int(n))
