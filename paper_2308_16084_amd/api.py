"""Python binding of the P2M C interface (argument marshalling only).

Every step of a query runs in libp2m.so; torch tensors provide device memory
and the stream.  Names follow the C calls in include/p2m.h.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import BuildOpts, BuildStats, P2MError, QueryOpts, check, lib

VERTEX, EDGE, FACE, NONE = 0, 1, 2, 3
OUT_OF_DOMAIN, NONFINITE = 1, 2
TABLE_FLOODING, TABLE_ALL_PAIRS, TABLE_EVERYTHING, TABLE_FLOODING_DEVICE = 0, 1, 2, 3


def prim_type(prim):
    return (np.asarray(prim).astype(np.int64) & 0xFFFFFFFF) >> 30


def prim_id(prim):
    return np.asarray(prim).astype(np.int64) & 0x3FFFFFFF


def _ptr(a) -> ctypes.c_void_p:
    if a is None:
        return ctypes.c_void_p(0)
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(a.data_ptr())


def _torch():
    import torch
    return torch


def _stream(stream=None) -> ctypes.c_void_p:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_tensor(x, dtype, shape_tail, name):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if tuple(x.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [n, {', '.join(map(str, shape_tail))}]")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return x


class Mesh:
    """A triangle mesh (optionally with free segments: a mixed primitive set)
    with its precomputed KD tree, Voronoi graph and interception table."""

    def __init__(self, V=None, F=None, segments=None, _handle=None):
        self._h = ctypes.c_void_p(0)
        self.device = None
        if _handle is not None:
            self._h = _handle
            return
        V = np.ascontiguousarray(np.asarray(V, dtype=np.float32).reshape(-1, 3))
        F = np.ascontiguousarray(np.asarray(F if F is not None else np.zeros((0, 3)), dtype=np.int32).reshape(-1, 3))
        if segments is None:
            check(lib().p2m_mesh_create(_ptr(V), V.shape[0], _ptr(F), F.shape[0], ctypes.byref(self._h)))
        else:
            S = np.ascontiguousarray(np.asarray(segments, dtype=np.int32).reshape(-1, 2))
            check(lib().p2m_mesh_create_mixed(_ptr(V), V.shape[0], _ptr(F) if len(F) else None, F.shape[0],
                                              _ptr(S) if len(S) else None, S.shape[0], ctypes.byref(self._h)))
        self.nv, self.nf = V.shape[0], F.shape[0]

    @classmethod
    def load(cls, path: str) -> "Mesh":
        h = ctypes.c_void_p(0)
        check(lib().p2m_load(path.encode(), ctypes.byref(h)))
        m = cls(_handle=h)
        nv, nf = ctypes.c_int64(), ctypes.c_int64()
        check(lib().p2m_mesh_counts(m._h, ctypes.byref(nv), None, ctypes.byref(nf)))
        m.nv, m.nf = nv.value, nf.value
        return m

    @classmethod
    def cached(cls, V, F, domain, cache_dir: str | None, segments=None, **precompute_kw) -> tuple["Mesh", dict]:
        """Precompute, or load the structures saved by an earlier call with
        the same mesh, domain and options from cache_dir (None: no cache)."""
        import hashlib
        import os
        V = np.ascontiguousarray(np.asarray(V, dtype=np.float32).reshape(-1, 3))
        F = np.ascontiguousarray(np.asarray(F, dtype=np.int32).reshape(-1, 3))
        h = hashlib.sha256()
        h.update(V.tobytes())
        h.update(F.tobytes())
        if segments is not None:
            h.update(b"segments")
            h.update(np.ascontiguousarray(np.asarray(segments, dtype=np.int32)).tobytes())
        h.update(np.asarray(domain, dtype=np.float64).tobytes())
        h.update(repr(sorted(precompute_kw.items())).encode())
        path = os.path.join(cache_dir, f"mesh_{h.hexdigest()[:24]}.p2m") if cache_dir else None
        if path and os.path.exists(path):
            try:
                return cls.load(path), {"loaded_from": path}
            except P2MError:
                pass
        m = cls(V, F, segments=segments)
        st = m.precompute(domain=domain, **precompute_kw)
        if path:
            os.makedirs(cache_dir, exist_ok=True)
            tmp = path + f".tmp{os.getpid()}"
            m.save(tmp)
            os.replace(tmp, path)
        return m, st

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().p2m_mesh_destroy(h)
            except Exception:
                pass
            self._h = ctypes.c_void_p(0)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    # ------------------------------------------------------------- host
    def edges(self) -> np.ndarray:
        ne = ctypes.c_int64()
        check(lib().p2m_mesh_edges(self._h, ctypes.byref(ne), None))
        E = np.zeros((ne.value, 2), np.int32)
        check(lib().p2m_mesh_edges(self._h, ctypes.byref(ne), _ptr(E)))
        return E

    def precompute(self, domain=None, threads: int = 0, margin_rel: float = 0.0,
                   table_mode: int = TABLE_FLOODING, device_visit_cap: int = 0) -> dict:
        o = BuildOpts()
        if domain is None:
            o.use_default_domain = 1
        else:
            lo, hi = domain
            for k in range(3):
                o.domain_lo[k] = float(lo[k])
                o.domain_hi[k] = float(hi[k])
        o.num_threads = int(threads)
        o.margin_rel = float(margin_rel)
        o.table_mode = int(table_mode)
        o.device_visit_cap = int(device_visit_cap)
        st = BuildStats()
        check(lib().p2m_precompute(self._h, ctypes.byref(o), ctypes.byref(st)))
        return st.as_dict()

    def table(self) -> tuple[np.ndarray, np.ndarray]:
        nnz = ctypes.c_int64()
        check(lib().p2m_mesh_table(self._h, ctypes.byref(nnz), None, None))
        off = np.zeros(2 * self.nv + 1, np.uint32)
        ent = np.zeros(max(1, nnz.value), np.int32)
        check(lib().p2m_mesh_table(self._h, ctypes.byref(nnz), _ptr(off), _ptr(ent)))
        return off, ent[:nnz.value]

    def table_boxes(self) -> np.ndarray:
        """Entry boxes uint16 [nnz, 6] (lower xyz, upper xyz in D's 16-bit frame)."""
        off, _ = self.table()
        boxes = np.zeros((max(1, int(off[-1])), 6), np.uint16)
        check(lib().p2m_mesh_table_boxes(self._h, _ptr(boxes)))
        return boxes[:int(off[-1])]

    def neighbors(self) -> tuple[np.ndarray, np.ndarray]:
        nnz = ctypes.c_int64()
        check(lib().p2m_mesh_neighbors(self._h, ctypes.byref(nnz), None, None))
        off = np.zeros(self.nv + 1, np.int64)
        nb = np.zeros(max(1, nnz.value), np.int32)
        check(lib().p2m_mesh_neighbors(self._h, ctypes.byref(nnz), _ptr(off), _ptr(nb)))
        return off, nb[:nnz.value]

    def kdtree(self) -> tuple[np.ndarray, np.ndarray]:
        n = self.nv
        xyz = np.zeros((n, 3), np.float32)
        vid = np.zeros(n, np.int32)
        check(lib().p2m_mesh_kdtree(self._h, _ptr(xyz), _ptr(vid)))
        return xyz, vid

    def save(self, path: str) -> None:
        check(lib().p2m_save(self._h, path.encode()))

    def query_host(self, q, threads: int = 0) -> dict:
        """Multi-threaded CPU P2M query (same tree, table and float32 code as the kernel)."""
        q = np.ascontiguousarray(np.asarray(q, dtype=np.float32).reshape(-1, 3))
        n = q.shape[0]
        prim = np.zeros(n, np.int32)
        closest = np.zeros((n, 3), np.float32)
        dist = np.zeros(n, np.float32)
        status = np.zeros(n, np.uint8)
        cnt = np.zeros(8, np.int64)
        check(lib().p2m_query_host(self._h, _ptr(q), n, _ptr(prim), _ptr(closest), _ptr(dist), _ptr(status),
                                   int(threads), _ptr(cnt)))
        return {"prim": prim, "closest": closest, "dist": dist, "status": status,
                "nodes": int(cnt[0]), "edges": int(cnt[1]), "faces": int(cnt[2]), "steps": int(cnt[3]),
                "edge_forms": int(cnt[4]), "face_forms": int(cnt[5]), "rescans": int(cnt[6]),
                "rescan_exact": int(cnt[7])}

    # ----------------------------------------------------------- device
    def upload(self, device: int = 0, stream=None) -> int:
        nbytes = ctypes.c_int64()
        check(lib().p2m_upload(self._h, int(device), _stream(stream), ctypes.byref(nbytes)))
        self.device = int(device)
        return nbytes.value

    def query(self, q, sort: bool | None = None, block_size: int = 0, out: dict | None = None, status: bool = True,
              for_backward: bool = False, profile: bool = False, traversal: int = 0, stream=None,
              noalloc: bool = False, lds_levels: int = 0) -> dict:
        """P2M query of a CUDA float32 [n,3] tensor; returns device tensors.
        sort: Morton-order the batch first (None: the library's default, on
        from 2^19 queries).  noalloc: call p2m_query_noalloc (the library
        allocates nothing; pass `out` to allocate nothing here either)."""
        torch = _torch()
        q = _dev_tensor(q, torch.float32, (3,), "q")
        n = q.shape[0]
        dev = q.device
        if out is None:
            out = {"prim": torch.empty(n, dtype=torch.int32, device=dev),
                   "closest": torch.empty((n, 3), dtype=torch.float32, device=dev),
                   "dist": torch.empty(n, dtype=torch.float32, device=dev)}
            if status:
                out["status"] = torch.empty(n, dtype=torch.uint8, device=dev)
            if for_backward:
                out["bary"] = torch.empty((n, 3), dtype=torch.float32, device=dev)
                out["pvid"] = torch.empty((n, 3), dtype=torch.int32, device=dev)
        o = QueryOpts()
        o.sort_queries = -1 if sort is None else (1 if sort else 0)
        o.block_size = int(block_size)
        o.profile = 1 if profile else 0
        o.traversal = int(traversal)
        o.lds_levels = int(lds_levels)
        fn = lib().p2m_query_noalloc if noalloc else lib().p2m_query
        check(fn(self._h, _ptr(q), n, _ptr(out["prim"]), _ptr(out["closest"]), _ptr(out["dist"]),
                 _ptr(out.get("status")), _ptr(out.get("bary")), _ptr(out.get("pvid")), ctypes.byref(o),
                 _stream(stream)))
        return out

    def query_profile(self) -> tuple[float, float, float]:
        """(ordering, query kernel, answer write-out) ms of the last profiled query."""
        a, b, c = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
        check(lib().p2m_query_profile(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def nearest_vertex(self, q, traversal: int = 0, stream=None):
        torch = _torch()
        q = _dev_tensor(q, torch.float32, (3,), "q")
        n = q.shape[0]
        vid = torch.empty(n, dtype=torch.int32, device=q.device)
        d2 = torch.empty(n, dtype=torch.float32, device=q.device)
        check(lib().p2m_nearest_vertex(self._h, _ptr(q), n, _ptr(vid), _ptr(d2), int(traversal), _stream(stream)))
        return vid, d2

    def order_queries(self, q, stream=None):
        torch = _torch()
        q = _dev_tensor(q, torch.float32, (3,), "q")
        n = q.shape[0]
        keys = torch.empty(n, dtype=torch.int32, device=q.device)
        perm = torch.empty(n, dtype=torch.int32, device=q.device)
        check(lib().p2m_order_queries(self._h, _ptr(q), n, _ptr(keys), _ptr(perm), _stream(stream)))
        return keys, perm

    def query_backward(self, q, fwd: dict, grad_dist, grad_q=True, grad_V=None, stream=None):
        """grad_q [n,3] (new tensor or None) and grad_V accumulated into the given [nv,3] tensor."""
        torch = _torch()
        q = _dev_tensor(q, torch.float32, (3,), "q")
        n = q.shape[0]
        for k, tail, dt in (("closest", (3,), torch.float32), ("bary", (3,), torch.float32),
                            ("pvid", (3,), torch.int32)):
            if fwd.get(k) is not None:
                _dev_tensor(fwd[k], dt, tail, k)
                if fwd[k].shape[0] != n:
                    raise ValueError(f"{k} must have {n} rows")
        if fwd["dist"].shape != (n,) or fwd["dist"].dtype != torch.float32 or not fwd["dist"].is_contiguous():
            raise ValueError(f"dist must be a contiguous float32 tensor of shape [{n}]")
        if grad_V is not None:
            _dev_tensor(grad_V, torch.float32, (3,), "grad_V")
            if grad_V.shape[0] != self.nv:
                raise ValueError(f"grad_V must have shape [{self.nv}, 3] (one row per mesh vertex)")
            if grad_V.data_ptr() % 16:
                raise ValueError("grad_V must be 16-byte aligned")
        gq = torch.empty((n, 3), dtype=torch.float32, device=q.device) if grad_q else None
        grad_dist = grad_dist.contiguous().to(torch.float32)
        if grad_dist.shape != (n,) or grad_dist.device != q.device:
            raise ValueError(f"grad_dist must have shape [{n}] on the queries' device")
        check(lib().p2m_query_backward(self._h, _ptr(q), n, _ptr(fwd["closest"]), _ptr(fwd["dist"]),
                                       _ptr(fwd.get("bary")), _ptr(fwd.get("pvid")), _ptr(grad_dist),
                                       _ptr(gq), _ptr(grad_V), _stream(stream)))
        return gq, grad_V


class Batch:
    """Many precomputed meshes in one device arena, queried in one launch."""

    def __init__(self, meshes, device: int = 0, stream=None):
        self._h = ctypes.c_void_p(0)
        self.meshes = list(meshes)
        arr = (ctypes.c_void_p * len(self.meshes))(*[m.handle.value for m in self.meshes])
        check(lib().p2m_batch_create(arr, len(self.meshes), int(device), _stream(stream), ctypes.byref(self._h)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().p2m_batch_destroy(h)
            except Exception:
                pass
            self._h = ctypes.c_void_p(0)

    @staticmethod
    def _offsets(q_offsets):
        off = np.ascontiguousarray(np.asarray(q_offsets, dtype=np.int64))
        return off

    def _outs(self, q, out, status=True):
        torch = _torch()
        n = q.shape[0]
        if out is None:
            out = {"prim": torch.empty(n, dtype=torch.int32, device=q.device),
                   "closest": torch.empty((n, 3), dtype=torch.float32, device=q.device),
                   "dist": torch.empty(n, dtype=torch.float32, device=q.device)}
            if status:
                out["status"] = torch.empty(n, dtype=torch.uint8, device=q.device)
        return out

    def query(self, q, q_offsets, out: dict | None = None, graph: bool = True, stream=None,
              status: bool = True) -> dict:
        torch = _torch()
        q = _dev_tensor(q, torch.float32, (3,), "q")
        off = self._offsets(q_offsets)
        if off.shape[0] != len(self.meshes) + 1 or off[-1] != q.shape[0]:
            raise ValueError("q_offsets must have len(meshes)+1 entries ending at len(q)")
        out = self._outs(q, out, status)
        fn = lib().p2m_batch_query if graph else lib().p2m_batch_query_eager
        check(fn(self._h, _ptr(q), _ptr(off), _ptr(out["prim"]), _ptr(out["closest"]), _ptr(out["dist"]),
                 _ptr(out.get("status")), _stream(stream)))
        return out

    def order_queries(self, q, q_offsets, stream=None):
        """The batched query's ordering: (sorted keys uint32 viewed as int32,
        perm int32) of the stable per-mesh sort by 24-bit Morton key."""
        torch = _torch()
        q = _dev_tensor(q, torch.float32, (3,), "q")
        off = self._offsets(q_offsets)
        if off.shape[0] != len(self.meshes) + 1 or off[-1] != q.shape[0]:
            raise ValueError("q_offsets must have len(meshes)+1 entries ending at len(q)")
        n = q.shape[0]
        keys = torch.empty(n, dtype=torch.int32, device=q.device)
        perm = torch.empty(n, dtype=torch.int32, device=q.device)
        check(lib().p2m_batch_order_queries(self._h, _ptr(q), _ptr(off), _ptr(keys), _ptr(perm), _stream(stream)))
        return keys, perm

    def set_shape(self, block: int, queries_per_lane: int, traversal: int) -> None:
        check(lib().p2m_batch_set_shape(self._h, int(block), int(queries_per_lane), int(traversal)))

    def shape(self) -> tuple[int, int, int]:
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().p2m_batch_get_shape(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def set_lds_levels(self, levels: int) -> None:
        """Tree levels the per-lane tree search (traversal 1) stages in LDS."""
        check(lib().p2m_batch_set_lds_levels(self._h, int(levels)))

    def lds_levels(self) -> int:
        x = ctypes.c_int()
        check(lib().p2m_batch_get_lds_levels(self._h, ctypes.byref(x)))
        return x.value

    def set_schedule(self, persistent: bool) -> None:
        check(lib().p2m_batch_set_schedule(self._h, 1 if persistent else 0))

    def schedule(self) -> bool:
        x = ctypes.c_int()
        check(lib().p2m_batch_get_schedule(self._h, ctypes.byref(x)))
        return bool(x.value)

    def autotune(self, q, q_offsets, out: dict | None = None, stream=None) -> tuple[int, int, int]:
        torch = _torch()
        q = _dev_tensor(q, torch.float32, (3,), "q")
        off = self._offsets(q_offsets)
        out = self._outs(q, out, status=False)
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().p2m_batch_autotune(self._h, _ptr(q), _ptr(off), _ptr(out["prim"]), _ptr(out["closest"]),
                                       _ptr(out["dist"]), _stream(stream), ctypes.byref(a), ctypes.byref(b),
                                       ctypes.byref(c)))
        return a.value, b.value, c.value


def precompute_many(items, cache_dir: str | None = None, workers: int = 0, **kw) -> list:
    """Precompute several meshes concurrently (one host thread each; the C
    calls release the interpreter lock).  items: (V, F, domain) tuples.
    Returns the Mesh objects in the same order."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    if workers <= 0:
        workers = max(1, len(os.sched_getaffinity(0)))

    def one(it):
        V, F, dom = it
        return Mesh.cached(V, F, dom, cache_dir, threads=1, **kw)[0]

    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(one, items))


def _make_function():
    torch = _torch()

    class P2MDistance(torch.autograd.Function):
        """dist = P2MDistance.apply(q, V, mesh): unsigned point-to-mesh distance.

        Forward runs the P2M query kernel; backward runs the hand-written
        backward kernel, giving d dist / d q and d dist / d V.  V is the
        mesh's vertex-position tensor, [nv,3] float32 on the queries' device;
        the forward answers from the positions the mesh was precomputed and
        uploaded with, so V must hold those positions (after V changes, build
        and upload the mesh again).
        """

        @staticmethod
        def forward(ctx, q, V, mesh):
            if not isinstance(V, torch.Tensor) or V.dtype != torch.float32 or tuple(V.shape) != (mesh.nv, 3):
                raise ValueError(f"V must be a float32 tensor of shape [{mesh.nv}, 3] (the mesh's vertices)")
            if V.device != q.device:
                raise ValueError("V must be on the queries' device")
            fwd = mesh.query(q.detach().contiguous(), for_backward=True, status=False)
            ctx.mesh = mesh
            ctx.save_for_backward(q, fwd["closest"], fwd["dist"], fwd["bary"], fwd["pvid"])
            ctx.V_shape = V.shape
            ctx.mark_non_differentiable(fwd["prim"], fwd["closest"])
            return fwd["dist"], fwd["prim"], fwd["closest"]

        @staticmethod
        def backward(ctx, g_dist, g_prim=None, g_closest=None):
            q, closest, dist, bary, pvid = ctx.saved_tensors
            need_q, need_V = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            gV = torch.zeros(ctx.V_shape, dtype=torch.float32, device=q.device) if need_V else None
            fwd = {"closest": closest, "dist": dist, "bary": bary, "pvid": pvid}
            gq, gV = ctx.mesh.query_backward(q.detach().contiguous(), fwd, g_dist, grad_q=need_q, grad_V=gV)
            return gq, gV, None

    return P2MDistance


_P2MDistance = None


def p2m_distance(q, V, mesh):
    """Differentiable distance (and primitive codes, closest points) of q to the mesh."""
    global _P2MDistance
    if _P2MDistance is None:
        _P2MDistance = _make_function()
    return _P2MDistance.apply(q, V, mesh)


__all__ = ["Mesh", "Batch", "precompute_many", "p2m_distance", "P2MError", "prim_type", "prim_id", "VERTEX", "EDGE", "FACE", "NONE",
           "OUT_OF_DOMAIN", "NONFINITE", "TABLE_FLOODING", "TABLE_ALL_PAIRS", "TABLE_EVERYTHING", "TABLE_FLOODING_DEVICE", "_lib"]
