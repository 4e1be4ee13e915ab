"""Thin Python binding of the C ABI in ``include/gwn.h`` (argument marshalling only).

Every computation runs in the HIP kernels of ``libgwn.so``; this module only
passes torch device pointers, sizes and the current HIP stream through ctypes.
If the library is missing, :func:`load` raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# GWN_LIB selects another build of the library (e.g. one with sanitized host code)
LIB_PATH = os.environ.get("GWN_LIB") or os.path.join(_PKG, "libgwn.so")

GWN_PREC_FP32 = 0
GWN_PREC_FP64 = 1
_PREC = {"fp32": GWN_PREC_FP32, "fp64": GWN_PREC_FP64, GWN_PREC_FP32: GWN_PREC_FP32, GWN_PREC_FP64: GWN_PREC_FP64}

_lib = None


class GwnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gwn status {status}: {msg}")
        self.status = status


class MeshInfo(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("nf", ctypes.c_int64), ("nboundary", ctypes.c_int64),
                ("nloops", ctypes.c_int64), ("nnodes", ctypes.c_int64), ("bvh_depth", ctypes.c_int32),
                ("qshift", ctypes.c_int32), ("bbox", ctypes.c_double * 6), ("qlo", ctypes.c_double * 3),
                ("build_ms", ctypes.c_double), ("nunique", ctypes.c_int64), ("axis", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("proj_area", ctypes.c_double * 3)]


class QueryTuning(ctypes.Structure):
    _fields_ = [("split_max_points", ctypes.c_int32 * 2), ("order_min_points", ctypes.c_int32),
                ("grid_samples_per_lane", ctypes.c_int32 * 2), ("tuned", ctypes.c_int32)]


class AutotuneOpts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("grid_nz", ctypes.c_int32), ("reps", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("cache", ctypes.c_char_p)]


class BuildOpts(ctypes.Structure):
    _fields_ = [("weld_positions", ctypes.c_int32), ("axis", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


_AXIS = {"z": 0, "x": 1, "y": 2, "auto": -1}


def load():
    """Load libgwn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python -m paper_2605_01536_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.gwn_build_mesh.argtypes = [vp, vp, vp, i64, i64, vp, i64, vp, ctypes.POINTER(vp)]
    L.gwn_build_mesh_opts.argtypes = [vp, vp, vp, i64, i64, vp, i64, ctypes.POINTER(BuildOpts), vp,
                                      ctypes.POINTER(vp)]
    L.gwn_build_mesh_opts.restype = ctypes.c_int
    L.gwn_mesh_info_get.argtypes = [vp, ctypes.POINTER(MeshInfo)]
    L.gwn_mesh_destroy.argtypes = [vp]
    L.gwn_query_batch.argtypes = [vp, vp, vp, vp, i64, i64, i32, vp, vp, vp]
    L.gwn_query_grid.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int64), i32, vp, vp, vp]
    L.gwn_query_crossings.argtypes = [vp, vp, vp, vp, i64, i64, vp, vp, vp]
    L.gwn_query_crossings.restype = ctypes.c_int
    L.gwn_query_gradient.argtypes = [vp, vp, vp, vp, i64, i64, i32, vp, vp]
    L.gwn_query_gradient.restype = ctypes.c_int
    L.gwn_query_grid_gradient.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int64), i32, vp, vp]
    L.gwn_query_grid_gradient.restype = ctypes.c_int
    L.gwn_query_direct.argtypes = [vp, vp, vp, vp, i64, i64, i32, vp, vp]
    L.gwn_query_direct.restype = ctypes.c_int
    L.gwn_status_str.argtypes = [ctypes.c_int]
    L.gwn_status_str.restype = ctypes.c_char_p
    L.gwn_last_error.restype = ctypes.c_char_p
    for f in ("gwn_build_mesh", "gwn_mesh_info_get", "gwn_mesh_destroy", "gwn_query_batch", "gwn_query_grid"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        L = load()
        raise GwnError(status, L.gwn_last_error().decode())


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int:
    return int(t.data_ptr()) if t is not None else 0


def _points(Q, name="Q"):
    """An (n, 3) CUDA tensor as contiguous float32 (the layout the C ABI reads)."""
    import torch
    if not (isinstance(Q, torch.Tensor) and Q.is_cuda and Q.dim() == 2 and Q.shape[1] == 3):
        raise ValueError(f"{name} must be an (n, 3) CUDA tensor")
    return Q.to(torch.float32).contiguous()


def _out(t, shape, dtype, device, name):
    """A caller-supplied output must match exactly (the kernels write shape[0] rows);
    None allocates one."""
    import torch
    shape = tuple(int(x) for x in shape)
    if t is None:
        return torch.empty(shape, device=device, dtype=dtype)
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()
            and tuple(t.shape) == shape):
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor of shape {shape}")
    return t


def _wdtype(p):
    import torch
    return torch.float64 if p == GWN_PREC_FP64 else torch.float32


class Mesh:
    """A soup built on the device: V (nv, 3) float32 and F (nf, 3) int32 CUDA tensors.
    weld=True merges vertices with equal positions before the boundary is extracted;
    axis ("z", "x", "y" or "auto") is the direction of the crossing ray."""

    def __init__(self, V, F, stream=None, weld: bool = False, axis: str = "z"):
        import torch
        L = load()
        if V.dim() != 2 or V.shape[1] != 3 or F.dim() != 2 or F.shape[1] != 3:
            raise ValueError("V must be (nv, 3) and F (nf, 3)")
        V = V.to(device="cuda", dtype=torch.float32).contiguous()
        F = F.to(device="cuda", dtype=torch.int32).contiguous()
        self._h = ctypes.c_void_p()
        base = _ptr(V)
        opts = BuildOpts(int(bool(weld)), _AXIS[axis])
        _check(L.gwn_build_mesh_opts(base, base + 4, base + 8, 3, V.shape[0], _ptr(F), F.shape[0],
                                     ctypes.byref(opts), _stream(stream), ctypes.byref(self._h)))

    def info(self) -> dict:
        inf = MeshInfo()
        _check(load().gwn_mesh_info_get(self._h, ctypes.byref(inf)))
        return {"nv": inf.nv, "nf": inf.nf, "nboundary": inf.nboundary, "nloops": inf.nloops,
                "nnodes": inf.nnodes, "bvh_depth": inf.bvh_depth, "qshift": inf.qshift,
                "bbox": list(inf.bbox), "qlo": list(inf.qlo), "build_ms": inf.build_ms, "nunique": inf.nunique,
                "axis": "zxy"[inf.axis], "proj_area": list(inf.proj_area)}

    @property
    def handle(self):
        return self._h

    def tuning(self) -> dict:
        """The mesh's query tuning (gwn_mesh_get_tuning); 0 = built-in rule, -1 = never."""
        L = load()
        L.gwn_mesh_get_tuning.argtypes = [ctypes.c_void_p, ctypes.POINTER(QueryTuning)]
        L.gwn_mesh_get_tuning.restype = ctypes.c_int
        q = QueryTuning()
        _check(L.gwn_mesh_get_tuning(self._h, ctypes.byref(q)))
        return {"split_max_points": list(q.split_max_points), "order_min_points": q.order_min_points,
                "grid_samples_per_lane": list(q.grid_samples_per_lane), "tuned": q.tuned}

    def set_tuning(self, split_max_points=(0, 0), order_min_points=0, grid_samples_per_lane=(0, 0)):
        """gwn_mesh_set_tuning; pairs are indexed by precision (fp32, fp64)."""
        L = load()
        L.gwn_mesh_set_tuning.argtypes = [ctypes.c_void_p, ctypes.POINTER(QueryTuning)]
        L.gwn_mesh_set_tuning.restype = ctypes.c_int
        q = QueryTuning((ctypes.c_int32 * 2)(*split_max_points), int(order_min_points),
                        (ctypes.c_int32 * 2)(*grid_samples_per_lane), 0)
        _check(L.gwn_mesh_set_tuning(self._h, ctypes.byref(q)))

    def autotune(self, prec="fp32", grid_nz: int = 0, reps: int = 0, cache: str | None = None, stream=None) -> dict:
        """gwn_mesh_autotune for one precision; returns the tuning it set."""
        L = load()
        L.gwn_mesh_autotune.argtypes = [ctypes.c_void_p, ctypes.POINTER(AutotuneOpts), ctypes.c_void_p]
        L.gwn_mesh_autotune.restype = ctypes.c_int
        o = AutotuneOpts(_PREC[prec], int(grid_nz), int(reps), 0, os.fsencode(cache) if cache else None)
        _check(L.gwn_mesh_autotune(self._h, ctypes.byref(o), _stream(stream)))
        return self.tuning()

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().gwn_mesh_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_mesh(V, F, stream=None, weld: bool = False, axis: str = "z") -> Mesh:
    return Mesh(V, F, stream, weld=weld, axis=axis)


def query_batch(mesh: Mesh, Q, prec="fp32", want_chi=False, out=None, chi_out=None, stream=None):
    """w for points Q (n, 3) float32 CUDA tensor; returns w (and chi if requested)."""
    import torch
    L = load()
    p = _PREC[prec]
    Q = _points(Q)
    n = Q.shape[0]
    out = _out(out, (n,), _wdtype(p), Q.device, "out")
    if want_chi or chi_out is not None:
        chi_out = _out(chi_out, (n,), torch.int32, Q.device, "chi_out")
    base = _ptr(Q)
    _check(L.gwn_query_batch(mesh.handle, base, base + 4, base + 8, 3, n, p, _ptr(out),
                             _ptr(chi_out) if chi_out is not None else None, _stream(stream)))
    return (out, chi_out) if want_chi else out


def query_crossings(mesh: Mesh, Q, stream=None):
    """(chi along +z, chi along -z) per point, int32 CUDA tensors."""
    import torch
    L = load()
    Q = _points(Q)
    n = Q.shape[0]
    up = torch.empty(n, device=Q.device, dtype=torch.int32)
    dn = torch.empty(n, device=Q.device, dtype=torch.int32)
    base = _ptr(Q)
    _check(L.gwn_query_crossings(mesh.handle, base, base + 4, base + 8, 3, n, _ptr(up), _ptr(dn), _stream(stream)))
    return up, dn


def query_gradient(mesh: Mesh, Q, prec="fp32", out=None, stream=None):
    """grad w at each query point, (n, 3) float32 or float64 (Supp. Alg. 3)."""
    import torch
    L = load()
    p = _PREC[prec]
    Q = _points(Q)
    n = Q.shape[0]
    out = _out(out, (n, 3), _wdtype(p), Q.device, "out")
    base = _ptr(Q)
    _check(L.gwn_query_gradient(mesh.handle, base, base + 4, base + 8, 3, n, p, _ptr(out), _stream(stream)))
    return out


def query_direct(mesh: Mesh, Q, prec="fp32", out=None, stream=None):
    """w by the direct per-triangle solid-angle sum (O(F) per point; the baseline)."""
    import torch
    L = load()
    p = _PREC[prec]
    Q = _points(Q)
    n = Q.shape[0]
    out = _out(out, (n,), _wdtype(p), Q.device, "out")
    base = _ptr(Q)
    _check(L.gwn_query_direct(mesh.handle, base, base + 4, base + 8, 3, n, p, _ptr(out), _stream(stream)))
    return out


def query_grid(mesh: Mesh, origin, spacing, dims, prec="fp32", want_chi=False, out=None, chi_out=None, stream=None):
    """w on the cell-centred grid origin + (idx + 0.5) * spacing, flattened z fastest."""
    import torch
    L = load()
    p = _PREC[prec]
    if len(dims) != 3 or min(int(x) for x in dims) < 0:
        raise ValueError("dims must be three non-negative sizes")
    n = int(dims[0]) * int(dims[1]) * int(dims[2])
    out = _out(out, (n,), _wdtype(p), "cuda", "out")
    if want_chi or chi_out is not None:
        chi_out = _out(chi_out, (n,), torch.int32, "cuda", "chi_out")
    o = (ctypes.c_double * 3)(*[float(x) for x in origin])
    s = (ctypes.c_double * 3)(*[float(x) for x in spacing])
    d = (ctypes.c_int64 * 3)(*[int(x) for x in dims])
    _check(L.gwn_query_grid(mesh.handle, o, s, d, p, _ptr(out), _ptr(chi_out) if chi_out is not None else None,
                            _stream(stream)))
    return (out, chi_out) if want_chi else out


def query_grid_gradient(mesh: Mesh, origin, spacing, dims, prec="fp32", out=None, stream=None):
    """grad w on the cell-centred grid of query_grid, (nx * ny * nz, 3), z fastest."""
    L = load()
    p = _PREC[prec]
    if len(dims) != 3 or min(int(x) for x in dims) < 0:
        raise ValueError("dims must be three non-negative sizes")
    n = int(dims[0]) * int(dims[1]) * int(dims[2])
    out = _out(out, (n, 3), _wdtype(p), "cuda", "out")
    o = (ctypes.c_double * 3)(*[float(x) for x in origin])
    s = (ctypes.c_double * 3)(*[float(x) for x in spacing])
    d = (ctypes.c_int64 * 3)(*[int(x) for x in dims])
    _check(L.gwn_query_grid_gradient(mesh.handle, o, s, d, p, _ptr(out), _stream(stream)))
    return out


class MultiOpts(ctypes.Structure):
    _fields_ = [("item_queries", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32), ("order", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("tune_cache", ctypes.c_char_p)]


class MultiInfo(ctypes.Structure):
    _fields_ = [("nmesh", ctypes.c_int32), ("nqueries", ctypes.c_int64), ("nitems", ctypes.c_int32),
                ("item_queries", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32), ("order", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("tuned", ctypes.c_int32), ("est_pairs", ctypes.c_double),
                ("tuned_ms", ctypes.c_double)]


def _load_multi(L):
    if getattr(L, "_multi_ready", False):
        return
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.gwn_multi_create.argtypes = [ctypes.POINTER(vp), i32, vp, vp, vp, i64, ctypes.POINTER(ctypes.c_int64), i32, vp,
                                   vp, ctypes.POINTER(MultiOpts), vp, ctypes.POINTER(vp)]
    L.gwn_multi_run.argtypes = [vp, vp]
    L.gwn_multi_info_get.argtypes = [vp, ctypes.POINTER(MultiInfo)]
    L.gwn_multi_destroy.argtypes = [vp]
    for f in ("gwn_multi_create", "gwn_multi_run", "gwn_multi_info_get", "gwn_multi_destroy"):
        getattr(L, f).restype = ctypes.c_int
    L._multi_ready = True


class MultiPlan:
    """Captured multi-mesh evaluation: meshes[m] owns queries Q[offsets[m]:offsets[m+1]]."""

    def __init__(self, meshes, Q, offsets, w_out=None, chi_out=None, item_queries=0, waves_per_simd=0, order=0,
                 autotune=False, tune_cache=None, stream=None, prec="fp32"):
        import torch
        L = load()
        _load_multi(L)
        prec = _PREC[prec]
        self._meshes = list(meshes)
        self._Q = _points(Q)
        n = int(offsets[-1])
        if len(offsets) != len(self._meshes) + 1 or self._Q.shape[0] < n:
            raise ValueError("offsets must have nmesh + 1 entries ending at most at len(Q)")
        self.w = _out(w_out, (n,), torch.float64 if prec == GWN_PREC_FP64 else torch.float32, Q.device, "w_out")
        self.chi = _out(chi_out, (n,), torch.int32, Q.device, "chi_out") if chi_out is not None else None
        hs = (ctypes.c_void_p * len(self._meshes))(*[m.handle.value for m in self._meshes])
        offs = (ctypes.c_int64 * len(offsets))(*[int(o) for o in offsets])
        self._cache = tune_cache.encode() if tune_cache else None
        opts = MultiOpts(int(item_queries), int(waves_per_simd), int(order), int(bool(autotune)), self._cache)
        base = _ptr(self._Q)
        self._h = ctypes.c_void_p()
        _check(L.gwn_multi_create(hs, len(self._meshes), base, base + 4, base + 8, 3, offs, int(prec),
                                  _ptr(self.w), _ptr(self.chi) if self.chi is not None else None,
                                  ctypes.byref(opts), _stream(stream), ctypes.byref(self._h)))

    def run(self, stream=None):
        _check(load().gwn_multi_run(self._h, _stream(stream)))
        return self.w

    def info(self) -> dict:
        inf = MultiInfo()
        _check(load().gwn_multi_info_get(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in MultiInfo._fields_}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().gwn_multi_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PatchOpts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("eps", ctypes.c_double), ("max_depth", ctypes.c_int32)]


class PatchesInfo(ctypes.Structure):
    _fields_ = [("npatch", ctypes.c_int64), ("ncurves", ctypes.c_int64), ("tau", ctypes.c_double),
                ("eps", ctypes.c_double), ("max_depth", ctypes.c_int32), ("diag", ctypes.c_double)]


def _load_patches(L):
    if getattr(L, "_patches_ready", False):
        return
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    L.gwn_patches_build.argtypes = [vp, i64, ctypes.POINTER(PatchOpts), vp, ctypes.POINTER(vp)]
    L.gwn_patches_info_get.argtypes = [vp, ctypes.POINTER(PatchesInfo)]
    L.gwn_patches_query.argtypes = [vp, vp, vp, vp, i64, i64, vp, vp, vp, vp]
    L.gwn_patches_destroy.argtypes = [vp]
    L.gwn_patches_query_stats.argtypes = [vp, vp, vp, vp, i64, i64, vp, ctypes.POINTER(ctypes.c_int64), vp]
    L.gwn_patches_query_grid.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64), vp, vp, vp,
                                         ctypes.POINTER(ctypes.c_int64), vp]
    for f in ("gwn_patches_build", "gwn_patches_info_get", "gwn_patches_query", "gwn_patches_destroy",
              "gwn_patches_query_stats", "gwn_patches_query_grid"):
        getattr(L, f).restype = ctypes.c_int
    L._patches_ready = True


class Patches:
    """A surface of tensor-product cubic Bezier patches: P is a CUDA float64
    tensor (npatch, 16, 3), control point P[k, 4 i + j] with i along u."""

    def __init__(self, P, tau=0.0, eps=0.0, max_depth=0, stream=None):
        import torch
        L = load()
        _load_patches(L)
        if not (torch.is_tensor(P) and P.is_cuda and P.dtype == torch.float64 and P.dim() == 3
                and P.shape[1:] == (16, 3)):
            raise ValueError("P must be a CUDA float64 tensor of shape (npatch, 16, 3)")
        self._P = P.contiguous()
        opts = PatchOpts(float(tau), float(eps), int(max_depth))
        self._h = ctypes.c_void_p()
        _check(L.gwn_patches_build(_ptr(self._P), self._P.shape[0], ctypes.byref(opts), _stream(stream),
                                   ctypes.byref(self._h)))

    def info(self) -> dict:
        inf = PatchesInfo()
        _check(load().gwn_patches_info_get(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in PatchesInfo._fields_}

    def query(self, Q, want_chi=False, out=None, stream=None):
        """w (float64) per point of Q (n, 3) float32; with want_chi also the
        crossing counts and the chosen direction index per point."""
        import torch
        L = load()
        Q = _points(Q)
        n = Q.shape[0]
        out = _out(out, (n,), torch.float64, Q.device, "out")
        chi = torch.empty(n, dtype=torch.int32, device=Q.device) if want_chi else None
        dr = torch.empty(n, dtype=torch.int32, device=Q.device) if want_chi else None
        base = _ptr(Q)
        _check(L.gwn_patches_query(self._h, base, base + 4, base + 8, 3, n, _ptr(out),
                                   _ptr(chi) if chi is not None else None, _ptr(dr) if dr is not None else None,
                                   _stream(stream)))
        return (out, chi, dr) if want_chi else out

    def query_grid(self, origin, spacing, dims, want_chi=False, out=None, stream=None, counts=None):
        """w (float64) on the cell-centred grid origin + (idx + 0.5) * spacing, z fastest (columns
        share their vertical ray); with want_chi also crossing counts and direction indices; with
        counts (a list) the call also appends (quadrature intervals, sub-patch cells)."""
        import torch
        L = load()
        if len(dims) != 3 or min(int(x) for x in dims) < 0:
            raise ValueError("dims must be three non-negative sizes")
        n = int(dims[0]) * int(dims[1]) * int(dims[2])
        out = _out(out, (n,), torch.float64, "cuda", "out")
        chi = torch.empty(n, dtype=torch.int32, device="cuda") if want_chi else None
        dr = torch.empty(n, dtype=torch.int32, device="cuda") if want_chi else None
        o = (ctypes.c_double * 3)(*[float(x) for x in origin])
        s = (ctypes.c_double * 3)(*[float(x) for x in spacing])
        d = (ctypes.c_int64 * 3)(*[int(x) for x in dims])
        cnt = (ctypes.c_int64 * 2)() if counts is not None else None
        _check(L.gwn_patches_query_grid(self._h, o, s, d, _ptr(out), _ptr(chi) if chi is not None else None,
                                        _ptr(dr) if dr is not None else None, cnt, _stream(stream)))
        if counts is not None:
            counts.extend([int(cnt[0]), int(cnt[1])])
        return (out, chi, dr) if want_chi else out

    def query_stats(self, Q, stream=None):
        """(w, quadrature intervals, sub-patch cells) of one evaluation of Q."""
        import torch
        L = load()
        Q = _points(Q)
        out = torch.empty(Q.shape[0], dtype=torch.float64, device=Q.device)
        counts = (ctypes.c_int64 * 2)()
        base = _ptr(Q)
        _check(L.gwn_patches_query_stats(self._h, base, base + 4, base + 8, 3, Q.shape[0], _ptr(out), counts,
                                         _stream(stream)))
        return out, int(counts[0]), int(counts[1])

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().gwn_patches_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MLP_NPARAMS = 57985


def _target(T, Q):
    import torch
    if not (isinstance(T, torch.Tensor) and T.is_cuda and T.dim() == 1 and T.shape[0] == Q.shape[0]):
        raise ValueError("target must be a 1-D CUDA tensor with one value per point")
    return T.to(torch.float32).contiguous()


class SurrogateCfg(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_train", ctypes.c_int64), ("box_lo", ctypes.c_double * 3),
                ("box_hi", ctypes.c_double * 3), ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("lr", ctypes.c_float), ("lr_final", ctypes.c_float), ("stop_epoch", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


BAND_HALF = 0   # |prediction - 1/2| < band
BAND_FRAC = 1   # |frac(prediction) - 1/2| < band
_RULE = {"half": BAND_HALF, "frac": BAND_FRAC, BAND_HALF: BAND_HALF, BAND_FRAC: BAND_FRAC}


def _load_mlp(L):
    if getattr(L, "_mlp_ready", False):
        return
    vp, i64, i32, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float
    L.gwn_mlp_create.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(vp)]
    L.gwn_mlp_destroy.argtypes = [vp]
    L.gwn_mlp_get_state.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int64)]
    L.gwn_mlp_set_state.argtypes = [vp, vp, vp, vp, vp, i64]
    L.gwn_mlp_forward.argtypes = [vp, vp, vp, vp, i64, i64, vp, vp]
    L.gwn_mlp_loss_grad.argtypes = [vp, vp, vp, vp, i64, vp, i64, vp, ctypes.POINTER(f32), vp]
    L.gwn_mlp_train_step.argtypes = [vp, vp, vp, vp, i64, vp, i64, f32, ctypes.POINTER(f32), vp]
    L.gwn_surrogate_query.argtypes = [vp, vp, vp, vp, vp, i64, i64, f32, i32, vp, vp, ctypes.POINTER(ctypes.c_int64),
                                      vp]
    L.gwn_surrogate_train.argtypes = [vp, vp, ctypes.POINTER(SurrogateCfg), vp, vp, i64, vp,
                                      ctypes.POINTER(ctypes.c_int64), vp]
    L.gwn_surrogate_save.argtypes = [vp, ctypes.c_char_p]
    L.gwn_surrogate_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
    L.gwn_surrogate_destroy.argtypes = [vp]
    for f in ("gwn_mlp_create", "gwn_mlp_destroy", "gwn_mlp_get_state", "gwn_mlp_set_state", "gwn_mlp_forward",
              "gwn_mlp_loss_grad", "gwn_mlp_train_step", "gwn_surrogate_query", "gwn_surrogate_train",
              "gwn_surrogate_save", "gwn_surrogate_load", "gwn_surrogate_destroy"):
        getattr(L, f).restype = ctypes.c_int
    L._mlp_ready = True


class Surrogate:
    """Fourier-feature MLP trained and evaluated by the library's MFMA kernels."""

    def __init__(self, seed: int = 0, sigma: float = 2.0, _handle=None):
        L = load()
        _load_mlp(L)
        if _handle is not None:
            self._h = _handle
            return
        self._h = ctypes.c_void_p()
        _check(L.gwn_mlp_create(int(seed), float(sigma), ctypes.byref(self._h)))

    @classmethod
    def load(cls, path: str) -> "Surrogate":
        """A network restored from a checkpoint written by save() (gwn_surrogate_load)."""
        L = load()
        _load_mlp(L)
        h = ctypes.c_void_p()
        _check(L.gwn_surrogate_load(os.fsencode(path), ctypes.byref(h)))
        return cls(_handle=h)

    def save(self, path: str):
        """The complete training state in the library's checkpoint format (gwn_surrogate_save)."""
        _check(load().gwn_surrogate_save(self._h, os.fsencode(path)))

    def state(self) -> dict:
        import numpy as np
        th = np.zeros(MLP_NPARAMS, np.float32)
        m = np.zeros(MLP_NPARAMS, np.float32)
        v = np.zeros(MLP_NPARAMS, np.float32)
        G = np.zeros(96, np.float32)
        step = ctypes.c_int64(0)
        _check(load().gwn_mlp_get_state(self._h, th.ctypes.data, m.ctypes.data, v.ctypes.data, G.ctypes.data,
                                        ctypes.byref(step)))
        return {"theta": th, "m": m, "v": v, "G": G.reshape(32, 3), "step": int(step.value)}

    def load_state(self, st: dict):
        import numpy as np
        arrs = {k: np.ascontiguousarray(st[k], np.float32).ravel() for k in ("theta", "m", "v", "G") if k in st}
        p = {k: (arrs[k].ctypes.data if k in arrs else None) for k in ("theta", "m", "v", "G")}
        _check(load().gwn_mlp_set_state(self._h, p["theta"], p["m"], p["v"], p["G"], int(st.get("step", -1))))

    def train(self, mesh, epochs: int, batch: int = 8192, lr: float = 2e-3, lr_final: float = 1e-4,
              n_train: int = 0, seed: int = 0, box=None, X=None, T=None, stop_epoch: int = 0, stream=None):
        """gwn_surrogate_train: mini-batch Adam with per-pass device shuffles and a cosine
        learning rate, on n_train generated points labelled by the exact path (or on the
        caller's points X (n, 3), with labels T or labelled on mesh).  Returns the mean
        batch loss of each pass trained by this call."""
        import numpy as np
        L = load()
        cfg = SurrogateCfg()
        cfg.seed = int(seed)
        cfg.n_train = int(n_train)
        if box is not None:
            for a in range(3):
                cfg.box_lo[a] = float(box[0][a])
                cfg.box_hi[a] = float(box[1][a])
        cfg.epochs, cfg.batch, cfg.lr, cfg.lr_final = int(epochs), int(batch), float(lr), float(lr_final)
        cfg.stop_epoch = int(stop_epoch)
        n = 0
        if X is not None:
            X = _points(X, "X")
            n = X.shape[0]
            if T is not None:
                T = _target(T, X)
        elif T is not None:
            raise ValueError("labels T need their points X")
        losses = np.zeros(max(1, int(epochs)), np.float32)
        ran = ctypes.c_int64(0)
        _check(L.gwn_surrogate_train(self._h, mesh.handle if mesh is not None else None, ctypes.byref(cfg),
                                     _ptr(X) if X is not None else None, _ptr(T) if T is not None else None, n,
                                     losses.ctypes.data, ctypes.byref(ran), _stream(stream)))
        return losses[:ran.value].tolist()

    def forward(self, Q, out=None, stream=None):
        import torch
        Q = _points(Q)
        n = Q.shape[0]
        out = _out(out, (n,), torch.float32, Q.device, "out")
        b = _ptr(Q)
        _check(load().gwn_mlp_forward(self._h, b, b + 4, b + 8, 3, n, _ptr(out), _stream(stream)))
        return out

    def loss_grad(self, Q, target, stream=None):
        import torch
        Q = _points(Q)
        target = _target(target, Q)
        g = torch.empty(MLP_NPARAMS, device=Q.device, dtype=torch.float32)
        loss = ctypes.c_float(0)
        b = _ptr(Q)
        _check(load().gwn_mlp_loss_grad(self._h, b, b + 4, b + 8, 3, _ptr(target), Q.shape[0], _ptr(g),
                                        ctypes.byref(loss), _stream(stream)))
        return float(loss.value), g

    def train_step(self, Q, target, lr: float, want_loss: bool = True, stream=None):
        Q = _points(Q)
        target = _target(target, Q)
        loss = ctypes.c_float(0)
        b = _ptr(Q)
        _check(load().gwn_mlp_train_step(self._h, b, b + 4, b + 8, 3, _ptr(target), Q.shape[0], float(lr),
                                         ctypes.byref(loss) if want_loss else None, _stream(stream)))
        return float(loss.value) if want_loss else None

    def query(self, mesh: Mesh, Q, band: float, out=None, want_mask: bool = False, rule="half", stream=None):
        """Prediction, with exact re-evaluation where the fallback rule holds: rule "half",
        |prediction - 1/2| < band; rule "frac", |frac(prediction) - 1/2| < band."""
        import torch
        Q = _points(Q)
        n = Q.shape[0]
        out = _out(out, (n,), torch.float32, Q.device, "out")
        mask = torch.empty(n, device=Q.device, dtype=torch.uint8) if want_mask else None
        nfb = ctypes.c_int64(0)
        b = _ptr(Q)
        _check(load().gwn_surrogate_query(self._h, mesh.handle, b, b + 4, b + 8, 3, n, float(band), _RULE[rule],
                                          _ptr(out), _ptr(mask) if mask is not None else None, ctypes.byref(nfb),
                                          _stream(stream)))
        return (out, mask, int(nfb.value)) if want_mask else (out, int(nfb.value))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().gwn_surrogate_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _load_prims(L):
    if getattr(L, "_prims_ready", False):
        return
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    for f in ("gwn_radix_sort_u32", "gwn_radix_sort_u64"):
        getattr(L, f).argtypes = [vp, vp, vp, vp, i64, i32, i32, vp]
        getattr(L, f).restype = ctypes.c_int
    for f in ("gwn_scan_exclusive_sum_i32", "gwn_scan_inclusive_max_i32"):
        getattr(L, f).argtypes = [vp, vp, i64, vp]
        getattr(L, f).restype = ctypes.c_int
    L._prims_ready = True


def radix_sort(keys, vals=None, begin_bit: int = 0, end_bit: int | None = None, stream=None):
    """Stable device sort of a 1-D CUDA tensor of uint32 or uint64 keys (given as int32 / int64
    tensors, reinterpreted) by bits [begin_bit, end_bit); returns (sorted keys, payloads or None)."""
    import torch
    L = load()
    _load_prims(L)
    if not (isinstance(keys, torch.Tensor) and keys.is_cuda and keys.dim() == 1
            and keys.dtype in (torch.int32, torch.int64)):
        raise ValueError("keys must be a 1-D CUDA int32 or int64 tensor")
    keys = keys.contiguous()
    wide = keys.dtype == torch.int64
    end_bit = (64 if wide else 32) if end_bit is None else end_bit
    kout = torch.empty_like(keys)
    vout = None
    if vals is not None:
        if not (isinstance(vals, torch.Tensor) and vals.is_cuda and vals.dtype == torch.int32
                and vals.shape == keys.shape):
            raise ValueError("vals must be a CUDA int32 tensor shaped like keys")
        vals = vals.contiguous()
        vout = torch.empty_like(vals)
    f = L.gwn_radix_sort_u64 if wide else L.gwn_radix_sort_u32
    _check(f(_ptr(keys), _ptr(kout), _ptr(vals) if vals is not None else None,
             _ptr(vout) if vout is not None else None, keys.shape[0], int(begin_bit), int(end_bit), _stream(stream)))
    return kout, vout


def scan(x, op: str = "exclusive_sum", stream=None):
    """Device prefix scan of a 1-D CUDA int32 tensor: "exclusive_sum" or "inclusive_max"."""
    import torch
    L = load()
    _load_prims(L)
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dim() == 1 and x.dtype == torch.int32):
        raise ValueError("x must be a 1-D CUDA int32 tensor")
    x = x.contiguous()
    out = torch.empty_like(x)
    f = {"exclusive_sum": L.gwn_scan_exclusive_sum_i32, "inclusive_max": L.gwn_scan_inclusive_max_i32}[op]
    _check(f(_ptr(x), _ptr(out), x.shape[0], _stream(stream)))
    return out


NOALLOC_MAX_POINTS = 1048576


def query_batch_noalloc(mesh: Mesh, Q, prec="fp32", want_chi=False, out=None, chi_out=None, stream=None):
    """gwn_query_batch_noalloc: query_batch with the library's fixed per-GPU scratch instead of
    allocations (at most NOALLOC_MAX_POINTS points; calls overlapping on one GPU race)."""
    import torch
    L = load()
    if not getattr(L, "_noalloc_ready", False):
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.gwn_query_batch_noalloc.argtypes = [vp, vp, vp, vp, i64, i64, i32, vp, vp, vp]
        L.gwn_query_batch_noalloc.restype = ctypes.c_int
        L._noalloc_ready = True
    p = _PREC[prec]
    Q = _points(Q)
    n = Q.shape[0]
    out = _out(out, (n,), _wdtype(p), Q.device, "out")
    if want_chi or chi_out is not None:
        chi_out = _out(chi_out, (n,), torch.int32, Q.device, "chi_out")
    base = _ptr(Q)
    _check(L.gwn_query_batch_noalloc(mesh.handle, base, base + 4, base + 8, 3, n, p, _ptr(out),
                                     _ptr(chi_out) if chi_out is not None else None, _stream(stream)))
    return (out, chi_out) if want_chi else out
