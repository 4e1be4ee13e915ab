"""CPU oracle for generalized winding numbers -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It is independent of the GPU library
(no shared sources, headers or constants) and implements, in plain FP64 C:

* ``direct``     -- Eq. 2 with the per-triangle signed solid angle of Eq. 6,
                    accumulated in double-double (ground truth, Sec. 5.2).
* ``antipodal``  -- Eq. 10 / Alg. 1 with x0 = +z and exact quantised
                    predicates with symbolic perturbation (Supp. Sec. 2.1).
* ``chi``        -- signed crossings of the +z and -z rays (Sec. 3.2).
* ``gradient``   -- grad w by Supp. Alg. 3 (boundary term only; the integer
                    part is locally constant), any axis.
* ``distance``   -- point-to-soup distance (Ericson 2005), to mask queries
                    on or near the surface where w is undefined (Sec. 3.1).
* ``boundary``   -- the cancelled directed boundary chain (Sec. 4.1).
* ``weld``       -- merge vertices with equal coordinates onto one index.
* ``parametric`` -- Alg. 2 for tensor-product cubic Bezier patches: chi by
                    ray-driven subdivision to bilinear pieces, the boundary
                    curves' integral of Alg. 2's f by adaptive GK15 (Sec. 4.4).
* ``bezier_boundary`` -- the patches' boundary curves after equal curves
                    traversed both ways cancel.

The C sources are ``gwn_oracle.c`` and ``param_oracle.c``; ``build()``
compiles them with gcc into ``liboracle.so`` next to them (no FP contraction,
OpenMP over queries).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gwn_oracle.c")
_SRC_PARAM = os.path.join(_HERE, "param_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_F32 = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_F64 = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_I64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_U8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_VP = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (always when force=True)."""
    stale = not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                                     os.path.getmtime(_SRC_PARAM))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", _SRC, _SRC_PARAM, "-o", tmp, "-lquadmath", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(path: str) -> str:
    """Compile the oracle with AddressSanitizer and UndefinedBehaviorSanitizer
    (any undefined behaviour aborts) into `path`; load it by setting
    GWN_ORACLE_LIB=path in a process started with the sanitizer runtimes
    preloaded (LD_PRELOAD)."""
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           _SRC, _SRC_PARAM, "-o", path, "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True)
    return path


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("GWN_ORACLE_LIB")
        if not path:
            build()
            path = _LIB
        L = ctypes.CDLL(path)
        L.oracle_quant_params.argtypes = [_F32, _i64, _F64, _F64, ctypes.POINTER(_i32)]
        L.oracle_quantize.argtypes = [_F32, _i64, _F64, _i32, _I64, _U8]
        L.oracle_orient2d_sos.argtypes = [_i64] * 6
        L.oracle_orient2d_sos.restype = ctypes.c_int
        L.oracle_plane_sos.argtypes = [_I64, _I64, _I64, _I64]
        L.oracle_plane_sos.restype = ctypes.c_int
        L.oracle_boundary.argtypes = [_I32, _i64, ctypes.c_int, _VP, _VP, _i64]
        L.oracle_boundary.restype = _i64
        L.oracle_chi.argtypes = [_F32, _i64, _I32, _i64, _F32, _i64, ctypes.c_int, _I32, _I32]
        L.oracle_antipodal.argtypes = [_F32, _i64, _I32, _i64, _F32, _i64, ctypes.c_int, _F64, _F64, _I32, _I32]
        L.oracle_direct.argtypes = [_F32, _i64, _I32, _i64, _F32, _i64, _F64]
        L.oracle_solid_angle.argtypes = [_F64, _F64, _F64, _F64]
        L.oracle_solid_angle.restype = ctypes.c_double
        L.oracle_distance.argtypes = [_F32, _i64, _I32, _i64, _F32, _i64, ctypes.c_double, _F64]
        L.oracle_distance2.argtypes = [_F32, _i64, _I32, _i64, _F32, _i64, ctypes.c_double, ctypes.c_int, _F64]
        L.oracle_gradient.argtypes = [_F32, _i64, _I32, _i64, _F32, _i64, _F64, _F64, _F64]
        L.oracle_weld.argtypes = [_F32, _i64, _I32, _i64, _I32]
        L.oracle_weld.restype = _i64
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_param_boundary.argtypes = [_i64, _F64, _i64, _F64, _F64, ctypes.c_double, ctypes.c_int, _F64]
        L.oracle_param_chi.argtypes = [_i64, _F64, _i64, _F64, _F64, ctypes.c_double, ctypes.c_double, _I32, _U8]
        L.oracle_gk15_poly.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        _lib = L
    return _lib


def _mesh(V, F):
    V = np.ascontiguousarray(V, dtype=np.float32).reshape(-1, 3)
    F = np.ascontiguousarray(F, dtype=np.int32).reshape(-1, 3)
    return V, F


def _pts(Q):
    return np.ascontiguousarray(Q, dtype=np.float32).reshape(-1, 3)


def quant_params(V):
    """(bbox[6], lo[3], k) of the 30-bit fixed-point grid for vertex set V."""
    V = np.ascontiguousarray(V, dtype=np.float32).reshape(-1, 3)
    bbox = np.zeros(6)
    lo = np.zeros(3)
    k = _i32(0)
    lib().oracle_quant_params(V, V.shape[0], bbox, lo, ctypes.byref(k))
    return bbox, lo, int(k.value)


def quantize(P, lo, k):
    P = _pts(P)
    q = np.zeros((P.shape[0], 3), dtype=np.int64)
    ib = np.zeros(P.shape[0], dtype=np.uint8)
    lib().oracle_quantize(P, P.shape[0], np.ascontiguousarray(lo, dtype=np.float64), int(k), q, ib)
    return q, ib.astype(bool)


def orient2d_sos(x0, y0, x1, y1, qx, qy) -> int:
    return int(lib().oracle_orient2d_sos(int(x0), int(y0), int(x1), int(y1), int(qx), int(qy)))


def plane_sos(p0, p1, p2, q) -> int:
    a = [np.ascontiguousarray(v, dtype=np.int64) for v in (p0, p1, p2, q)]
    return int(lib().oracle_plane_sos(*a))


def boundary(F, cancel: bool = True):
    F = np.ascontiguousarray(F, dtype=np.int32).reshape(-1, 3)
    n = lib().oracle_boundary(F, F.shape[0], int(cancel), None, None, 0)
    fr = np.zeros(max(n, 1), dtype=np.int32)
    to = np.zeros(max(n, 1), dtype=np.int32)
    lib().oracle_boundary(F, F.shape[0], int(cancel), fr.ctypes.data, to.ctypes.data, n)
    return fr[:n], to[:n]


def chi(V, F, Q, use_bins: bool = True):
    """(chi along +z, chi along -z) per query, int32."""
    V, F = _mesh(V, F)
    Q = _pts(Q)
    up = np.zeros(Q.shape[0], dtype=np.int32)
    dn = np.zeros(Q.shape[0], dtype=np.int32)
    lib().oracle_chi(V, V.shape[0], F, F.shape[0], Q, Q.shape[0], int(use_bins), up, dn)
    return up, dn


def antipodal(V, F, Q, cancel: bool = True, full: bool = False):
    """O2: w per query (float64); with full=True also (S, chi_up, chi_down)."""
    V, F = _mesh(V, F)
    Q = _pts(Q)
    n = Q.shape[0]
    w = np.zeros(n)
    S = np.zeros(n)
    up = np.zeros(n, dtype=np.int32)
    dn = np.zeros(n, dtype=np.int32)
    lib().oracle_antipodal(V, V.shape[0], F, F.shape[0], Q, n, int(cancel), w, S, up, dn)
    return (w, S, up, dn) if full else w


def direct(V, F, Q):
    """O1: direct sum of signed solid angles / 4 pi, double-double accumulation."""
    V, F = _mesh(V, F)
    Q = _pts(Q)
    w = np.zeros(Q.shape[0])
    lib().oracle_direct(V, V.shape[0], F, F.shape[0], Q, Q.shape[0], w)
    return w


def gradient(V, F, Q, axis=(0.0, 0.0, 1.0), with_l1: bool = False):
    """O4: grad w per query, (n, 3) float64, with x0 = axis normalised; with
    with_l1=True also the per-query sum of edge-term norms / 4 pi."""
    V, F = _mesh(V, F)
    Q = _pts(Q)
    a = np.asarray(axis, dtype=np.float64)
    a = np.ascontiguousarray(a / np.linalg.norm(a))
    g = np.zeros((Q.shape[0], 3))
    l1 = np.zeros(Q.shape[0])
    lib().oracle_gradient(V, V.shape[0], F, F.shape[0], Q, Q.shape[0], a, g, l1)
    return (g, l1) if with_l1 else g


def weld(V, F):
    """(F with equal positions merged onto their smallest index, number of distinct positions)."""
    V, F = _mesh(V, F)
    out = np.zeros_like(F)
    n = lib().oracle_weld(V, V.shape[0], F, F.shape[0], out)
    return out, int(n)


def solid_angle(v0, v1, v2, p) -> float:
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (v0, v1, v2, p)]
    return float(lib().oracle_solid_angle(*a))


def distance(V, F, Q, cutoff: float, use_bins: bool = True):
    """min(distance to the soup, cutoff) per query."""
    V, F = _mesh(V, F)
    Q = _pts(Q)
    d = np.zeros(Q.shape[0])
    lib().oracle_distance2(V, V.shape[0], F, F.shape[0], Q, Q.shape[0], float(cutoff), int(use_bins), d)
    return d


def num_threads() -> int:
    return int(lib().oracle_num_threads())


# ---------------------------------------------------------------- parametric
# Ray directions tried in turn (Sec. 4.4.1 shoots another ray when a hit is
# ambiguous): +z, then three fixed unit vectors in general position.
PARAM_DIRS = np.array([[0.0, 0.0, 1.0], [0.36, 0.48, 0.8], [-0.48, 0.6, 0.64], [0.6, -0.64, 0.48]])


def bezier_curves(P):
    """The four boundary curves of each patch, counter-clockwise in (u, v):
    (n, 4 curves, 4 points, 3) from patches (n, 16, 3) (index 4 i + j, i along u)."""
    P = np.asarray(P, dtype=np.float64).reshape(-1, 4, 4, 3)
    c0 = P[:, :, 0]              # v = 0, u 0 -> 1
    c1 = P[:, 3, :]              # u = 1, v 0 -> 1
    c2 = P[:, ::-1, 3]           # v = 1, u 1 -> 0
    c3 = P[:, 0, ::-1]           # u = 0, v 1 -> 0
    return np.stack([c0, c1, c2, c3], axis=1)


def bezier_boundary(P):
    """Boundary curves (m, 4, 3) of the patch set: a curve and the same curve
    traversed backwards (equal control points) cancel, as interior mesh edges do
    (Sec. 4.1); what remains is kept with its net multiplicity."""
    C = bezier_curves(P).reshape(-1, 4, 3) + 0.0   # -0 and +0 are the same point
    net = {}
    first = {}
    for c in C:
        key = c.tobytes()
        rkey = c[::-1].copy().tobytes()
        if rkey in net:
            net[rkey] -= 1
        else:
            net[key] = net.get(key, 0) + 1
            first.setdefault(key, c)
    out = []
    for key, m in net.items():
        c = first[key]
        for _ in range(abs(m)):
            out.append(c if m > 0 else c[::-1])
    return np.array(out, dtype=np.float64).reshape(-1, 4, 3)


def param_chi(P, Q, d, tau, margin=1e-9):
    """(chi, ambiguous) along unit direction d for patches P (n, 16, 3)."""
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(-1, 48)
    Q = np.ascontiguousarray(Q, dtype=np.float64).reshape(-1, 3)
    chi = np.zeros(Q.shape[0], dtype=np.int32)
    amb = np.zeros(Q.shape[0], dtype=np.uint8)
    lib().oracle_param_chi(P.shape[0], P, Q.shape[0], Q, np.ascontiguousarray(d, dtype=np.float64), float(tau),
                           float(margin), chi, amb)
    return chi, amb.astype(bool)


def param_boundary(curves, Q, d, eps=1e-12, maxdepth=50):
    """Sum over the curves of the adaptive-GK15 integral of Alg. 2's f with x0 = d."""
    C = np.ascontiguousarray(curves, dtype=np.float64).reshape(-1, 12)
    Q = np.ascontiguousarray(Q, dtype=np.float64).reshape(-1, 3)
    S = np.zeros(Q.shape[0])
    lib().oracle_param_boundary(C.shape[0], C, Q.shape[0], Q, np.ascontiguousarray(d, dtype=np.float64),
                                float(eps), int(maxdepth), S)
    return S


def gk15_poly(k, a, b):
    """(K15, G7) of t^k on [a, b] (test of the quadrature table)."""
    K, G = ctypes.c_double(), ctypes.c_double()
    lib().oracle_gk15_poly(int(k), float(a), float(b), ctypes.byref(K), ctypes.byref(G))
    return K.value, G.value


def parametric(P, Q, eps=1e-12, tau_rel=1e-9, margin=1e-9, dirs=None):
    """Alg. 2: (w, chi, direction index) per query for cubic Bezier patches
    P (n, 16, 3).  Each query takes the first direction of ``dirs`` whose ray
    has no ambiguous hit; w = chi + boundary integral for that direction
    (direction index -1 and NaN where every direction is ambiguous)."""
    P = np.asarray(P, dtype=np.float64).reshape(-1, 16, 3)
    Q = np.asarray(Q, dtype=np.float64).reshape(-1, 3)
    dirs = PARAM_DIRS if dirs is None else np.asarray(dirs, dtype=np.float64)
    diag = float(np.linalg.norm(P.reshape(-1, 3).max(0) - P.reshape(-1, 3).min(0))) if P.size else 1.0
    curves = bezier_boundary(P)
    n = Q.shape[0]
    w = np.full(n, np.nan)
    chi = np.zeros(n, dtype=np.int32)
    di = np.full(n, -1, dtype=np.int32)
    todo = np.arange(n)
    for k, d in enumerate(dirs):
        if todo.size == 0:
            break
        c, amb = param_chi(P, Q[todo], d, tau_rel * diag, margin)
        sel = np.flatnonzero(~amb)
        if sel.size:
            S = param_boundary(curves, Q[todo[sel]], d, eps) if len(curves) else np.zeros(sel.size)
            # Alg. 2's integrand is 0/0 where the boundary passes exactly through
            # -x0 (v = 0 and X = 0): such a direction counts as ambiguous too
            bad = ~np.isfinite(S)
            amb[sel[bad]] = True
            good = sel[~bad]
            w[todo[good]] = c[good] + S[~bad]
            chi[todo[good]] = c[good]
            di[todo[good]] = k
        todo = todo[amb]
    return w, chi, di

