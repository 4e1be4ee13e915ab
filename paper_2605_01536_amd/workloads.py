"""Seeded synthetic workloads (triangle soups and query sets).

This module only *generates inputs*: positions, triangle indices and query
points, drawn from NumPy's PCG64 generator with a fixed seed per workload.
It holds none of the winding-number arithmetic, so both the CPU oracle and
the GPU path can consume its output without sharing any of the method.

The shapes follow the paper's workload style (open, self-intersecting and
non-manifold soups, grid and random queries; Sec. 5.1 measures on open
meshes with queries in the bounding box), scaled to the five sizes used by
the tests and the benchmark:

* ``icosphere``      closed unit icosphere, 3 subdivisions (642 V, 1280 F),
                     10,000 uniform queries in [-1.5, 1.5]^3.
* ``torus_soup``     torus R=1, r=0.3 on a 250x200 quad grid (100k tris),
                     vertex noise, 20 % of triangles deleted, 5 % duplicated
                     with jitter; 1M uniform + 1M near-surface queries.
* ``ellipsoid_batch`` 256 soups, each a union of 1-8 random ellipsoids with
                     log-uniform triangle and query counts.
* ``opened_spheres`` 64 overlapping spheres/ellipsoids in [-1,1]^3, each a
                     UV grid with one random spherical cap removed (~1M
                     tris); queried on a dense regular grid.
* surrogate set      the opened-spheres generator at ~500k triangles.

All positions are produced in float64 and returned as float32; indices are
int32 with counter-clockwise (outward) orientation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Soup", "GridSpec", "icosphere", "uv_ellipsoid", "torus_soup",
    "opened_spheres", "ellipsoid_union", "ellipsoid_batch", "uniform_box",
    "near_surface", "config1", "config2", "config3", "config4", "config5",
    "grid_points",
]


@dataclass
class Soup:
    V: np.ndarray            # (nv, 3) float32
    F: np.ndarray            # (nf, 3) int32
    meta: dict = field(default_factory=dict)

    @property
    def nv(self) -> int:
        return int(self.V.shape[0])

    @property
    def nf(self) -> int:
        return int(self.F.shape[0])

    def bbox(self):
        V = self.V.astype(np.float64)
        return V.min(axis=0), V.max(axis=0)


@dataclass
class GridSpec:
    """Cell-centred regular grid: point (i,j,k) = float32(origin + (idx+0.5)*spacing),
    flattened with z fastest: out[(i*ny + j)*nz + k]."""
    origin: tuple
    spacing: tuple
    dims: tuple

    @property
    def n(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])


def grid_points(g: GridSpec, idx: np.ndarray | None = None) -> np.ndarray:
    """Coordinates of grid points (all, or the flat indices ``idx``) as float32,
    evaluated as float64 origin + (i + 0.5) * spacing then rounded once."""
    nx, ny, nz = (int(d) for d in g.dims)
    if idx is None:
        idx = np.arange(nx * ny * nz, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    k = idx % nz
    j = (idx // nz) % ny
    i = idx // (nz * ny)
    o = np.asarray(g.origin, dtype=np.float64)
    s = np.asarray(g.spacing, dtype=np.float64)
    P = np.stack([o[0] + (i + 0.5) * s[0], o[1] + (j + 0.5) * s[1], o[2] + (k + 0.5) * s[2]], axis=1)
    return P.astype(np.float32)


# ----------------------------------------------------------------------------
# primitive surfaces
# ----------------------------------------------------------------------------

def icosphere(levels: int = 3) -> Soup:
    """Icosahedron refined by midpoint subdivision, new vertices projected to the
    unit sphere in float64; outward counter-clockwise faces."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    V = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(levels):
        cache = {}
        newF = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]

        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            newF += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = newF
    Va = np.array(V, dtype=np.float64)
    Fa = np.array(F, dtype=np.int32)
    _orient_outward(Va, Fa)
    return Soup(Va.astype(np.float32), Fa, {"kind": "icosphere", "levels": levels})


def _orient_outward(V: np.ndarray, F: np.ndarray) -> None:
    """Flip all faces if the signed volume of a closed surface is negative."""
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum()
    if vol < 0:
        F[:, [1, 2]] = F[:, [2, 1]]


def uv_ellipsoid(n_lat: int, n_lon: int) -> tuple[np.ndarray, np.ndarray]:
    """Closed UV sphere of unit radius: two pole vertices plus (n_lat-1) rings of
    n_lon vertices; 2*n_lon*(n_lat-1) triangles, outward orientation."""
    rings = []
    for i in range(1, n_lat):
        th = math.pi * i / n_lat
        ph = 2.0 * math.pi * np.arange(n_lon) / n_lon
        rings.append(np.stack([math.sin(th) * np.cos(ph), math.sin(th) * np.sin(ph),
                               np.full(n_lon, math.cos(th))], axis=1))
    V = np.concatenate([np.array([[0.0, 0.0, 1.0]]), *rings, np.array([[0.0, 0.0, -1.0]])], axis=0)
    south = V.shape[0] - 1
    F = []
    j = np.arange(n_lon)
    jn = (j + 1) % n_lon
    # north fan
    F.append(np.stack([np.zeros(n_lon, dtype=np.int64), 1 + j, 1 + jn], axis=1))
    for r in range(n_lat - 2):
        a = 1 + r * n_lon + j
        b = 1 + r * n_lon + jn
        c = 1 + (r + 1) * n_lon + j
        d = 1 + (r + 1) * n_lon + jn
        F.append(np.stack([a, c, d], axis=1))
        F.append(np.stack([a, d, b], axis=1))
    last = 1 + (n_lat - 2) * n_lon
    F.append(np.stack([last + j, np.full(n_lon, south), last + jn], axis=1))
    F = np.concatenate(F, axis=0).astype(np.int32)
    _orient_outward(V, F)
    return V, F


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _lat_lon_for(n_tris: int) -> tuple[int, int]:
    n_lat = max(3, int(round(math.sqrt(max(n_tris, 8) / 4.0))))
    return n_lat, 2 * n_lat


def uniform_box(rng: np.random.Generator, n: int, lo, hi) -> np.ndarray:
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return (lo + (hi - lo) * rng.random((n, 3))).astype(np.float32)


def near_surface(rng: np.random.Generator, soup: Soup, n: int, sigma: float) -> np.ndarray:
    """Area-weighted random surface points (uniform barycentric) plus N(0, sigma^2 I)."""
    V = soup.V.astype(np.float64)
    a, b, c = V[soup.F[:, 0]], V[soup.F[:, 1]], V[soup.F[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    p = area / area.sum()
    t = rng.choice(soup.nf, size=n, p=p)
    u = rng.random(n)
    v = rng.random(n)
    flip = u + v > 1.0
    u[flip], v[flip] = 1.0 - u[flip], 1.0 - v[flip]
    P = a[t] + u[:, None] * (b[t] - a[t]) + v[:, None] * (c[t] - a[t])
    P += sigma * rng.standard_normal((n, 3))
    return P.astype(np.float32)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def torus_soup(seed: int = 2, n_u: int = 250, n_v: int = 200, R: float = 1.0, r: float = 0.3,
               noise: float = 1e-3, delete_frac: float = 0.2, dup_frac: float = 0.05) -> Soup:
    rng = np.random.default_rng(seed)
    u = 2 * math.pi * np.arange(n_u) / n_u
    v = 2 * math.pi * np.arange(n_v) / n_v
    U, Vv = np.meshgrid(u, v, indexing="ij")
    X = np.stack([(R + r * np.cos(Vv)) * np.cos(U), (R + r * np.cos(Vv)) * np.sin(U), r * np.sin(Vv)], axis=-1)
    V = X.reshape(-1, 3)
    i, j = np.meshgrid(np.arange(n_u), np.arange(n_v), indexing="ij")
    i, j = i.ravel(), j.ravel()
    idx = lambda a, b: (a % n_u) * n_v + (b % n_v)
    F = np.concatenate([np.stack([idx(i, j), idx(i + 1, j), idx(i + 1, j + 1)], 1),
                        np.stack([idx(i, j), idx(i + 1, j + 1), idx(i, j + 1)], 1)], 0).astype(np.int32)
    _orient_outward(V, F)
    V = V + noise * rng.standard_normal(V.shape)
    nf0 = F.shape[0]
    keep = rng.permutation(nf0)[: nf0 - int(round(delete_frac * nf0))]
    keep.sort()
    F = F[keep]
    ndup = int(round(dup_frac * nf0))
    pick = rng.choice(F.shape[0], size=ndup, replace=False)
    newV = V[F[pick].reshape(-1)] + noise * rng.standard_normal((3 * ndup, 3))
    newF = (V.shape[0] + np.arange(3 * ndup)).reshape(ndup, 3)
    V = np.concatenate([V, newV], 0)
    F = np.concatenate([F, newF], 0).astype(np.int32)
    return Soup(V.astype(np.float32), F, {"kind": "torus_soup", "seed": seed})


def opened_spheres(seed: int = 4, n_surf: int = 64, tris_per_surf: int = 19600,
                   cap_deg=(15.0, 75.0), semi=(0.15, 0.5)) -> Soup:
    """Overlapping spheres (p=0.5) and ellipsoids inside [-1,1]^3, each a closed UV
    grid with the triangles whose centroid direction lies in a random spherical
    cap removed (one boundary loop per surface)."""
    rng = np.random.default_rng(seed)
    n_lat = max(3, int(round(math.sqrt(tris_per_surf / 4.0))))
    n_lon = 2 * n_lat
    V0, F0 = uv_ellipsoid(n_lat, n_lon)
    cen0 = V0[F0].mean(axis=1)
    cen0 /= np.linalg.norm(cen0, axis=1, keepdims=True)
    Vs, Fs = [], []
    off = 0
    for _ in range(n_surf):
        if rng.random() < 0.5:
            ax = np.full(3, rng.uniform(*semi))
        else:
            ax = rng.uniform(semi[0], semi[1], size=3)
        Rm = _random_rotation(rng)
        Rb = ax.max()
        c = rng.uniform(-1.0 + Rb, 1.0 - Rb, size=3)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        half = math.radians(rng.uniform(*cap_deg))
        keep = cen0 @ d <= math.cos(half)
        V = (V0 * ax) @ Rm.T + c
        Vs.append(V)
        Fs.append(F0[keep] + off)
        off += V.shape[0]
    V = np.concatenate(Vs, 0)
    F = np.concatenate(Fs, 0).astype(np.int32)
    return Soup(V.astype(np.float32), F, {"kind": "opened_spheres", "seed": seed,
                                          "n_surf": n_surf, "n_lat": n_lat, "n_lon": n_lon})


def ellipsoid_union(rng: np.random.Generator, n_tris: int, remove_frac: float) -> Soup:
    ne = int(rng.integers(1, 9))
    axes = rng.uniform(0.2, 1.0, size=(ne, 3))
    cen = rng.uniform(-1.0, 1.0, size=(ne, 3))
    area = axes[:, 0] * axes[:, 1] + axes[:, 1] * axes[:, 2] + axes[:, 0] * axes[:, 2]
    share = area / area.sum()
    Vs, Fs = [], []
    off = 0
    for e in range(ne):
        n_lat, n_lon = _lat_lon_for(int(share[e] * n_tris))
        V, F = uv_ellipsoid(n_lat, n_lon)
        V = (V * axes[e]) @ _random_rotation(rng).T + cen[e]
        Vs.append(V)
        Fs.append(F + off)
        off += V.shape[0]
    V = np.concatenate(Vs, 0)
    F = np.concatenate(Fs, 0)
    nrem = int(round(remove_frac * F.shape[0]))
    keep = np.sort(rng.permutation(F.shape[0])[nrem:])
    return Soup(V.astype(np.float32), F[keep].astype(np.int32), {"kind": "ellipsoid_union", "n_ell": ne})


def ellipsoid_batch(seed: int = 3, n_mesh: int = 256, tri_range=(1_000, 200_000),
                    q_range=(10_000, 1_000_000)):
    """Many soups of uneven size; returns (soups, queries) with queries uniform
    in each soup's bounding box."""
    rng = np.random.default_rng(seed)
    soups, queries = [], []
    for _ in range(n_mesh):
        nt = int(round(math.exp(rng.uniform(math.log(tri_range[0]), math.log(tri_range[1])))))
        rf = rng.uniform(0.0, 0.3)
        nq = int(round(math.exp(rng.uniform(math.log(q_range[0]), math.log(q_range[1])))))
        s = ellipsoid_union(rng, nt, rf)
        lo, hi = s.bbox()
        soups.append(s)
        queries.append(uniform_box(rng, nq, lo, hi))
    return soups, queries


# ----------------------------------------------------------------------------
# the five named configurations
# ----------------------------------------------------------------------------

def wavy_sheets(seed: int = 6, n_sheets: int = 6, n: int = 40) -> Soup:
    """n_sheets open, gently waving sheets stacked along z over [-1, 1]^2, each an
    n x n vertex grid: vertical rays cross every sheet, horizontal ones few (the
    case the ray-axis choice is for)."""
    rng = np.random.default_rng(seed)
    u, v = np.meshgrid(np.linspace(-1, 1, n), np.linspace(-1, 1, n), indexing="ij")
    idx = np.arange(n * n).reshape(n, n)
    a, b, c, d = idx[:-1, :-1], idx[1:, :-1], idx[1:, 1:], idx[:-1, 1:]
    quad = np.concatenate([np.stack([a, b, c], -1).reshape(-1, 3), np.stack([a, c, d], -1).reshape(-1, 3)])
    Vs, Fs = [], []
    for k in range(n_sheets):
        ph = rng.uniform(0, 2 * np.pi, size=2)
        z = (2.0 * (k + 0.5) / n_sheets - 1.0) * 0.9 + 0.04 * np.sin(3 * u + ph[0]) * np.cos(2 * v + ph[1])
        Vs.append(np.stack([u, v, z], -1).reshape(-1, 3))
        Fs.append(quad + k * n * n)
    return Soup(np.concatenate(Vs).astype(np.float32), np.concatenate(Fs).astype(np.int32), {"seed": seed})


def explode(soup: Soup, seed: int | None = None) -> Soup:
    """The same triangles with three private vertex copies each, as an STL file
    stores them (no shared indices); with a seed, the triangle order is shuffled."""
    V = soup.V[soup.F.reshape(-1)].astype(np.float32)
    F = np.arange(V.shape[0], dtype=np.int32).reshape(-1, 3)
    if seed is not None:
        F = F[np.random.default_rng(seed).permutation(F.shape[0])]
    return Soup(V, np.ascontiguousarray(F))


def config1(n_query: int = 10_000):
    """Closed icosphere, 1280 triangles, uniform queries in [-1.5, 1.5]^3 (seed 1)."""
    rng = np.random.default_rng(1)
    s = icosphere(3)
    Q = uniform_box(rng, n_query, (-1.5,) * 3, (1.5,) * 3)
    return s, Q


def config2(n_uniform: int = 1_000_000, n_near: int = 1_000_000):
    """Open torus soup (~85k triangles) with uniform-in-bbox and near-surface queries (seed 2)."""
    s = torus_soup(seed=2)
    rng = np.random.default_rng(102)
    lo, hi = s.bbox()
    diag = float(np.linalg.norm(hi - lo))
    Qu = uniform_box(rng, n_uniform, lo, hi)
    Qn = near_surface(rng, s, n_near, 1e-3 * diag)
    return s, np.concatenate([Qu, Qn], 0)


def config3(n_mesh: int = 256, **kw):
    """256 ellipsoid-union soups with log-uniform triangle and query counts (seed 3)."""
    return ellipsoid_batch(seed=3, n_mesh=n_mesh, **kw)


def config4(n: int = 512, **kw):
    """~1M-triangle opened-spheres soup queried on an n^3 cell-centred grid over [-1,1]^3 (seed 4)."""
    s = opened_spheres(seed=4, **kw)
    g = GridSpec(origin=(-1.0, -1.0, -1.0), spacing=(2.0 / n,) * 3, dims=(n, n, n))
    return s, g


def config5(n_train: int = 10_000_000, n_infer: int = 16_000_000):
    """~500k-triangle opened-spheres soup; uniform training and inference points in [-1,1]^3 (seed 5)."""
    s = opened_spheres(seed=5, tris_per_surf=9216)
    rng = np.random.default_rng(105)
    Xtr = uniform_box(rng, n_train, (-1.0,) * 3, (1.0,) * 3) if n_train else None
    Xin = uniform_box(rng, n_infer, (-1.0,) * 3, (1.0,) * 3) if n_infer else None
    return s, Xtr, Xin
