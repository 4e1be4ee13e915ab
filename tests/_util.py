"""Shared helpers for the test suite (inputs and comparisons only)."""
import numpy as np

import oracle as O

TOL_FP32 = 1e-4   # |w_gpu - w_oracle| bound for the FP32 path
TOL_FP64 = 1e-5   # ... and for the FP64 path
NEAR_FRAC = 1e-4  # queries closer than this fraction of the bbox diagonal are excluded from w checks


def diag_of(V):
    V = np.asarray(V, np.float64)
    return float(np.linalg.norm(V.max(0) - V.min(0)))


def off_surface_mask(V, F, Q, frac=NEAR_FRAC):
    cut = frac * diag_of(V)
    return O.distance(V, F, Q, cut * 2.0) > cut


def compare(w_gpu, chi_gpu, V, F, Q, tol, label=""):
    """chi must match the oracle bit for bit; w within tol where defined."""
    w_o, S, up, dn = O.antipodal(V, F, Q, full=True)
    chi_bad = np.flatnonzero(np.asarray(chi_gpu) != up)
    assert chi_bad.size == 0, f"{label}: chi mismatch at {chi_bad[:10]} gpu={np.asarray(chi_gpu)[chi_bad[:10]]} oracle={up[chi_bad[:10]]}"
    m = off_surface_mask(V, F, Q)
    err = np.abs(np.asarray(w_gpu, np.float64) - w_o)
    e = float(err[m].max()) if m.any() else 0.0
    assert e <= tol, f"{label}: max |w - oracle| = {e:.3e} > {tol:.1e} (n={m.sum()})"
    return e, int(m.sum())


def fan_soup(lengths, seed):
    """One triangle fan per entry: a wavy polygon of L boundary vertices around a
    raised centre, the fans scattered over [-1, 1]^3 (boundary loops of exactly
    those lengths)."""
    rng = np.random.default_rng(seed)
    Vs, Fs, nv = [], [], 0
    for k, L in enumerate(lengths):
        c = rng.uniform(-0.6, 0.6, size=3)
        r = rng.uniform(0.15, 0.4)
        a = np.sort(rng.uniform(0, 2 * np.pi, size=L)) if k % 2 else np.linspace(0, 2 * np.pi, L, endpoint=False)
        ring = np.stack([c[0] + r * np.cos(a), c[1] + r * np.sin(a) * rng.uniform(0.5, 1.0),
                         c[2] + 0.3 * r * np.sin(3 * a + k)], axis=1)
        V = np.concatenate([ring, [c + [0, 0, rng.uniform(-0.2, 0.2)]]])
        F = np.stack([np.arange(L), (np.arange(L) + 1) % L, np.full(L, L)], axis=1)
        if k % 3 == 1:
            F = F[:, [1, 0, 2]]                         # the other orientation
        Vs.append(V)
        Fs.append(F + nv)
        nv += L + 1
    return np.concatenate(Vs).astype(np.float32), np.concatenate(Fs).astype(np.int32)


def flat_bezier_patch(x0, x1, y0, y1, z=0.0):
    """A planar bicubic patch over [x0, x1] x [y0, y1] at height z (normal +z), (16, 3)."""
    P = np.zeros((4, 4, 3))
    for i in range(4):
        for j in range(4):
            P[i, j] = [x0 + (x1 - x0) * i / 3, y0 + (y1 - y0) * j / 3, z]
    return P.reshape(16, 3)


def bezier_cube():
    """The unit cube as six planar bicubic patches with outward normals, (6, 16, 3)."""
    faces = [((0, 0, 0), (0, 1, 0), (1, 0, 0)), ((0, 0, 1), (1, 0, 0), (0, 1, 0)),
             ((0, 0, 0), (1, 0, 0), (0, 0, 1)), ((0, 1, 0), (0, 0, 1), (1, 0, 0)),
             ((0, 0, 0), (0, 0, 1), (0, 1, 0)), ((1, 0, 0), (0, 1, 0), (0, 0, 1))]
    out = []
    for o, U, V in faces:
        o, U, V = (np.array(x, dtype=np.float64) for x in (o, U, V))
        out.append(np.array([o + U * i / 3 + V * j / 3 for i in range(4) for j in range(4)]))
    return np.array(out)


def bezier_tessellate(P, n):
    """(V float32, F int32): each cubic patch of P (m, 16, 3) sampled on an
    (n + 1) x (n + 1) parameter grid, two triangles per cell, same orientation."""
    P = np.asarray(P, dtype=np.float64).reshape(-1, 4, 4, 3)
    t = np.linspace(0.0, 1.0, n + 1)
    s = 1.0 - t
    B = np.stack([s ** 3, 3 * s * s * t, 3 * s * t * t, t ** 3], axis=1)
    Vs, Fs, off = [], [], 0
    idx = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
    a, b, c, d = idx[:-1, :-1].ravel(), idx[1:, :-1].ravel(), idx[1:, 1:].ravel(), idx[:-1, 1:].ravel()
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    for Pk in P:
        S = np.einsum("ai,bj,ijc->abc", B, B, Pk)
        Vs.append(S.reshape(-1, 3))
        Fs.append(F + off)
        off += S.shape[0] * S.shape[1]
    return np.concatenate(Vs).astype(np.float32), np.concatenate(Fs).astype(np.int32)
