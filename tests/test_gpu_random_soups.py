"""Randomised soups against the oracle: uniform, lattice-snapped (coincident
vertices, shared coordinates), layered and clustered vertex sets; random
triangles with duplicates, flips and zero-area needles; queries on lattice
points, on vertical lines through vertices and far away; the ray along z, x, y
or the automatic choice, with and without welding; and multi-mesh plans built
from the same meshes, bit for bit against the single-mesh calls.  Crossing
counts must match the oracle exactly, w within the path's tolerance off the
surface (zero-area triangles count as surface)."""
import os

import numpy as np
import pytest

from tests._util import TOL_FP32, TOL_FP64, compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _soup(seed):
    rng = np.random.default_rng(seed)
    kind = seed % 4
    nv = int(rng.integers(3, 400))
    if kind == 0:
        V = rng.uniform(-1, 1, (nv, 3))
    elif kind == 1:
        V = np.round(rng.uniform(-1, 1, (nv, 3)) * 4) / 4
    elif kind == 2:
        V = rng.uniform(-1, 1, (nv, 3))
        V[:, 2] = np.round(V[:, 2] * 2) / 2
    else:
        base = rng.uniform(-1, 1, (max(3, nv // 4), 3))
        V = base[rng.integers(0, len(base), nv)] + rng.normal(0, 1e-3, (nv, 3)) * (rng.uniform(size=(nv, 1)) < 0.5)
    V = V.astype(np.float32) + np.float32(0.0)
    nf = int(rng.integers(1, 600))
    F = rng.integers(0, nv, (nf, 3)).astype(np.int32)
    if rng.uniform() < 0.5:
        d = F[rng.integers(0, nf, nf // 4 + 1)]
        flip = rng.uniform(size=len(d)) < 0.5
        d[flip] = d[flip][:, [1, 0, 2]]
        F = np.concatenate([F, d])
    nq = int(rng.integers(1, 1500))
    Q = rng.uniform(-1.3, 1.3, (nq, 3))
    if kind in (1, 2):
        Q[: nq // 3] = np.round(Q[: nq // 3] * 4) / 4
    k = min(nq // 4, nv)
    if k > 0:
        idx = rng.integers(0, nv, k)
        Q[-k:, :2] = V[idx, :2]
        Q[-k:, 2] = V[idx, 2] + rng.choice([-0.5, -0.1, 0.1, 0.7], k)
    far = rng.uniform(size=nq) < 0.1
    Q[far] *= rng.choice([1e3, 1e5, 1e6], int(far.sum()))[:, None]
    return V, F, Q.astype(np.float32)


def _weld(V, F):
    Vu, inv = np.unique(V, axis=0, return_inverse=True)
    return Vu.astype(np.float32), inv.reshape(-1)[F].astype(np.int32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _grid_points(lo, sp, dims):
    ii, jj, kk = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    P = np.stack([lo[0] + (ii + 0.5) * sp[0], lo[1] + (jj + 0.5) * sp[1], lo[2] + (kk + 0.5) * sp[2]], -1)
    return P.reshape(-1, 3).astype(np.float32)


@pytest.mark.parametrize("block", range(8))
def test_random_soups_against_oracle_and_plans(gwn, monkeypatch, block):
    kept = []
    for seed in range(block * 100, block * 100 + 100):
        V, F, Q = _soup(seed)
        axis = ["z", "x", "y", "auto"][(seed // 4) % 4]
        weld = seed % 3 == 0
        m = gwn.Mesh(_dev(V), _dev(F), weld=weld, axis=axis)
        a = "zxy".index(m.info()["axis"])
        perm = [a % 3, (a + 1) % 3, (a + 2) % 3]   # the oracle sees the mesh's frame
        Vo, Fo = _weld(V, F) if weld else (V, F)
        if seed % 5 == 0:
            monkeypatch.setenv("GWN_SPLIT_BOUNDARY", "1")
        for prec, tol in (("fp32", TOL_FP32), ("fp64", TOL_FP64)):
            w, chi = gwn.query_batch(m, _dev(Q), prec=prec, want_chi=True)
            compare(w.cpu().numpy(), chi.cpu().numpy(), Vo[:, perm], Fo, Q[:, perm], tol,
                    f"seed {seed} {prec} axis {axis} weld {weld}")
        monkeypatch.delenv("GWN_SPLIT_BOUNDARY", raising=False)
        if seed % 4 == 0:   # a small grid over the soup's box (70 samples per column)
            lo = V.min(0).astype(np.float64) - 0.1
            dims = (5, 4, 70)
            sp = (V.max(0).astype(np.float64) + 0.1 - lo) / np.array(dims)
            P = _grid_points(lo, sp, dims)
            for prec, tol in (("fp32", TOL_FP32), ("fp64", TOL_FP64)):
                wg, cg = gwn.query_grid(m, tuple(lo), tuple(sp), dims, prec=prec, want_chi=True)
                compare(wg.cpu().numpy().reshape(-1), cg.cpu().numpy().reshape(-1), Vo[:, perm], Fo, P[:, perm],
                        tol, f"seed {seed} grid {prec} axis {axis} weld {weld}")
        kept.append((m, Q))
    # the same meshes and points as one plan, in input and in Morton order
    monkeypatch.setenv("GWN_SPLIT_BOUNDARY", "0")
    meshes = [k[0] for k in kept]
    offs = np.concatenate([[0], np.cumsum([k[1].shape[0] for k in kept])]).astype(np.int64)
    Qd = _dev(np.concatenate([k[1] for k in kept]))
    for prec, order, iq in (("fp32", 0, 0), ("fp32", 2, 64), ("fp64", 2, 128)):
        chi = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
        w = gwn.MultiPlan(meshes, Qd, offs, chi_out=chi, prec=prec, order=order, item_queries=iq).run().clone()
        for i, mm in enumerate(meshes):
            a, b = int(offs[i]), int(offs[i + 1])
            wb, cb = gwn.query_batch(mm, Qd[a:b], prec=prec, want_chi=True)
            assert torch.equal(cb, chi[a:b]), (prec, order, i)
            assert torch.equal(wb, w[a:b]), (prec, order, i)
