"""GPU parity of the parametric-surface path (cubic Bezier patches, Alg. 2's
decomposition) against the CPU oracle, closed forms and invariants."""
import numpy as np
import pytest

import oracle as O
from tests._util import bezier_cube, bezier_tessellate, flat_bezier_patch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_PARAM = 1e-7   # both sides FP64; quadrature tolerances 1e-11 (GPU) and 1e-12 (oracle) per interval


def _dev(P):
    return torch.from_numpy(np.ascontiguousarray(P, dtype=np.float64)).cuda()


def _q(Q):
    return torch.from_numpy(np.ascontiguousarray(Q, dtype=np.float32)).cuda()


def _far(P, Q, cut):
    V, F = bezier_tessellate(P, 64)
    return O.distance(V, F, np.asarray(Q, np.float32), cut) >= cut


def _compare(gwn, P, Q, label, tol=TOL_PARAM, cut=1e-3):
    Q = np.asarray(Q, np.float32)
    pt = gwn.Patches(_dev(P))
    w, chi, dr = pt.query(_q(Q), want_chi=True)
    torch.cuda.synchronize()
    w, chi, dr = w.cpu().numpy(), chi.cpu().numpy(), dr.cpu().numpy()
    wo, co, do = O.parametric(P, Q.astype(np.float64))
    far = _far(P, Q, cut) & (dr >= 0) & (do >= 0)
    assert far.sum() > 0.8 * len(Q), f"{label}: only {far.sum()} of {len(Q)} comparable"
    err = np.abs(w - wo)[far]
    assert err.max() <= tol, f"{label}: max |w - oracle| = {err.max():.3e}"
    same = far & (dr == do)
    assert np.array_equal(chi[same], co[same]), f"{label}: chi differs"
    return w, chi, dr


@pytest.mark.parametrize("h", [0.05, 0.7, 3.0])
def test_flat_square_closed_form(gwn, h):
    P = flat_bezier_patch(-1, 1, -1, 1)[None]
    h = float(np.float32(h))   # the query as the FP32 input holds it
    exact = np.arcsin(1.0 / (1.0 + h * h)) / np.pi
    pt = gwn.Patches(_dev(P))
    w, chi, dr = pt.query(_q([[0, 0, h], [0, 0, -h], [0.3, -0.2, h]]), want_chi=True)
    w = w.cpu().numpy()
    assert abs(w[0] + exact) < 1e-12 and abs(w[1] - exact) < 1e-12
    assert pt.info()["ncurves"] == 4


def test_closed_cube(gwn):
    C = bezier_cube()
    pt = gwn.Patches(_dev(C))
    assert pt.info()["ncurves"] == 0
    Q = np.random.default_rng(0).uniform(-0.5, 1.5, size=(2000, 3)).astype(np.float32)
    w, chi, dr = pt.query(_q(Q), want_chi=True)
    inside = np.all((Q > 0) & (Q < 1), axis=1)
    assert np.array_equal(w.cpu().numpy(), inside.astype(np.float64))
    assert (dr.cpu().numpy() >= 0).all()


@pytest.mark.parametrize("seed", range(3))
def test_random_patches_against_oracle(gwn, seed):
    # cubic patches with control points uniform in the unit cube (the paper's
    # synthetic benchmark) and queries around them
    rng = np.random.default_rng(300 + seed)
    P = rng.uniform(0, 1, size=(int(rng.integers(2, 7)), 16, 3))
    Q = rng.uniform(-0.5, 1.5, size=(300, 3))
    _compare(gwn, P, Q, f"random{seed}")


def test_closed_curved_pillow(gwn):
    # two curved patches sharing their four boundary curves (a closed surface):
    # every curve cancels and w is the crossing count, agreeing with the oracle
    rng = np.random.default_rng(11)
    A = rng.uniform(0, 1, size=(4, 4, 3))
    B = A.copy()
    B[1:3, 1:3] += rng.uniform(-0.6, 0.6, size=(2, 2, 3))   # interior control points only
    B = B[::-1]                                              # the other orientation
    P = np.stack([A.reshape(16, 3), B.reshape(16, 3)])
    assert len(O.bezier_boundary(P)) == 0
    Q = rng.uniform(-0.3, 1.3, size=(400, 3))
    w, chi, dr = _compare(gwn, P, Q, "pillow")
    assert np.array_equal(w[dr >= 0], np.round(w[dr >= 0]))


def test_shared_edges_and_orientation(gwn):
    # a strip of four patches sharing edges (curves cancel pairwise), and the
    # strip reversed (w changes sign)
    rng = np.random.default_rng(21)
    G = np.zeros((13, 4, 3))
    for i in range(13):
        for j in range(4):
            G[i, j] = [i / 4.0, j / 3.0, 0.3 * np.sin(i / 2.0) * np.cos(j)]
    G[:, :, 2] += rng.uniform(-0.05, 0.05, size=(13, 4))
    P = np.stack([G[3 * k:3 * k + 4].reshape(16, 3) for k in range(4)])
    assert len(O.bezier_boundary(P)) == 10
    Q = rng.uniform([-0.3, -0.3, -0.6], [3.3, 1.3, 0.6], size=(300, 3))
    w, _, dr = _compare(gwn, P, Q, "strip")
    Pr = P.reshape(-1, 4, 4, 3)[:, ::-1].reshape(-1, 16, 3)
    wr = gwn.Patches(_dev(Pr)).query(_q(Q)).cpu().numpy()
    ok = np.isfinite(w) & np.isfinite(wr)
    assert np.abs(w + wr)[ok].max() < 1e-9


def test_edge_cases(gwn):
    P = np.random.default_rng(3).uniform(0, 1, size=(2, 16, 3))
    pt = gwn.Patches(_dev(P))
    assert pt.query(torch.zeros((0, 3), device="cuda")).numel() == 0
    empty = gwn.Patches(torch.zeros((0, 16, 3), dtype=torch.float64, device="cuda"))
    w = empty.query(_q(np.random.default_rng(4).uniform(size=(100, 3))))
    assert float(w.abs().max()) == 0.0
    Pn = P.copy()
    Pn[1, 5, 2] = np.nan
    with pytest.raises(gwn.GwnError) as ei:
        gwn.Patches(_dev(Pn))
    assert ei.value.status == 1


@pytest.mark.parametrize("seed", range(2))
def test_grid_ray_reuse_equals_single_rays(gwn, seed):
    # the column path (one line per column, samples count the crossings above
    # them) against single rays at the same points and the oracle; the grid
    # puts columns exactly through control points and patch corners (ambiguous
    # lines fall back to single rays)
    rng = np.random.default_rng(500 + seed)
    P = np.round(rng.uniform(0, 1, size=(5, 16, 3)) * 8) / 8
    dims = (9, 11, 70)
    origin, spacing = (-0.0625, -0.0625, -0.3), (0.125, 0.125, 1.6 / 70)
    pt = gwn.Patches(_dev(P))
    wg, cg, dg = pt.query_grid(origin, spacing, dims, want_chi=True)
    ii, jj, kk = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    Q = np.stack([(np.float64(origin[c]) + ([ii, jj, kk][c].ravel() + 0.5) * spacing[c]) for c in range(3)],
                 axis=1).astype(np.float32)
    wb, cb, db = pt.query(_q(Q), want_chi=True)
    wg, cg, dg = wg.cpu().numpy(), cg.cpu().numpy(), dg.cpu().numpy()
    wb, cb, db = wb.cpu().numpy(), cb.cpu().numpy(), db.cpu().numpy()
    same = (dg == db) & (dg >= 0)
    assert same.mean() > 0.5
    assert np.array_equal(cg[same], cb[same])
    ok = np.isfinite(wg) & np.isfinite(wb)
    assert np.abs(wg - wb)[ok].max() < 1e-9
    _compare(gwn, P, Q[::7], f"grid{seed}")



def test_many_curves_against_oracle(gwn):
    # 100 random patches (400 boundary curves) as in the benchmark: the wave's
    # interval queue refills and runs near its capacity
    rng = np.random.default_rng(7)
    P = rng.uniform(0, 1, size=(100, 16, 3))
    Q = rng.uniform(-0.2, 1.2, size=(400, 3))
    _compare(gwn, P, Q, "100 patches", cut=1e-3)


def test_rays_grazing_boundary_curves(gwn):
    # queries straight below and above points of curved boundary curves (and
    # corners): their +z rays pass within the FP32 rounding of the curve, where
    # the crossing count and the boundary integrand are both near their jumps;
    # the GPU and the oracle re-shoot or resolve them alike
    rng = np.random.default_rng(31)
    P = rng.uniform(0, 1, size=(3, 16, 3))
    C = O.bezier_boundary(P)
    pts = []
    for c in C[::2]:
        for t in (0.0, 1.0 / 3.0, 0.5, 0.71):
            b = np.array([(1 - t) ** 3, 3 * (1 - t) ** 2 * t, 3 * (1 - t) * t * t, t ** 3])
            X = b @ c
            pts += [X - [0, 0, 0.4], X + [0, 0, 0.3]]
    Q = np.array(pts, dtype=np.float32)
    pt = gwn.Patches(_dev(P))
    w, chi, dr = pt.query(_q(Q), want_chi=True)
    w, dr = w.cpu().numpy(), dr.cpu().numpy()
    wo, co, do = O.parametric(P, Q.astype(np.float64))
    ok = (dr >= 0) & (do >= 0) & _far(P, Q, 1e-3)
    assert ok.sum() > 0.5 * len(Q)
    assert np.isfinite(w[dr >= 0]).all()
    assert np.abs(w - wo)[ok].max() < 1e-6


def _stacked_bumps(n, rng):
    # n copies of one curved patch (a bump over [-1, 1]^2) stacked 0.01 apart
    # in z with small shifts in x and y: a vertical line meets all of them, so
    # more cells wait than the shared queues hold and lanes follow the rest alone
    B = flat_bezier_patch(-1, 1, -1, 1).reshape(4, 4, 3).copy()
    B[1:3, 1:3, 2] += 0.3
    P = np.stack([B.reshape(16, 3) + [rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05), 0.01 * k]
                  for k in range(n)])
    return P


def test_stacked_patches_overflow_the_cell_queues(gwn):
    rng = np.random.default_rng(41)
    P = _stacked_bumps(256, rng)
    Q = np.concatenate([rng.uniform([-0.6, -0.6, -0.5], [0.6, 0.6, 3.5], size=(60, 3)),
                        rng.uniform([-0.6, -0.6, 0.0], [0.6, 0.6, 0.3], size=(20, 3))])
    w, chi, dr = _compare(gwn, P, Q, "stacked", cut=1e-3)
    # the grid path (a workgroup per column) against single rays at the same points
    pt = gwn.Patches(_dev(P))
    dims = (6, 5, 40)
    origin, spacing = (-0.55, -0.5, -0.4), (0.2, 0.2, 0.1)
    wg, cg, dg = pt.query_grid(origin, spacing, dims, want_chi=True)
    ii, jj, kk = np.meshgrid(*[np.arange(m) for m in dims], indexing="ij")
    G = np.stack([(np.float64(origin[c]) + ([ii, jj, kk][c].ravel() + 0.5) * spacing[c]) for c in range(3)],
                 axis=1).astype(np.float32)
    wb, cb, db = pt.query(_q(G), want_chi=True)
    wg, cg, dg = wg.cpu().numpy(), cg.cpu().numpy(), dg.cpu().numpy()
    wb, cb, db = wb.cpu().numpy(), cb.cpu().numpy(), db.cpu().numpy()
    same = (dg == db) & (dg >= 0)
    assert same.mean() > 0.5
    assert np.array_equal(cg[same], cb[same])
    ok = np.isfinite(wg) & np.isfinite(wb)
    assert np.abs(wg - wb)[ok].max() < 1e-9


def test_grid_calls_on_several_streams(gwn):
    # a grid call forks its boundary term onto the handle's side stream and
    # joins it back: calls on different streams, back to back without waiting
    # in between, each give what one call alone gives
    rng = np.random.default_rng(61)
    P = rng.uniform(0, 1, size=(8, 16, 3))
    pt = gwn.Patches(_dev(P))
    dims = (7, 6, 50)
    origin, spacing = (-0.2, -0.2, -0.2), (0.2, 0.24, 0.028)
    ref = pt.query_grid(origin, spacing, dims)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    n = int(np.prod(dims))
    outs = [torch.full((n,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(4)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.current_stream(), torch.cuda.Stream()]
    for o, s in zip(outs, streams):
        pt.query_grid(origin, spacing, dims, out=o, stream=s)
    torch.cuda.synchronize()
    for o in outs:
        assert np.array_equal(o.cpu().numpy(), ref, equal_nan=True)
    pt.close()
