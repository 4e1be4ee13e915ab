"""The ray axis option: meshes built for x0 = +x, +y or the automatically chosen
axis (least projected area).  w and its gradient must not depend on the axis
(Prop. 4.2); the crossing counts along axis a must equal the oracle's +z counts
for the cyclically permuted input whose third coordinate is a, bit for bit."""
import numpy as np
import pytest

import oracle as O
from paper_2605_01536_amd import workloads as W
from tests._util import TOL_FP32, TOL_FP64, off_surface_mask

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FRAME = {"z": [0, 1, 2], "x": [1, 2, 0], "y": [2, 0, 1]}   # world components of the frame axes


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _check(G, V, F, Q, axis, prec):
    m = G.Mesh(_dev(V), _dev(F), axis=axis)
    assert m.info()["axis"] == axis
    w, chi = G.query_batch(m, _dev(Q), prec=prec, want_chi=True)
    p = FRAME[axis]
    up, _ = O.chi(V[:, p], F, Q[:, p])
    assert np.array_equal(chi.cpu().numpy(), up)
    mask = off_surface_mask(V, F, Q)
    err = np.abs(w.cpu().numpy().astype(np.float64) - O.antipodal(V, F, Q))[mask]
    assert err.max() <= (TOL_FP32 if prec == "fp32" else TOL_FP64)
    return m


@pytest.mark.parametrize("axis", ["x", "y"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_axis_tiny_and_torus(gwn, axis, prec):
    rng = np.random.default_rng(31)
    V = (np.round(rng.uniform(-1, 1, size=(120, 3)) * 16) / 16).astype(np.float32)
    F = rng.integers(0, 120, size=(40, 3)).astype(np.int32)
    Q = (np.round(rng.uniform(-1.2, 1.2, size=(1500, 3)) * 16) / 16).astype(np.float32)
    _check(gwn, V, F, Q, axis, prec)
    s, Q = W.config2(n_uniform=1500, n_near=1500)
    _check(gwn, s.V, s.F, Q, axis, prec)


@pytest.mark.parametrize("axis", ["x", "y"])
def test_axis_grid_gradient_crossings(gwn, axis):
    s = W.opened_spheres(seed=44, n_surf=5, tris_per_surf=500)
    mz = gwn.Mesh(_dev(s.V), _dev(s.F))
    ma = gwn.Mesh(_dev(s.V), _dev(s.F), axis=axis)
    g = W.GridSpec(origin=(-1.05, -0.97, -1.1), spacing=(0.1, 0.09, 0.007), dims=(21, 23, 313))
    P = W.grid_points(g)
    w, chi = gwn.query_grid(ma, g.origin, g.spacing, g.dims, want_chi=True)
    p = FRAME[axis]
    up, dn = O.chi(s.V[:, p], s.F, P[:, p])
    assert np.array_equal(chi.cpu().numpy(), up)
    wz = gwn.query_batch(mz, _dev(P))
    mask = off_surface_mask(s.V, s.F, P)
    assert float((w - wz).abs().cpu().numpy()[mask].max()) < 2e-6
    # gradients against the oracle taken with the same axis and with +z
    Q = P[::37]
    ga = gwn.query_gradient(ma, _dev(Q), prec="fp64").cpu().numpy()
    ref = O.gradient(s.V, s.F, Q, axis=np.eye(3)[p[2]])
    m2 = off_surface_mask(s.V, s.F, Q)
    assert np.abs(ga - ref)[m2].max() < 1e-9
    # both crossing directions
    cu, cd = gwn.query_crossings(ma, _dev(P))
    assert np.array_equal(cu.cpu().numpy(), up) and np.array_equal(cd.cpu().numpy(), dn)
    # the direct sum does not care about the frame
    wd = gwn.query_direct(ma, _dev(Q), prec="fp64").cpu().numpy()
    assert np.abs(wd - O.direct(s.V, s.F, Q))[m2].max() < 1e-9


def test_auto_axis_picks_least_projected_area(gwn):
    # a stack of wavy sheets over x-y: vertical rays cross every sheet, rays along
    # x or y cross few
    s = W.wavy_sheets(seed=3, n_sheets=6, n=40)
    V, F = s.V, s.F
    rng = np.random.default_rng(3)
    m = gwn.Mesh(_dev(V), _dev(F), axis="auto")
    info = m.info()
    A = info["proj_area"]
    assert info["axis"] in ("x", "y") and A[2] > 5 * max(A[0], A[1])
    Q = rng.uniform(-1.1, 1.1, size=(3000, 3)).astype(np.float32)
    w, chi = gwn.query_batch(m, _dev(Q), want_chi=True)
    p = FRAME[info["axis"]]
    assert np.array_equal(chi.cpu().numpy(), O.chi(V[:, p], F, Q[:, p])[0])
    mask = off_surface_mask(V, F, Q)
    assert np.abs(w.cpu().numpy() - O.antipodal(V, F, Q))[mask].max() < TOL_FP32


def test_multi_plan_with_mixed_axes(gwn):
    soups = [W.opened_spheres(seed=50 + i, n_surf=2, tris_per_surf=300) for i in range(3)]
    meshes = [gwn.Mesh(_dev(s.V), _dev(s.F), axis=a) for s, a in zip(soups, ["z", "x", "y"])]
    rng = np.random.default_rng(1)
    qs = [rng.uniform(-1.1, 1.1, size=(n, 3)).astype(np.float32) for n in (3000, 1777, 4097)]
    offs = np.concatenate([[0], np.cumsum([q.shape[0] for q in qs])]).astype(np.int64)
    Q = _dev(np.concatenate(qs))
    plan = gwn.MultiPlan(meshes, Q, offs, chi_out=torch.empty(int(offs[-1]), device="cuda", dtype=torch.int32))
    w = plan.run()
    torch.cuda.synchronize()
    for i, m in enumerate(meshes):
        a, b = int(offs[i]), int(offs[i + 1])
        wr, cr = gwn.query_batch(m, Q[a:b], want_chi=True)
        assert torch.equal(plan.chi[a:b], cr)
        assert float((w[a:b] - wr).abs().max()) < 1e-6
