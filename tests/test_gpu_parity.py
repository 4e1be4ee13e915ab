"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Crossing counts must match bit for bit on every query (they come from exact
integer predicates with symbolic perturbation on both sides); w must agree
within 1e-4 (FP32 path) or 1e-5 (FP64 path) wherever the query is farther
than 1e-4 of the bounding-box diagonal from the surface (w is undefined on
it).  Sizes span several tiles with ragged tails; the full-size workloads are
checked on sampled outputs in the same launch configuration the benchmark
times.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2605_01536_amd import workloads as W
from tests._util import TOL_FP32, TOL_FP64, compare, diag_of, fan_soup

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    return t.cuda() if dtype is None else t.to("cuda", dtype)


def _run_batch(G, V, F, Q, prec):
    m = G.Mesh(_dev(V), _dev(F))
    w, chi = G.query_batch(m, _dev(Q), prec=prec, want_chi=True)
    torch.cuda.synchronize()
    return m, w.cpu().numpy(), chi.cpu().numpy()


OCT_V = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float32)
OCT_F = np.array([[0, 1, 2]], np.int32)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("fp64", 1e-13)])
def test_closed_form_cases(gwn, prec, tol):
    # octant triangle: p=0 (vertex on the ray, perturbation limit) and p=(.1,.1,0)
    Q = np.array([[0, 0, 0], [0.1, 0.1, 0]], np.float32)
    _, w, chi = _run_batch(gwn, OCT_V, OCT_F, Q, prec)
    assert w[0] == pytest.approx(0.125, abs=tol)
    assert chi.tolist() == [1, 1]
    assert w[1] == pytest.approx(O.direct(OCT_V, OCT_F, Q[1:])[0], abs=max(tol, 1e-12))
    # square on its axis
    V = np.array([[-1, -1, 0], [1, -1, 0], [1, 1, 0], [-1, 1, 0]], np.float32)
    F = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    h = float(np.float32(0.5))
    _, w, chi = _run_batch(gwn, V, F, np.array([[0, 0, -h], [0, 0, h]], np.float32), prec)
    ref = math.asin(1 / (1 + h * h)) / math.pi
    assert chi.tolist() == [1, 0]
    assert w[0] == pytest.approx(ref, abs=max(tol, 1e-7)) and w[1] == pytest.approx(-ref, abs=max(tol, 1e-7))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_icosphere_config(gwn, prec):
    s, Q = W.config1()
    Q = np.concatenate([[[0, 0, 0]], Q]).astype(np.float32)
    m, w, chi = _run_batch(gwn, s.V, s.F, Q, prec)
    assert m.info()["nboundary"] == 0
    up, _ = O.chi(s.V, s.F, Q)
    assert np.array_equal(chi, up)
    assert w[0] == 1.0
    assert np.array_equal(w, chi.astype(w.dtype))       # B = 0: w is exactly chi


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tiny_soups(gwn, seed, prec):
    rng = np.random.default_rng(500 + seed)
    nt = int(rng.integers(1, 80))
    V = rng.uniform(-1, 1, size=(3 * nt, 3)).astype(np.float32)
    if seed % 2:
        V = (np.round(V * 32) / 32).astype(np.float32)     # coincident coordinates, exact grid hits
    F = rng.integers(0, V.shape[0], size=(nt, 3)).astype(np.int32)
    Q = rng.uniform(-1.3, 1.3, size=(777, 3)).astype(np.float32)
    if seed % 2:
        Q[:300] = np.round(Q[:300] * 32) / 32              # queries on vertex/edge lines
    Q[-5:] = [[5, 5, 0], [-4, 0, 0.1], [0, 7, -2], [0.3, 0.2, 9], [0.1, -0.2, -9]]   # outside the grid box
    _, w, chi = _run_batch(gwn, V, F, Q, prec)
    compare(w, chi, V, F, Q, TOL_FP32 if prec == "fp32" else TOL_FP64, f"tiny{seed}-{prec}")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_torus_soup_subset(gwn, prec):
    s, Q = W.config2(n_uniform=3000, n_near=3000)
    Q = Q[:5999]          # ragged against the 64/256-lane tiles
    m, w, chi = _run_batch(gwn, s.V, s.F, Q, prec)
    info = m.info()
    fr, _ = O.boundary(s.F)
    assert info["nboundary"] == len(fr)
    compare(w, chi, s.V, s.F, Q, TOL_FP32 if prec == "fp32" else TOL_FP64, f"torus-{prec}")


def test_torus_soup_full_size_sampled(gwn):
    # the full 2M-query launch; 2500 sampled outputs checked against the oracle
    s, Q = W.config2()
    m, w, chi = _run_batch(gwn, s.V, s.F, Q, "fp32")
    idx = np.random.default_rng(0).choice(Q.shape[0], 2500, replace=False)
    compare(w[idx], chi[idx], s.V, s.F, Q[idx], TOL_FP32, "torus-full")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("dims", [(13, 11, 700), (9, 17, 65), (5, 4, 3)])
def test_grid_small_mesh_all_points(gwn, prec, dims):
    s = W.opened_spheres(seed=40, n_surf=6, tris_per_surf=800)
    g = W.GridSpec(origin=(-1.05, -0.97, -1.1), spacing=(2.1 / dims[0], 1.9 / dims[1], 2.2 / dims[2]), dims=dims)
    m = gwn.Mesh(_dev(s.V), _dev(s.F))
    w, chi = gwn.query_grid(m, g.origin, g.spacing, g.dims, prec=prec, want_chi=True)
    torch.cuda.synchronize()
    P = W.grid_points(g)
    compare(w.cpu().numpy(), chi.cpu().numpy(), s.V, s.F, P, TOL_FP32 if prec == "fp32" else TOL_FP64,
            f"grid{dims}-{prec}")
    # the batch path on the same points gives the same crossings and w
    wb, cb = gwn.query_batch(m, _dev(P), prec=prec, want_chi=True)
    assert torch.equal(cb, chi)
    assert float((wb.double() - w.double()).abs().max()) < (1e-6 if prec == "fp32" else 1e-12)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("zb", ["1", "8"])
def test_grid_long_boundary_loops(gwn, monkeypatch, prec, zb):
    # boundary loops around the lengths where the grid kernel's vertex ring fills
    # (64 vertices at a time), wraps (128 slots) and flushes (32 edges), and
    # pairs its edges four at a time, plus single-edge and short loops
    lengths = [3, 4, 5, 31, 32, 33, 34, 63, 64, 65, 66, 127, 128, 129, 130, 131, 191, 192, 193, 256, 257, 300]
    V, F = fan_soup(lengths, seed=77)
    monkeypatch.setenv("GWN_GRID_SAMPLES_PER_LANE", zb)
    m = gwn.Mesh(_dev(V), _dev(F))
    info = m.info()
    assert info["nloops"] == len(lengths) and info["nboundary"] == sum(lengths)
    g = W.GridSpec(origin=(-1.0, -0.93, -1.07), spacing=(2.0 / 15, 1.9 / 13, 2.1 / 200), dims=(15, 13, 200))
    w, chi = gwn.query_grid(m, g.origin, g.spacing, g.dims, prec=prec, want_chi=True)
    torch.cuda.synchronize()
    P = W.grid_points(g)
    compare(w.cpu().numpy(), chi.cpu().numpy(), V, F, P, TOL_FP32 if prec == "fp32" else TOL_FP64,
            f"fans-zb{zb}-{prec}")
    wb, cb = gwn.query_batch(m, _dev(P), prec=prec, want_chi=True)
    assert torch.equal(cb, chi)
    assert float((wb.double() - w.double()).abs().max()) < (1e-6 if prec == "fp32" else 1e-12)


def test_grid_full_size_sampled(gwn):
    # the 1M-triangle soup on the 512^3 grid the benchmark times; sampled outputs
    s, g = W.config4()
    m = gwn.Mesh(_dev(s.V), _dev(s.F))
    w, chi = gwn.query_grid(m, g.origin, g.spacing, g.dims, prec="fp32", want_chi=True)
    torch.cuda.synchronize()
    idx = np.random.default_rng(1).choice(g.n, 1500, replace=False)
    it = torch.from_numpy(idx).cuda()
    P = W.grid_points(g, idx)
    e, n = compare(w[it].cpu().numpy(), chi[it].cpu().numpy(), s.V, s.F, P, TOL_FP32, "grid512")
    assert n > 1000


def test_grid_far_columns_and_ray_hits_vertices(gwn):
    # grid extending far outside the fixed-point box; columns through mesh vertices
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0.5], [0.5, 0.5, 1]], np.float32)
    F = np.array([[0, 1, 4], [1, 3, 4], [3, 2, 4]], np.int32)
    g = W.GridSpec(origin=(-3.0, -3.0, -1.0), spacing=(0.25, 0.25, 0.0625), dims=(32, 32, 48))
    m = gwn.Mesh(_dev(V), _dev(F))
    w, chi = gwn.query_grid(m, g.origin, g.spacing, g.dims, prec="fp32", want_chi=True)
    P = W.grid_points(g)
    compare(w.cpu().numpy(), chi.cpu().numpy(), V, F, P, TOL_FP32, "grid-far")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("zb", ["1", "2", "4", "8"])
def test_grid_columns_through_boundary_vertices(gwn, monkeypatch, prec, zb):
    # lattice soups on a grid whose columns pass exactly through boundary vertices
    # and along edges (N = 0, the exact atan2 branch in the middle of an edge
    # pair), loops of many lengths (every tail of the pair loop), for each number
    # of samples per lane; against the oracle and against the per-point kernel
    monkeypatch.setenv("GWN_GRID_SAMPLES_PER_LANE", zb)
    # z samples off the lattice, then on it (samples at the vertices' heights)
    for g, seed in ((W.GridSpec(origin=(-1.0625, -1.0625, -1.3), spacing=(0.125, 0.125, 2.6 / 130),
                                dims=(18, 18, 130)), 17),
                    (W.GridSpec(origin=(-1.0625, -1.0625, -1.3), spacing=(0.125, 0.125, 2.6 / 130),
                                dims=(18, 18, 130)), 18),
                    (W.GridSpec(origin=(-1.0625, -1.0625, -1.0625), spacing=(0.125, 0.125, 0.125),
                                dims=(18, 18, 140)), 19)):
        P = W.grid_points(g)
        rng = np.random.default_rng(seed)
        V = (rng.integers(-8, 9, size=(120, 3)) / 8).astype(np.float32)
        F = rng.integers(0, 120, size=(50 + 13 * (seed - 17), 3)).astype(np.int32)
        m = gwn.Mesh(_dev(V), _dev(F))
        assert m.info()["nloops"] >= 3
        w, chi = gwn.query_grid(m, g.origin, g.spacing, g.dims, prec=prec, want_chi=True)
        compare(w.cpu().numpy(), chi.cpu().numpy(), V, F, P, TOL_FP32 if prec == "fp32" else TOL_FP64,
                f"lattice{seed}-zb{zb}-{prec}")
        wb, cb = gwn.query_batch(m, _dev(P), prec=prec, want_chi=True)
        assert torch.equal(cb, chi)
        d = (wb.double() - w.double()).abs().cpu().numpy()
        assert np.median(d) < (1e-7 if prec == "fp32" else 1e-14)


@pytest.mark.parametrize("seed", range(20))
def test_random_lattice_soups(gwn, monkeypatch, seed):
    # seeded lattice soups (shared, repeated and collinear vertices, zero-area and
    # duplicated triangles) on grids whose columns and samples sit on the lattice,
    # a random number of samples per lane, FP32 and FP64, against the oracle;
    # batch points at the same places as a cross-check of the column form
    rng = np.random.default_rng(1000 + seed)
    nv = int(rng.integers(20, 200))
    V = (rng.integers(-6, 7, size=(nv, 3)) / 6).astype(np.float32)
    F = rng.integers(0, nv, size=(int(rng.integers(5, 120)), 3)).astype(np.int32)
    F[::7] = F[::7][:, [0, 0, 1]]                      # some degenerate triangles
    F = np.concatenate([F, F[: len(F) // 5]])          # some duplicates
    monkeypatch.setenv("GWN_GRID_SAMPLES_PER_LANE", str(int(rng.choice([1, 2, 4, 8]))))
    h = 1 / 6
    g = W.GridSpec(origin=(-1 - h / 2 * rng.integers(0, 2), -1 - h / 2, -1.3 + h * rng.integers(0, 2)),
                   spacing=(h, h, h / int(rng.integers(1, 4))), dims=(13, 13, int(rng.integers(60, 300))))
    P = W.grid_points(g)
    m = gwn.Mesh(_dev(V), _dev(F))
    for prec, tol in (("fp32", TOL_FP32), ("fp64", TOL_FP64)):
        w, chi = gwn.query_grid(m, g.origin, g.spacing, g.dims, prec=prec, want_chi=True)
        compare(w.cpu().numpy(), chi.cpu().numpy(), V, F, P, tol, f"lattice-rand{seed}-{prec}")
        wb, cb = gwn.query_batch(m, _dev(P), prec=prec, want_chi=True)
        assert torch.equal(cb, chi)


def test_edge_cases(gwn):
    # nq = 0 is a no-op
    m = gwn.Mesh(_dev(OCT_V), _dev(OCT_F))
    out = gwn.query_batch(m, torch.zeros((0, 3), device="cuda"))
    assert out.numel() == 0
    # empty mesh: w = 0 everywhere
    m0 = gwn.Mesh(torch.zeros((0, 3), device="cuda"), torch.zeros((0, 3), dtype=torch.int32, device="cuda"))
    w, chi = gwn.query_batch(m0, torch.rand((100, 3), device="cuda"), want_chi=True)
    assert float(w.abs().max()) == 0.0 and int(chi.abs().max()) == 0
    # degenerate and duplicated triangles
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.5, 0.5, 0.5]], np.float32)
    F = np.array([[0, 1, 2], [0, 1, 2], [3, 3, 1], [0, 1, 1], [0, 2, 3]], np.int32)
    Q = np.random.default_rng(3).uniform(-0.5, 1.5, size=(500, 3)).astype(np.float32)
    _, w, chi = _run_batch(gwn, V, F, Q, "fp32")
    compare(w, chi, V, F, Q, TOL_FP32, "degenerate")
    # invalid input is rejected with GWN_E_INVALID
    with pytest.raises(gwn.GwnError) as ei:
        gwn.Mesh(_dev(OCT_V), _dev(np.array([[0, 1, 3]], np.int32)))
    assert ei.value.status == 1
    Vn = OCT_V.copy()
    Vn[1, 2] = np.nan
    with pytest.raises(gwn.GwnError) as ei:
        gwn.Mesh(_dev(Vn), _dev(OCT_F))
    assert ei.value.status == 1


def test_deterministic(gwn):
    s, Q = W.config2(n_uniform=20000, n_near=20000)
    m = gwn.Mesh(_dev(s.V), _dev(s.F))
    Qd = _dev(Q)
    a = gwn.query_batch(m, Qd)
    b = gwn.query_batch(m, Qd)
    assert torch.equal(a, b)
    m2 = gwn.Mesh(_dev(s.V), _dev(s.F))
    assert m2.info()["nboundary"] == m.info()["nboundary"]
    assert torch.equal(gwn.query_batch(m2, Qd), a)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_point_results_independent_of_the_batch(gwn, prec):
    # per-lane edge pairs are chosen per point, so a point's w is the same bits
    # in a large batch (traversal order by x, y), a smaller one (no reordering)
    # and a shuffled one
    s, Q = W.config2(n_uniform=150_000, n_near=150_000)
    m = gwn.Mesh(_dev(s.V), _dev(s.F))
    w_all = gwn.query_batch(m, _dev(Q), prec=prec)
    sub = Q[::15][:20_000]
    w_sub = gwn.query_batch(m, _dev(sub), prec=prec)
    perm = np.random.default_rng(8).permutation(sub.shape[0])
    w_shuf = gwn.query_batch(m, _dev(sub[perm]), prec=prec)
    assert torch.equal(w_sub, w_all[::15][:20_000])
    assert torch.equal(w_shuf, w_sub[torch.from_numpy(perm).cuda()])


def test_launch_splitting_is_invisible(gwn, monkeypatch):
    # batches and grids larger than one launch are split; force tiny launches and
    # compare every output bit for bit with the single-launch result
    s = W.opened_spheres(seed=41, n_surf=4, tris_per_surf=300)
    m = gwn.Mesh(_dev(s.V), _dev(s.F))
    Q = _dev(np.random.default_rng(2).uniform(-1.2, 1.2, size=(5000, 3)).astype(np.float32))
    g = W.GridSpec(origin=(-1.0, -1.0, -1.0), spacing=(0.05, 0.05, 0.01), dims=(21, 19, 600))

    def run():
        w, c = gwn.query_batch(m, Q, want_chi=True)
        wg, cg = gwn.query_grid(m, g.origin, g.spacing, g.dims, want_chi=True)
        return [w, c, wg, cg, gwn.query_gradient(m, Q), gwn.query_direct(m, Q[:1000])]

    ref = run()
    monkeypatch.setenv("GWN_MAX_LAUNCH_QUERIES", "768")
    out = run()
    torch.cuda.synchronize()
    for a, b in zip(ref, out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("case", ["tiny", "torus", "grid512", "closed"])
def test_crossings_both_directions(gwn, case):
    # chi along +z and along the antipode -z, bit for bit against the oracle
    if case == "tiny":
        rng = np.random.default_rng(77)
        V = (np.round(rng.uniform(-1, 1, size=(150, 3)) * 16) / 16).astype(np.float32)
        F = rng.integers(0, 150, size=(50, 3)).astype(np.int32)
        Q = (np.round(rng.uniform(-1.2, 1.2, size=(3001, 3)) * 16) / 16).astype(np.float32)
    elif case == "torus":
        s, Q = W.config2(n_uniform=2000, n_near=2000)
        V, F = s.V, s.F
    elif case == "grid512":
        s, g = W.config4()
        V, F = s.V, s.F
        Q = W.grid_points(g, np.random.default_rng(4).choice(g.n, 2000, replace=False))
    else:
        s, Q = W.config1()
        V, F = s.V, s.F
    m = gwn.Mesh(_dev(V), _dev(F))
    up, dn = gwn.query_crossings(m, _dev(Q))
    ou, od = O.chi(V, F, Q)
    assert np.array_equal(up.cpu().numpy(), ou)
    assert np.array_equal(dn.cpu().numpy(), od)
    _, chi = gwn.query_batch(m, _dev(Q), want_chi=True)
    assert torch.equal(chi, up)
    if case == "closed":
        assert torch.equal(up, dn)


def test_binding_rejects_mismatched_tensors(gwn):
    m = gwn.Mesh(_dev(OCT_V), _dev(OCT_F))
    Q = torch.rand((100, 3), device="cuda")
    with pytest.raises(ValueError):
        gwn.query_batch(m, Q, out=torch.empty(99, device="cuda"))
    with pytest.raises(ValueError):
        gwn.query_batch(m, Q, prec="fp64", out=torch.empty(100, device="cuda"))
    with pytest.raises(ValueError):
        gwn.query_gradient(m, Q, out=torch.empty((100, 2), device="cuda"))
    with pytest.raises(ValueError):
        gwn.query_batch(m, torch.rand((100, 2), device="cuda"))
    with pytest.raises(ValueError):
        gwn.Mesh(_dev(OCT_V[:, :2].copy()), _dev(OCT_F))


def test_batch_beyond_one_launch(gwn):
    # 2^30 + 4099 points: the largest single launch plus a ragged second one
    # (13 GB of points); sampled outputs around the split against the oracle
    n = (1 << 30) + 4099
    gen = torch.Generator(device="cuda")
    gen.manual_seed(123)
    Q = torch.rand((n, 3), device="cuda", generator=gen) * 3.0 - 1.0
    m = gwn.Mesh(_dev(OCT_V), _dev(OCT_F))
    w = torch.full((n,), float("nan"), device="cuda")
    chi = torch.full((n,), -7, device="cuda", dtype=torch.int32)
    gwn.query_batch(m, Q, out=w, chi_out=chi)
    torch.cuda.synchronize()
    assert not bool(torch.isnan(w).any()) and int(chi.min()) >= 0
    idx = np.concatenate([np.arange((1 << 30) - 300, (1 << 30) + 300), np.arange(n - 200, n),
                          np.random.default_rng(9).choice(n, 1000, replace=False)])
    it = torch.from_numpy(idx).cuda()
    P = Q[it].cpu().numpy()
    del Q
    compare(w[it].cpu().numpy(), chi[it].cpu().numpy(), OCT_V, OCT_F, P, TOL_FP32, "beyond-one-launch")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_astronomically_far_queries(gwn, prec):
    # scaled coordinates overflow FP32 here; w and its gradient are ~0 there
    s = W.opened_spheres(seed=40, n_surf=3, tris_per_surf=300)
    # (FAR queries take offsets in units of 2^e cells; without that FP32 N, D
    # and rho^2 overflow beyond ~1e10 mesh sizes)
    Q = np.array([[1e35, 0, 0], [0, -1e36, 0.5], [3e38, 3e38, 3e38], [0.1, 0.2, 1e35], [0.1, 0.2, -1e35],
                  [-2e34, 0.3, -1e37], [5e3, 1, 2], [-3e6, 2e6, 1e6], [1e11, -1e11, 0.5], [7e15, 0.1, -3e15],
                  [0.1, 0.2, 1e12], [0.1, 0.2, -1e12]], np.float32)
    m = gwn.Mesh(_dev(s.V), _dev(s.F))
    w, chi = gwn.query_batch(m, _dev(Q), prec=prec, want_chi=True)
    g = gwn.query_gradient(m, _dev(Q), prec=prec)
    w, chi, g = w.cpu().numpy(), chi.cpu().numpy(), g.cpu().numpy()
    up, _ = O.chi(s.V, s.F, Q)
    assert np.array_equal(chi, up)
    assert np.isfinite(w).all() and np.isfinite(g).all()
    assert np.abs(w - O.direct(s.V, s.F, Q)).max() < 1e-6
    assert np.abs(w).max() < 1e-6 and np.abs(g).max() < 1e-6


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_grid_descending_and_flat_z(gwn, prec):
    # negative spacing (samples fall in z along a column, so the sample blocks'
    # smallest z descend) and zero z spacing (every sample of a column equal)
    s = W.opened_spheres(seed=41, n_surf=4, tris_per_surf=500)
    m = gwn.Mesh(_dev(s.V), _dev(s.F))
    tol = TOL_FP32 if prec == "fp32" else TOL_FP64
    for g in (W.GridSpec(origin=(1.05, 1.0, 1.1), spacing=(-0.2, -0.18, -2.2 / 600), dims=(11, 12, 600)),
              W.GridSpec(origin=(-1.0, -1.0, 0.37), spacing=(0.25, 0.25, 0.0), dims=(8, 8, 130))):
        w, chi = gwn.query_grid(m, g.origin, g.spacing, g.dims, prec=prec, want_chi=True)
        P = W.grid_points(g)
        compare(w.cpu().numpy(), chi.cpu().numpy(), s.V, s.F, P, tol, f"grid-z{g.spacing[2]:+.3g}-{prec}")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("zb", ["", "1", "2", "4", "8"])
def test_grid_descending_z_with_clamped_blocks(gwn, monkeypatch, prec, zb):
    # negative z spacing with column lengths whose last chunk fills only its
    # first block of 64 samples (the later blocks hold clamped copies of the
    # column's last sample, with the same smallest z): the blocks' order must not
    # be taken for ascending there; the chosen and each forced samples per lane
    if zb:
        monkeypatch.setenv("GWN_GRID_SAMPLES_PER_LANE", zb)
    s = W.opened_spheres(seed=43, n_surf=3, tris_per_surf=400)
    m = gwn.Mesh(_dev(s.V), _dev(s.F))
    tol = TOL_FP32 if prec == "fp32" else TOL_FP64
    for nz in (7, 70, 130, 150, 257, 520):
        g = W.GridSpec(origin=(-0.93, -0.87, 1.1), spacing=(0.31, 0.29, -2.2 / nz), dims=(6, 5, nz))
        w, chi = gwn.query_grid(m, g.origin, g.spacing, g.dims, prec=prec, want_chi=True)
        P = W.grid_points(g)
        compare(w.cpu().numpy(), chi.cpu().numpy(), s.V, s.F, P, tol, f"desc-nz{nz}-zb{zb}-{prec}")
        wb, cb = gwn.query_batch(m, _dev(P), prec=prec, want_chi=True)
        assert torch.equal(cb, chi)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_grid_columns_far_in_z(gwn, prec):
    # columns inside the box whose samples lie far above and below it: every
    # sample far (FP32 cell offsets overflow to infinity), and a column mixing
    # near and far samples in one wave; finite, and against the oracle
    s = W.opened_spheres(seed=40, n_surf=3, tris_per_surf=300)
    m = gwn.Mesh(_dev(s.V), _dev(s.F))
    tol = TOL_FP32 if prec == "fp32" else TOL_FP64
    for g in (W.GridSpec(origin=(-0.5, -0.5, 1e30), spacing=(0.25, 0.25, 1e29), dims=(4, 4, 64)),
              W.GridSpec(origin=(-0.5, -0.5, -3e4), spacing=(0.25, 0.25, 937.5), dims=(4, 4, 64)),
              W.GridSpec(origin=(-0.5, -0.5, -3e4), spacing=(0.25, 0.25, 117.1875), dims=(4, 4, 512))):
        w, chi = gwn.query_grid(m, g.origin, g.spacing, g.dims, prec=prec, want_chi=True)
        w, chi = w.cpu().numpy(), chi.cpu().numpy()
        assert np.isfinite(w).all()
        P = W.grid_points(g)
        compare(w, chi, s.V, s.F, P, tol, f"far-z-{prec}")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_grid_boundary_vertices_around_the_far_cone(gwn, prec):
    # An open, slightly wavy disk (96 boundary vertices on a ring of radius 0.3
    # at height ~0.3) over a grid whose columns lie 0 to ~0.6 (horizontally)
    # from the ring's vertices and whose samples run from below the disk to
    # above it.  The grid kernel takes s = l - r_z for a vertex whose every
    # sample below it lies within 60 degrees of the vertical around the column
    # (r_z^2 <= 3 rho^2), and the reciprocal form otherwise; here both occur in
    # every column, along with blocks of samples straddling a vertex's height.
    n = 96
    ang = 2.0 * np.pi * np.arange(n) / n
    ring = np.stack([0.3 * np.cos(ang), 0.3 * np.sin(ang), 0.3 + 0.02 * np.sin(3.0 * ang)], 1)
    V = np.concatenate([[[0.01, -0.02, 0.36]], ring]).astype(np.float32)
    F = np.array([[0, 1 + i, 1 + (i + 1) % n] for i in range(n)], np.int32)
    m = gwn.Mesh(_dev(V), _dev(F))
    assert m.info()["nboundary"] == n
    g = W.GridSpec(origin=(-0.6, -0.6, -0.3), spacing=(0.075, 0.075, 0.8 / 512), dims=(16, 16, 512))
    w, chi = gwn.query_grid(m, g.origin, g.spacing, g.dims, prec=prec, want_chi=True)
    P = W.grid_points(g)
    e, k = compare(w.cpu().numpy(), chi.cpu().numpy(), V, F, P, TOL_FP32 if prec == "fp32" else TOL_FP64,
                   f"far-cone-{prec}")
    assert k > 0.99 * P.shape[0]
    # the same points through the batch path, which keeps the reciprocal form
    wb = gwn.query_batch(m, _dev(P), prec=prec).cpu().numpy()
    assert np.abs(wb.astype(np.float64) - w.cpu().numpy()).max() < (2e-6 if prec == "fp32" else 1e-12)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_welded_exploded_soup(gwn, prec):
    # STL-style input: every triangle with its own vertices; welding on the
    # device recovers the indexed boundary, and w / chi match the oracle
    s = W.opened_spheres(seed=42, n_surf=5, tris_per_surf=600)
    e = W.explode(s, seed=3)
    e.V[::7] = np.where(e.V[::7] == 0, np.float32(-0.0), e.V[::7])      # signed zeros weld too
    Fw, n = O.weld(e.V, e.F)
    mw = gwn.Mesh(_dev(e.V), _dev(e.F), weld=True)
    info = mw.info()
    assert info["nunique"] == n
    assert info["nboundary"] == len(O.boundary(Fw)[0]) == len(O.boundary(s.F)[0])
    m0 = gwn.Mesh(_dev(e.V), _dev(e.F))
    assert m0.info()["nboundary"] == 3 * s.nf and m0.info()["nunique"] == e.V.shape[0]
    Q = np.random.default_rng(8).uniform(-1.1, 1.1, size=(2500, 3)).astype(np.float32)
    w, chi = gwn.query_batch(mw, _dev(Q), prec=prec, want_chi=True)
    compare(w.cpu().numpy(), chi.cpu().numpy(), e.V, e.F, Q, TOL_FP32 if prec == "fp32" else TOL_FP64, "welded")
    w0 = gwn.query_batch(m0, _dev(Q), prec=prec).cpu().numpy()
    assert np.abs(w0 - w.cpu().numpy()).max() < (1e-4 if prec == "fp32" else 1e-9)


def test_traversal_order_is_invisible(gwn, monkeypatch):
    # Morton-ordered traversal of the crossing kernels changes which lane handles
    # which point, never a result
    s, g = W.config4()
    m = gwn.Mesh(_dev(s.V), _dev(s.F))
    P = _dev(W.grid_points(g, np.random.default_rng(5).choice(g.n, 70001, replace=False)))
    out = {}
    for flag in ("0", "1"):
        monkeypatch.setenv("GWN_ORDER_QUERIES", flag)
        w, c = gwn.query_batch(m, P, want_chi=True)
        up, dn = gwn.query_crossings(m, P)
        out[flag] = (w, c, up, dn)
    for a, b in zip(out["0"], out["1"]):
        assert torch.equal(a, b)


@pytest.mark.parametrize("seed", range(4))
def test_wave_traversal_small_meshes(gwn, monkeypatch, seed):
    # the ordered, wave-uniform crossing traversal forced on small soups (a single
    # triangle as the whole tree, rays through vertices) against the oracle
    monkeypatch.setenv("GWN_ORDER_QUERIES", "1")
    rng = np.random.default_rng(700 + seed)
    nt = [1, 2, 37, 500][seed]
    V = (np.round(rng.uniform(-1, 1, size=(3 * nt, 3)) * 8) / 8).astype(np.float32)
    F = rng.integers(0, V.shape[0], size=(nt, 3)).astype(np.int32)
    Q = (np.round(rng.uniform(-1.2, 1.2, size=(4097, 3)) * 8) / 8).astype(np.float32)
    Q[-3:] = [[9, 9, 0], [-9, 0, 1], [0, 0, 9]]
    m = gwn.Mesh(_dev(V), _dev(F))
    w, chi = gwn.query_batch(m, _dev(Q), want_chi=True)
    up, dn = gwn.query_crossings(m, _dev(Q))
    ou, od = O.chi(V, F, Q)
    assert np.array_equal(up.cpu().numpy(), ou) and np.array_equal(dn.cpu().numpy(), od)
    compare(w.cpu().numpy(), chi.cpu().numpy(), V, F, Q, TOL_FP32, f"wave{seed}")


def test_every_entry_point_on_empty_inputs(gwn):
    # an empty mesh gives w = 0, chi = 0 and a zero gradient everywhere; zero
    # points and zero grid sizes are no-ops
    m0 = gwn.Mesh(torch.zeros((0, 3), device="cuda"), torch.zeros((0, 3), dtype=torch.int32, device="cuda"))
    Q = torch.rand((300, 3), device="cuda")
    for prec in ("fp32", "fp64"):
        w, c = gwn.query_grid(m0, (-1, -1, -1), (0.1, 0.1, 0.1), (7, 5, 70), prec=prec, want_chi=True)
        assert float(w.abs().max()) == 0.0 and int(c.abs().max()) == 0
        assert float(gwn.query_gradient(m0, Q, prec=prec).abs().max()) == 0.0
        assert float(gwn.query_direct(m0, Q, prec=prec).abs().max()) == 0.0
    up, dn = gwn.query_crossings(m0, Q)
    assert int(up.abs().max()) == 0 and int(dn.abs().max()) == 0
    m = gwn.Mesh(_dev(OCT_V), _dev(OCT_F))
    E = torch.zeros((0, 3), device="cuda")
    assert gwn.query_batch(m, E).numel() == 0
    assert gwn.query_gradient(m, E).numel() == 0
    assert gwn.query_direct(m, E).numel() == 0
    assert gwn.query_crossings(m, E)[0].numel() == 0
    assert gwn.query_grid(m, (0, 0, 0), (1, 1, 1), (0, 4, 4)).numel() == 0
    assert gwn.query_grid(m, (0, 0, 0), (1, 1, 1), (4, 4, 0)).numel() == 0


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_split_boundary_path(gwn, monkeypatch, prec):
    # few points, many boundary edges: one workgroup per point with the edges
    # split among its lanes; forced on tiny soups (runs shorter than a lane's
    # share, loops ending inside a run) and taken by default on the torus soup
    tol = TOL_FP32 if prec == "fp32" else TOL_FP64
    rng = np.random.default_rng(91)
    V = (np.round(rng.uniform(-1, 1, size=(90, 3)) * 16) / 16).astype(np.float32)
    F = rng.integers(0, 90, size=(30, 3)).astype(np.int32)
    Q = (np.round(rng.uniform(-1.2, 1.2, size=(700, 3)) * 16) / 16).astype(np.float32)
    Q[-3:] = [[5, 5, 0], [-4, 0, 0.1], [0.1, 0.2, -9]]
    monkeypatch.setenv("GWN_SPLIT_BOUNDARY", "1")
    _, w, chi = _run_batch(gwn, V, F, Q, prec)
    compare(w, chi, V, F, Q, tol, f"split-tiny-{prec}")
    monkeypatch.delenv("GWN_SPLIT_BOUNDARY")
    s, Q = W.config2(n_uniform=1500, n_near=1500)
    m, w, chi = _run_batch(gwn, s.V, s.F, Q, prec)      # 3,000 points, 63k edges: split by default
    compare(w, chi, s.V, s.F, Q, tol, f"split-torus-{prec}")
    monkeypatch.setenv("GWN_SPLIT_BOUNDARY", "0")
    w1 = gwn.query_batch(m, _dev(Q), prec=prec).cpu().numpy()
    assert np.abs(w1 - w).max() < (1e-5 if prec == "fp32" else 1e-11)
