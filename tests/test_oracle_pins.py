"""Pins for the CPU oracle against facts fixed by the paper and by mathematics.

Every check here is independent of the oracle's own formulas: closed-form solid
angles, Girard's spherical excess (Eq. 5) against the Van Oosterom-Strackee
form (Eq. 6), exact rational brute force for the perturbed predicates
(Supp. Sec. 2.1), invariants of Eq. 2 (linearity, orientation, rotation),
the auxiliary-triangle identity per triangle (Eq. 9), the cancellation of
interior edges (Sec. 4.1), and the robustness experiment of Supp. Sec. 2.1
(queries in a tiny square around a ray grazing a boundary vertex or edge).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_2605_01536_amd import workloads as W

OCT_V = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float32)
OCT_F = np.array([[0, 1, 2]], np.int32)


# ---------------------------------------------------------------- closed forms

def test_octant_triangle_from_origin_is_one_eighth():
    # The octant triangle covers exactly 1/8 of the sphere around the origin (Eq. 1);
    # its vertex (0,0,1) lies on the +z ray, so O2 exercises the on-ray limit.
    assert O.direct(OCT_V, OCT_F, [[0, 0, 0]])[0] == pytest.approx(0.125, abs=1e-15)
    w, S, up, dn = O.antipodal(OCT_V, OCT_F, [[0, 0, 0]], full=True)
    assert up[0] == 1 and dn[0] == 0
    assert w[0] == pytest.approx(0.125, abs=1e-15)
    assert S[0] == pytest.approx(-3.5 * math.pi, abs=1e-13)


def _girard_signed_area(a, b, c):
    """Signed spherical-triangle area by Girard's theorem (Eq. 5): interior angles
    from tangent vectors, area = alpha + beta + gamma - pi, sign of det[a,b,c]."""
    A, B, C = (np.asarray(v, float) / np.linalg.norm(v) for v in (a, b, c))

    def angle(P, Q, R):
        t1 = Q - np.dot(P, Q) * P
        t2 = R - np.dot(P, R) * P
        return math.atan2(np.linalg.norm(np.cross(t1, t2)), np.dot(t1, t2))

    area = angle(A, B, C) + angle(B, C, A) + angle(C, A, B) - math.pi
    return math.copysign(area, np.linalg.det(np.stack([A, B, C])))


def test_eq6_against_girard_random_triangles():
    rng = np.random.default_rng(11)
    for _ in range(300):
        v = rng.standard_normal((3, 3))
        p = rng.standard_normal(3) * 0.3
        om = O.solid_angle(v[0], v[1], v[2], p)
        g = _girard_signed_area(v[0] - p, v[1] - p, v[2] - p)
        assert om == pytest.approx(g, abs=1e-10)


def test_worked_example_p_off_axis_matches_girard():
    p = np.array([0.1, 0.1, 0.0], np.float32).astype(np.float64)
    g = _girard_signed_area(OCT_V[0] - p, OCT_V[1] - p, OCT_V[2] - p) / (4 * math.pi)
    w, S, up, dn = O.antipodal(OCT_V, OCT_F, [p], full=True)
    assert up[0] == 1  # the +z ray from p meets the triangle, normal (1,1,1): +1 (Sec. 3.2)
    assert w[0] == pytest.approx(g, abs=1e-12)
    assert O.direct(OCT_V, OCT_F, [p])[0] == pytest.approx(g, abs=1e-14)


@pytest.mark.parametrize("h", [0.5, 0.1, 2.0])
def test_square_on_axis_closed_form(h):
    # Solid angle of a 2x2 square seen on its axis at height h: 4 asin(1/(1+h^2)).
    V = np.array([[-1, -1, 0], [1, -1, 0], [1, 1, 0], [-1, 1, 0]], np.float32)
    F = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    h = float(np.float32(h))          # the query is stored in float32
    ref = math.asin(1.0 / (1.0 + h * h)) / math.pi
    below = O.antipodal(V, F, [[0, 0, -h]], full=True)
    above = O.antipodal(V, F, [[0, 0, h]], full=True)
    assert below[0][0] == pytest.approx(ref, abs=1e-7)   # normal +z; query on the back side
    assert above[0][0] == pytest.approx(-ref, abs=1e-7)
    assert below[2][0] == 1 and above[2][0] == 0
    assert O.direct(V, F, [[0, 0, -h]])[0] == pytest.approx(ref, abs=1e-14)


def _hemisphere(n_lat=6, n_lon=17):
    V = [[0.0, 0.0, 1.0]]
    for i in range(1, n_lat + 1):
        th = 0.5 * math.pi * i / n_lat
        for j in range(n_lon):
            ph = 2 * math.pi * j / n_lon
            V.append([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    F = []
    for j in range(n_lon):
        F.append([0, 1 + j, 1 + (j + 1) % n_lon])
    for r in range(n_lat - 1):
        for j in range(n_lon):
            a, b = 1 + r * n_lon + j, 1 + r * n_lon + (j + 1) % n_lon
            c, d = a + n_lon, b + n_lon
            F += [[a, c, d], [a, d, b]]
    return np.array(V, np.float32), np.array(F, np.int32)


def test_open_hemisphere_centre_is_one_half():
    # Boundary on the equator projects to a great circle from the centre, so the
    # triangulated hemisphere subtends exactly 2 pi; the pole vertex is on the ray.
    V, F = _hemisphere()
    d = O.direct(V, F, [[0, 0, 0]])[0]
    w = O.antipodal(V, F, [[0, 0, 0]])[0]
    assert abs(abs(d) - 0.5) < 1e-6 and abs(abs(w) - 0.5) < 1e-6
    assert w == pytest.approx(d, abs=1e-12)
    # outward faces (normal away from the centre): w > 0 on the side opposite the normal
    assert w > 0


def test_icosphere_inside_outside():
    s, Q = W.config1(2000)
    wa, S, up, dn = O.antipodal(s.V, s.F, np.concatenate([[[0, 0, 0]], Q]), full=True)
    assert wa[0] == 1.0
    assert np.all(S == 0.0)                 # closed mesh: no boundary (Sec. 4.1)
    assert set(np.unique(wa)) <= {0.0, 1.0}
    wd = O.direct(s.V, s.F, Q)
    far = np.linalg.norm(Q, axis=1) > 1.05
    assert np.all(wa[1:][far] == 0.0)
    assert np.max(np.abs(wd - wa[1:])) < 1e-12


def test_far_field_vanishes():
    s = W.torus_soup(seed=2, n_u=40, n_v=30)
    q = np.array([[1e3, -2e3, 5e2]], np.float32)
    area = 0.5 * np.linalg.norm(np.cross(s.V[s.F[:, 1]] - s.V[s.F[:, 0]], s.V[s.F[:, 2]] - s.V[s.F[:, 0]]), axis=1).sum()
    bound = area / (4 * math.pi * (np.linalg.norm(q) - 2) ** 2)
    assert abs(O.antipodal(s.V, s.F, q)[0]) <= bound
    assert abs(O.direct(s.V, s.F, q)[0]) <= bound


# ---------------------------------------------------------------- quantisation

def test_quantisation_rule_by_hand():
    V = np.array([[0, 0, 0], [1, 1, 1]], np.float32)
    bbox, lo, k = O.quant_params(V)
    assert list(bbox) == [0, 0, 0, 1, 1, 1]
    assert list(lo) == [-0.75] * 3
    assert k == 28                      # 2.5 * 2^28 <= 2^30 - 1 < 2.5 * 2^29
    q, ib = O.quantize(np.array([[0, 0, 0], [1, 1, 1], [-0.75, 0, 5], [-0.76, 0, 0], [0, 0, -9]], np.float32), lo, k)
    assert q[0].tolist() == [201326592] * 3
    assert q[1].tolist() == [469762048] * 3
    assert ib.tolist() == [True, True, True, False, True]
    assert q[2, 0] == 0 and q[2, 2] == 2 ** 30      # z above the box clamps to 2^30
    assert q[4, 2] == -1                            # z below clamps to -1


# ---------------------------------------------------------------- exact predicates

def _orient_brute(x0, y0, x1, y1, qx, qy):
    e1, e2 = Fraction(1, 2 ** 100), Fraction(1, 2 ** 200)
    v = (qx + e1 - x0) * (y0 - y1) + (qy + e2 - y0) * (x1 - x0)
    return (v > 0) - (v < 0)


def _plane_brute(p0, p1, p2, q):
    u = [p1[i] - p0[i] for i in range(3)]
    v = [p2[i] - p0[i] for i in range(3)]
    n = [u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]]
    # f(q + eps) with eps = (2^-200, 2^-400, 2^-600), scaled by 2^600 to stay in integers
    f = sum(n[i] * (p0[i] - q[i]) for i in range(3)) * 2 ** 600
    f -= n[0] * 2 ** 400 + n[1] * 2 ** 200 + n[2]
    return (f > 0) - (f < 0)


@pytest.mark.parametrize("span", [3, 1000, 2 ** 30 - 1])
def test_orient2d_sos_matches_rational_brute_force(span):
    rng = np.random.default_rng(span)
    X = rng.integers(0, span + 1, size=(20000, 6))
    for row in X:
        a = [int(v) for v in row]
        assert O.orient2d_sos(*a) == _orient_brute(*a)
    # collinear and coincident configurations
    for _ in range(3000):
        x0, y0, dx, dy = (int(v) for v in rng.integers(0, 50, 4))
        t = int(rng.integers(-3, 4))
        args = (x0, y0, x0 + dx, y0 + dy, x0 + t * dx, y0 + t * dy)
        assert O.orient2d_sos(*args) == _orient_brute(*args)


@pytest.mark.parametrize("span", [3, 2 ** 30 - 1])
def test_plane_sos_matches_rational_brute_force(span):
    rng = np.random.default_rng(7 + span)
    for _ in range(4000):
        P = [[int(v) for v in rng.integers(0, span + 1, 3)] for _ in range(4)]
        assert O.plane_sos(*P) == _plane_brute(*P)
    # query on the plane of a tilted triangle
    for _ in range(2000):
        p0 = [int(v) for v in rng.integers(0, 20, 3)]
        u = [int(v) for v in rng.integers(-5, 6, 3)]
        v = [int(v) for v in rng.integers(-5, 6, 3)]
        s, t = int(rng.integers(-2, 3)), int(rng.integers(-2, 3))
        q = [p0[i] + s * u[i] + t * v[i] for i in range(3)]
        p1 = [p0[i] + u[i] for i in range(3)]
        p2 = [p0[i] + v[i] for i in range(3)]
        assert O.plane_sos(p0, p1, p2, q) == _plane_brute(p0, p1, p2, q)


# ---------------------------------------------------------------- boundary chain

def test_boundary_chain_cancellation():
    s = W.icosphere(2)
    assert len(O.boundary(s.F)[0]) == 0
    fr, to = O.boundary(OCT_F)
    assert sorted(zip(fr.tolist(), to.tolist())) == [(0, 1), (1, 2), (2, 0)]
    # two triangles sharing an edge consistently: shared edge cancels
    fr, to = O.boundary(np.array([[0, 1, 2], [0, 2, 3]]))
    assert sorted(zip(fr.tolist(), to.tolist())) == [(0, 1), (1, 2), (2, 3), (3, 0)]
    # the same triangle twice: every edge with multiplicity 2
    fr, to = O.boundary(np.array([[0, 1, 2], [0, 1, 2]]))
    assert len(fr) == 6
    # inconsistently oriented neighbours: shared edge survives twice (net multiplicity 2)
    fr, to = O.boundary(np.array([[0, 1, 2], [0, 3, 2]]))
    assert sorted(zip(fr.tolist(), to.tolist())).count((2, 0)) == 2
    # every vertex of the chain has in-degree == out-degree
    s = W.torus_soup(seed=2, n_u=40, n_v=30)
    fr, to = O.boundary(s.F)
    assert np.array_equal(np.bincount(fr, minlength=s.nv), np.bincount(to, minlength=s.nv))
    # degenerate index triangle contributes nothing
    assert len(O.boundary(np.array([[4, 4, 5]]))[0]) == 0


# ---------------------------------------------------------------- invariants

def _tiny_soup(rng, nt, dyadic):
    if dyadic:
        V = rng.integers(-64, 65, size=(3 * nt, 3)).astype(np.float32) / 64.0
    else:
        V = rng.uniform(-1, 1, size=(3 * nt, 3)).astype(np.float32)
    # share some vertices so that interior edges exist
    F = rng.integers(0, V.shape[0], size=(nt, 3)).astype(np.int32)
    return V, F


def _off_surface(V, F, Q, frac):
    lo, hi = V.min(0), V.max(0)
    diag = float(np.linalg.norm(hi - lo))
    return O.distance(V, F, Q, 1.0) > frac * diag


@pytest.mark.parametrize("seed", range(8))
def test_tiny_soups_antipodal_equals_direct(seed):
    rng = np.random.default_rng(100 + seed)
    dy = seed % 2 == 0
    V, F = _tiny_soup(rng, int(rng.integers(1, 65)), dyadic=dy)
    if dy:
        Q = (rng.integers(-80, 81, size=(400, 3)) / 128.0 + 1.0 / 1024).astype(np.float32)
    else:
        Q = rng.uniform(-1.2, 1.2, size=(400, 3)).astype(np.float32)
    m = _off_surface(V, F, Q, 1e-3)
    wa = O.antipodal(V, F, Q)
    wd = O.direct(V, F, Q)
    tol = 1e-12 if dy else 1e-6
    assert np.max(np.abs(wa - wd)[m]) < tol


def test_all_edges_equals_cancelled_chain():
    s = W.torus_soup(seed=2, n_u=30, n_v=20)
    Q = W.uniform_box(np.random.default_rng(3), 300, *s.bbox())
    a = O.antipodal(s.V, s.F, Q, cancel=True)
    b = O.antipodal(s.V, s.F, Q, cancel=False)
    assert np.max(np.abs(a - b)) < 1e-11


def test_per_triangle_auxiliary_identity():
    # Eq. 9 for one triangle: sum of the three auxiliary areas = Area(T) - 4 pi s [ray hits T].
    rng = np.random.default_rng(5)
    for _ in range(200):
        V = rng.uniform(-1, 1, (3, 3)).astype(np.float32)
        p = rng.uniform(-1, 1, (1, 3)).astype(np.float32)
        w, S, up, dn = O.antipodal(V, OCT_F, p, full=True)
        area = O.solid_angle(*V.astype(float), p[0].astype(float))
        assert S[0] == pytest.approx(area - 4 * math.pi * up[0], abs=2e-6)


def test_orientation_union_duplicate_linearity():
    rng = np.random.default_rng(9)
    V1, F1 = _tiny_soup(rng, 20, dyadic=False)
    V2, F2 = _tiny_soup(rng, 15, dyadic=False)
    Q = rng.uniform(-1, 1, size=(200, 3)).astype(np.float32)
    V = np.concatenate([V1, V2])
    F = np.concatenate([F1, F2 + V1.shape[0]])
    m = _off_surface(V, F, Q, 1e-3)
    w1, w2, w12 = O.antipodal(V, F1, Q), O.antipodal(V, F2 + V1.shape[0], Q), O.antipodal(V, F, Q)
    assert np.max(np.abs((w1 + w2 - w12)[m])) < 1e-9
    flip = F[:, [0, 2, 1]]
    assert np.max(np.abs((O.antipodal(V, flip, Q) + w12)[m])) < 1e-9
    dup = np.concatenate([F, F])
    assert np.max(np.abs((O.antipodal(V, dup, Q) - 2 * w12)[m])) < 1e-9


@pytest.mark.parametrize("perm", ["yzx", "zxy", "x-y-z", "-xy-z"])
def test_ray_direction_independence(perm):
    # Rotating the scene changes which world axis the +z ray follows (x0 in
    # {+-x, +-y, +-z}); w must not change (Prop. 4.2: w does not depend on x0).
    s = W.torus_soup(seed=2, n_u=30, n_v=20)
    Q = W.uniform_box(np.random.default_rng(4), 300, *s.bbox())
    R = {"yzx": [[0, 1, 0], [0, 0, 1], [1, 0, 0]], "zxy": [[0, 0, 1], [1, 0, 0], [0, 1, 0]],
         "x-y-z": [[1, 0, 0], [0, -1, 0], [0, 0, -1]], "-xy-z": [[-1, 0, 0], [0, 1, 0], [0, 0, -1]]}[perm]
    R = np.array(R, np.float32)
    m = _off_surface(s.V, s.F, Q, 1e-3)
    a = O.antipodal(s.V, s.F, Q)
    b = O.antipodal(s.V @ R.T, s.F, Q @ R.T)
    assert np.max(np.abs(a - b)[m]) < 1e-6


# ---------------------------------------------------------------- robustness (Supp. Sec. 2.1)

@pytest.mark.parametrize("center", [(0.0, 0.0), (0.5, 0.0), (0.25, 0.25)])
def test_grazing_ray_square_has_no_integer_jumps(center):
    # queries on a 1e-6 square whose +z rays graze a boundary vertex, a boundary
    # edge, or the shared interior edge of a fan; the antipodal result must stay
    # within round-off of the direct sum (no off-by-integer errors).
    V = np.array([[0, 0, 1], [1, 0, 1], [0, 1, 1], [-1, -0.5, 1.3], [0.5, -1, 0.7]], np.float32)
    F = np.array([[0, 1, 2], [0, 2, 3], [0, 4, 1]], np.int32)
    g = np.linspace(-0.5e-6, 0.5e-6, 41)
    X, Y = np.meshgrid(g + center[0], g + center[1], indexing="ij")
    Q = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1).astype(np.float32)
    Q = np.concatenate([Q, np.array([[center[0], center[1], 0]], np.float32)])
    wa = O.antipodal(V, F, Q)
    wd = O.direct(V, F, Q)
    assert np.max(np.abs(wa - wd)) < 1e-6


def test_query_exactly_below_boundary_vertex_takes_perturbation_limit():
    V = np.array([[0.25, 0.5, 1.0], [1, 0, 1.2], [0, 1, 0.8]], np.float32)
    q = np.array([[0.25, 0.5, -0.3]], np.float32)      # vertex 0 exactly on the +z ray
    wa = O.antipodal(V, OCT_F, q)[0]
    assert wa == pytest.approx(O.direct(V, OCT_F, q)[0], abs=1e-7)


# ---------------------------------------------------------------- crossing count

def test_chi_binned_equals_brute_force_and_closed_mesh_parity():
    s, Q = W.config2(n_uniform=1500, n_near=1500)
    u1, d1 = O.chi(s.V, s.F, Q, use_bins=True)
    u2, d2 = O.chi(s.V, s.F, Q, use_bins=False)
    assert np.array_equal(u1, u2) and np.array_equal(d1, d2)
    # closed watertight mesh: chi(+z) == chi(-z) == inside indicator
    s, Q = W.config1(3000)
    u, d = O.chi(s.V, s.F, Q)
    assert np.array_equal(u, d)
    assert set(np.unique(u)) <= {0, 1}


# ---------------------------------------------------------------- distance

def test_point_triangle_distance_closed_forms():
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    Q = np.array([[0.2, 0.2, 0.5], [-1, -1, 0], [0.5, -2, 0], [2, 2, 1]], np.float32)
    d = O.distance(V, OCT_F, Q, 10.0)
    assert d[0] == pytest.approx(0.5, abs=1e-7)
    assert d[1] == pytest.approx(math.sqrt(2), abs=1e-7)
    assert d[2] == pytest.approx(2.0, abs=1e-7)
    assert d[3] == pytest.approx(math.sqrt(1.5 ** 2 * 2 + 1), abs=1e-6)
    assert O.distance(V, OCT_F, Q[3:], 0.1)[0] == pytest.approx(0.1)


def test_binned_distance_equals_brute_force():
    s, Q = W.config2(n_uniform=800, n_near=800)
    for cut in (1e-3, 2e-2):
        a = O.distance(s.V, s.F, Q, cut, use_bins=True)
        b = O.distance(s.V, s.F, Q, cut, use_bins=False)
        assert np.array_equal(a, b)


# ---------------------------------------------------------------- gradient (Supp. Alg. 3)

def _grad_case(seed=3, n=40):
    s = W.opened_spheres(seed=seed, n_surf=2, tris_per_surf=200)
    rng = np.random.default_rng(seed)
    P = rng.uniform(-1.2, 1.2, size=(n, 3))
    P = (np.round(P * 2**16) / 2**16).astype(np.float32)      # p +- 2^-10 stays exact in float32
    P = P[O.distance(s.V, s.F, P, 1.0) > 0.15]
    return s.V, s.F, P


def test_gradient_matches_finite_differences_of_direct_sum():
    # central differences of the direct triangle sum O1 (a different formula: no
    # boundary, no axis), Richardson-extrapolated to O(h^4)
    V, F, P = _grad_case()
    assert len(P) > 20

    def fd(h):
        G = np.zeros((len(P), 3))
        for a in range(3):
            e = np.zeros(3, np.float32)
            e[a] = h
            G[:, a] = (O.direct(V, F, P + e) - O.direct(V, F, P - e)) / (2 * h)
        return G

    h = 2.0 ** -10
    G = (4 * fd(h / 2) - fd(h)) / 3
    g = O.gradient(V, F, P)
    assert np.abs(g).max() > 0.05
    assert np.abs(G - g).max() < 1e-9


def test_gradient_biot_savart_segments():
    # grad of the solid angle bounded by a polygon is the field of a unit current
    # along it: per straight segment (r_a x r_b)(l_a + l_b) / (l_a l_b (l_a l_b + r_a.r_b))
    V, F, P = _grad_case(seed=5)
    fr, to = O.boundary(F)
    Pd = P.astype(np.float64)
    ra = V[fr].astype(np.float64)[None] - Pd[:, None]
    rb = V[to].astype(np.float64)[None] - Pd[:, None]
    la, lb = np.linalg.norm(ra, axis=2), np.linalg.norm(rb, axis=2)
    fac = (la + lb) / (la * lb * (la * lb + (ra * rb).sum(2)))
    B = (np.cross(ra, rb) * fac[..., None]).sum(1) / (4 * np.pi)
    g, l1 = O.gradient(V, F, P, with_l1=True)
    # Alg. 3's per-edge terms grow where a boundary vertex lies near the axis
    # through p and cancel in the sum; the rounding error scales with their norms
    err = np.abs(B - g).max(1)
    assert (err < 1e-11 * np.maximum(1.0, l1)).all()
    assert err[l1 < 10].max() < 1e-13


@pytest.mark.parametrize("axis", [(0, 0, -1), (1, 0, 0), (0.3, -0.5, 0.8)])
def test_gradient_independent_of_axis(axis):
    V, F, P = _grad_case(seed=7)
    g0, l0 = O.gradient(V, F, P, with_l1=True)
    g1, l1 = O.gradient(V, F, P, axis=axis, with_l1=True)
    # per-edge terms differ between axes; their sum may not (rounding of d, whose
    # parts can cancel, bounds the difference)
    assert np.abs(g1 - g0).max() < 1e-11 * max(1.0, l0.max(), l1.max())
    assert np.abs(g0).max() > 0.05


def test_gradient_of_closed_mesh_is_zero_and_far_field_decays():
    s, Q = W.config1()
    assert np.abs(O.gradient(s.V, s.F, Q[:50])).max() == 0.0
    # one triangle: |grad w| falls off like r^-3 along a ray
    g = O.gradient(OCT_V, OCT_F, [[10, 11, 12], [20, 22, 24]])
    ratio = np.linalg.norm(g[0]) / np.linalg.norm(g[1])
    assert 7.0 < ratio < 9.0


def _near_axis_case():
    # queries 0.7 below boundary vertices, 1e-7..1e-6 off their vertical line:
    # Alg. 1's D and Alg. 3's d cancel to ~(rho/l)^2 there
    s = W.opened_spheres(seed=40, n_surf=3, tris_per_surf=300)
    fr, _ = O.boundary(s.F)
    rng = np.random.default_rng(0)
    Q = []
    for v in s.V[fr[rng.choice(len(fr), min(40, len(fr)), replace=False)]].astype(np.float64):
        for rho in (1e-7, 3e-7, 1e-6):
            ang = rng.uniform(0, 2 * np.pi)
            Q.append([v[0] + rho * np.cos(ang), v[1] + rho * np.sin(ang), v[2] - 0.7])
    Q = np.array(Q, np.float32)
    return s.V, s.F, Q[O.distance(s.V, s.F, Q, 1.0) > 0.01]


def test_near_axis_antipodal_matches_direct():
    V, F, Q = _near_axis_case()
    assert len(Q) > 60
    assert np.abs(O.antipodal(V, F, Q) - O.direct(V, F, Q)).max() < 1e-12


def test_near_axis_gradient_matches_biot_savart_and_other_axes():
    V, F, Q = _near_axis_case()
    g, l1 = O.gradient(V, F, Q, with_l1=True)
    assert l1.max() > 1e5             # individual edge terms are huge and cancel
    fr, to = O.boundary(F)
    Pd = Q.astype(np.float64)
    ra = V[fr].astype(np.float64)[None] - Pd[:, None]
    rb = V[to].astype(np.float64)[None] - Pd[:, None]
    la, lb = np.linalg.norm(ra, axis=2), np.linalg.norm(rb, axis=2)
    B = (np.cross(ra, rb) * ((la + lb) / (la * lb * (la * lb + (ra * rb).sum(2))))[..., None]).sum(1) / (4 * np.pi)
    assert np.abs(B - g).max() < 1e-8
    assert np.abs(O.gradient(V, F, Q, axis=(0.3, 0.4, -0.5)) - g).max() < 1e-8


def test_weld_restores_the_indexed_boundary():
    # an exploded soup (private vertex copies per triangle) has every edge on the
    # boundary; welding equal positions gives back the indexed mesh's chain
    s = W.opened_spheres(seed=40, n_surf=3, tris_per_surf=300)
    e = W.explode(s, seed=1)
    assert len(O.boundary(e.F)[0]) == 3 * s.nf
    Fw, n = O.weld(e.V, e.F)
    assert n == len(np.unique(s.V[np.unique(s.F)], axis=0))
    key = lambda V, fr, to: sorted(map(tuple, np.concatenate([V[fr], V[to]], axis=1).tolist()))
    assert key(e.V, *O.boundary(Fw)) == key(s.V, *O.boundary(s.F))
    Q = np.random.default_rng(2).uniform(-1.2, 1.2, size=(300, 3)).astype(np.float32)
    w0, w1 = O.antipodal(s.V, s.F, Q), O.antipodal(e.V, Fw, Q)
    assert np.abs(w0 - w1).max() < 1e-12
    # +0 and -0 are one position
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [-0.0, 0, -0.0]], np.float32)
    Fz, n = O.weld(V, np.array([[0, 1, 2], [3, 2, 1]], np.int32))
    assert n == 3 and Fz[1].tolist() == [0, 2, 1]


def test_distance_to_zero_area_triangles():
    # A zero-area triangle is still part of the soup: as a point set it is its
    # segments, so the distance is the distance to them (closed forms below).
    # Two coincident corners (a needle), collinear distinct corners, and all
    # three at one point; the closest-point region tests would divide 0 by 0 on
    # the zero-length edge of the needle.
    needle_V = np.array([[0, 0, 1], [0, 0, 1], [0, 0, 0]], np.float32)
    line_V = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], np.float32)
    point_V = np.array([[0.5, 0.5, 0.5]] * 3, np.float32)
    F = np.array([[0, 1, 2]], np.int32)
    cases = [
        (needle_V, [[0, 0, 0], [0, 0, 0.5], [0, 0, 1], [1, 0, 0.5], [0, 0, -2], [0, 3, 0.5]], [0, 0, 0, 1, 2, 3]),
        (line_V, [[1, 1, 0], [3, 0, 0], [-1, 0, 0], [0.5, 0, 0], [2, 0, 2]], [1, 1, 1, 0, 2]),
        (point_V, [[0.5, 0.5, 0.5], [0.5, 0.5, 1.5], [1.5, 0.5, 0.5]], [0, 1, 1]),
    ]
    for V, Q, want in cases:
        Q = np.array(Q, np.float32)
        for bins in (True, False):
            d = O.distance(V, F, Q, 10.0, use_bins=bins)
            assert np.allclose(d, want, rtol=0, atol=1e-12), (V.tolist(), d.tolist(), want)
