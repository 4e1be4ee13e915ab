"""Pins of the parametric-surface oracle (Alg. 2 on cubic Bezier patches)
against the quadrature table's exactness, closed forms, an independent
formula (the direct triangle sum of a fine triangulation) and invariants."""
import numpy as np
import pytest

import oracle as O
from tests._util import bezier_tessellate, flat_bezier_patch, bezier_cube


def test_gk15_table_exactness():
    # the 15-point Kronrod rule integrates polynomials of degree <= 23 exactly,
    # its embedded 7-point Gauss rule those of degree <= 13 (and not 14)
    a, b = -0.3, 1.7
    for k in range(24):
        K, G = O.gk15_poly(k, a, b)
        exact = (b ** (k + 1) - a ** (k + 1)) / (k + 1)
        assert abs(K - exact) <= 1e-13 * max(1.0, abs(exact)), k
        if k <= 13:
            assert abs(G - exact) <= 1e-13 * max(1.0, abs(exact)), k
    K, G = O.gk15_poly(14, a, b)
    exact = (b ** 15 - a ** 15) / 15
    assert abs(G - exact) > 1e-8 * abs(exact) and abs(K - exact) < 1e-12 * abs(exact)


@pytest.mark.parametrize("h", [0.05, 0.3, 1.0, 2.5, 10.0])
def test_flat_square_on_its_axis(h):
    # a 2 x 2 square (a planar bicubic patch, normal +z) seen from (0, 0, +-h):
    # |w| = asin(1 / (1 + h^2)) / pi, negative on the normal's side
    P = flat_bezier_patch(-1, 1, -1, 1)[None]
    exact = np.arcsin(1.0 / (1.0 + h * h)) / np.pi
    w, chi, di = O.parametric(P, np.array([[0.0, 0.0, h], [0.0, 0.0, -h]]))
    assert np.all(di >= 0)
    assert abs(w[0] + exact) < 1e-12 and abs(w[1] - exact) < 1e-12
    # the other orientation (u and v swapped) flips the sign
    Pf = P.reshape(1, 4, 4, 3).transpose(0, 2, 1, 3).reshape(1, 16, 3)
    wf, _, _ = O.parametric(Pf, np.array([[0.0, 0.0, h]]))
    assert abs(wf[0] - exact) < 1e-12


def test_closed_cube_is_an_inside_test():
    # six planar patches sharing their edges: every boundary curve cancels and
    # w is the crossing count alone, 1 inside and 0 outside
    C = bezier_cube()
    assert len(O.bezier_boundary(C)) == 0
    Q = np.random.default_rng(0).uniform(-0.5, 1.5, size=(300, 3))
    w, chi, di = O.parametric(C, Q)
    inside = np.all((Q > 0) & (Q < 1), axis=1)
    assert np.all(di >= 0)
    assert np.array_equal(w, inside.astype(float))


def test_curved_patches_match_fine_triangulations():
    # random cubic patches (control points in the unit cube, as in the paper's
    # 100-patch benchmark) against the direct triangle sum over an n x n
    # triangulation of each patch: the difference falls as n^-2
    rng = np.random.default_rng(5)
    P = rng.uniform(0, 1, size=(3, 16, 3))
    Q = rng.uniform(-0.5, 1.5, size=(60, 3))
    w, chi, di = O.parametric(P, Q)
    assert np.all(di >= 0)
    errs = []
    for n in (48, 96):
        V, F = bezier_tessellate(P, n)
        wm = O.direct(V, F, Q.astype(np.float32))
        far = O.distance(V, F, Q.astype(np.float32), 0.05) >= 0.05
        errs.append(float(np.abs(w - wm)[far].max()))
        assert far.sum() > 40
    assert errs[1] < 1e-4 and errs[1] < errs[0] / 3.0, errs


def test_direction_independence_and_linearity():
    rng = np.random.default_rng(8)
    P = rng.uniform(0, 1, size=(4, 16, 3))
    Q = rng.uniform(-0.5, 1.5, size=(80, 3))
    w, _, di = O.parametric(P, Q)
    w2, _, di2 = O.parametric(P, Q, dirs=O.PARAM_DIRS[1:])
    ok = (di >= 0) & (di2 >= 0)
    assert ok.all()
    assert np.abs(w - w2).max() < 1e-10
    # union = sum; a patch with u reversed has the opposite orientation
    wa, _, _ = O.parametric(P[:2], Q)
    wb, _, _ = O.parametric(P[2:], Q)
    assert np.abs(w - (wa + wb)).max() < 1e-10
    Pr = P.reshape(-1, 4, 4, 3)[:, ::-1].reshape(-1, 16, 3)
    wr, _, _ = O.parametric(Pr, Q)
    assert np.abs(w + wr).max() < 1e-10


def test_boundary_cancellation():
    # two patches sharing an edge leave 6 curves; a patch with its reversed copy
    # leaves none and w = 0
    A = flat_bezier_patch(0, 1, 0, 1)
    B = flat_bezier_patch(1, 2, 0, 1)
    assert len(O.bezier_boundary(np.stack([A, B]))) == 6
    Ar = A.reshape(4, 4, 3)[::-1].reshape(16, 3)
    assert len(O.bezier_boundary(np.stack([A, Ar]))) == 0
    Q = np.random.default_rng(2).uniform(-1, 2, size=(50, 3))
    w, _, di = O.parametric(np.stack([A, Ar]), Q)
    assert np.all(di >= 0) and np.abs(w).max() == 0.0
