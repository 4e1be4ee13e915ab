"""Per-mesh query tuning: explicit settings take the paths they name with the
results the paths guarantee (crossing counts always bit-equal; the Morton
order never changes w; the split form and the samples per lane agree to
rounding, against the oracle too), and the autotuner times the candidates,
sets a tuning within the candidate ranges, and stores and reuses it through
its cache."""
import json

import numpy as np
import pytest

from paper_2605_01536_amd import workloads as W
from tests._util import TOL_FP32, TOL_FP64, compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torus(gwn):
    s = W.torus_soup(seed=2)
    return s, gwn.Mesh(torch.from_numpy(s.V).cuda(), torch.from_numpy(s.F).cuda())


def test_set_and_get_tuning(gwn, torus):
    s, m = torus
    assert m.tuning() == {"split_max_points": [0, 0], "order_min_points": 0, "grid_samples_per_lane": [0, 0],
                          "tuned": 0}
    m.set_tuning((1024, -1), 1 << 16, (4, 2))
    assert m.tuning()["split_max_points"] == [1024, -1] and m.tuning()["grid_samples_per_lane"] == [4, 2]
    for bad in (dict(split_max_points=(-2, 0)), dict(order_min_points=-5), dict(grid_samples_per_lane=(3, 0)),
                dict(grid_samples_per_lane=(0, 8))):
        with pytest.raises(gwn.GwnError):
            m.set_tuning(**bad)
    m.set_tuning()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_explicit_tuning_paths_agree(gwn, torus, prec, monkeypatch):
    for v in ("GWN_SPLIT_BOUNDARY", "GWN_ORDER_QUERIES", "GWN_GRID_SAMPLES_PER_LANE"):
        monkeypatch.delenv(v, raising=False)
    s, m = torus
    p = 0 if prec == "fp32" else 1
    lo, hi = s.bbox()
    Q = torch.from_numpy(W.uniform_box(np.random.default_rng(11), 300_000, lo, hi)).cuda()
    tol = TOL_FP32 if prec == "fp32" else TOL_FP64
    # ordering on from 2 points versus never: the same bits
    m.set_tuning(order_min_points=2)
    w1, c1 = gwn.query_batch(m, Q, prec=prec, want_chi=True)
    m.set_tuning(order_min_points=-1)
    w2, c2 = gwn.query_batch(m, Q, prec=prec, want_chi=True)
    assert torch.equal(w1, w2) and torch.equal(c1, c2)
    # a 20,000-point batch split (tuned threshold) and per lane (never): same chi, w to rounding, both at the oracle
    q = Q[:20_000]
    split = [0, 0]
    split[p] = 32768
    m.set_tuning(split_max_points=tuple(split))
    ws, cs = gwn.query_batch(m, q, prec=prec, want_chi=True)
    split[p] = -1
    m.set_tuning(split_max_points=tuple(split))
    wl, cl = gwn.query_batch(m, q, prec=prec, want_chi=True)
    assert torch.equal(cs, cl)
    assert (ws.double() - wl.double()).abs().max().item() < (1e-5 if prec == "fp32" else 1e-12)
    idx = np.random.default_rng(3).choice(20_000, 400, replace=False)
    compare(ws.cpu().numpy()[idx], cs.cpu().numpy()[idx], s.V, s.F, q.cpu().numpy()[idx], tol, "split")
    # grid samples per lane: every allowed value against the oracle on a small grid
    g = W.GridSpec(origin=tuple(float(x) for x in lo), spacing=tuple(float(x) for x in (hi - lo) / [12, 10, 300]),
                   dims=(12, 10, 300))
    P = W.grid_points(g)
    pick = np.random.default_rng(4).choice(g.n, 500, replace=False)
    ref = None
    for zb in ((1, 2, 4, 8) if prec == "fp32" else (1, 2, 4)):
        z = [0, 0]
        z[p] = zb
        m.set_tuning(grid_samples_per_lane=tuple(z))
        w, c = gwn.query_grid(m, g.origin, g.spacing, g.dims, prec=prec, want_chi=True)
        if ref is None:
            ref = c.clone()
        assert torch.equal(c, ref)
        compare(w.cpu().numpy()[pick], c.cpu().numpy()[pick], s.V, s.F, P[pick], tol, f"zb={zb}")
    m.set_tuning()


def test_autotune_sets_and_caches_a_tuning(gwn, tmp_path, monkeypatch):
    for v in ("GWN_SPLIT_BOUNDARY", "GWN_ORDER_QUERIES", "GWN_GRID_SAMPLES_PER_LANE"):
        monkeypatch.delenv(v, raising=False)
    s = W.opened_spheres(seed=44, n_surf=16, tris_per_surf=4000)
    V, F = torch.from_numpy(s.V).cuda(), torch.from_numpy(s.F).cuda()
    m = gwn.Mesh(V, F)
    cache = str(tmp_path / "tune.jsonl")
    t = m.autotune("fp32", grid_nz=256, reps=2, cache=cache)
    assert t["tuned"] & 1
    sm = t["split_max_points"][0]
    assert sm == -1 or (256 <= sm <= 32768 and sm & (sm - 1) == 0)
    om = t["order_min_points"]
    assert om == -1 or ((1 << 14) <= om <= (1 << 20) and om & (om - 1) == 0)
    assert t["grid_samples_per_lane"][0] in (1, 2, 4, 8)
    lines = [json.loads(x) for x in open(cache)]
    assert len(lines) == 1 and "prec=0" in lines[0]["key"] and "nz=256" in lines[0]["key"]
    # a second mesh of the same size takes the stored choice without timing
    m2 = gwn.Mesh(V, F)
    t2 = m2.autotune("fp32", grid_nz=256, cache=cache)
    assert t2 == t and len(open(cache).readlines()) == 1
    # and the tuned mesh answers like the untuned one (chi bit-equal, w to rounding)
    Q = torch.rand((50_000, 3), device="cuda") * 2 - 1
    w1, c1 = gwn.query_batch(m, Q, want_chi=True)
    m3 = gwn.Mesh(V, F)
    w3, c3 = gwn.query_batch(m3, Q, want_chi=True)
    assert torch.equal(c1, c3) and (w1 - w3).abs().max().item() < 1e-5
    print("tuned:", t)
