"""Parity at the full sizes of the named workloads, sampled where the oracle
cannot take every point:

* the 512^3 grid of the 1.05M-triangle opened-spheres soup in all-FP64 (the
  precision sweep's second arm), chi bit-exact and w within 1e-5 of the FP64
  oracle on 2,000 sampled points (Sec. 5.2 reports both precisions);
* the 256-soup batched workload as one captured plan: every point bit-equal to
  the single-mesh batch call, and 8 points per soup against the oracle.
"""
import numpy as np
import pytest

from paper_2605_01536_amd import workloads as W
from tests._util import TOL_FP32, TOL_FP64, compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_opened_spheres_grid_512_fp64_sampled(gwn):
    s, g = W.config4()
    m = gwn.Mesh(_dev(s.V), _dev(s.F))
    w, chi = gwn.query_grid(m, g.origin, g.spacing, g.dims, prec="fp64", want_chi=True)
    torch.cuda.synchronize()
    assert w.dtype == torch.float64 and w.shape[0] == 512 ** 3
    idx = np.sort(np.random.default_rng(4242).choice(g.n, 2000, replace=False))
    it = _dev(idx)
    P = W.grid_points(g, idx)
    e, n = compare(w[it].cpu().numpy(), chi[it].cpu().numpy(), s.V, s.F, P, TOL_FP64, "grid512-fp64")
    assert n > 1900
    # the FP32 arm on the same sample agrees with the FP64 one within the FP32 bar
    w32 = gwn.query_grid(m, g.origin, g.spacing, g.dims, prec="fp32")
    d = (w32[it].double() - w[it]).abs().max().item()
    assert d <= TOL_FP32, d


def test_ellipsoid_batch_256_soups_one_plan(gwn, monkeypatch):
    # batches of at most 8,192 points would take the split-boundary kernel (another
    # summation order); every soup here has at least 10,000 points, but keep the
    # per-point kernel explicitly
    monkeypatch.setenv("GWN_SPLIT_BOUNDARY", "0")
    soups, queries = W.config3()
    assert len(soups) == 256
    meshes = [gwn.Mesh(_dev(s.V), _dev(s.F)) for s in soups]
    offs = np.concatenate([[0], np.cumsum([q.shape[0] for q in queries])]).astype(np.int64)
    Q = _dev(np.concatenate(queries))
    nq = int(offs[-1])
    chi = torch.empty(nq, dtype=torch.int32, device="cuda")
    # the schedule the autotuner picks on this workload (128-query items, 8 waves
    # per SIMD, largest cost first, each soup's points in Morton order), fixed
    plan = gwn.MultiPlan(meshes, Q, offs, chi_out=chi, item_queries=128, waves_per_simd=8, order=2)
    w = plan.run().clone()
    torch.cuda.synchronize()
    inf = plan.info()
    assert inf["nmesh"] == 256 and inf["nqueries"] == nq
    wb = torch.empty(nq, device="cuda")
    cb = torch.empty(nq, dtype=torch.int32, device="cuda")
    for i, m in enumerate(meshes):
        a, b = int(offs[i]), int(offs[i + 1])
        gwn.query_batch(m, Q[a:b], out=wb[a:b], chi_out=cb[a:b])
    torch.cuda.synchronize()
    assert torch.equal(cb, chi)
    assert torch.equal(wb, w)
    rng = np.random.default_rng(7)
    worst = 0.0
    for i, s in enumerate(soups):
        a, b = int(offs[i]), int(offs[i + 1])
        idx = np.sort(rng.choice(b - a, 8, replace=False)) + a
        it = _dev(idx)
        e, _ = compare(w[it].cpu().numpy(), chi[it].cpu().numpy(), s.V, s.F, queries[i][idx - a], TOL_FP32,
                       f"soup {i}")
        worst = max(worst, e)
    print(f"256 soups, {nq} points: bit-equal to per-soup calls; max |w - oracle| over 2,048 samples {worst:.2e}")
