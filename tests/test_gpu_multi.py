"""Batched multi-mesh plans (one captured graph with a persistent kernel)
against the single-mesh path and the CPU oracle."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2605_01536_amd import workloads as W
from tests._util import TOL_FP32, TOL_FP64, compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _batch_of(gwn, n_mesh, seed, q_range=(200, 5000), tri_range=(100, 20000)):
    soups, queries = W.ellipsoid_batch(seed=seed, n_mesh=n_mesh, tri_range=tri_range, q_range=q_range)
    meshes = [gwn.Mesh(torch.from_numpy(s.V).cuda(), torch.from_numpy(s.F).cuda()) for s in soups]
    offs = np.concatenate([[0], np.cumsum([q.shape[0] for q in queries])]).astype(np.int64)
    Q = torch.from_numpy(np.concatenate(queries)).cuda()
    return soups, queries, meshes, offs, Q


def test_multi_equals_single_mesh_path_and_oracle(gwn, monkeypatch):
    # the per-point batch kernel runs the persistent kernel's arithmetic; small
    # batches would otherwise take the split-boundary path (other summation order)
    monkeypatch.setenv("GWN_SPLIT_BOUNDARY", "0")
    soups, queries, meshes, offs, Q = _batch_of(gwn, 24, seed=33)
    chi = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
    plan = gwn.MultiPlan(meshes, Q, offs, chi_out=chi)
    w = plan.run().clone()
    torch.cuda.synchronize()
    for m, s in enumerate(soups):
        a, b = int(offs[m]), int(offs[m + 1])
        wb, cb = gwn.query_batch(meshes[m], Q[a:b], want_chi=True)
        assert torch.equal(cb, chi[a:b])
        assert torch.equal(wb, w[a:b])        # same per-query arithmetic, bit for bit
    rng = np.random.default_rng(0)
    for m in rng.choice(len(soups), 6, replace=False):
        a, b = int(offs[m]), int(offs[m + 1])
        idx = rng.choice(b - a, min(300, b - a), replace=False)
        compare(w[a:b][torch.from_numpy(idx).cuda()].cpu().numpy(), chi[a:b][torch.from_numpy(idx).cuda()].cpu().numpy(),
                soups[m].V, soups[m].F, queries[m][idx], TOL_FP32, f"multi mesh {m}")


def test_multi_far_and_mixed_queries(gwn, monkeypatch):
    # per-lane edge pairs: queries inside a mesh's box in x and y but far from it
    # in z (single edges), far in x and y (far path) and ordinary ones, mixed in
    # the same waves; bit for bit the single-mesh path, and against the oracle
    monkeypatch.setenv("GWN_SPLIT_BOUNDARY", "0")
    soups, queries, meshes, offs, Q = _batch_of(gwn, 6, seed=35, q_range=(300, 900))
    Qh = Q.cpu().numpy()
    rng = np.random.default_rng(9)
    pick = rng.choice(Qh.shape[0], Qh.shape[0] // 3, replace=False)
    Qh[pick[0::3], 2] = np.float32(1e6) * np.sign(rng.standard_normal(pick[0::3].size)).astype(np.float32)
    Qh[pick[1::3], 2] = np.float32(3e35)
    Qh[pick[2::3], 0] = np.float32(-4e7)
    Q = torch.from_numpy(Qh).cuda()
    plan = gwn.MultiPlan(meshes, Q, offs)
    w = plan.run().clone()
    torch.cuda.synchronize()
    assert torch.isfinite(w).all()
    for m, s in enumerate(soups):
        a, b = int(offs[m]), int(offs[m + 1])
        wb, cb = gwn.query_batch(meshes[m], Q[a:b], want_chi=True)
        assert torch.equal(wb, w[a:b])
        compare(wb.cpu().numpy(), cb.cpu().numpy(), s.V, s.F, Qh[a:b], TOL_FP32, f"far-mixed-{m}")


@pytest.mark.parametrize("sched", [dict(item_queries=64, waves_per_simd=1, order=1),
                                   dict(item_queries=512, waves_per_simd=8, order=0),
                                   dict(item_queries=100, waves_per_simd=3, order=0),
                                   dict(item_queries=128, waves_per_simd=8, order=2),
                                   dict(item_queries=64, waves_per_simd=4, order=3)])
def test_schedules_agree(gwn, sched):
    soups, queries, meshes, offs, Q = _batch_of(gwn, 12, seed=34)
    ref = gwn.MultiPlan(meshes, Q, offs).run().clone()
    p = gwn.MultiPlan(meshes, Q, offs, **sched)
    inf = p.info()
    assert inf["item_queries"] % 64 == 0 and inf["nitems"] > 0 and inf["order"] == sched["order"]
    # the same bits whatever the schedule, Morton-ordered queries included
    assert torch.equal(p.run(), ref)
    assert torch.equal(p.run(), ref)


def test_graph_replays_with_eager_work_between(gwn):
    soups, queries, meshes, offs, Q = _batch_of(gwn, 10, seed=35)
    plan = gwn.MultiPlan(meshes, Q, offs)
    first = plan.run().clone()
    for rep in range(4):
        plan.w.fill_(-7.0)                                   # eager work on the same buffers
        junk = torch.randn(1 << 20, device="cuda").sum()      # unrelated eager kernels
        torch.cuda.synchronize()
        out = plan.run()
        torch.cuda.synchronize()
        assert torch.equal(out, first), f"replay {rep} differs"
        assert float(junk) == float(junk)


def test_autotune_and_cache(gwn, tmp_path):
    soups, queries, meshes, offs, Q = _batch_of(gwn, 16, seed=36)
    cache = str(tmp_path / "tune.jsonl")
    p1 = gwn.MultiPlan(meshes, Q, offs, autotune=True, tune_cache=cache)
    i1 = p1.info()
    assert i1["tuned"] == 1 and i1["tuned_ms"] > 0
    assert os.path.exists(cache) and "item_queries" in open(cache).read()
    w1 = p1.run().clone()
    p2 = gwn.MultiPlan(meshes, Q, offs, autotune=True, tune_cache=cache)   # served from the cache
    i2 = p2.info()
    assert i2["tuned"] == 1 and i2["tuned_ms"] == 0.0
    assert (i2["item_queries"], i2["waves_per_simd"], i2["order"]) == (i1["item_queries"], i1["waves_per_simd"], i1["order"])
    assert torch.equal(p2.run(), w1)


def test_multi_rejects_bad_arguments(gwn):
    soups, queries, meshes, offs, Q = _batch_of(gwn, 3, seed=37)
    with pytest.raises(gwn.GwnError):
        gwn.MultiPlan(meshes, Q, [1] + list(offs[1:]))
    with pytest.raises(gwn.GwnError):
        gwn.MultiPlan(meshes, Q, [0, 10, 5, int(offs[-1])])
    for bad in (4, -1):
        with pytest.raises(gwn.GwnError) as ei:
            gwn.MultiPlan(meshes, Q, offs, order=bad)
        assert ei.value.status == 1


def test_multi_fp64_equals_single_mesh_path_and_oracle(gwn, monkeypatch):
    # FP64 geometry in the persistent kernel: bit for bit the FP64 batch path
    # (ordinary, far-in-z and far-in-x/y queries), and the oracle within TOL_FP64
    monkeypatch.setenv("GWN_SPLIT_BOUNDARY", "0")
    soups, queries, meshes, offs, Q = _batch_of(gwn, 10, seed=38, q_range=(300, 2000))
    Qh = Q.cpu().numpy()
    rng = np.random.default_rng(11)
    pick = rng.choice(Qh.shape[0], Qh.shape[0] // 4, replace=False)
    Qh[pick[0::2], 2] = np.float32(1e6)
    Qh[pick[1::2], 0] = np.float32(-4e7)
    Q = torch.from_numpy(Qh).cuda()
    chi = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
    plan = gwn.MultiPlan(meshes, Q, offs, chi_out=chi, prec="fp64")
    w = plan.run().clone()
    torch.cuda.synchronize()
    assert w.dtype == torch.float64 and torch.isfinite(w).all()
    w32 = gwn.MultiPlan(meshes, Q, offs).run()
    for m, s in enumerate(soups):
        a, b = int(offs[m]), int(offs[m + 1])
        wb, cb = gwn.query_batch(meshes[m], Q[a:b], prec="fp64", want_chi=True)
        assert torch.equal(cb, chi[a:b])
        assert torch.equal(wb, w[a:b])
        idx = rng.choice(b - a, min(200, b - a), replace=False)
        ti = torch.from_numpy(idx).cuda()
        compare(w[a:b][ti].cpu().numpy(), chi[a:b][ti].cpu().numpy(), s.V, s.F, Qh[a:b][idx], TOL_FP64,
                f"multi fp64 mesh {m}")
    # the two precisions agree to the FP32 bound
    assert float((w32.double() - w).abs().max()) < TOL_FP32


@pytest.mark.parametrize("sched", [dict(item_queries=64, waves_per_simd=2, order=1),
                                   dict(item_queries=256, waves_per_simd=8, order=2)])
def test_schedules_agree_fp64(gwn, sched):
    soups, queries, meshes, offs, Q = _batch_of(gwn, 8, seed=39)
    ref = gwn.MultiPlan(meshes, Q, offs, prec="fp64").run().clone()
    assert torch.equal(gwn.MultiPlan(meshes, Q, offs, prec="fp64", **sched).run(), ref)


def test_multi_rejects_unknown_precision(gwn):
    import ctypes
    soups, queries, meshes, offs, Q = _batch_of(gwn, 2, seed=40)
    L = gwn.load()
    gwn.MultiPlan(meshes, Q, offs).close()          # binds the multi entry points
    hs = (ctypes.c_void_p * 2)(*[m.handle.value for m in meshes])
    o = (ctypes.c_int64 * 3)(*[int(x) for x in offs])
    w = torch.empty(int(offs[-1]), dtype=torch.float64, device="cuda")
    h = ctypes.c_void_p()
    base = Q.data_ptr()
    st = L.gwn_multi_create(hs, 2, base, base + 4, base + 8, 3, o, 2, w.data_ptr(), None, None, None,
                            ctypes.byref(h))
    assert st == 1 and not h.value


def test_multi_empty_meshes_and_queryless_meshes(gwn, monkeypatch):
    # empty meshes, meshes without queries and meshes with one query in one
    # plan, in both precisions, input or Morton order, tuned or not: every
    # replay equal to the single-mesh calls bit for bit
    from tests.test_gpu_random_soups import _soup
    monkeypatch.setenv("GWN_SPLIT_BOUNDARY", "0")
    rng = np.random.default_rng(5)
    meshes, qs = [], []
    for k in range(40):
        if k % 7 == 3:
            V, F = np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32)
        else:
            V, F, _ = _soup(1000 + k)
        meshes.append(gwn.Mesh(torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()))
        nq = 0 if k % 5 == 2 else (1 if k % 11 == 4 else int(rng.integers(1, 400)))
        qs.append(rng.uniform(-1.2, 1.2, (nq, 3)).astype(np.float32))
    offs = np.concatenate([[0], np.cumsum([q.shape[0] for q in qs])]).astype(np.int64)
    Q = torch.from_numpy(np.concatenate(qs)).cuda()
    for prec, order, iq, tune in (("fp32", 0, 0, False), ("fp32", 2, 64, False), ("fp64", 3, 128, False),
                                  ("fp32", 0, 0, True)):
        chi = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
        plan = gwn.MultiPlan(meshes, Q, offs, chi_out=chi, prec=prec, order=order, item_queries=iq, autotune=tune)
        w = plan.run().clone()
        assert torch.equal(plan.run(), w)
        for i, m in enumerate(meshes):
            a, b = int(offs[i]), int(offs[i + 1])
            wb, cb = gwn.query_batch(m, Q[a:b], prec=prec, want_chi=True)
            assert torch.equal(wb, w[a:b]) and torch.equal(cb, chi[a:b]), (prec, order, i)
