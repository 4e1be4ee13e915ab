"""Surrogate MLP kernels (bf16 MFMA forward/backward, Adam) against the FP64
reference in oracle/mlp_ref.py, plus the band-fallback query against the
exact path."""
import numpy as np
import pytest

from oracle import mlp_ref as R
from paper_2605_01536_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _sur(gwn, seed=3, sigma=1.5):
    return gwn.Surrogate(seed=seed, sigma=sigma)


def _points(n, seed):
    return np.random.default_rng(seed).uniform(-1, 1, (n, 3)).astype(np.float32)


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 4097])
def test_forward_matches_reference(gwn, n):
    s = _sur(gwn)
    st = s.state()
    P = _points(n, 10 + n)
    y = s.forward(torch.from_numpy(P).cuda()).cpu().numpy().astype(np.float64)
    y_ref, _ = R.forward(st["theta"].astype(np.float64), st["G"].astype(np.float64), P, bf16=True)
    err = np.abs(y - y_ref)
    assert np.median(err) < 2e-4 * (1 + np.median(np.abs(y_ref)))
    assert err.max() < 5e-3 * (1 + np.abs(y_ref).max())


def test_gradient_matches_reference(gwn):
    s = _sur(gwn, seed=5)
    st = s.state()
    P = _points(3000, 7)
    t = np.random.default_rng(8).uniform(-0.5, 1.5, 3000).astype(np.float32)
    loss, g = s.loss_grad(torch.from_numpy(P).cuda(), torch.from_numpy(t).cuda())
    g = g.cpu().numpy().astype(np.float64)
    loss_ref, g_ref = R.loss_and_grad(st["theta"].astype(np.float64), st["G"].astype(np.float64), P, t, bf16=True)
    assert loss == pytest.approx(loss_ref, rel=2e-3)
    for (a, b, c) in R.offsets():
        for lo, hi in ((a, b), (b, c)):
            gg, gr = g[lo:hi], g_ref[lo:hi]
            rel = np.linalg.norm(gg - gr) / max(np.linalg.norm(gr), 1e-12)
            assert rel < 3e-2, f"params [{lo},{hi}): relative error {rel:.3e}"
    cos = g @ g_ref / (np.linalg.norm(g) * np.linalg.norm(g_ref))
    assert cos > 0.9995


def test_adam_step_matches_reference(gwn):
    s = _sur(gwn, seed=6)
    P = torch.from_numpy(_points(2048, 11)).cuda()
    t = torch.rand(2048, device="cuda")
    st0 = s.state()
    _, g = s.loss_grad(P, t)
    s.train_step(P, t, 1e-3)
    st1 = s.state()
    th_ref, m_ref, v_ref = R.adam_step(st0["theta"].astype(np.float64), np.zeros(R.N_PARAMS), np.zeros(R.N_PARAMS),
                                       g.cpu().numpy().astype(np.float64), 1, 1e-3)
    assert st1["step"] == 1
    assert np.max(np.abs(st1["theta"] - th_ref)) < 2e-6
    assert np.max(np.abs(st1["m"] - m_ref)) < 1e-6 * (1 + np.abs(m_ref).max())


def test_training_reduces_loss_on_winding_labels(gwn):
    soup = W.opened_spheres(seed=41, n_surf=6, tris_per_surf=600)
    m = gwn.Mesh(torch.from_numpy(soup.V).cuda(), torch.from_numpy(soup.F).cuda())
    X = torch.rand((40000, 3), device="cuda") * 2 - 1
    T = gwn.query_batch(m, X)
    s = _sur(gwn, seed=7, sigma=1.5)
    l0, _ = s.loss_grad(X, T)
    losses = gwn.train_surrogate(s, X, T, epochs=6, batch=4096, lr=3e-3, lr_final=3e-4)
    l1, _ = s.loss_grad(X, T)
    assert l1 < 0.2 * l0, (l0, l1, losses[-3:])


def test_checkpoint_resume_is_bit_identical(gwn, tmp_path):
    P = torch.from_numpy(_points(8192, 12)).cuda()
    t = torch.rand(8192, device="cuda")
    batches = [torch.arange(i * 1024, (i + 1) * 1024, device="cuda") for i in range(8)]
    a = _sur(gwn, seed=9)
    for i in range(4):
        a.train_step(P[batches[i]], t[batches[i]], 1e-3, want_loss=False)
    path = str(tmp_path / "ckpt.npz")
    a.save(path)
    for i in range(4, 8):
        a.train_step(P[batches[i]], t[batches[i]], 1e-3, want_loss=False)
    b = _sur(gwn, seed=123)          # different init, overwritten by the checkpoint
    b.load(path)
    for i in range(4, 8):
        b.train_step(P[batches[i]], t[batches[i]], 1e-3, want_loss=False)
    sa, sb = a.state(), b.state()
    for k in ("theta", "m", "v", "G"):
        assert np.array_equal(sa[k], sb[k]), k
    assert sa["step"] == sb["step"] == 8
    assert torch.equal(a.forward(P), b.forward(P))


def test_band_query_matches_network_and_exact_path(gwn):
    soup = W.opened_spheres(seed=42, n_surf=5, tris_per_surf=800)
    m = gwn.Mesh(torch.from_numpy(soup.V).cuda(), torch.from_numpy(soup.F).cuda())
    X = torch.rand((20000, 3), device="cuda") * 2 - 1
    T = gwn.query_batch(m, X)
    s = _sur(gwn, seed=8, sigma=1.5)
    gwn.train_surrogate(s, X, T, epochs=3, batch=4096, lr=3e-3)
    Q = torch.rand((30001, 3), device="cuda") * 2 - 1
    y = s.forward(Q)
    exact = gwn.query_batch(m, Q)
    w0, mask0, n0 = s.query(m, Q, 0.0, want_mask=True)
    assert n0 == 0 and torch.equal(w0, y) and int(mask0.sum()) == 0
    wa, maska, na = s.query(m, Q, 1e9, want_mask=True)
    assert na == Q.shape[0] and torch.equal(wa, exact)
    w3, mask3, n3 = s.query(m, Q, 0.3, want_mask=True)
    sel = (y - 0.5).abs() < 0.3
    assert torch.equal(mask3.bool(), sel) and n3 == int(sel.sum())
    assert torch.equal(w3[sel], exact[sel]) and torch.equal(w3[~sel], y[~sel])
