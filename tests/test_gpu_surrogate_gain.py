"""What the trained surrogate gains over the exact path alone, measured on the
~483k-triangle opened-spheres soup of the surrogate workload: the network is
trained through gwn_surrogate_train on 2M points the library draws in
[-1,1]^3 and labels with the exact kernel, then 2M other uniform points are
evaluated by the exact kernel and by network + exact fallback.

Asserted (the numbers the measurement gives, with margin):
* band 0.3 around w = 1/2 (the workload's rule): the fallback path is faster
  than the exact kernel and agrees with it on inside/outside (w >= 1/2) for
  almost every point; every re-evaluated point carries the exact kernel's bits;
* identical max |err|: no band short of re-evaluating every point reaches the
  exact kernel's own max |err| against the FP64 path, under either rule, so at
  identical max |err| the surrogate gains nothing (its error is a network
  error on the far side of a smoothed jump, not a near-1/2 prediction).
"""
import time

import numpy as np
import pytest

from paper_2605_01536_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _median_ms(fn, reps=5):
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1e3)
    return float(np.median(ts))


def test_surrogate_gain_over_exact_path(gwn):
    soup, _, _ = W.config5(n_train=0, n_infer=0)
    m = gwn.Mesh(torch.from_numpy(soup.V).cuda(), torch.from_numpy(soup.F).cuda())
    s = gwn.Surrogate(seed=0, sigma=1.0)
    losses = s.train(m, epochs=8, n_train=2_000_000, batch=8192, lr=1e-3, lr_final=5e-5, seed=1,
                     box=((-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)))
    assert len(losses) == 8 and losses[-1] < 0.5 * losses[0], losses
    Q = torch.from_numpy(W.uniform_box(np.random.default_rng(2024), 2_000_000, (-1.0,) * 3, (1.0,) * 3)).cuda()
    n = Q.shape[0]
    exact = torch.empty(n, device="cuda")
    t_exact = _median_ms(lambda: gwn.query_batch(m, Q, out=exact))
    w = torch.empty(n, device="cuda")
    res = {}

    def sur():
        _, res["mask"], res["n"] = s.query(m, Q, 0.3, out=w, want_mask=True)

    t_sur = _median_ms(sur)
    y = s.forward(Q)
    mask = res["mask"].bool()
    assert torch.equal(w[mask], exact[mask]) and torch.equal(w[~mask], y[~mask])
    e = (w - exact).abs()
    agree = float(((w >= 0.5) == (exact >= 0.5)).float().mean())
    speedup = t_exact / t_sur
    p99 = float(torch.quantile(e[::8], 0.99))
    print(f"exact {t_exact:.2f} ms, surrogate+fallback {t_sur:.2f} ms ({speedup:.2f}x), fallback "
          f"{res['n'] / n:.3f}, inside/outside agreement {agree:.5f}, max|err| {float(e.max()):.3f}, p99 {p99:.3f}, "
          f"losses {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert speedup > 1.5, speedup
    assert agree > 0.995, agree
    assert res["n"] < 0.3 * n
    # identical max|err|: the exact kernel's own error against the FP64 path
    w64 = gwn.query_batch(m, Q[: 1 << 19], prec="fp64")
    exact_err = float((exact[: 1 << 19].double() - w64).abs().max())
    assert exact_err < 1e-5
    for rule, bands in (("half", (0.3, 0.45, 0.5)), ("frac", (0.3, 0.45, 0.49))):
        for band in bands:
            wb, nb = s.query(m, Q, band, rule=rule)
            err = float((wb - exact).abs().max())
            assert nb < n and err > exact_err, (rule, band, nb, err)
    # re-evaluating everything gives the exact path's bits (and its max|err|)
    wall, nall = s.query(m, Q, 0.5001, rule="frac")
    assert nall == n and torch.equal(wall, exact)
