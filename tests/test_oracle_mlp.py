"""Pins for the FP64 surrogate reference: its gradient against central finite
differences, closed forms of GELU and of the first Adam step, bf16 rounding."""
import math

import numpy as np
import pytest

from oracle import mlp_ref as R


def _params(rng, scale=0.2):
    return rng.normal(0, scale, R.N_PARAMS)


def test_parameter_count_and_layout():
    assert R.N_PARAMS == 57985
    off = R.offsets()
    assert off[0] == (0, 8192, 8320) and off[4] == (57856, 57984, 57985)


def test_gelu_closed_forms():
    z = np.array([0.0, 1.0, -1.0, 6.0, -6.0])
    g = R.gelu(z)
    assert g[0] == 0.0
    assert g[1] == pytest.approx(0.8413447460685429, abs=1e-15)     # Phi(1)
    assert g[2] == pytest.approx(-0.15865525393145707, abs=1e-15)
    assert g[3] == pytest.approx(6.0, abs=1e-8) and abs(g[4]) < 1e-8
    assert R.gelu_grad(np.array([0.0]))[0] == 0.5
    h = 1e-6
    zz = np.linspace(-3, 3, 13)
    fd = (R.gelu(zz + h) - R.gelu(zz - h)) / (2 * h)
    assert np.max(np.abs(fd - R.gelu_grad(zz))) < 1e-8


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.0e-3], np.float32)
    r = R.round_bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie -> even
    assert r[2] == 1.0 + 2 ** -7            # above the tie -> up
    assert r[3] == -2.5
    assert abs(r[4] - 3e-3) / 3e-3 < 2 ** -8


@pytest.mark.parametrize("bf16", [False])
def test_gradient_matches_central_differences(bf16):
    rng = np.random.default_rng(0)
    theta = _params(rng)
    G = rng.normal(0, 1.0, (32, 3))
    P = rng.uniform(-1, 1, (20, 3))
    t = rng.uniform(-1, 2, 20)
    loss, g = R.loss_and_grad(theta, G, P, t)
    idx = np.concatenate([rng.choice(R.N_PARAMS, 40, replace=False), [8191, 8192, 57983, 57984, 24703, 41216]])
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        lp, _ = R.loss_and_grad(tp, G, P, t)
        lm, _ = R.loss_and_grad(tm, G, P, t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, f"param {i}: fd {fd} vs {g[i]}"


def test_first_adam_step_is_signed_learning_rate():
    rng = np.random.default_rng(1)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = R.adam_step(th, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    assert np.allclose(th - new, 1e-3 * np.sign(g), atol=1e-9)
