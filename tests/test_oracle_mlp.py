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


def test_half_rounding():
    x = np.array([1.0, 1.0 + 2 ** -11, 1.0 + 3 * 2 ** -12, 70000.0, -70000.0, 2.0 ** -20, 1e-9, 65504.0])
    r = R.round_half(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie -> even
    assert r[2] == 1.0 + 2 ** -10           # above the tie -> up
    assert r[3] == 65504.0 and r[4] == -65504.0   # saturated, not infinite
    assert r[5] == 2.0 ** -20               # a subnormal, exact
    assert r[6] == 0.0                      # below half of the smallest subnormal (2^-25)
    assert r[7] == 65504.0


def test_half_operands_of_bf16_weights_are_exact():
    # bf16 keeps 8 significant bits and half 11, so a bf16 weight in the half
    # normal range converts exactly; the half forward then differs from the bf16
    # forward only by the layer inputs' rounding (half: 2^-11 relative, bf16:
    # 2^-8), so it lies closer to the unrounded network (both keep bf16 weights)
    rng = np.random.default_rng(4)
    w = R.round_bf16(rng.choice([-1, 1], 4000) * rng.uniform(1, 2, 4000) * 2.0 ** rng.integers(-14, 15, 4000))
    assert np.array_equal(R.round_half(w), w)
    theta = rng.normal(0, 0.1, R.N_PARAMS)
    G = rng.normal(0, 1.0, (32, 3))
    P = rng.uniform(-1, 1, (300, 3))
    y, _ = R.forward(theta, G, P)
    yh, (xs, _) = R.forward(theta, G, P, half=True)
    yb, _ = R.forward(theta, G, P, bf16=True)
    assert all(np.array_equal(R.round_half(x), x) for x in xs)
    eh, eb = np.abs(yh - y).max(), np.abs(yb - y).max()
    assert eh < eb, (eh, eb)


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
