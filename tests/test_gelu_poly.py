"""The inference GELU's polynomial in the kernel source is the one the committed
fitting script produces, and its packed half-precision evaluation meets the
stated bound against GELU(z) = z Phi(z) computed from math.erf in FP64."""
import math
import os
import re
import subprocess
import sys

import numpy as np

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2605_01536_amd", "csrc")

# |GELU error| / |z| of the half evaluation: 2.4e-3 on Phi (the fit with half
# coefficients, 1.2e-3, and the rounding of each half operation), plus the
# final product's rounding (2^-11 relative)
BOUND = 2.9e-3


def _kernel():
    src = open(os.path.join(CSRC, "mlp.hip")).read()
    table = re.search(r"kGeluH\[\]\s*=\s*\{([^}]*)\}", src).group(1)
    c = float(re.search(r"kGeluHC\s*=\s*([0-9.]+)f", src).group(1))
    return [float(x.strip().rstrip("f")) for x in table.split(",")], c


def _h(a):
    # one rounding to IEEE half (round to nearest even), back to float64
    return np.asarray(a, np.float64).astype(np.float16).astype(np.float64)


def _eval_half(table, c, z):
    # the kernel's arithmetic, each packed half operation rounded once: z to
    # half, t = clamp(z s + 1/2, 0, 1) with s = 1/(2c) in half, u = 2t - 1,
    # v = u^2, Horner with fused multiply-adds, Phi = u Q + 1/2, GELU = z Phi
    s = float(np.float16(0.5 / c))
    zh = _h(np.asarray(z, np.float32))
    t = np.clip(_h(zh * s + 0.5), 0.0, 1.0)
    u = _h(2.0 * t - 1.0)
    v = _h(u * u)
    q = np.full_like(v, table[0])
    for a in table[1:]:
        q = _h(q * v + a)
    return _h(zh * _h(u * q + 0.5))


def _gelu(z):
    z = np.asarray(z, np.float64)
    return z * 0.5 * (1.0 + np.vectorize(math.erf)(z / math.sqrt(2.0)))


def test_table_matches_generator():
    table, c = _kernel()
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_gelu_poly.py"), "4", repr(c)], capture_output=True,
                         text=True, check=True).stdout
    gen = [float(x.strip().rstrip("f")) for x in re.search(r"\{([^}]*)\}", out).group(1).split(",")]
    assert gen == table
    # every coefficient is a half-precision value (the kernel converts them exactly)
    assert all(float(np.float16(a)) == a for a in table)


def test_half_gelu_error_bound():
    table, c = _kernel()
    z = np.linspace(-30.0, 30.0, 600001).astype(np.float32)
    g = _eval_half(table, c, z)
    zz = z.astype(np.float64)
    err = np.abs(g - _gelu(zz))
    assert np.all(err <= BOUND * np.abs(zz)), float((err / np.maximum(np.abs(zz), 1e-30)).max())
    # exact at 0; odd part: GELU(z) - GELU(-z) = z up to the bound
    assert _eval_half(table, c, np.float32(0.0)) == 0.0
    assert np.all(np.abs((g - _eval_half(table, c, -z)) - zz) <= 2 * BOUND * np.abs(zz))
    # saturates to z and to (nearly) 0 far out
    far = np.abs(zz) > 6
    assert np.all(np.abs(g[far & (zz > 0)] - zz[far & (zz > 0)]) <= BOUND * zz[far & (zz > 0)])
    assert np.all(np.abs(g[far & (zz < 0)]) <= BOUND * np.abs(zz[far & (zz < 0)]))


def test_half_gelu_against_a_sampled_grid_of_small_z():
    # where the activations mostly fall (|z| <= 3), the mean error is far below
    # the worst case: the fit's error oscillates in sign
    table, c = _kernel()
    z = np.random.default_rng(0).normal(0.0, 1.0, 200000).astype(np.float32)
    e = _eval_half(table, c, z) - _gelu(z.astype(np.float64))
    assert abs(float(np.mean(e))) < 2e-4 and float(np.sqrt(np.mean(e * e))) < 1.5e-3
