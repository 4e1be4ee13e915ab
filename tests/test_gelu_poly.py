"""The inference GELU's polynomial in the kernel source is the one the committed
fitting script produces, and its float32 evaluation meets the stated bound
against GELU(z) = z Phi(z) computed from math.erf in FP64."""
import math
import os
import re
import subprocess
import sys

import numpy as np

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2605_01536_amd", "csrc")


def _kernel_table():
    src = open(os.path.join(CSRC, "mlp.hip")).read()
    m = re.search(r"kGeluP\[\]\s*=\s*\{([^}]*)\}", src)
    return [np.float32(x.strip().rstrip("f")) for x in m.group(1).split(",")]


def _eval_f32(table, z):
    # the kernel's arithmetic: clamp, square, Horner with fused multiply-adds, fma(zc, P, 1/2), product
    z = np.asarray(z, dtype=np.float32)
    zc = np.clip(z, np.float32(-4.0), np.float32(4.0))
    x = (zc * zc).astype(np.float32)
    p = np.full_like(x, table[0])
    for a in table[1:]:
        p = (p.astype(np.float64) * x + np.float64(a)).astype(np.float32)
    h = (zc.astype(np.float64) * p + 0.5).astype(np.float32)
    return (z * h).astype(np.float32)


def test_table_matches_generator():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_gelu_poly.py"), "7", "4.0"], capture_output=True,
                         text=True, check=True).stdout
    gen = [np.float32(x.strip().rstrip("f")) for x in re.search(r"\{([^}]*)\}", out).group(1).split(",")]
    assert gen == _kernel_table()


def test_float32_gelu_error_bound():
    z = np.linspace(-30.0, 30.0, 600001).astype(np.float32)
    g = _eval_f32(_kernel_table(), z).astype(np.float64)
    zz = z.astype(np.float64)
    ref = zz * 0.5 * (1.0 + np.vectorize(math.erf)(zz / math.sqrt(2.0)))
    err = np.abs(g - ref)
    assert np.all(err <= 5.3e-5 * np.abs(zz) + 1e-30), float((err / np.maximum(np.abs(zz), 1e-30)).max())
    # exact at 0, odd part exact: GELU(z) - GELU(-z) = z
    assert _eval_f32(_kernel_table(), np.float32(0.0)) == 0.0
    # saturates to z and to (nearly) 0 far out
    assert np.allclose(g[zz > 6], zz[zz > 6], rtol=5.3e-5, atol=0) and np.all(np.abs(g[zz < -6]) <= 5.3e-5 * np.abs(zz[zz < -6]))
