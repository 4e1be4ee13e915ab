"""The FP32 arctangent polynomial in the kernel header is the one the committed
fitting script produces, and it meets its stated error bound."""
import os
import re
import subprocess
import sys

import numpy as np

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2605_01536_amd", "csrc")


def _kernel_table():
    src = open(os.path.join(CSRC, "gwn_kernels.h")).read()
    m = re.search(r"kAtanQ\[8\]\s*=\s*\{([^}]*)\}", src)
    return [float(x.strip().rstrip("f")) for x in m.group(1).split(",")]


def test_table_matches_generator():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_atan_poly.py"), "7"], capture_output=True,
                         text=True, check=True).stdout
    gen = [float(x.strip().rstrip("f")) for x in re.search(r"\{([^}]*)\}", out).group(1).split(",")]
    assert np.allclose(gen, _kernel_table(), rtol=0, atol=0)


def test_polynomial_relative_error_in_float32():
    q = [np.float32(c) for c in _kernel_table()]
    t = np.linspace(-1, 1, 200001, dtype=np.float32)
    t = t[t != 0]
    x = (t * t).astype(np.float32)
    acc = np.full_like(x, q[0])
    for c in q[1:]:
        acc = (acc * x + c).astype(np.float32)
    a = ((t * x).astype(np.float32) * acc + t).astype(np.float32).astype(np.float64)
    ref = np.arctan(t.astype(np.float64))
    rel = np.abs(a - ref) / np.abs(ref)
    assert rel.max() < 2e-7
    assert abs(np.mean((a - ref) / np.abs(ref))) < 1e-8     # no systematic bias


def _pair_table():
    src = open(os.path.join(CSRC, "gwn_kernels.h")).read()
    m = re.search(r"kAtanP\[5\]\s*=\s*\{([^}]*)\}", src)
    return [float(x.strip().rstrip("f")) for x in m.group(1).split(",")]


def _inv_tan():
    src = open(os.path.join(CSRC, "gwn_kernels.h")).read()
    return float(re.search(r"kInvTan\s*=\s*([0-9.]+)f", src).group(1))


def test_pair_table_matches_generator():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_atan_poly.py"), "4", "pform"], capture_output=True,
                         text=True, check=True).stdout
    gen = [float(x.strip().rstrip("f")) for x in re.search(r"\{([^}]*)\}", out).group(1).split(",")]
    assert np.allclose(gen, _pair_table(), rtol=0, atol=0)


def test_pair_polynomial_relative_error_in_float32():
    # the edge-pair arctangent t P(t^2) on |t| <= tan(pi/8) (slightly beyond,
    # for rounding), with the product taken as the kernel's final FMA does
    q = [np.float32(c) for c in _pair_table()]
    tm = np.tan(np.pi / 8) * (1 + 1e-6)
    t = np.linspace(-tm, tm, 200001).astype(np.float32)
    t = t[t != 0]
    x = (t * t).astype(np.float32)
    p = np.full_like(x, q[0])
    for c in q[1:]:
        p = (p * x + c).astype(np.float32)
    a = (t.astype(np.float64) * p.astype(np.float64)).astype(np.float32).astype(np.float64)
    ref = np.arctan(t.astype(np.float64))
    rel = (a - ref) / np.abs(ref)
    assert np.abs(rel).max() < 1.5e-7
    assert abs(np.mean(rel)) < 3e-8          # small systematic bias


def test_pair_window_keeps_product_in_range():
    # |N| < D / kInvTan for both edges (kInvTan >= cot(pi/16)) puts the product
    # (D1 + i N1)(D2 + i N2) in the right half-plane with |Im/Re| < tan(pi/8),
    # evaluated in float32 as the kernel does (N1 N2 rounded first, then FMAs)
    k = _inv_tan()
    assert k >= 1 / np.tan(np.pi / 16)
    rng = np.random.default_rng(0)
    D1 = rng.uniform(1e-3, 1e4, 200000).astype(np.float32)
    D2 = rng.uniform(1e-3, 1e4, 200000).astype(np.float32)
    N1 = (D1 / np.float32(k) * rng.uniform(-1, 1, D1.size).astype(np.float32)).astype(np.float32)
    N2 = (D2 / np.float32(k) * rng.uniform(-1, 1, D2.size).astype(np.float32)).astype(np.float32)
    edge = rng.random(D1.size) < 0.1          # at the window's edge
    N1[edge] = np.nextafter((D1[edge] / np.float32(k)).astype(np.float32), np.float32(0))
    N2[edge] = -np.nextafter((D2[edge] / np.float32(k)).astype(np.float32), np.float32(0))
    n12 = (N1.astype(np.float64) * N2).astype(np.float32)
    re = (D1.astype(np.float64) * D2 - n12).astype(np.float32)
    im = (D1.astype(np.float64) * N2 + (N1.astype(np.float64) * D2).astype(np.float32)).astype(np.float32)
    assert (re > 0).all()
    t = im.astype(np.float64) / re
    assert np.abs(t).max() <= np.tan(np.pi / 8) * (1 + 1e-6)
    # and the pair's angle is the sum of the two
    ang = np.arctan(t)
    ref = np.arctan(N1.astype(np.float64) / D1) + np.arctan(N2.astype(np.float64) / D2)
    assert np.abs(ang - ref).max() < 1e-6
