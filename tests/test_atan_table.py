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
