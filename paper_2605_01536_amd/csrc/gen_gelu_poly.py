#!/usr/bin/env python3
"""Fit the polynomial of the surrogate's inference GELU.

GELU(z) = z Phi(z), Phi the standard normal CDF.  For |z| <= c the kernel
evaluates Phi(z) - 1/2 (odd in z) as z P(z^2), P a polynomial of degree `deg`;
beyond c it clamps z to +-c, i.e. takes Phi = 1/2 +- (Phi(c) - 1/2), which is
off by at most 1 - Phi(c) (3.2e-5 for c = 4).  P is chosen by the Remez
exchange algorithm to minimise the maximum absolute error of z P(z^2) against
Phi(z) - 1/2 on [0, c]:

    e(x) = sqrt(x) P(x) - (Phi(sqrt x) - 1/2),   x = z^2 in [0, c^2],

i.e. a weighted minimax fit of G(x) = (Phi(sqrt x) - 1/2) / sqrt(x) with
weight sqrt(x).  The exchange works in t = x / c^2 in [0, 1] (c = 4: an exact
power-of-two scaling) and the coefficients are scaled back to x.

    python gen_gelu_poly.py [deg [c]]       # float32 table, coefficients highest first

The printed table is the kGeluP table of mlp.hip; the script also reports the
fitted error and the error of the kernel's float32 evaluation,
z * fma(zc, P(zc^2), 1/2) with zc = clamp(z, -c, c), against GELU in FP64.
"""
import math
import sys

import numpy as np


def phi_half(z):
    """Phi(z) - 1/2 = erf(z / sqrt 2) / 2."""
    return 0.5 * np.vectorize(math.erf)(np.asarray(z, dtype=np.float64) / math.sqrt(2.0))


def G(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.full_like(x, 1.0 / math.sqrt(2.0 * math.pi))
    nz = x > 0
    s = np.sqrt(x[nz])
    out[nz] = phi_half(s) / s
    return out


def remez(deg, c, iters=100, grid=200001):
    n = deg + 1
    x2 = c * c
    k = np.arange(n + 1)
    ref = 0.5 - 0.5 * np.cos(np.pi * k / n)     # in t = x / c^2
    ref[0] = 1e-9
    T = np.linspace(1e-9, 1.0, grid)
    GT = G(T * x2)
    WT = np.sqrt(T * x2)
    coef, err = None, None
    for _ in range(iters):
        A = np.zeros((n + 1, n + 1))
        w = np.sqrt(ref * x2)
        for i, ti in enumerate(ref):
            A[i, :n] = ti ** np.arange(n)
            A[i, n] = (-1) ** i / w[i]
        sol = np.linalg.solve(A, G(ref * x2))
        coef = sol[:n]
        err = WT * (np.polyval(coef[::-1], T) - GT)
        sgn = np.sign(err)
        idx = []
        start = 0
        for i in range(1, len(T) + 1):
            if i == len(T) or sgn[i] != sgn[start]:
                seg = np.arange(start, i)
                idx.append(seg[np.argmax(np.abs(err[seg]))])
                start = i
        if len(idx) < n + 1:
            break
        while len(idx) > n + 1:
            e = np.abs(err[idx])
            if e[0] < e[-1]:
                idx.pop(0)
            else:
                idx.pop()
        new = T[idx]
        if np.allclose(new, ref, rtol=0, atol=1e-14):
            break
        ref = new
    # coefficients of P in x: b_i t^i = b_i (x / c^2)^i
    return coef / x2 ** np.arange(n), float(np.max(np.abs(err)))


def gelu_f32(table, c, z):
    """The kernel's float32 evaluation (each operation rounded to float32)."""
    z = np.asarray(z, dtype=np.float32)
    zc = np.clip(z, np.float32(-c), np.float32(c)).astype(np.float32)
    x = (zc * zc).astype(np.float32)
    p = np.full_like(x, np.float32(table[0]))
    for a in table[1:]:
        p = (p.astype(np.float64) * x + np.float64(np.float32(a))).astype(np.float32)   # fma: one rounding
    h = (zc.astype(np.float64) * p + 0.5).astype(np.float32)                           # fma
    return (z * h).astype(np.float32)


def gelu_ref(z):
    z = np.asarray(z, dtype=np.float64)
    return z * (0.5 + phi_half(z))


def main():
    deg = int(sys.argv[1]) if len(sys.argv) > 1 else 7
    c = float(sys.argv[2]) if len(sys.argv) > 2 else 4.0
    coef, emax = remez(deg, c)
    table = [np.float32(a) for a in coef[::-1]]
    z = np.linspace(-12.0, 12.0, 480001)
    g32 = gelu_f32(table, c, z).astype(np.float64)
    ref = gelu_ref(z.astype(np.float32).astype(np.float64))
    zz = z.astype(np.float32).astype(np.float64)
    dphi = np.abs(g32 / np.where(zz == 0, 1.0, zz) - ref / np.where(zz == 0, 1.0, zz))[zz != 0]
    tail = 0.5 - float(phi_half(np.array([c]))[0])
    print(f"// P of degree {deg} in x = z^2, |z| <= {c}: minimax |z P(z^2) - (Phi(z) - 1/2)| {emax:.3e}, "
          f"clamp tail {tail:.3e}; float32 evaluation: max |Phi error| {dphi.max():.3e}")
    print("constexpr float kGeluP[] = {" + ", ".join(f"{a!r}f".replace("np.float32(", "").replace(")", "")
                                                   for a in table) + "};")


if __name__ == "__main__":
    main()
