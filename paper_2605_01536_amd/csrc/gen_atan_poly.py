#!/usr/bin/env python3
"""Fit the arctangent polynomial used by the FP32 boundary kernels.

atan(t) for t in [0, 1] is written as t + t * x * Q(x) with x = t^2 and Q a
polynomial of degree `deg`.  Q is chosen by the Remez exchange algorithm to
minimise the maximum *relative* error of atan:

    e(x) = x * (Q(x) - h(x)) / g(x),   g(x) = atan(sqrt x)/sqrt x,
                                       h(x) = (g(x) - 1) / x,

i.e. a weighted minimax fit of h with weight x / g(x).  Usage:

    python gen_atan_poly.py [deg]     # prints the coefficients, highest first

The printed table is pasted into query.hip (kAtanQ); the script also reports
the fitted error and the error of the same Horner evaluation in float32.
"""
import sys

import numpy as np


def g(x):
    x = np.asarray(x, dtype=np.float64)
    s = np.sqrt(x)
    out = np.ones_like(x)
    nz = s > 0
    out[nz] = np.arctan(s[nz]) / s[nz]
    return out


def h(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.full_like(x, -1.0 / 3.0)
    big = x > 1e-4
    out[big] = (g(x[big]) - 1.0) / x[big]
    xs = x[~big]   # series: atan(t)/t = 1 - x/3 + x^2/5 - x^3/7 + ...
    out[~big] = -1.0 / 3.0 + xs / 5.0 - xs ** 2 / 7.0 + xs ** 3 / 9.0
    return out


def weight(x):
    return np.asarray(x, dtype=np.float64) / g(x)


def remez(deg, iters=60, grid=200001):
    n = deg + 1
    # initial reference: Chebyshev extrema mapped to (0, 1]
    k = np.arange(n + 1)
    ref = 0.5 - 0.5 * np.cos(np.pi * k / n)
    ref[0] = 1e-6
    X = np.linspace(1e-6, 1.0, grid)
    coef = None
    for _ in range(iters):
        A = np.zeros((n + 1, n + 1))
        for i, xi in enumerate(ref):
            A[i, :n] = xi ** np.arange(n)
            A[i, n] = (-1) ** i / weight(np.array([xi]))[0]
        rhs = h(ref)
        sol = np.linalg.solve(A, rhs)
        coef = sol[:n]
        err = weight(X) * (np.polyval(coef[::-1], X) - h(X))
        # new reference: one extremum per sign-alternating segment
        sgn = np.sign(err)
        idx = []
        start = 0
        for i in range(1, len(X) + 1):
            if i == len(X) or sgn[i] != sgn[start]:
                seg = np.arange(start, i)
                idx.append(seg[np.argmax(np.abs(err[seg]))])
                start = i
        if len(idx) < n + 1:
            break
        # keep the n+1 largest-alternating extrema
        while len(idx) > n + 1:
            e = np.abs(err[idx])
            if e[0] < e[-1]:
                idx.pop(0)
            else:
                idx.pop()
        new = X[idx]
        if np.allclose(new, ref, rtol=0, atol=1e-12):
            break
        ref = new
    return coef, float(np.max(np.abs(err)))


def horner_f32(coef_hi_first, t):
    t = np.float32(t)
    x = (t * t).astype(np.float32)
    q = np.full_like(x, np.float32(coef_hi_first[0]))
    for c in coef_hi_first[1:]:
        q = (q * x + np.float32(c)).astype(np.float32)
    tx = (t * x).astype(np.float32)
    return (tx * q + t).astype(np.float32)


def main():
    deg = int(sys.argv[1]) if len(sys.argv) > 1 else 7
    coef, emax = remez(deg)
    hi_first = coef[::-1]
    t = np.linspace(0.0, 1.0, 400001)[1:]
    ref = np.arctan(t.astype(np.float32).astype(np.float64))
    f32 = horner_f32([np.float32(c) for c in hi_first], t.astype(np.float32)).astype(np.float64)
    rel = np.abs(f32 - ref) / ref
    print(f"// degree {deg} in x = t^2; minimax relative error {emax:.3e}; "
          f"float32 Horner: max rel {rel.max():.3e}, mean rel {np.mean(rel):.3e}, "
          f"mean signed rel {np.mean((f32 - ref) / ref):.3e}")
    print("constexpr float kAtanQ[] = {" + ", ".join(f"{np.float32(c)!r}f".replace("np.float32(", "").replace(")", "")
                                                 for c in hi_first) + "};")


if __name__ == "__main__":
    main()
