#!/usr/bin/env python3
"""Fit the arctangent polynomial used by the FP32 boundary kernels.

atan(t) for t in [0, 1] is written as t + t * x * Q(x) with x = t^2 and Q a
polynomial of degree `deg`.  Q is chosen by the Remez exchange algorithm to
minimise the maximum *relative* error of atan:

    e(x) = x * (Q(x) - h(x)) / g(x),   g(x) = atan(sqrt x)/sqrt x,
                                       h(x) = (g(x) - 1) / x,

i.e. a weighted minimax fit of h with weight x / g(x).  Usage:

    python gen_atan_poly.py [deg]            # float32 table, coefficients highest first
    python gen_atan_poly.py deg double       # float64 table for |t| <= tan(pi/8)
    python gen_atan_poly.py deg pair         # float32 table for |t| <= tan(pi/8)
    python gen_atan_poly.py deg pform        # float32 table of P for |t| <= tan(pi/8)

The "pform" table writes atan(t) = t * P(x) instead, P of degree `deg` fitted
to g(x) = atan(sqrt x)/sqrt x by the Remez exchange for minimax relative error,
so that a sum of arctangents accumulates as fma(t, P(x), acc).

The printed table is pasted into gwn_kernels.h (kAtanQ, kAtanP); the script
also reports the fitted error and the error of the same Horner evaluation in
float32.
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
    """(atan(sqrt x)/sqrt x - 1)/x; the alternating series -1/3 + x/5 - x^2/7 + ...
    below x = 1/4 (60 terms: error < 4^-60), the closed form above it."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    big = x >= 0.25
    out[big] = (g(x[big]) - 1.0) / x[big]
    xs = x[~big]
    acc = np.zeros_like(xs)
    for k in range(60, 0, -1):
        acc = acc * xs + (-1.0) ** k / (2 * k + 1)
    out[~big] = acc
    return out


def weight(x):
    return np.asarray(x, dtype=np.float64) / g(x)


def unit_weight(x):
    return np.ones_like(np.asarray(x, dtype=np.float64))


def remez(deg, iters=60, grid=200001, xmax=1.0, wfun=weight):
    n = deg + 1
    # initial reference: Chebyshev extrema mapped to (0, xmax]
    k = np.arange(n + 1)
    ref = xmax * (0.5 - 0.5 * np.cos(np.pi * k / n))
    lo = 1e-6 * xmax if wfun is weight else 0.0
    ref[0] = max(ref[0], lo)
    X = np.linspace(lo, xmax, grid)
    coef = None
    for _ in range(iters):
        A = np.zeros((n + 1, n + 1))
        for i, xi in enumerate(ref):
            A[i, :n] = xi ** np.arange(n)
            A[i, n] = (-1) ** i / wfun(np.array([xi]))[0]
        rhs = h(ref)
        sol = np.linalg.solve(A, rhs)
        coef = sol[:n]
        err = wfun(X) * (np.polyval(coef[::-1], X) - h(X))
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


def remez_g(deg, xmax, iters=80, grid=200001):
    """Minimax relative fit of g on [0, xmax] by a polynomial of degree deg."""
    n = deg + 1
    k = np.arange(n + 1)
    ref = xmax * (0.5 - 0.5 * np.cos(np.pi * k / n))
    X = np.linspace(0.0, xmax, grid)
    gx = g(X)
    coef, err = None, None
    for _ in range(iters):
        A = np.zeros((n + 1, n + 1))
        gr = g(ref)
        for i, xi in enumerate(ref):
            A[i, :n] = xi ** np.arange(n)
            A[i, n] = (-1) ** i * gr[i]
        coef = np.linalg.solve(A, gr)[:n]
        err = (np.polyval(coef[::-1], X) - gx) / gx
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
        while len(idx) > n + 1:
            e = np.abs(err[idx])
            if e[0] < e[-1]:
                idx.pop(0)
            else:
                idx.pop()
        new = X[idx]
        if np.allclose(new, ref, rtol=0, atol=1e-13):
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
    if len(sys.argv) > 2 and sys.argv[2] == "double":
        # |t| <= tan(pi/8): x = t^2 <= 3 - 2 sqrt 2
        xmax = 3.0 - 2.0 * np.sqrt(2.0)
        # near-minimax: interpolate h at the Chebyshev nodes of [0, xmax] and convert
        # to powers of x (well conditioned on this short interval); atan's relative
        # error is then <= x max|Q - h|
        from numpy.polynomial import Chebyshev, Polynomial
        j = np.arange(deg + 1)
        xn = 0.5 * xmax * (1.0 - np.cos(np.pi * (j + 0.5) / (deg + 1)))
        cheb = Chebyshev.fit(xn, h(xn), deg, domain=[0.0, xmax])
        coef = cheb.convert(kind=Polynomial).coef
        X = np.linspace(0.0, xmax, 200001)
        emax = float(np.max(np.abs(np.polyval(coef[::-1], X) - h(X))))
        hi_first = coef[::-1]
        t = np.linspace(0.0, np.sqrt(xmax), 400001)[1:]
        x = t * t
        q = np.full_like(x, hi_first[0])
        for c in hi_first[1:]:
            q = q * x + c
        a = t + (t * x) * q
        rel = np.abs(a - np.arctan(t)) / np.arctan(t)
        print(f"// degree {deg} in x = t^2 on |t| <= tan(pi/8); max |Q - h| {emax:.3e}; float64 Horner: max rel {rel.max():.3e}")
        print(f"constexpr double kAtanQd[{deg + 1}] = {{" + ", ".join(repr(float(c)) for c in hi_first) + "};")
        return
    if len(sys.argv) > 2 and sys.argv[2] == "pform":
        xmax = 3.0 - 2.0 * np.sqrt(2.0)
        coef, emax = remez_g(deg, xmax)
        hi_first = [np.float32(c) for c in coef[::-1]]
        t = np.linspace(0.0, np.sqrt(xmax), 400001)[1:].astype(np.float32)
        x = (t * t).astype(np.float32)
        q = np.full_like(x, hi_first[0])
        for c in hi_first[1:]:
            q = (q * x + c).astype(np.float32)
        a = (t.astype(np.float64) * q.astype(np.float64)).astype(np.float32).astype(np.float64)
        ref = np.arctan(t.astype(np.float64))
        rel = np.abs(a - ref) / ref
        print(f"// P of degree {deg} in x = t^2 on |t| <= tan(pi/8); minimax relative error {emax:.3e}; "
              f"float32 Horner: max rel {rel.max():.3e}, mean signed rel {np.mean((a - ref) / ref):.3e}")
        print("constexpr float kAtanP[] = {" + ", ".join(f"{c!r}f".replace("np.float32(", "").replace(")", "")
                                                      for c in hi_first) + "};")
        return
    pair = len(sys.argv) > 2 and sys.argv[2] == "pair"
    tmax = np.sqrt(3.0 - 2.0 * np.sqrt(2.0)) if pair else 1.0
    coef, emax = remez(deg, xmax=tmax * tmax)
    hi_first = coef[::-1]
    t = np.linspace(0.0, tmax, 400001)[1:]
    ref = np.arctan(t.astype(np.float32).astype(np.float64))
    f32 = horner_f32([np.float32(c) for c in hi_first], t.astype(np.float32)).astype(np.float64)
    rel = np.abs(f32 - ref) / ref
    print(f"// degree {deg} in x = t^2; minimax relative error {emax:.3e}; "
          f"float32 Horner: max rel {rel.max():.3e}, mean rel {np.mean(rel):.3e}, "
          f"mean signed rel {np.mean((f32 - ref) / ref):.3e}")
    print(f"constexpr float {'kAtanQp' if pair else 'kAtanQ'}[] = {{" + ", ".join(f"{np.float32(c)!r}f".replace("np.float32(", "").replace(")", "")
                                                 for c in hi_first) + "};")


if __name__ == "__main__":
    main()
