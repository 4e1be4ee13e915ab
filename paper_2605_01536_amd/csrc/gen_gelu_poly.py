#!/usr/bin/env python3
"""Fit the polynomial of the surrogate's inference GELU.

GELU(z) = z Phi(z), Phi the standard normal CDF.  For |z| <= c the kernel
evaluates Phi(z) - 1/2 (odd in z) as z P(z^2), P a polynomial of degree `deg`;
beyond c it clamps z to +-c, i.e. takes Phi = 1/2 +- (Phi(c) - 1/2), which is
off by at most 1 - Phi(c) (2.3e-4 for c = 3.5).  P is chosen by the Remez
exchange algorithm to minimise the maximum absolute error of z P(z^2) against
Phi(z) - 1/2 on [0, c]:

    e(x) = sqrt(x) P(x) - (Phi(sqrt x) - 1/2),   x = z^2 in [0, c^2],

i.e. a weighted minimax fit of G(x) = (Phi(sqrt x) - 1/2) / sqrt(x) with
weight sqrt(x), found in t = x / c^2 in [0, 1].  The kernel evaluates it in
packed half precision in the variable v = u^2, u = clamp(z / c, -1, 1), as
Phi(z) - 1/2 = u Q(v) with Q(v) = c P(c^2 v); the coefficients of Q are then
rounded to half precision one at a time (half_table), the others re-fitted
after each.

    python gen_gelu_poly.py [deg [c]]       # half-exact table, coefficients highest first

The printed table is the kGeluH table of mlp.hip; the script also reports the
fitted error and the error of the kernel's half-precision evaluation
(gelu_half) against GELU in FP64.
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


def half_scale(c):
    """The kernel's t = z s + 1/2 takes s = 1/(2c) rounded to half precision, so
    u = 2t - 1 is z / c_eff with c_eff = 1 / (2 s)."""
    return 0.5 / float(np.float16(0.5 / c))


def half_table(deg, c, grid=4001):
    """Q(v) with Phi(z) - 1/2 = u Q(u^2), u = z / c_eff in [-1, 1], and half-
    precision coefficients.  Start from the minimax fit (remez, scaled from x =
    z^2 to v = u^2), then round one coefficient at a time, highest power first:
    of the two half values around it keep the one after which the remaining
    coefficients, re-fitted for minimax absolute error of u Q(u^2) against
    Phi(c_eff u) - 1/2 on a grid of u in [0, 1] (a linear programme), give the
    smaller error."""
    from scipy.optimize import linprog
    ce = half_scale(c)
    coef, _ = remez(deg, ce)
    n = deg + 1
    q = ce * coef * (ce * ce) ** np.arange(n)          # Q(v) = c_eff P(c_eff^2 v)
    u = np.linspace(0.0, 1.0, grid)
    v = u * u
    g = phi_half(ce * u)
    B = u[:, None] * v[:, None] ** np.arange(n)         # column i: u v^i

    def refit(fixed):
        # minimise e over the free coefficients with |B q - g| <= e
        free = [i for i in range(n) if i not in fixed]
        rest = g - sum(B[:, i] * fixed[i] for i in fixed) if fixed else g.copy()
        if not free:
            return {}, float(np.abs(rest).max())
        A = B[:, free]
        m = len(free)
        ones = np.ones((grid, 1))
        res = linprog(np.r_[np.zeros(m), 1.0], A_ub=np.block([[A, -ones], [-A, -ones]]), b_ub=np.r_[rest, -rest],
                      bounds=[(None, None)] * m + [(0, None)], method="highs")
        return dict(zip(free, res.x[:m])), float(res.x[m])

    fixed = {}
    cur = dict(enumerate(q))
    for i in range(n - 1, -1, -1):
        h = np.float16(cur[i])
        cands = {float(h), float(np.nextafter(h, np.float16(np.inf))), float(np.nextafter(h, np.float16(-np.inf)))}
        best = None
        for cand in sorted(cands):
            sol, err = refit({**fixed, i: cand})
            if best is None or err < best[2]:
                best = (cand, sol, err)
        fixed[i] = best[0]
        cur = {**fixed, **best[1]}
    table = [np.float16(fixed[i]) for i in range(n - 1, -1, -1)]   # highest power first
    return table, best[2]


def f16(a):
    return np.asarray(a, np.float64).astype(np.float16).astype(np.float64)


def gelu_half(table, c, z):
    """The kernel's packed half evaluation, each operation rounded once to half
    precision: z to half, t = clamp(z s + 1/2, 0, 1) (the FMA's output clamp),
    u = 2t - 1, v = u u, Horner with FMAs, Phi = u Q + 1/2, GELU = z Phi."""
    s = float(np.float16(0.5 / c))
    zh = f16(np.asarray(z, dtype=np.float32))
    t = np.clip(f16(zh * s + 0.5), 0.0, 1.0)
    u = f16(2.0 * t - 1.0)
    v = f16(u * u)
    p = np.full_like(v, float(table[0]))
    for a in table[1:]:
        p = f16(p * v + float(a))
    phi = f16(u * p + 0.5)
    return f16(zh * phi), phi


def gelu_ref(z):
    z = np.asarray(z, dtype=np.float64)
    return z * (0.5 + phi_half(z))


def main():
    deg = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    c = float(sys.argv[2]) if len(sys.argv) > 2 else 3.5
    table, efit = half_table(deg, c)
    z = np.linspace(-12.0, 12.0, 480001).astype(np.float32)
    gh, phi = gelu_half(table, c, z)
    zz = z.astype(np.float64)
    dphi = np.abs(phi - (0.5 + phi_half(zz))).max()
    tail = 0.5 - float(phi_half(np.array([half_scale(c)]))[0])
    print(f"// Q of degree {deg} in v = u^2, u = clamp(z / c, -1, 1), c = {c} (c_eff {half_scale(c):.6f} with the "
          f"half-precision scale): minimax |u Q(u^2) - (Phi(z) - 1/2)| {efit:.3e} with half coefficients, clamp "
          f"tail {tail:.3e}; half-precision evaluation: max |Phi error| {dphi:.3e}")
    print("constexpr float kGeluH[] = {" + ", ".join(f"{float(a)!r}f" for a in table) + "};")


if __name__ == "__main__":
    main()
