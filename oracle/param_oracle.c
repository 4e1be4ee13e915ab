/*
 * param_oracle.c -- CPU oracle for the generalized winding number of surfaces
 * made of tensor-product cubic Bezier patches (Sec. 4.4, Alg. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * headers, tables or constants with the GPU library.
 *
 * Patch: 16 control points P[i][j] (i along u, j along v), stored at
 * (4 i + j) * 3, S(u, v) = sum_ij B_i(u) B_j(v) P[i][j] with the cubic
 * Bernstein basis.  Its normal is S_u x S_v; its boundary runs counter-
 * clockwise in (u, v) (v = 0, then u = 1, then v = 1 backwards, then u = 0
 * backwards), i.e. counter-clockwise about the normal, as a triangle's
 * (v0, v1, v2) runs about (v1 - v0) x (v2 - v0).  Curves: 4 control points
 * (12 doubles) each.
 *
 * w(p) = chi(x0) + sum over boundary curves of the integral over [0, 1] of
 * Alg. 2's f(t) = (w(t) - d eta(t)) / (4 pi), where with
 * Gamma = (phi(t) - p) / |phi(t) - p| and x1 = -x0:
 *   X = x0 - (x0 . Gamma) Gamma,    d eta = Gamma . (X x X') / |X|^2,
 *   v = Gamma - (x1 . Gamma) x1,    w     = x1 . (v x v') / |v|^2,
 * (Prop. 5.2: the spherical winding number at x1 plus the rotation of the
 * height-gradient field relative to parallel transport).  Integrals by
 * adaptive 15-point Gauss-Kronrod (Sec. 4.4 names GK15), bisecting an
 * interval while |K15 - G7| exceeds the tolerance.
 *
 * chi(x0): signed count of crossings of the ray p + t x0, t > 0, +1 where
 * the ray has positive dot product with the normal.  Patches whose control
 * points' bounding box meets the ray are bisected in u and v (de Casteljau)
 * until the control net lies within tau of the bilinear patch through its
 * corners (the Hausdorff criterion of Sec. 4.4.1), then the ray meets that
 * bilinear patch: the problem projected along x0 onto a plane is the planar
 * inverse of a bilinear map, a quadratic in v.  A hit that is tangent or lies
 * within a small margin of a leaf's edge (at the patch's boundary: within 4 tau,
 * the chord's distance from the exact curve, counting near misses) makes the
 * query ambiguous for this direction (Sec. 4.4.1 shoots another ray in such
 * cases).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PO_PI 3.14159265358979323846

/* Gauss-Kronrod 15 / Gauss 7 abscissae and weights on [-1, 1] (the standard
 * published table; node k and -node k share a weight) */
static const double po_xk[8] = {0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
                                0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
                                0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
                                0.207784955007898467600689403773245, 0.0};
static const double po_wk[8] = {0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
                                0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
                                0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
                                0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
/* Gauss 7 uses the odd-indexed Kronrod nodes 1, 3, 5 and the centre */
static const double po_wg[4] = {0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
                                0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

static inline double po_dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static inline void po_cross(const double* a, const double* b, double* o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* cubic Bezier point and derivative (Bernstein form) */
static void po_cubic(const double* C, double t, double* X, double* dX)
{
    const double s = 1.0 - t;
    const double b0 = s * s * s, b1 = 3.0 * s * s * t, b2 = 3.0 * s * t * t, b3 = t * t * t;
    const double d0 = -3.0 * s * s, d1 = 3.0 * s * s - 6.0 * s * t, d2 = 6.0 * s * t - 3.0 * t * t, d3 = 3.0 * t * t;
    for (int c = 0; c < 3; ++c) {
        X[c] = b0 * C[c] + b1 * C[3 + c] + b2 * C[6 + c] + b3 * C[9 + c];
        dX[c] = d0 * C[c] + d1 * C[3 + c] + d2 * C[6 + c] + d3 * C[9 + c];
    }
}

/* Alg. 2's f(phi, t) */
static double po_f(const double* C, double t, const double* p, const double* x0)
{
    double phi[3], dphi[3];
    po_cubic(C, t, phi, dphi);
    double r[3] = {phi[0] - p[0], phi[1] - p[1], phi[2] - p[2]};
    const double L = sqrt(po_dot(r, r));
    double G[3] = {r[0] / L, r[1] / L, r[2] / L};
    const double dg = po_dot(dphi, G);
    double Gp[3] = {(dphi[0] - dg * G[0]) / L, (dphi[1] - dg * G[1]) / L, (dphi[2] - dg * G[2]) / L};
    /* the vector field at Gamma and its derivative */
    const double hg = po_dot(x0, G), hgp = po_dot(x0, Gp);
    double X[3], Xp[3], XxXp[3];
    for (int c = 0; c < 3; ++c) {
        X[c] = x0[c] - hg * G[c];
        Xp[c] = -hgp * G[c] - hg * Gp[c];
    }
    po_cross(X, Xp, XxXp);
    const double deta = po_dot(G, XxXp) / po_dot(X, X);
    /* tangent of the geodesic from x1 = -x0 towards Gamma, and its rotation rate */
    const double x1[3] = {-x0[0], -x0[1], -x0[2]};
    const double a = po_dot(x1, G), ap = po_dot(x1, Gp);
    double v[3], vp[3], vxvp[3];
    for (int c = 0; c < 3; ++c) {
        v[c] = G[c] - a * x1[c];
        vp[c] = Gp[c] - ap * x1[c];
    }
    po_cross(v, vp, vxvp);
    const double w = po_dot(x1, vxvp) / po_dot(v, v);
    return (w - deta) / (4.0 * PO_PI);
}

/* K15 and G7 of f on [a, b] */
static void po_gk15_rule(const double* C, const double* p, const double* x0, double a, double b, double* K, double* G)
{
    const double c = 0.5 * (a + b), h = 0.5 * (b - a);
    const double fc = po_f(C, c, p, x0);
    double k = po_wk[7] * fc, g = po_wg[3] * fc;
    for (int i = 0; i < 7; ++i) {
        const double f1 = po_f(C, c - h * po_xk[i], p, x0), f2 = po_f(C, c + h * po_xk[i], p, x0);
        k += po_wk[i] * (f1 + f2);
        if (i & 1) g += po_wg[i >> 1] * (f1 + f2);
    }
    *K = k * h;
    *G = g * h;
}

static double po_adapt(const double* C, const double* p, const double* x0, double a, double b, double eps, int depth,
                       int maxdepth)
{
    double K, G;
    po_gk15_rule(C, p, x0, a, b, &K, &G);
    if (!(fabs(K - G) > eps) || depth >= maxdepth) return K; /* a NaN integrand is accepted as it is */
    const double m = 0.5 * (a + b);
    return po_adapt(C, p, x0, a, m, eps, depth + 1, maxdepth) + po_adapt(C, p, x0, m, b, eps, depth + 1, maxdepth);
}

/* sum over curves of the adaptive GK15 integral of Alg. 2's f, per query */
void oracle_param_boundary(int64_t ncurves, const double* curves, int64_t nq, const double* Q, const double* x0,
                           double eps, int maxdepth, double* S_out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nq; ++i) {
        double s = 0.0, comp = 0.0;
        for (int64_t c = 0; c < ncurves; ++c) {
            const double x = po_adapt(curves + 12 * c, Q + 3 * i, x0, 0.0, 1.0, eps, 0, maxdepth);
            const double y = x - comp, t = s + y; /* Kahan */
            comp = (t - s) - y;
            s = t;
        }
        S_out[i] = s;
    }
}

/* GK15 applied once to a function given by samples: the test of the table
 * (polynomial exactness) calls it with f(t) = t^k on [a, b] */
void oracle_gk15_poly(int k, double a, double b, double* K, double* G)
{
    const double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double kk = po_wk[7] * pow(c, k), gg = po_wg[3] * pow(c, k);
    for (int i = 0; i < 7; ++i) {
        const double f1 = pow(c - h * po_xk[i], k), f2 = pow(c + h * po_xk[i], k);
        kk += po_wk[i] * (f1 + f2);
        if (i & 1) gg += po_wg[i >> 1] * (f1 + f2);
    }
    *K = kk * h;
    *G = gg * h;
}

/* ---------------------------------------------------------------- chi */

/* split a cubic (4 points of stride st, 3 coordinates) at 1/2 into lo and hi */
static void po_split4(const double* P, int st, double* lo, double* hi, int sto)
{
    for (int c = 0; c < 3; ++c) {
        const double p0 = P[c], p1 = P[st + c], p2 = P[2 * st + c], p3 = P[3 * st + c];
        const double a = 0.5 * (p0 + p1), b = 0.5 * (p1 + p2), d = 0.5 * (p2 + p3);
        const double e = 0.5 * (a + b), f = 0.5 * (b + d), g = 0.5 * (e + f);
        lo[c] = p0; lo[sto + c] = a; lo[2 * sto + c] = e; lo[3 * sto + c] = g;
        hi[c] = g; hi[sto + c] = f; hi[2 * sto + c] = d; hi[3 * sto + c] = p3;
    }
}

/* 48 doubles -> four quarters (u low/high x v low/high) */
static void po_split_patch(const double* P, double* q00, double* q10, double* q01, double* q11)
{
    double ul[48], uh[48];
    for (int j = 0; j < 4; ++j) po_split4(P + 3 * j, 12, ul + 3 * j, uh + 3 * j, 12); /* along u (index i) */
    for (int i = 0; i < 4; ++i) {
        po_split4(ul + 12 * i, 3, q00 + 12 * i, q01 + 12 * i, 3); /* along v (index j) */
        po_split4(uh + 12 * i, 3, q10 + 12 * i, q11 + 12 * i, 3);
    }
}

/* largest distance of the control net from the bilinear patch through the corners */
static double po_bilinear_dev(const double* P)
{
    const double* A = P;               /* (0,0) */
    const double* B = P + 3 * 12;      /* (1,0): i = 3, j = 0 */
    const double* Cc = P + 3 * 15;     /* (1,1) */
    const double* D = P + 3 * 3;       /* (0,1) */
    double m = 0.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            const double u = i / 3.0, v = j / 3.0;
            double e2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double bl = (1 - u) * (1 - v) * A[c] + u * (1 - v) * B[c] + u * v * Cc[c] + (1 - u) * v * D[c];
                const double e = P[3 * (4 * i + j) + c] - bl;
                e2 += e * e;
            }
            if (e2 > m) m = e2;
        }
    return sqrt(m);
}

typedef struct {
    const double* p;
    const double* d;
    double e1[3], e2[3]; /* orthonormal basis of the plane across d */
    double tau;
    double margin;       /* parameter distance to a leaf edge that counts as ambiguous */
    int chi;
    int amb;
} po_ray;

/* does the ray meet the bounding box of the control points? (slab test) */
static int po_box_hit(const po_ray* R, const double* P)
{
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int k = 0; k < 16; ++k)
        for (int c = 0; c < 3; ++c) {
            if (P[3 * k + c] < lo[c]) lo[c] = P[3 * k + c];
            if (P[3 * k + c] > hi[c]) hi[c] = P[3 * k + c];
        }
    double t0 = 0.0, t1 = 1e300;
    for (int c = 0; c < 3; ++c) {
        const double pad = 1e-12 * (1.0 + fabs(lo[c]) + fabs(hi[c]));
        if (R->d[c] == 0.0) {
            if (R->p[c] < lo[c] - pad || R->p[c] > hi[c] + pad) return 0;
        } else {
            double a = (lo[c] - pad - R->p[c]) / R->d[c], b = (hi[c] + pad - R->p[c]) / R->d[c];
            if (a > b) { const double s = a; a = b; b = s; }
            if (a > t0) t0 = a;
            if (b < t1) t1 = b;
            if (t0 > t1) return 0;
        }
    }
    return 1;
}

static inline double po_x2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

/* the ray against the bilinear patch through the corners of the leaf P; bedge:
 * bits 0..3 where the leaf's u = 0, u = 1, v = 0, v = 1 edge is on the patch
 * boundary, whose margin also covers the chord's distance (up to tau) from the
 * exact boundary curve */
static void po_leaf_hits(po_ray* R, const double* P, int bedge)
{
    const double* c3[4] = {P, P + 3 * 12, P + 3 * 15, P + 3 * 3}; /* (0,0) (1,0) (1,1) (0,1) */
    double q2[4][2];
    for (int k = 0; k < 4; ++k) {
        double r[3] = {c3[k][0] - R->p[0], c3[k][1] - R->p[1], c3[k][2] - R->p[2]};
        q2[k][0] = po_dot(r, R->e1);
        q2[k][1] = po_dot(r, R->e2);
    }
    /* planar: 0 = a + u E + v F + u v G, with the ray's foot at the origin */
    const double Ex = q2[1][0] - q2[0][0], Ey = q2[1][1] - q2[0][1];
    const double Fx = q2[3][0] - q2[0][0], Fy = q2[3][1] - q2[0][1];
    const double Gx = q2[0][0] - q2[1][0] + q2[2][0] - q2[3][0], Gy = q2[0][1] - q2[1][1] + q2[2][1] - q2[3][1];
    const double Hx = -q2[0][0], Hy = -q2[0][1];
    /* (H - v F) x (E + v G) = 0 */
    const double k2 = -po_x2(Fx, Fy, Gx, Gy);
    const double k1 = po_x2(Hx, Hy, Gx, Gy) - po_x2(Fx, Fy, Ex, Ey);
    const double k0 = po_x2(Hx, Hy, Ex, Ey);
    double vs[2];
    int nv = 0;
    const double scale = fabs(k2) + fabs(k1) + fabs(k0);
    if (scale == 0.0) {
        R->amb = 1; /* degenerate leaf seen edge-on */
        return;
    }
    if (fabs(k2) <= 1e-14 * scale) {
        if (k1 != 0.0) vs[nv++] = -k0 / k1;
    } else {
        const double disc = k1 * k1 - 4.0 * k2 * k0;
        if (disc < 0.0) return;
        const double sq = sqrt(disc);
        const double qq = -0.5 * (k1 + (k1 >= 0.0 ? sq : -sq));
        vs[nv++] = qq / k2;
        if (qq != 0.0) vs[nv++] = k0 / qq;
        if (disc == 0.0) nv = 1;
    }
    for (int s = 0; s < nv; ++s) {
        const double v = vs[s];
        const double mx = Ex + v * Gx, my = Ey + v * Gy;
        const double den = mx * mx + my * my;
        if (den == 0.0) { R->amb = 1; continue; }
        const double u = ((Hx - v * Fx) * mx + (Hy - v * Fy) * my) / den;
        double mu0 = R->margin, mu1 = R->margin, mv0 = R->margin, mv1 = R->margin;
        if (bedge) {
            double eu[3], ev[3];
            for (int c = 0; c < 3; ++c) {
                eu[c] = c3[1][c] - c3[0][c];
                ev[c] = c3[3][c] - c3[0][c];
            }
            const double lu = sqrt(po_dot(eu, eu)), lv = sqrt(po_dot(ev, ev));
            const double bu = lu > 0.0 ? 4.0 * R->tau / lu : 1.0, bv = lv > 0.0 ? 4.0 * R->tau / lv : 1.0;
            if ((bedge & 1) && bu > mu0) mu0 = bu;
            if ((bedge & 2) && bu > mu1) mu1 = bu;
            if ((bedge & 4) && bv > mv0) mv0 = bv;
            if ((bedge & 8) && bv > mv1) mv1 = bv;
        }
        if (u < -mu0 || u > 1.0 + mu1 || v < -mv0 || v > 1.0 + mv1) continue;
        if (u < mu0 || u > 1.0 - mu1 || v < mv0 || v > 1.0 - mv1) { R->amb = 1; continue; }
        /* 3D point, ray parameter and normal of the bilinear patch */
        double X[3], Su[3], Sv[3], n[3];
        for (int c = 0; c < 3; ++c) {
            X[c] = (1 - u) * (1 - v) * c3[0][c] + u * (1 - v) * c3[1][c] + u * v * c3[2][c] + (1 - u) * v * c3[3][c];
            Su[c] = (1 - v) * (c3[1][c] - c3[0][c]) + v * (c3[2][c] - c3[3][c]);
            Sv[c] = (1 - u) * (c3[3][c] - c3[0][c]) + u * (c3[2][c] - c3[1][c]);
        }
        double r[3] = {X[0] - R->p[0], X[1] - R->p[1], X[2] - R->p[2]};
        const double t = po_dot(r, R->d);
        po_cross(Su, Sv, n);
        const double nn = sqrt(po_dot(n, n));
        const double nd = po_dot(n, R->d);
        if (!(nn > 0.0) || fabs(nd) < 1e-9 * nn) { R->amb = 1; continue; }
        if (fabs(t) <= 1e-12 * (1.0 + sqrt(po_dot(r, r)))) { R->amb = 1; continue; } /* on the surface */
        if (t <= 0.0) continue;
        R->chi += nd > 0.0 ? 1 : -1;
    }
}

/* (i, j): the cell of this sub-patch among the 2^depth x 2^depth of its patch */
static void po_patch_ray(po_ray* R, const double* P, int depth, int64_t i, int64_t j)
{
    if (!po_box_hit(R, P)) return;
    if (depth >= 30 || po_bilinear_dev(P) <= R->tau) {
        const int64_t last = ((int64_t)1 << depth) - 1;
        po_leaf_hits(R, P, (i == 0 ? 1 : 0) | (i == last ? 2 : 0) | (j == 0 ? 4 : 0) | (j == last ? 8 : 0));
        return;
    }
    double q[4][48];
    po_split_patch(P, q[0], q[1], q[2], q[3]); /* (u, v) low-low, high-low, low-high, high-high */
    po_patch_ray(R, q[0], depth + 1, 2 * i, 2 * j);
    po_patch_ray(R, q[1], depth + 1, 2 * i + 1, 2 * j);
    po_patch_ray(R, q[2], depth + 1, 2 * i, 2 * j + 1);
    po_patch_ray(R, q[3], depth + 1, 2 * i + 1, 2 * j + 1);
}

/* chi along direction d for every query; amb_out[i] = 1 where a hit was tangent,
 * on the surface, or within `margin` (in a leaf's parameters) of a leaf edge */
void oracle_param_chi(int64_t npatch, const double* P, int64_t nq, const double* Q, const double* d, double tau,
                      double margin, int32_t* chi_out, uint8_t* amb_out)
{
    /* a basis of the plane across d */
    double e1[3], e2[3];
    const double ax = fabs(d[0]), ay = fabs(d[1]), az = fabs(d[2]);
    double h[3] = {0, 0, 0};
    if (ax <= ay && ax <= az) h[0] = 1; else if (ay <= az) h[1] = 1; else h[2] = 1;
    po_cross(d, h, e1);
    const double n1 = sqrt(po_dot(e1, e1));
    for (int c = 0; c < 3; ++c) e1[c] /= n1;
    po_cross(d, e1, e2);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nq; ++i) {
        po_ray R;
        R.p = Q + 3 * i;
        R.d = d;
        memcpy(R.e1, e1, sizeof e1);
        memcpy(R.e2, e2, sizeof e2);
        R.tau = tau;
        R.margin = margin;
        R.chi = 0;
        R.amb = 0;
        for (int64_t k = 0; k < npatch; ++k) po_patch_ray(&R, P + 48 * k, 0, 0, 0);
        chi_out[i] = R.chi;
        amb_out[i] = (uint8_t)R.amb;
    }
}
