/*
 * gwn_oracle.c -- CPU oracle for generalized winding numbers of triangle soups.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * headers, tables or constants with the GPU library; both implement the same
 * published definitions independently.
 *
 * Contents (all arithmetic in IEEE double, compiled without FP contraction):
 *
 *   O1  oracle_direct      w(p) = (1/4pi) sum_T Area_{S^2_p}(T)          [Eq. 2]
 *       per-triangle signed solid angle by the Van Oosterom-Strackee
 *       formula [Eq. 6] written for unnormalised vectors (both atan2
 *       arguments scaled by |a||b||c| > 0), accumulated in double-double
 *       (the paper's accuracy study, Sec. 5.2, uses a double-double
 *       accumulator for its ground truth).
 *
 *   O2  oracle_antipodal   w(p) = chi(x0) + (1/4pi) sum_{(a,b) in dM} Area(a^, b^, x1)
 *       [Eq. 10, Alg. 1] with x0 = +z, x1 = -z (the robustness section,
 *       Supp. Sec. 2.1, fixes d = (0,0,1)).  The boundary dM is the net
 *       directed edge chain left after interior edges cancel (Sec. 4.1).
 *       chi is the signed count of crossings of the +z ray, +1 when the ray
 *       has positive dot product with the triangle normal (Sec. 3.2).
 *       Crossing tests and the atan2 branch use exact integer predicates on
 *       a 30-bit fixed-point copy of the input with symbolic perturbation of
 *       the query, q_eps = q + (e1, e2, e3), 0 < e3 << e2 << e1
 *       (Supp. Sec. 2.1).  The boundary term is the literal Alg. 1
 *       expression on unit vectors, summed with Neumaier compensation.
 *       Domain: its d = 1 + x1.a^ + x1.b^ + a^.b^ cancels in double when a
 *       boundary vertex lies far above the query compared with its x/y
 *       offset (relative offsets below ~1e-8, e.g. queries ~1e8 soup sizes
 *       below the soup); there O1 is the reference.  The same holds for the
 *       d of O4.
 *
 *   O4  oracle_gradient    grad w(p) = (1/4pi) sum_{(a,b) in dM} grad Area(a^, b^, x1)
 *       [Supp. Sec. 4, Alg. 3]: the integer part is locally constant, so
 *       only the boundary term is differentiated.  For each boundary edge
 *       the derivative of 2 atan2(n, d) with respect to p is taken by the
 *       chain rule through n = x1.(r0 x r1) and
 *       d = l0 l1 + l1 x1.r0 + l0 x1.r1 + r0.r1, with the axis x0 (x1 = -x0)
 *       an argument: the gradient does not depend on it.  FP64 throughout,
 *       Neumaier-compensated per component; also returns the sum of the
 *       per-edge term norms (the scale of the rounding error).
 *
 *   O3  oracle_distance    unsigned point-to-soup distance (closest point on
 *       a triangle by Voronoi-region classification, Ericson 2005,
 *       "Real-Time Collision Detection", Sec. 5.1.5).  Used only to mask
 *       queries that lie too close to the surface, where w is undefined.
 *
 * Readings taken where the paper is silent:
 *   - quantisation box: bbox expanded by 0.75 * max extent on every side,
 *     scale 2^k with k the largest integer such that 2.5 * extent * 2^k
 *     <= 2^30 - 1; q = rint((x - lo) * 2^k) in double.
 *   - geometry of the boundary term for queries whose quantised x and y lie
 *     in [0, 2^30 - 1]: x/y offsets from the quantised grid, z offset from
 *     the raw input; the jump decisions come from the same integers.  Other
 *     queries use raw offsets (no decision is needed there: the +z ray meets
 *     no triangle and every boundary edge has D > 0).
 *   - a boundary vertex whose quantised x/y coincide with the query's and
 *     which lies above it sits on the ray; its edge terms take the limit
 *     under the perturbation q_eps.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_QMAX ((int64_t)1073741823) /* 2^30 - 1 */
#define OR_PI 3.14159265358979323846

typedef __int128 i128;

/* ------------------------------------------------------------------------ */
/* quantisation                                                              */
/* ------------------------------------------------------------------------ */

int oracle_quant_params(const float* V, int64_t nv, double* bbox6, double* lo3, int32_t* k_out)
{
    double mn[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
    for (int64_t i = 0; i < nv; ++i) {
        for (int a = 0; a < 3; ++a) {
            double x = (double)V[3 * i + a];
            if (i == 0 || x < mn[a]) mn[a] = x;
            if (i == 0 || x > mx[a]) mx[a] = x;
        }
    }
    double e = 0.0;
    for (int a = 0; a < 3; ++a)
        if (mx[a] - mn[a] > e) e = mx[a] - mn[a];
    if (!(e > 0.0)) e = 1.0;
    for (int a = 0; a < 3; ++a) {
        bbox6[a] = mn[a];
        bbox6[3 + a] = mx[a];
        lo3[a] = mn[a] - 0.75 * e;
    }
    double ext = 2.5 * e;
    int k = 0;
    if (ldexp(ext, 0) <= (double)OR_QMAX) {
        while (ldexp(ext, k + 1) <= (double)OR_QMAX) ++k;
    } else {
        while (ldexp(ext, k) > (double)OR_QMAX) --k;
    }
    *k_out = k;
    return 0;
}

static inline double or_qcoord(double x, double lo, double scale)
{
    return rint((x - lo) * scale);
}

/* quantise n points; returns in-box flag per point (x and y inside [0, 2^30-1]);
 * z is clamped to [-1, 2^30]. */
void oracle_quantize(const float* P, int64_t n, const double* lo3, int32_t k, int64_t* q_out, uint8_t* inbox)
{
    double scale = ldexp(1.0, k);
    for (int64_t i = 0; i < n; ++i) {
        double t[3];
        for (int a = 0; a < 3; ++a) t[a] = or_qcoord((double)P[3 * i + a], lo3[a], scale);
        int ib = (t[0] >= 0.0 && t[0] <= (double)OR_QMAX && t[1] >= 0.0 && t[1] <= (double)OR_QMAX);
        double z = t[2];
        if (!(z >= -1.0)) z = -1.0;
        if (z > (double)(OR_QMAX + 1)) z = (double)(OR_QMAX + 1);
        q_out[3 * i + 0] = ib ? (int64_t)t[0] : 0;
        q_out[3 * i + 1] = ib ? (int64_t)t[1] : 0;
        q_out[3 * i + 2] = (int64_t)z;
        if (inbox) inbox[i] = (uint8_t)ib;
    }
}

/* ------------------------------------------------------------------------ */
/* exact predicates with symbolic perturbation (Supp. Sec. 2.1)              */
/* ------------------------------------------------------------------------ */

static inline int sgn64(int64_t v) { return (v > 0) - (v < 0); }
static inline int sgn128(i128 v) { return (v > 0) - (v < 0); }

/* Sign of the classification of q_eps = (qx+e1, qy+e2) against the directed
 * edge (x0,y0)->(x1,y1): (x+e1-x0)(y0-y1) + (y+e2-y0)(x1-x0), evaluated by
 * coefficient signs in lexicographic order: real part, e1, e2. */
int oracle_orient2d_sos(int64_t x0, int64_t y0, int64_t x1, int64_t y1, int64_t qx, int64_t qy)
{
    int64_t real = (qx - x0) * (y0 - y1) + (qy - y0) * (x1 - x0);
    if (real != 0) return sgn64(real);
    if (y0 - y1 != 0) return sgn64(y0 - y1);
    return sgn64(x1 - x0);
}

/* Which side of the supporting plane of triangle (p0,p1,p2) the perturbed
 * query lies on: sign of f(q_eps) = n . (p0 - q_eps), n = (p1-p0) x (p2-p0),
 * i.e. f - n_x e1 - n_y e2 - n_z e3 in lexicographic order. */
int oracle_plane_sos(const int64_t* p0, const int64_t* p1, const int64_t* p2, const int64_t* q)
{
    int64_t ux = p1[0] - p0[0], uy = p1[1] - p0[1], uz = p1[2] - p0[2];
    int64_t vx = p2[0] - p0[0], vy = p2[1] - p0[1], vz = p2[2] - p0[2];
    int64_t nx = uy * vz - uz * vy;
    int64_t ny = uz * vx - ux * vz;
    int64_t nz = ux * vy - uy * vx;
    i128 f = (i128)nx * (p0[0] - q[0]) + (i128)ny * (p0[1] - q[1]) + (i128)nz * (p0[2] - q[2]);
    if (f != 0) return sgn128(f);
    if (nx != 0) return -sgn64(nx);
    if (ny != 0) return -sgn64(ny);
    return -sgn64(nz);
}

/* Crossing of the vertical line through q_eps with triangle t.  Returns 0 on
 * a miss; otherwise +1/-1 = sign s of the projected orientation, and *above
 * tells whether the crossing lies on the +z side of the query. */
static int or_line_hit(const int64_t* P0, const int64_t* P1, const int64_t* P2, const int64_t* q, int* above)
{
    int e0 = oracle_orient2d_sos(P0[0], P0[1], P1[0], P1[1], q[0], q[1]);
    int e1 = oracle_orient2d_sos(P1[0], P1[1], P2[0], P2[1], q[0], q[1]);
    int e2 = oracle_orient2d_sos(P2[0], P2[1], P0[0], P0[1], q[0], q[1]);
    if (e0 == 0 || e0 != e1 || e0 != e2) return 0;
    int64_t nz = (P1[0] - P0[0]) * (P2[1] - P0[1]) - (P1[1] - P0[1]) * (P2[0] - P0[0]);
    int side = oracle_plane_sos(P0, P1, P2, q);
    *above = (side == sgn64(nz));
    return e0;
}

/* ------------------------------------------------------------------------ */
/* boundary chain (Sec. 4.1: interior edges cancel)                          */
/* ------------------------------------------------------------------------ */

typedef struct { int64_t lo, hi; int sign; } or_edge;

static int or_edge_cmp(const void* A, const void* B)
{
    const or_edge* a = (const or_edge*)A;
    const or_edge* b = (const or_edge*)B;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
    return 0;
}

/* Net directed boundary of the 2-chain given by the triangles, by vertex
 * index: for each unordered pair {u,v}, m = #(u->v) - #(v->u), emitted |m|
 * times in the direction of its sign.  With cancel == 0 every triangle edge
 * is emitted as is.  Writes up to cap edges; returns the total count. */
int64_t oracle_boundary(const int32_t* F, int64_t nf, int cancel, int32_t* from, int32_t* to, int64_t cap)
{
    or_edge* E = (or_edge*)malloc(sizeof(or_edge) * (size_t)(3 * nf + 1));
    int64_t ne = 0;
    for (int64_t t = 0; t < nf; ++t) {
        for (int c = 0; c < 3; ++c) {
            int64_t u = F[3 * t + c], v = F[3 * t + (c + 1) % 3];
            if (u == v) continue;
            if (!cancel) {
                if (ne < cap) { from[ne] = (int32_t)u; to[ne] = (int32_t)v; }
                ++ne;
                continue;
            }
            E[ne].lo = u < v ? u : v;
            E[ne].hi = u < v ? v : u;
            E[ne].sign = u < v ? 1 : -1;
            ++ne;
        }
    }
    if (!cancel) { free(E); return ne; }
    qsort(E, (size_t)ne, sizeof(or_edge), or_edge_cmp);
    int64_t nb = 0;
    for (int64_t i = 0; i < ne;) {
        int64_t j = i;
        int64_t m = 0;
        while (j < ne && E[j].lo == E[i].lo && E[j].hi == E[i].hi) { m += E[j].sign; ++j; }
        int64_t cnt = m > 0 ? m : -m;
        for (int64_t r = 0; r < cnt; ++r) {
            if (nb < cap) {
                from[nb] = (int32_t)(m > 0 ? E[i].lo : E[i].hi);
                to[nb] = (int32_t)(m > 0 ? E[i].hi : E[i].lo);
            }
            ++nb;
        }
        i = j;
    }
    free(E);
    return nb;
}

/* ------------------------------------------------------------------------ */
/* uniform xy bins over the quantised triangles (oracle-side accelerator;    */
/* a plain bucket grid, unrelated to any GPU structure)                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t G;
    int64_t x0, y0, span;      /* bin b covers [x0 + b*span/G, ...) */
    int64_t* start;            /* G*G+1 */
    int64_t* items;            /* triangle ids */
} or_bins;

static inline int64_t or_bin_of(const or_bins* B, int64_t v, int64_t origin)
{
    int64_t b = (int64_t)(((i128)(v - origin) * B->G) / B->span);
    if (b < 0) b = 0;
    if (b >= B->G) b = B->G - 1;
    return b;
}

static void or_bins_build(or_bins* B, const int64_t* QV, const int32_t* F, int64_t nf)
{
    int64_t mnx = 0, mxx = 0, mny = 0, mxy = 0;
    for (int64_t t = 0; t < nf; ++t)
        for (int c = 0; c < 3; ++c) {
            int64_t x = QV[3 * F[3 * t + c]], y = QV[3 * F[3 * t + c] + 1];
            if ((t == 0 && c == 0) || x < mnx) mnx = x;
            if ((t == 0 && c == 0) || x > mxx) mxx = x;
            if ((t == 0 && c == 0) || y < mny) mny = y;
            if ((t == 0 && c == 0) || y > mxy) mxy = y;
        }
    int64_t G = (int64_t)sqrt((double)nf / 2.0);
    if (G < 1) G = 1;
    if (G > 2048) G = 2048;
    B->G = G;
    B->x0 = mnx;
    B->y0 = mny;
    int64_t sx = mxx - mnx + 1, sy = mxy - mny + 1;
    B->span = sx > sy ? sx : sy;
    B->start = (int64_t*)calloc((size_t)(G * G + 1), sizeof(int64_t));
    for (int pass = 0; pass < 2; ++pass) {
        int64_t* fill = NULL;
        if (pass == 1) {
            for (int64_t i = 0; i < G * G; ++i) B->start[i + 1] += B->start[i];
            B->items = (int64_t*)malloc(sizeof(int64_t) * (size_t)(B->start[G * G] + 1));
            fill = (int64_t*)calloc((size_t)(G * G), sizeof(int64_t));
        }
        for (int64_t t = 0; t < nf; ++t) {
            int64_t lx = 0, hx = 0, ly = 0, hy = 0;
            for (int c = 0; c < 3; ++c) {
                int64_t x = QV[3 * F[3 * t + c]], y = QV[3 * F[3 * t + c] + 1];
                if (c == 0 || x < lx) lx = x;
                if (c == 0 || x > hx) hx = x;
                if (c == 0 || y < ly) ly = y;
                if (c == 0 || y > hy) hy = y;
            }
            int64_t bx0 = or_bin_of(B, lx, B->x0), bx1 = or_bin_of(B, hx, B->x0);
            int64_t by0 = or_bin_of(B, ly, B->y0), by1 = or_bin_of(B, hy, B->y0);
            for (int64_t bx = bx0; bx <= bx1; ++bx)
                for (int64_t by = by0; by <= by1; ++by) {
                    int64_t b = bx * G + by;
                    if (pass == 0) B->start[b + 1]++;
                    else B->items[B->start[b] + fill[b]++] = t;
                }
        }
        if (pass == 1) free(fill);
    }
}

static void or_bins_free(or_bins* B) { free(B->start); free(B->items); }

/* ------------------------------------------------------------------------ */
/* chi: signed crossings along the vertical line through each query           */
/* ------------------------------------------------------------------------ */

static void or_quantize_vertices(const float* V, int64_t nv, const double* lo3, int32_t k, int64_t* QV)
{
    double scale = ldexp(1.0, k);
    for (int64_t i = 0; i < nv; ++i)
        for (int a = 0; a < 3; ++a) QV[3 * i + a] = (int64_t)or_qcoord((double)V[3 * i + a], lo3[a], scale);
}

static void or_chi_one(const int64_t* QV, const int32_t* F, int64_t nf, const or_bins* B,
                       const int64_t* q, int inbox, int32_t* up, int32_t* down)
{
    int32_t cu = 0, cd = 0;
    if (inbox) {
        const int64_t* list = NULL;
        int64_t n = nf;
        if (B) {
            if (q[0] < B->x0 || q[0] >= B->x0 + B->span || q[1] < B->y0 || q[1] >= B->y0 + B->span) {
                n = 0;
            } else {
                int64_t b = or_bin_of(B, q[0], B->x0) * B->G + or_bin_of(B, q[1], B->y0);
                list = B->items + B->start[b];
                n = B->start[b + 1] - B->start[b];
            }
        }
        for (int64_t ii = 0; ii < n; ++ii) {
            int64_t t = list ? list[ii] : ii;
            const int64_t* P0 = QV + 3 * F[3 * t];
            const int64_t* P1 = QV + 3 * F[3 * t + 1];
            const int64_t* P2 = QV + 3 * F[3 * t + 2];
            int above = 0;
            int s = or_line_hit(P0, P1, P2, q, &above);
            if (!s) continue;
            if (above) cu += s;
            else cd -= s;
        }
    }
    *up = cu;
    *down = cd;
}

/* chi(+z) and chi(-z) for every query; use_bins = 0 tests every triangle. */
void oracle_chi(const float* V, int64_t nv, const int32_t* F, int64_t nf, const float* Q, int64_t nq,
                int use_bins, int32_t* chi_up, int32_t* chi_down)
{
    double bbox[6], lo[3];
    int32_t k;
    oracle_quant_params(V, nv, bbox, lo, &k);
    int64_t* QV = (int64_t*)malloc(sizeof(int64_t) * (size_t)(3 * nv + 3));
    or_quantize_vertices(V, nv, lo, k, QV);
    or_bins B;
    int have_bins = use_bins && nf > 0;
    if (have_bins) or_bins_build(&B, QV, F, nf);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nq; ++i) {
        int64_t q[3];
        uint8_t ib;
        oracle_quantize(Q + 3 * i, 1, lo, k, q, &ib);
        int32_t u, d;
        or_chi_one(QV, F, nf, have_bins ? &B : NULL, q, ib, &u, &d);
        chi_up[i] = u;
        if (chi_down) chi_down[i] = d;
    }
    if (have_bins) or_bins_free(&B);
    free(QV);
}

/* ------------------------------------------------------------------------ */
/* O2: antipodal evaluation (Eq. 10, Alg. 1)                                  */
/* ------------------------------------------------------------------------ */

/* Alg. 1 SignedSphericalTriArea(A, B, x1) with x1 = (0,0,-1), written out:
 * N = A . (B x x1), D = 1 + A.B + A.x1 + B.x1. Returns (N, D). */
static inline void or_alg1_nd(const double* A, const double* B, double* N, double* D)
{
    const double x1[3] = {0.0, 0.0, -1.0};
    double c[3] = {B[1] * x1[2] - B[2] * x1[1], B[2] * x1[0] - B[0] * x1[2], B[0] * x1[1] - B[1] * x1[0]};
    *N = A[0] * c[0] + A[1] * c[1] + A[2] * c[2];
    *D = 1.0 + (A[0] * B[0] + A[1] * B[1] + A[2] * B[2]) + (A[0] * x1[0] + A[1] * x1[1] + A[2] * x1[2]) +
         (B[0] * x1[0] + B[1] * x1[1] + B[2] * x1[2]);
}

/* D adds terms of size up to 1 that cancel when both endpoints lie nearly on
 * the +z axis through the query (D ~ rho^2/l^2 there) or where the spherical
 * triangle's area crosses +-pi; below this bound its double rounding error is
 * no longer small against D, and the same expression is evaluated again in
 * IEEE binary128 from the (exact) double offsets. */
#define OR_ESCALATE 0x1p-10

static void or_alg1_nd_q(const double* ra, const double* rb, double* N, double* D)
{
    __float128 A[3], B[3];
    const __float128 la = sqrtq((__float128)ra[0] * ra[0] + (__float128)ra[1] * ra[1] + (__float128)ra[2] * ra[2]);
    const __float128 lb = sqrtq((__float128)rb[0] * rb[0] + (__float128)rb[1] * rb[1] + (__float128)rb[2] * rb[2]);
    for (int i = 0; i < 3; ++i) { A[i] = ra[i] / la; B[i] = rb[i] / lb; }
    /* x1 = (0, 0, -1): B x x1 = (-B_y, B_x, 0) */
    *N = (double)(A[0] * -B[1] + A[1] * B[0]);
    *D = (double)(1 + (A[0] * B[0] + A[1] * B[1] + A[2] * B[2]) - A[2] - B[2]);
}

/* Limit of 2*atan2(N, D) for an edge whose first (first_on=1) or second
 * endpoint lies on the +z ray, as the query moves to q_eps: that endpoint's
 * x/y offset becomes (-e1, -e2).  o = x/y offset of the other endpoint. */
static double or_axis_limit(int first_on, double ox, double oy)
{
    if (ox == 0.0 && oy == 0.0) return 0.0;
    if (first_on) {
        /* N ~ e1*oy - e2*ox, D ~ -e1*ox - e2*oy */
        if (oy != 0.0) return 2.0 * atan2(oy, -ox);
        return ox > 0.0 ? -2.0 * OR_PI : 0.0;
    }
    /* N ~ -e1*oy + e2*ox, D ~ -e1*ox - e2*oy */
    if (oy != 0.0) return 2.0 * atan2(-oy, -ox);
    return ox > 0.0 ? 2.0 * OR_PI : 0.0;
}

typedef struct {
    const float* V;
    const int64_t* QV;
    const int32_t* from;
    const int32_t* to;
    int64_t nb;
    double cell;
} or_bdry;

static double or_boundary_sum(const or_bdry* Bd, const float* p, const int64_t* q, int inbox)
{
    double s = 0.0, comp = 0.0; /* Neumaier */
    for (int64_t e = 0; e < Bd->nb; ++e) {
        int32_t ia = Bd->from[e], ib = Bd->to[e];
        double ra[3], rb[3];
        const int64_t* qa = Bd->QV + 3 * ia;
        const int64_t* qb = Bd->QV + 3 * ib;
        if (inbox) {
            ra[0] = (double)(qa[0] - q[0]) * Bd->cell;
            ra[1] = (double)(qa[1] - q[1]) * Bd->cell;
            rb[0] = (double)(qb[0] - q[0]) * Bd->cell;
            rb[1] = (double)(qb[1] - q[1]) * Bd->cell;
        } else {
            ra[0] = (double)Bd->V[3 * ia] - (double)p[0];
            ra[1] = (double)Bd->V[3 * ia + 1] - (double)p[1];
            rb[0] = (double)Bd->V[3 * ib] - (double)p[0];
            rb[1] = (double)Bd->V[3 * ib + 1] - (double)p[1];
        }
        ra[2] = (double)Bd->V[3 * ia + 2] - (double)p[2];
        rb[2] = (double)Bd->V[3 * ib + 2] - (double)p[2];
        int on_a = inbox && qa[0] == q[0] && qa[1] == q[1] && ra[2] > 0.0;
        int on_b = inbox && qb[0] == q[0] && qb[1] == q[1] && rb[2] > 0.0;
        double term;
        if (on_a && on_b) {
            term = 0.0;
        } else if (on_a) {
            term = or_axis_limit(1, rb[0], rb[1]);
        } else if (on_b) {
            term = or_axis_limit(0, ra[0], ra[1]);
        } else {
            double la = sqrt(ra[0] * ra[0] + ra[1] * ra[1] + ra[2] * ra[2]);
            double lb = sqrt(rb[0] * rb[0] + rb[1] * rb[1] + rb[2] * rb[2]);
            double A[3] = {ra[0] / la, ra[1] / la, ra[2] / la};
            double B[3] = {rb[0] / lb, rb[1] / lb, rb[2] / lb};
            double N, D;
            or_alg1_nd(A, B, &N, &D);
            if (fabs(D) < OR_ESCALATE) or_alg1_nd_q(ra, rb, &N, &D);
            if (inbox && D <= 0.0) {
                /* atan2 jumps where N changes sign with D < 0; N carries the
                 * sign of -orient2d(a, b, q_eps), the same polynomial as the
                 * ray-crossing edge test (Supp. Sec. 2.1). */
                int o = oracle_orient2d_sos(qa[0], qa[1], qb[0], qb[1], q[0], q[1]);
                if (o != 0) N = (o > 0 ? -1.0 : 1.0) * fabs(N);
            }
            term = 2.0 * atan2(N, D);
        }
        double t = s + term;
        if (fabs(s) >= fabs(term)) comp += (s - t) + term;
        else comp += (term - t) + s;
        s = t;
    }
    return s + comp;
}

/* O2 for every query.  cancel = 0 evaluates all 3F triangle edges instead of
 * the cancelled boundary chain.  w_out[i] = chi_up + S/(4 pi); s_out (nullable)
 * receives S; chi_up/chi_down (nullable) the crossing counts. */
int oracle_antipodal(const float* V, int64_t nv, const int32_t* F, int64_t nf, const float* Q, int64_t nq,
                     int cancel, double* w_out, double* s_out, int32_t* chi_up, int32_t* chi_down)
{
    double bbox[6], lo[3];
    int32_t k;
    oracle_quant_params(V, nv, bbox, lo, &k);
    int64_t* QV = (int64_t*)malloc(sizeof(int64_t) * (size_t)(3 * nv + 3));
    or_quantize_vertices(V, nv, lo, k, QV);
    int64_t nb = oracle_boundary(F, nf, cancel, NULL, NULL, 0);
    int32_t* from = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nb + 1));
    int32_t* to = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nb + 1));
    oracle_boundary(F, nf, cancel, from, to, nb);
    or_bins B;
    int have_bins = nf > 0;
    if (have_bins) or_bins_build(&B, QV, F, nf);
    or_bdry Bd = {V, QV, from, to, nb, ldexp(1.0, -k)};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nq; ++i) {
        int64_t q[3];
        uint8_t ib;
        oracle_quantize(Q + 3 * i, 1, lo, k, q, &ib);
        int32_t u, d;
        or_chi_one(QV, F, nf, have_bins ? &B : NULL, q, ib, &u, &d);
        double S = or_boundary_sum(&Bd, Q + 3 * i, q, ib);
        w_out[i] = (double)u + S / (4.0 * OR_PI);
        if (s_out) s_out[i] = S;
        if (chi_up) chi_up[i] = u;
        if (chi_down) chi_down[i] = d;
    }
    if (have_bins) or_bins_free(&B);
    free(from);
    free(to);
    free(QV);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O1: direct sum of signed solid angles (Eq. 2, Eq. 6), double-double sum    */
/* ------------------------------------------------------------------------ */

static inline void or_two_sum(double a, double b, double* s, double* e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *e = (a - av) + (b - bv);
    *s = x;
}

/* signed solid angle of one triangle seen from p: 2 atan2(a.(b x c),
 * |a||b||c| + (a.b)|c| + (a.c)|b| + (b.c)|a|) with a, b, c = vertices - p. */
double oracle_solid_angle(const double* v0, const double* v1, const double* v2, const double* p)
{
    double a[3], b[3], c[3];
    for (int i = 0; i < 3; ++i) { a[i] = v0[i] - p[i]; b[i] = v1[i] - p[i]; c[i] = v2[i] - p[i]; }
    double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    double lc = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    double bxc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
    double num = a[0] * bxc[0] + a[1] * bxc[1] + a[2] * bxc[2];
    double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    double ac = a[0] * c[0] + a[1] * c[1] + a[2] * c[2];
    double bc = b[0] * c[0] + b[1] * c[1] + b[2] * c[2];
    double den = la * lb * lc + ab * lc + ac * lb + bc * la;
    return 2.0 * atan2(num, den);
}

void oracle_direct(const float* V, int64_t nv, const int32_t* F, int64_t nf, const float* Q, int64_t nq, double* w_out)
{
    (void)nv;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nq; ++i) {
        double p[3] = {(double)Q[3 * i], (double)Q[3 * i + 1], (double)Q[3 * i + 2]};
        double hi = 0.0, lo = 0.0;
        for (int64_t t = 0; t < nf; ++t) {
            double v[3][3];
            for (int c = 0; c < 3; ++c)
                for (int a = 0; a < 3; ++a) v[c][a] = (double)V[3 * F[3 * t + c] + a];
            double om = oracle_solid_angle(v[0], v[1], v[2], p);
            double s, e;
            or_two_sum(hi, om, &s, &e);
            lo += e;
            or_two_sum(s, lo, &hi, &lo);
        }
        w_out[i] = (hi + lo) / (4.0 * OR_PI);
    }
}

/* ------------------------------------------------------------------------ */
/* Welding: equal positions become one index (the smallest)                   */
/* ------------------------------------------------------------------------ */

static const float* or_weld_V;

static int or_weld_cmp(const void* A, const void* B)
{
    const int64_t i = *(const int64_t*)A, j = *(const int64_t*)B;
    for (int a = 0; a < 3; ++a) {
        const float x = or_weld_V[3 * i + a], y = or_weld_V[3 * j + a];
        if (x < y) return -1;
        if (x > y) return 1;
    }
    return (i > j) - (i < j);
}

/* F_out = F with every index replaced by the smallest index whose vertex has
 * the same coordinates (float equality, so +0 == -0).  Returns the number of
 * distinct positions.  Not thread-safe (qsort comparator state). */
int64_t oracle_weld(const float* V, int64_t nv, const int32_t* F, int64_t nf, int32_t* F_out)
{
    int64_t* ord = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nv + 1));
    int32_t* rep = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nv + 1));
    for (int64_t i = 0; i < nv; ++i) ord[i] = i;
    or_weld_V = V;
    qsort(ord, (size_t)nv, sizeof(int64_t), or_weld_cmp);
    int64_t distinct = 0, first = 0;
    for (int64_t j = 0; j < nv; ++j) {
        const int64_t i = ord[j];
        int same = j > 0;
        for (int a = 0; a < 3 && same; ++a) same = V[3 * i + a] == V[3 * ord[j - 1] + a];
        if (!same) { first = i; ++distinct; }   /* sorted by index within equal positions */
        rep[i] = (int32_t)first;
    }
    for (int64_t t = 0; t < 3 * nf; ++t) F_out[t] = rep[F[t]];
    free(ord);
    free(rep);
    return distinct;
}

/* ------------------------------------------------------------------------ */
/* O4: gradient of w (Supp. Sec. 4, Alg. 3)                                    */
/* ------------------------------------------------------------------------ */

static inline double or_dot(const double* u, const double* v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; }

static inline void or_cross(const double* u, const double* v, double* out)
{
    out[0] = u[1] * v[2] - u[2] * v[1];
    out[1] = u[2] * v[0] - u[0] * v[2];
    out[2] = u[0] * v[1] - u[1] * v[0];
}

/* Neumaier step: running sum *s with compensation *c */
static inline void or_neumaier(double* s, double* c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
    else *c += (x - t) + *s;
    *s = t;
}

/* One edge's term c_n g_n + c_d g_d of Alg. 3 in double (x1 = -x0).  Returns 0
 * without a result when d is small against l0 l1 (see OR_ESCALATE). */
static int or_grad_edge(const double* r0, const double* r1, const double* x1, double* term)
{
    double v0[3], v1[3], r0xr1[3], r1xx1[3], x1xr0[3], gn[3], gd[3];
    const double l0 = sqrt(or_dot(r0, r0)), l1v = sqrt(or_dot(r1, r1));
    for (int a = 0; a < 3; ++a) { v0[a] = r0[a] / l0; v1[a] = r1[a] / l1v; }
    or_cross(r0, r1, r0xr1);
    const double n = or_dot(x1, r0xr1);
    const double d = l0 * l1v + l1v * or_dot(x1, r0) + l0 * or_dot(x1, r1) + or_dot(r0, r1);
    if (fabs(d) < OR_ESCALATE * l0 * l1v) return 0;
    /* derivatives of 2 atan2(n, d) with respect to n and d */
    const double cn = 2.0 * d / (n * n + d * d);
    const double cd = -2.0 * n / (n * n + d * d);
    /* dn/dp: n = r0.(r1 x x1) = r1.(x1 x r0), and dr0/dp = dr1/dp = -I */
    or_cross(r1, x1, r1xx1);
    or_cross(x1, r0, x1xr0);
    for (int a = 0; a < 3; ++a) gn[a] = -(r1xx1[a] + x1xr0[a]);
    /* dd/dr0 and dd/dr1; dd/dp is minus their sum */
    const double x1v0 = or_dot(x1, v0), x1v1 = or_dot(x1, v1);
    for (int a = 0; a < 3; ++a) {
        const double t1 = l1v * (x1[a] + v1[a] + (1.0 + x1v1) * v0[a]);
        const double t2 = l0 * (x1[a] + v0[a] + (1.0 + x1v0) * v1[a]);
        gd[a] = -(t1 + t2);
    }
    for (int a = 0; a < 3; ++a) term[a] = cn * gn[a] + cd * gd[a];
    return 1;
}

/* The same steps in binary128. */
static void or_grad_edge_q(const double* r0d, const double* r1d, const double* x1d, double* term)
{
    __float128 r0[3], r1[3], x1[3], v0[3], v1[3], gn[3], gd[3];
    for (int a = 0; a < 3; ++a) { r0[a] = r0d[a]; r1[a] = r1d[a]; x1[a] = x1d[a]; }
    const __float128 l0 = sqrtq(r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2]);
    const __float128 l1v = sqrtq(r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
    for (int a = 0; a < 3; ++a) { v0[a] = r0[a] / l0; v1[a] = r1[a] / l1v; }
    const __float128 c[3] = {r0[1] * r1[2] - r0[2] * r1[1], r0[2] * r1[0] - r0[0] * r1[2],
                             r0[0] * r1[1] - r0[1] * r1[0]};
    const __float128 n = x1[0] * c[0] + x1[1] * c[1] + x1[2] * c[2];
    const __float128 x1r0 = x1[0] * r0[0] + x1[1] * r0[1] + x1[2] * r0[2];
    const __float128 x1r1 = x1[0] * r1[0] + x1[1] * r1[1] + x1[2] * r1[2];
    const __float128 d = l0 * l1v + l1v * x1r0 + l0 * x1r1 + (r0[0] * r1[0] + r0[1] * r1[1] + r0[2] * r1[2]);
    const __float128 cn = 2 * d / (n * n + d * d), cd = -2 * n / (n * n + d * d);
    const __float128 r1xx1[3] = {r1[1] * x1[2] - r1[2] * x1[1], r1[2] * x1[0] - r1[0] * x1[2],
                                 r1[0] * x1[1] - r1[1] * x1[0]};
    const __float128 x1xr0[3] = {x1[1] * r0[2] - x1[2] * r0[1], x1[2] * r0[0] - x1[0] * r0[2],
                                 x1[0] * r0[1] - x1[1] * r0[0]};
    for (int a = 0; a < 3; ++a) gn[a] = -(r1xx1[a] + x1xr0[a]);
    const __float128 x1v0 = x1[0] * v0[0] + x1[1] * v0[1] + x1[2] * v0[2];
    const __float128 x1v1 = x1[0] * v1[0] + x1[1] * v1[1] + x1[2] * v1[2];
    for (int a = 0; a < 3; ++a) {
        const __float128 t1 = l1v * (x1[a] + v1[a] + (1 + x1v1) * v0[a]);
        const __float128 t2 = l0 * (x1[a] + v0[a] + (1 + x1v0) * v1[a]);
        gd[a] = -(t1 + t2);
    }
    for (int a = 0; a < 3; ++a) term[a] = (double)(cn * gn[a] + cd * gd[a]);
}

/* grad_out[3 * i ..], and l1_out[i] = sum over edges of |edge term| (may be NULL).
 * x0: unit axis; the boundary is the cancelled chain of oracle_boundary. */
void oracle_gradient(const float* V, int64_t nv, const int32_t* F, int64_t nf, const float* Q, int64_t nq,
                     const double* x0, double* grad_out, double* l1_out)
{
    (void)nv;
    int64_t nb = oracle_boundary(F, nf, 1, NULL, NULL, 0);
    int32_t* from = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nb + 1));
    int32_t* to = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nb + 1));
    oracle_boundary(F, nf, 1, from, to, nb);
    const double x1[3] = {-x0[0], -x0[1], -x0[2]};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nq; ++i) {
        const double p[3] = {(double)Q[3 * i], (double)Q[3 * i + 1], (double)Q[3 * i + 2]};
        double gs[3] = {0, 0, 0}, gc[3] = {0, 0, 0}, l1 = 0.0;
        for (int64_t e = 0; e < nb; ++e) {
            double r0[3], r1[3], term[3];
            for (int a = 0; a < 3; ++a) {
                r0[a] = (double)V[3 * from[e] + a] - p[a];
                r1[a] = (double)V[3 * to[e] + a] - p[a];
            }
            if (!or_grad_edge(r0, r1, x1, term)) or_grad_edge_q(r0, r1, x1, term);
            for (int a = 0; a < 3; ++a) or_neumaier(&gs[a], &gc[a], term[a]);
            l1 += sqrt(or_dot(term, term));
        }
        for (int a = 0; a < 3; ++a) grad_out[3 * i + a] = (gs[a] + gc[a]) / (4.0 * OR_PI);
        if (l1_out) l1_out[i] = l1 / (4.0 * OR_PI);
    }
    free(from);
    free(to);
}

/* ------------------------------------------------------------------------ */
/* O3: unsigned distance to the soup (Ericson 2005, Sec. 5.1.5)               */
/* ------------------------------------------------------------------------ */

/* squared distance from p to the nearest of the three segments of a zero-area
 * triangle (collinear or coincident corners): as a point set it is those
 * segments, and the region tests below would divide 0 by 0 on a zero-length
 * edge */
static double or_point_segs_dist2(const double* p, const double* a, const double* b, const double* c)
{
    double best = 1e300;
    const double* P[3] = {a, b, c};
    for (int e = 0; e < 3; ++e) {
        const double* u = P[e];
        const double* w = P[(e + 1) % 3];
        double d[3] = {w[0] - u[0], w[1] - u[1], w[2] - u[2]};
        double up[3] = {p[0] - u[0], p[1] - u[1], p[2] - u[2]};
        double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double t = dd > 0.0 ? (up[0] * d[0] + up[1] * d[1] + up[2] * d[2]) / dd : 0.0;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
        double r[3] = {up[0] - t * d[0], up[1] - t * d[1], up[2] - t * d[2]};
        double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (r2 < best) best = r2;
    }
    return best;
}

static double or_point_tri_dist2(const double* p, const double* a, const double* b, const double* c)
{
    double ab[3], ac[3], ap[3], q[3];
    for (int i = 0; i < 3; ++i) { ab[i] = b[i] - a[i]; ac[i] = c[i] - a[i]; ap[i] = p[i] - a[i]; }
    /* corners from float32 inputs: their differences and the products below are
     * exact in double, so the cross product is zero exactly when the corners
     * are collinear */
    if (ab[1] * ac[2] - ab[2] * ac[1] == 0.0 && ab[2] * ac[0] - ab[0] * ac[2] == 0.0 &&
        ab[0] * ac[1] - ab[1] * ac[0] == 0.0)
        return or_point_segs_dist2(p, a, b, c);
#define DOT(u, v) ((u)[0] * (v)[0] + (u)[1] * (v)[1] + (u)[2] * (v)[2])
    double d1 = DOT(ab, ap), d2 = DOT(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) { for (int i = 0; i < 3; ++i) q[i] = a[i]; goto done; }
    {
        double bp[3];
        for (int i = 0; i < 3; ++i) bp[i] = p[i] - b[i];
        double d3 = DOT(ab, bp), d4 = DOT(ac, bp);
        if (d3 >= 0.0 && d4 <= d3) { for (int i = 0; i < 3; ++i) q[i] = b[i]; goto done; }
        double vc = d1 * d4 - d3 * d2;
        if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
            double v = d1 / (d1 - d3);
            for (int i = 0; i < 3; ++i) q[i] = a[i] + v * ab[i];
            goto done;
        }
        double cp[3];
        for (int i = 0; i < 3; ++i) cp[i] = p[i] - c[i];
        double d5 = DOT(ab, cp), d6 = DOT(ac, cp);
        if (d6 >= 0.0 && d5 <= d6) { for (int i = 0; i < 3; ++i) q[i] = c[i]; goto done; }
        double vb = d5 * d2 - d1 * d6;
        if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
            double w = d2 / (d2 - d6);
            for (int i = 0; i < 3; ++i) q[i] = a[i] + w * ac[i];
            goto done;
        }
        double va = d3 * d6 - d5 * d4;
        if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
            double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
            for (int i = 0; i < 3; ++i) q[i] = b[i] + w * (c[i] - b[i]);
            goto done;
        }
        double den = va + vb + vc;
        if (den == 0.0) return or_point_segs_dist2(p, a, b, c); /* degenerate after rounding */
        double v = vb / den, w = vc / den;
        for (int i = 0; i < 3; ++i) q[i] = a[i] + ab[i] * v + ac[i] * w;
    }
done:
    {
        double d[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
        return DOT(d, d);
    }
#undef DOT
}

/* distance from each query to the nearest triangle, computed exactly for
 * triangles whose bounding box expanded by `cutoff` contains the query; the
 * result is min(distance, cutoff) (enough to mask near-surface queries).
 * With use_bins != 0 the candidate triangles come from a uniform x/y bucket
 * grid over the expanded boxes (same arithmetic, fewer candidates). */
void oracle_distance2(const float* V, int64_t nv, const int32_t* F, int64_t nf, const float* Q, int64_t nq,
                      double cutoff, int use_bins, double* d_out)
{
    (void)nv;
    int64_t G = 1;
    double x0 = 0.0, y0 = 0.0, cw = 1.0;
    int64_t* start = NULL;
    int64_t* items = NULL;
    if (use_bins && nf > 0) {
        double mnx = 1e300, mny = 1e300, mxx = -1e300, mxy = -1e300;
        for (int64_t i = 0; i < 3 * nf; ++i) {
            double x = (double)V[3 * F[i]], y = (double)V[3 * F[i] + 1];
            if (x < mnx) mnx = x;
            if (x > mxx) mxx = x;
            if (y < mny) mny = y;
            if (y > mxy) mxy = y;
        }
        G = (int64_t)sqrt((double)nf / 2.0);
        if (G < 1) G = 1;
        if (G > 2048) G = 2048;
        x0 = mnx - cutoff;
        y0 = mny - cutoff;
        double span = fmax(mxx - mnx, mxy - mny) + 2.0 * cutoff;
        cw = span / (double)G;
        if (!(cw > 0.0)) cw = 1.0;
        start = (int64_t*)calloc((size_t)(G * G + 1), sizeof(int64_t));
        int64_t* fill = NULL;
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1) {
                for (int64_t i = 0; i < G * G; ++i) start[i + 1] += start[i];
                /* a cutoff large against the triangles puts each in many buckets:
                 * past a bound (or if memory runs out) every query scans all triangles */
                if (start[G * G] <= 64 * nf + (1 << 20))
                    items = (int64_t*)malloc(sizeof(int64_t) * (size_t)(start[G * G] + 1));
                fill = items ? (int64_t*)calloc((size_t)(G * G), sizeof(int64_t)) : NULL;
                if (!items || !fill) {
                    free(items);
                    free(fill);
                    free(start);
                    items = NULL;
                    fill = NULL;
                    start = NULL;
                    break;
                }
            }
            for (int64_t t = 0; t < nf; ++t) {
                double lx = 1e300, hx = -1e300, ly = 1e300, hy = -1e300;
                for (int c = 0; c < 3; ++c) {
                    double x = (double)V[3 * F[3 * t + c]], y = (double)V[3 * F[3 * t + c] + 1];
                    if (x < lx) lx = x;
                    if (x > hx) hx = x;
                    if (y < ly) ly = y;
                    if (y > hy) hy = y;
                }
                int64_t bx0 = (int64_t)floor((lx - cutoff - x0) / cw), bx1 = (int64_t)floor((hx + cutoff - x0) / cw);
                int64_t by0 = (int64_t)floor((ly - cutoff - y0) / cw), by1 = (int64_t)floor((hy + cutoff - y0) / cw);
                if (bx0 < 0) bx0 = 0;
                if (by0 < 0) by0 = 0;
                if (bx1 >= G) bx1 = G - 1;
                if (by1 >= G) by1 = G - 1;
                for (int64_t bx = bx0; bx <= bx1; ++bx)
                    for (int64_t by = by0; by <= by1; ++by) {
                        int64_t b = bx * G + by;
                        if (pass == 0) start[b + 1]++;
                        else items[start[b] + fill[b]++] = t;
                    }
            }
        }
        free(fill);
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nq; ++i) {
        double p[3] = {(double)Q[3 * i], (double)Q[3 * i + 1], (double)Q[3 * i + 2]};
        double best = cutoff * cutoff;
        const int64_t* list = NULL;
        int64_t n = nf;
        if (start) {
            int64_t bx = (int64_t)floor((p[0] - x0) / cw), by = (int64_t)floor((p[1] - y0) / cw);
            if (bx < 0 || by < 0 || bx >= G || by >= G) {
                n = 0;
            } else {
                list = items + start[bx * G + by];
                n = start[bx * G + by + 1] - start[bx * G + by];
            }
        }
        for (int64_t ii = 0; ii < n; ++ii) {
            int64_t t = list ? list[ii] : ii;
            double v[3][3];
            int skip = 0;
            for (int a = 0; a < 3 && !skip; ++a) {
                double lo = 1e300, hi = -1e300;
                for (int c = 0; c < 3; ++c) {
                    double x = (double)V[3 * F[3 * t + c] + a];
                    v[c][a] = x;
                    if (x < lo) lo = x;
                    if (x > hi) hi = x;
                }
                if (p[a] < lo - cutoff || p[a] > hi + cutoff) skip = 1;
            }
            if (skip) continue;
            double d2 = or_point_tri_dist2(p, v[0], v[1], v[2]);
            if (d2 < best) best = d2;
        }
        d_out[i] = sqrt(best);
    }
    free(start);
    free(items);
}

void oracle_distance(const float* V, int64_t nv, const int32_t* F, int64_t nf, const float* Q, int64_t nq,
                     double cutoff, double* d_out)
{
    oracle_distance2(V, nv, F, nf, Q, nq, cutoff, 1, d_out);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
