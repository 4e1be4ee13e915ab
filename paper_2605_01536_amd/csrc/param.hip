// param.hip -- generalized winding numbers of surfaces made of tensor-product
// cubic Bezier patches (Sec. 4.4): w(p) = chi(x0) + boundary term, FP64.
//
// Patch: 16 control points P[i][j] (i along u, j along v) at (4 i + j) * 3;
// normal S_u x S_v; its boundary runs counter-clockwise in (u, v).  A boundary
// curve of one patch cancels the same curve traversed backwards by another
// (equal control points), as interior mesh edges do (Sec. 4.1).
//
// chi(x0): one wave per query, its lanes sharing out the patches.  The ray
// p + t x0 (t > 0) is tested against each patch by subdivision driven by the ray: a sub-patch is named by its
// level and (u, v) cell, its control points are extracted from the patch by
// de Casteljau on the cell's interval, the ray is tested against their
// bounding box (convex hull property), and a sub-patch whose control net lies
// within tau of the bilinear patch through its corners (Sec. 4.4.1's test for
// "approximately bilinear") is intersected as that bilinear patch.  A hit that
// is tangent, at the query, or near a leaf's edge makes the direction
// ambiguous; the lane then shoots the next of four fixed directions (Sec. 4.4.1
// shoots another ray in these cases).
//
// Boundary term, for the chosen x0 = d and x1 = -d: the area swept by the
// geodesic triangle (x1, Gamma(t), Gamma(t + dt)) on the unit sphere around p,
// i.e. Alg. 1's per-edge term of Eq. 10 in the limit of short edges.  In a
// frame (e1, e2, d) with r = phi(t) - p, l = |r|, s = l - r_z (= rho^2 /
// (l + r_z) for r_z > 0) it is
//     (1 / 4 pi) * integral of (r_y r'_x - r_x r'_y) / (l s) dt,
// the same N and s as the mesh kernels (Alg. 2 splits the same integral into
// the spherical winding number at x1 and the field's rotation, Prop. 5.2).
// Integrated by adaptive 15-point Gauss-Kronrod per curve (bisection while
// |K15 - G7| > eps, to a maximum depth).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "gwn_alloc.h"
#include "gwn_mesh.h"

struct gwn_patches_s {
    int device = 0;
    int64_t npatch = 0, ncurves = 0;
    double tau = 0.0, eps = 0.0, diag = 0.0;
    int max_depth = 25;
    double* patches = nullptr;   // npatch * 48
    double* boxes = nullptr;     // npatch * 8: lo xyz, hi xyz of the control points, the first
                                 // subdivision level worth testing for flatness, unused
    double* curves = nullptr;    // ncurves * 12
    // grid calls run the boundary term along the first direction on a stream
    // of their own, beside the column kernel; the mutex keeps each call's
    // fork and join of the two streams together
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    std::mutex grid_mu;
};

namespace gwn {
namespace {

constexpr int kNDir = 4;
// +z, then three unit vectors in general position
__constant__ double c_dirs[kNDir][3] = {{0.0, 0.0, 1.0}, {0.36, 0.48, 0.8}, {-0.48, 0.6, 0.64}, {0.6, -0.64, 0.48}};

// Kronrod nodes on [0, 1] of the 15-point rule (symmetric; the last is the
// centre) and weights; the embedded 7-point Gauss rule uses nodes 1, 3, 5 and
// the centre
__constant__ double c_gk_x[8] = {0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
                                 0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
                                 0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
                                 0.207784955007898467600689403773245, 0.0};
__constant__ double c_gk_w[8] = {0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
                                 0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
                                 0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
                                 0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
__constant__ double c_g7_w[4] = {0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
                                 0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

constexpr double kInv4Pi = 0.079577471545947667884441881686257;
constexpr int kMaxLevel = 28;     // sub-patch cells of 2^-28
constexpr int kRayStack = 3 * kMaxLevel + 4;
// Work bounds that keep every wave finite on degenerate input: a ray grazing a
// patch meets about 2^level cells per level; past kMaxCells cells the direction
// counts as ambiguous.  An integrand that is not finite is accepted as it is
// (w becomes NaN), and past kMaxIntervals intervals for one query the remaining
// ones are accepted without bisection.
constexpr int kMaxCells = 1 << 14;
constexpr long long kMaxIntervals = 1 << 18;

struct Frame {
    double e1[3], e2[3], d[3];   // right-handed: e1 x e2 = d
};

__device__ inline Frame make_frame(int k) {
    Frame f;
    for (int c = 0; c < 3; ++c) f.d[c] = c_dirs[k][c];
    // e2: d x (the axis least aligned with d), normalised; e1 = e2 x d
    const double ax = fabs(f.d[0]), ay = fabs(f.d[1]), az = fabs(f.d[2]);
    double h[3] = {0.0, 0.0, 0.0};
    if (ax <= ay && ax <= az) h[0] = 1.0;
    else if (ay <= az) h[1] = 1.0;
    else h[2] = 1.0;
    double e[3] = {f.d[1] * h[2] - f.d[2] * h[1], f.d[2] * h[0] - f.d[0] * h[2], f.d[0] * h[1] - f.d[1] * h[0]};
    const double n = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    for (int c = 0; c < 3; ++c) f.e2[c] = e[c] / n;   // d x h
    // e1 = e2 x d so that e1 x e2 = d
    f.e1[0] = f.e2[1] * f.d[2] - f.e2[2] * f.d[1];
    f.e1[1] = f.e2[2] * f.d[0] - f.e2[0] * f.d[2];
    f.e1[2] = f.e2[0] * f.d[1] - f.e2[1] * f.d[0];
    return f;
}

// control points of the cubic c0..c3 restricted to [a, b] within [0, 1]
__device__ inline void cubic_interval(double c0, double c1, double c2, double c3, double a, double b, double* o) {
    // left part at b: control points of [0, b]
    const double l01 = c0 + b * (c1 - c0), l12 = c1 + b * (c2 - c1), l23 = c2 + b * (c3 - c2);
    const double l012 = l01 + b * (l12 - l01), l123 = l12 + b * (l23 - l12);
    const double l0123 = l012 + b * (l123 - l012);
    const double L0 = c0, L1 = l01, L2 = l012, L3 = l0123;
    // right part of that at a / b: control points of [a, b]
    const double s = b > 0.0 ? a / b : 0.0;
    const double m01 = L0 + s * (L1 - L0), m12 = L1 + s * (L2 - L1), m23 = L2 + s * (L3 - L2);
    const double m012 = m01 + s * (m12 - m01), m123 = m12 + s * (m23 - m12);
    o[0] = m012 + s * (m123 - m012);
    o[1] = m123;
    o[2] = m23;
    o[3] = L3;
}

// control points (48) of the cell [iu h, (iu + 1) h] x [iv h, (iv + 1) h], h = 2^-level
__device__ inline void extract(const double* __restrict__ P, int level, unsigned iu, unsigned iv, double* S) {
    const double h = ldexp(1.0, -level);
    const double u0 = iu * h, u1 = (iu + 1) * h, v0 = iv * h, v1 = (iv + 1) * h;
    double T[48];
    for (int j = 0; j < 4; ++j)
        for (int c = 0; c < 3; ++c) {
            double o[4];
            cubic_interval(P[(0 + j) * 3 + c], P[(4 + j) * 3 + c], P[(8 + j) * 3 + c], P[(12 + j) * 3 + c], u0, u1, o);
            for (int i = 0; i < 4; ++i) T[(4 * i + j) * 3 + c] = o[i];
        }
    for (int i = 0; i < 4; ++i)
        for (int c = 0; c < 3; ++c) {
            double o[4];
            cubic_interval(T[(4 * i) * 3 + c], T[(4 * i + 1) * 3 + c], T[(4 * i + 2) * 3 + c], T[(4 * i + 3) * 3 + c],
                           v0, v1, o);
            for (int j = 0; j < 4; ++j) S[(4 * i + j) * 3 + c] = o[j];
        }
}

struct RayState {
    double p[3], d[3], e1[3], e2[3], invd[3];
    double tau, margin;
    int chi;
    bool amb;
    // line mode (a grid column): every hit along the whole line goes to an LDS
    // list of (z, sign); a full list makes the line ambiguous
    bool line = false;
    double* hz = nullptr;
    int* hs = nullptr;
    int* hn = nullptr;
    int hcap = 0;
};

__device__ inline bool ray_box(const RayState& R, const double* lo, const double* hi) {
    double t0 = R.line ? -1e300 : 0.0, t1 = 1e300;
    for (int c = 0; c < 3; ++c) {
        const double pad = 1e-12 * (1.0 + fabs(lo[c]) + fabs(hi[c]));
        const double l = lo[c] - pad, u = hi[c] + pad;
        if (R.d[c] == 0.0) {
            if (R.p[c] < l || R.p[c] > u) return false;
        } else {
            const double inv = R.invd[c];
            double a = (l - R.p[c]) * inv, b = (u - R.p[c]) * inv;
            if (a > b) {
                const double t = a;
                a = b;
                b = t;
            }
            t0 = fmax(t0, a);
            t1 = fmin(t1, b);
            if (t0 > t1) return false;
        }
    }
    return true;
}

// distance of the control net from the bilinear patch through its corners
__device__ inline double net_deviation(const double* S) {
    double m = 0.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            const double u = i * (1.0 / 3.0), v = j * (1.0 / 3.0);
            double e2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double b = (1.0 - u) * ((1.0 - v) * S[c] + v * S[9 + c]) +
                                 u * ((1.0 - v) * S[36 + c] + v * S[45 + c]);
                const double e = S[(4 * i + j) * 3 + c] - b;
                e2 += e * e;
            }
            m = fmax(m, e2);
        }
    return sqrt(m);
}

// the ray against the bilinear patch through the corners of S (00, 10, 11, 01
// at control points 0, 12, 15, 3): two planes through the ray, e1.(x - p) = 0
// and e2.(x - p) = 0, each bilinear in (u, v); eliminating u gives a quadratic
// in v
// bedge: bits 0..3 set where the leaf's u = 0, u = 1, v = 0, v = 1 edge lies on
// the patch's boundary; there the margin also covers the leaf chord's distance
// from the exact boundary curve (up to tau), so a ray that passes between them
// is ambiguous rather than counted against the wrong side
__device__ inline void bilinear_hits(RayState& R, const double* S, int bedge) {
    const double* q[4] = {S, S + 36, S + 45, S + 9};
    double f1[4], f2[4];
    for (int k = 0; k < 4; ++k) {
        const double r0 = q[k][0] - R.p[0], r1 = q[k][1] - R.p[1], r2 = q[k][2] - R.p[2];
        f1[k] = r0 * R.e1[0] + r1 * R.e1[1] + r2 * R.e1[2];
        f2[k] = r0 * R.e2[0] + r1 * R.e2[1] + r2 * R.e2[2];
    }
    // f(u, v) = a + b u + c v + d u v
    const double a1 = f1[0], b1 = f1[1] - f1[0], c1 = f1[3] - f1[0], d1 = f1[0] - f1[1] + f1[2] - f1[3];
    const double a2 = f2[0], b2 = f2[1] - f2[0], c2 = f2[3] - f2[0], d2 = f2[0] - f2[1] + f2[2] - f2[3];
    // (a2 + c2 v)(b1 + d1 v) - (a1 + c1 v)(b2 + d2 v) = 0
    const double A = c2 * d1 - c1 * d2;
    const double B = a2 * d1 + c2 * b1 - a1 * d2 - c1 * b2;
    const double C = a2 * b1 - a1 * b2;
    const double sc = fabs(A) + fabs(B) + fabs(C);
    if (sc == 0.0) {
        R.amb = true;
        return;
    }
    double roots[2];
    int nr = 0;
    if (fabs(A) <= 1e-14 * sc) {
        if (B != 0.0) roots[nr++] = -C / B;
    } else {
        const double disc = B * B - 4.0 * A * C;
        if (disc < 0.0) return;
        const double sq = sqrt(disc);
        const double qq = -0.5 * (B + (B >= 0.0 ? sq : -sq));
        roots[nr++] = qq / A;
        if (qq != 0.0 && disc > 0.0) roots[nr++] = C / qq;
    }
    for (int k = 0; k < nr; ++k) {
        const double v = roots[k];
        const double den1 = b1 + d1 * v, den2 = b2 + d2 * v;
        double u;
        if (fabs(den1) >= fabs(den2)) {
            if (den1 == 0.0) {
                R.amb = true;
                continue;
            }
            u = -(a1 + c1 * v) / den1;
        } else {
            u = -(a2 + c2 * v) / den2;
        }
        double mu0 = R.margin, mu1 = R.margin, mv0 = R.margin, mv1 = R.margin;
        if (bedge) {
            const double lu = sqrt((q[1][0] - q[0][0]) * (q[1][0] - q[0][0]) + (q[1][1] - q[0][1]) * (q[1][1] - q[0][1]) +
                                   (q[1][2] - q[0][2]) * (q[1][2] - q[0][2]));
            const double lv = sqrt((q[3][0] - q[0][0]) * (q[3][0] - q[0][0]) + (q[3][1] - q[0][1]) * (q[3][1] - q[0][1]) +
                                   (q[3][2] - q[0][2]) * (q[3][2] - q[0][2]));
            const double bu = lu > 0.0 ? 4.0 * R.tau / lu : 1.0, bv = lv > 0.0 ? 4.0 * R.tau / lv : 1.0;
            if (bedge & 1) mu0 = fmax(mu0, bu);
            if (bedge & 2) mu1 = fmax(mu1, bu);
            if (bedge & 4) mv0 = fmax(mv0, bv);
            if (bedge & 8) mv1 = fmax(mv1, bv);
        }
        if (u < -mu0 || u > 1.0 + mu1 || v < -mv0 || v > 1.0 + mv1) continue;
        if (u < mu0 || u > 1.0 - mu1 || v < mv0 || v > 1.0 - mv1) {
            R.amb = true;
            continue;
        }
        double X[3], Su[3], Sv[3];
        for (int c = 0; c < 3; ++c) {
            X[c] = (1.0 - u) * ((1.0 - v) * q[0][c] + v * q[3][c]) + u * ((1.0 - v) * q[1][c] + v * q[2][c]);
            Su[c] = (1.0 - v) * (q[1][c] - q[0][c]) + v * (q[2][c] - q[3][c]);
            Sv[c] = (1.0 - u) * (q[3][c] - q[0][c]) + u * (q[2][c] - q[1][c]);
        }
        const double n0 = Su[1] * Sv[2] - Su[2] * Sv[1], n1 = Su[2] * Sv[0] - Su[0] * Sv[2],
                     n2 = Su[0] * Sv[1] - Su[1] * Sv[0];
        const double nn = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        const double nd = n0 * R.d[0] + n1 * R.d[1] + n2 * R.d[2];
        const double r0 = X[0] - R.p[0], r1 = X[1] - R.p[1], r2 = X[2] - R.p[2];
        const double t = r0 * R.d[0] + r1 * R.d[1] + r2 * R.d[2];
        if (!(nn > 0.0) || fabs(nd) < 1e-9 * nn) {
            R.amb = true;
            continue;
        }
        if (R.line) {   // the samples of the column classify the hit later
            const int slot = atomicAdd(R.hn, 1);
            if (slot < R.hcap) {
                R.hz[slot] = X[2];
                R.hs[slot] = nd > 0.0 ? 1 : -1;
            } else {
                R.amb = true;
            }
            continue;
        }
        if (fabs(t) <= 1e-12 * (1.0 + sqrt(r0 * r0 + r1 * r1 + r2 * r2))) {
            R.amb = true;   // the query on the surface
            continue;
        }
        if (t > 0.0) R.chi += nd > 0.0 ? 1 : -1;
    }
}

// one patch: depth-first over sub-patch cells whose control-point box meets the ray
// (returns the number of cells extracted)
// (start: the cell to begin with, level << 58 | iu << 29 | iv; 0 = the whole patch)
__device__ int patch_ray(RayState& R, const double* __restrict__ P, int flat_level,
                         unsigned long long start = 0ull) {
    unsigned long long stk[kRayStack];
    int sp = 0;
    stk[sp++] = start;
    int cells = 0;
    while (sp > 0) {
        if (++cells > kMaxCells) {
            R.amb = true;
            return cells;
        }
        const unsigned long long code = stk[--sp];
        const int level = (int)(code >> 58);
        const unsigned iu = (unsigned)((code >> 29) & 0x1fffffffu), iv = (unsigned)(code & 0x1fffffffu);
        double S[48];
        extract(P, level, iu, iv, S);
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int k = 0; k < 16; ++k)
            for (int c = 0; c < 3; ++c) {
                lo[c] = fmin(lo[c], S[3 * k + c]);
                hi[c] = fmax(hi[c], S[3 * k + c]);
            }
        if (!ray_box(R, lo, hi)) continue;
        // the net's distance from bilinear falls about 4x per level: cells above
        // flat_level are subdivided without the test (a later leaf is as valid)
        if (level >= kMaxLevel || (level >= flat_level && net_deviation(S) <= R.tau)) {
            const unsigned last = (1u << level) - 1u;
            bilinear_hits(R, S, (iu == 0 ? 1 : 0) | (iu == last ? 2 : 0) | (iv == 0 ? 4 : 0) | (iv == last ? 8 : 0));
            continue;
        }
        if (sp + 4 > kRayStack) {   // cannot happen for depth-first with kRayStack >= 3 levels + 4
            R.amb = true;
            continue;
        }
        const unsigned long long nl = (unsigned long long)(level + 1) << 58;
        for (int c = 0; c < 4; ++c) {
            const unsigned long long cu = 2ull * iu + (c & 1), cv = 2ull * iv + (c >> 1);
            stk[sp++] = nl | (cu << 29) | cv;
        }
    }
    return cells;
}

// One wave per query: its lanes share the sub-patch cells of the crossings and
// the quadrature intervals of the boundary term through queues in LDS; the
// partial counts and sums are combined across the wave in a fixed butterfly
// order.  A direction is ambiguous for the query if it is for any lane.  STATS:
// also add the wave's quadrature intervals and sub-patch cells to stats[0],
// stats[1].
constexpr int kParamWaves = 4;   // waves (queries) per workgroup

__device__ inline double wave_sum(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// query points: strided FP32 arrays, or the cell-centred grid
// float(origin + (idx + 0.5) spacing) (each coordinate rounded once from FP64,
// as for meshes), flattened (i ny + j) nz + k
struct BatchPts {
    const float *x, *y, *z;
    long long qs;
    __device__ inline void get(long long i, double* p) const {
        p[0] = x[i * qs];
        p[1] = y[i * qs];
        p[2] = z[i * qs];
    }
};

__device__ inline float cell_coord(double o, double s, long long i) {
#pragma clang fp contract(off)   // the product and the sum rounded separately (no fused multiply-add)
    const double t = ((double)i + 0.5) * s;
    return (float)(o + t);
}

struct GridPts {
    double o[3], s[3];
    long long ny, nz;
    __device__ inline void get(long long i, double* p) const {
        const long long k = i % nz, ij = i / nz;
        p[0] = cell_coord(o[0], s[0], ij / ny);
        p[1] = cell_coord(o[1], s[1], ij % ny);
        p[2] = cell_coord(o[2], s[2], k);
    }
};

constexpr int kPending = -2;   // direction not decided yet (a grid column that needs single rays)

// crossings: chi and the chosen direction per query (-1: all ambiguous).
// PENDING: only the queries whose direction is kPending.  The wave's lanes share
// one LDS queue of sub-patch cells (patch, level, u cell, v cell): each round
// they take up to 64, test their boxes and intersect them or queue their
// quarters (placed by lane rank); patches enter while a round of them fits, and
// a lane whose quarters find no room follows them alone.
constexpr int kWaveCells = 256;   // sub-patch cells waiting, per wave
// a ray (or a column's line) that meets more cells than this in all patches
// together is taken as ambiguous, as one meeting kMaxCells in one patch is
constexpr long long kMaxQueueCells = 1ll << 20;

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int lane_rank(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

template <bool STATS, bool PENDING, class Pts>
__global__ __launch_bounds__(64 * kParamWaves) void k_param_chi(
    const double* __restrict__ patches, const double* __restrict__ boxes, long long npatch, Pts pts, long long nq,
    double tau, int* __restrict__ chi_out, int* __restrict__ dir_out, unsigned long long* __restrict__ stats) {
    const long long i = blockIdx.x * (long long)kParamWaves + (threadIdx.x >> 6);
    if (i >= nq) return;   // whole waves leave together
    if (PENDING && dir_out[i] != kPending) return;
    const int lane = threadIdx.x & 63;
    __shared__ unsigned long long wq[kParamWaves][kWaveCells];   // cell codes as patch_ray's
    __shared__ int wp[kParamWaves][kWaveCells];
    unsigned long long* Q = wq[threadIdx.x >> 6];
    int* QP = wp[threadIdx.x >> 6];
    RayState R;
    pts.get(i, R.p);
    R.tau = tau;
    R.margin = 1e-9;
    int dir = -1, chi = 0;
    long long ncell = 0;
    for (int k = 0; k < kNDir && dir < 0; ++k) {
        const Frame F = make_frame(k);
        for (int c = 0; c < 3; ++c) {
            R.d[c] = F.d[c];
            R.e1[c] = F.e1[c];
            R.e2[c] = F.e2[c];
            R.invd[c] = F.d[c] != 0.0 ? 1.0 / F.d[c] : 0.0;
        }
        R.chi = 0;
        R.amb = false;
        int n = 0;   // queue length (the same in every lane)
        long long next = 0, total = 0;
        while (true) {
            while (next < npatch && n <= kWaveCells - 64) {
                const long long pi = next + lane;
                const bool in = pi < npatch && ray_box(R, boxes + 8 * pi, boxes + 8 * pi + 3);
                const unsigned long long m = __builtin_amdgcn_ballot_w64(in);
                if (in) {
                    const int slot = n + lane_rank(m);
                    Q[slot] = 0ull;
                    QP[slot] = (int)pi;
                }
                n += __builtin_popcountll(m);
                next += 64;
            }
            wave_lds_sync();
            if (n == 0) break;   // every patch offered and every cell done
            const int take = min(n, 64);
            n -= take;
            total += take;
            if (total > kMaxQueueCells) {
                R.amb = true;
                break;
            }
            unsigned long long code = 0ull;
            int pi = 0;
            if (lane < take) {
                code = Q[n + lane];
                pi = QP[n + lane];
            }
            wave_lds_sync();
            bool split = false;
            const int level = (int)(code >> 58);
            const unsigned iu = (unsigned)((code >> 29) & 0x1fffffffu), iv = (unsigned)(code & 0x1fffffffu);
            const double* P = patches + 48 * (long long)pi;
            const int flat_level = (int)boxes[8 * (long long)pi + 6];
            if (lane < take) {
                double S[48];
                extract(P, level, iu, iv, S);
                ++ncell;
                double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
                for (int k2 = 0; k2 < 16; ++k2)
                    for (int c = 0; c < 3; ++c) {
                        lo[c] = fmin(lo[c], S[3 * k2 + c]);
                        hi[c] = fmax(hi[c], S[3 * k2 + c]);
                    }
                if (ray_box(R, lo, hi)) {
                    if (level >= kMaxLevel || (level >= flat_level && net_deviation(S) <= R.tau)) {
                        const unsigned last = (1u << level) - 1u;
                        bilinear_hits(R, S, (iu == 0 ? 1 : 0) | (iu == last ? 2 : 0) | (iv == 0 ? 4 : 0) |
                                                (iv == last ? 8 : 0));
                    } else {
                        split = true;
                    }
                }
            }
            const unsigned long long m = __builtin_amdgcn_ballot_w64(split);
            const int room = (kWaveCells - n) / 4;
            if (split) {
                const int rank = lane_rank(m);
                const unsigned long long nl = (unsigned long long)(level + 1) << 58;
                for (int c = 0; c < 4; ++c) {
                    const unsigned long long cu = 2ull * iu + (c & 1), cv = 2ull * iv + (c >> 1);
                    const unsigned long long child = nl | (cu << 29) | cv;
                    if (rank < room) {
                        Q[n + 4 * rank + c] = child;
                        QP[n + 4 * rank + c] = pi;
                    } else {   // no room: this lane alone
                        ncell += patch_ray(R, P, flat_level, child);
                    }
                }
            }
            n += 4 * min(__builtin_popcountll(m), room);
            wave_lds_sync();
            if (__builtin_amdgcn_ballot_w64(R.amb) != 0ull) break;
        }
        if (__builtin_amdgcn_ballot_w64(R.amb) == 0ull) {
            dir = k;
            int c = R.chi;
            for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
            chi = c;
        }
    }
    if (lane == 0) {
        chi_out[i] = dir >= 0 ? chi : 0;
        dir_out[i] = dir;
    }
    if constexpr (STATS) atomicAdd(&stats[1], (unsigned long long)ncell);
}

// Grid columns (Sec. 4.3.1's ray reuse): one workgroup per (i, j) column finds
// every crossing of the column's vertical line (+z) once, its lanes sharing out
// the patches; each sample's chi is the signed count of the crossings above it.
// A column whose line has an ambiguous hit, and a sample within the on-surface
// margin of a crossing, are left kPending for single rays.
constexpr int kMaxHits = 256;

constexpr int kColThreads = 256;   // one workgroup per column
constexpr int kCellQueue = 1024;   // sub-patch cells waiting, per workgroup

template <bool STATS>
__global__ __launch_bounds__(kColThreads) void k_param_cols(
    const double* __restrict__ patches, const double* __restrict__ boxes, long long npatch, GridPts g,
    long long ncols, double tau, int* __restrict__ chi_out, int* __restrict__ dir_out,
    unsigned long long* __restrict__ stats) {
    __shared__ double hz[kMaxHits];
    __shared__ int hs[kMaxHits];
    __shared__ unsigned long long queue[kCellQueue];   // cell codes as patch_ray's
    __shared__ int qpatch[kCellQueue];
    __shared__ int hn, amb_any, qn, qpush;
    const long long col = blockIdx.x;
    if (col >= ncols) return;   // the whole workgroup
    const int tid = threadIdx.x;
    if (tid == 0) {
        hn = 0;
        amb_any = 0;
        qn = 0;
    }
    __syncthreads();
    const long long ci = col / g.ny, cj = col - ci * g.ny;
    RayState R;
    R.p[0] = cell_coord(g.o[0], g.s[0], ci);
    R.p[1] = cell_coord(g.o[1], g.s[1], cj);
    R.p[2] = 0.0;
    R.tau = tau;
    R.margin = 1e-9;
    const Frame F = make_frame(0);
    for (int c = 0; c < 3; ++c) {
        R.d[c] = F.d[c];
        R.e1[c] = F.e1[c];
        R.e2[c] = F.e2[c];
        R.invd[c] = F.d[c] != 0.0 ? 1.0 / F.d[c] : 0.0;
    }
    R.chi = 0;
    R.amb = false;
    R.line = true;
    R.hz = hz;
    R.hs = hs;
    R.hn = &hn;
    R.hcap = kMaxHits;
    long long ncell = 0;
    // The whole workgroup works through one queue of cells (patch, level, u
    // cell, v cell) whose boxes the line may meet: each round every lane takes a
    // cell, tests its box, intersects it if flat, or queues its four quarters.
    // Patches whose box the line meets enter while the queue has room for a
    // full round of them; a cell whose quarters find no room is followed by its
    // lane alone.  Every cell is visited once in some order, and the crossings
    // are an integer sum, so the result does not depend on the schedule.
    long long next = 0, total = 0;
    while (true) {
        while (next < npatch && qn <= kCellQueue - kColThreads) {
            const long long pi = next + tid;
            const bool in = pi < npatch && ray_box(R, boxes + 8 * pi, boxes + 8 * pi + 3);
            __syncthreads();   // every lane has read qn
            if (in) {
                const int slot = atomicAdd(&qn, 1);   // < kCellQueue by the loop's condition
                queue[slot] = 0ull;
                qpatch[slot] = (int)pi;
            }
            next += kColThreads;
            __syncthreads();
        }
        const int n = qn;
        // n == 0 here only once every patch has been offered
        if (n == 0 || amb_any) break;   // an ambiguous line: its samples take single rays anyway
        const int take = min(n, kColThreads), base = n - take;
        total += take;
        if (total > kMaxQueueCells) {
            amb_any = 1;   // every lane writes the same value
            break;
        }
        unsigned long long code = 0ull;
        int pi = 0;
        if (tid < take) {
            code = queue[base + tid];
            pi = qpatch[base + tid];
        }
        __syncthreads();   // the taken slots have been read
        if (tid == 0) qpush = base;
        __syncthreads();
        if (tid < take) {
            const int level = (int)(code >> 58);
            const unsigned iu = (unsigned)((code >> 29) & 0x1fffffffu), iv = (unsigned)(code & 0x1fffffffu);
            const double* P = patches + 48 * (long long)pi;
            const int flat_level = (int)boxes[8 * (long long)pi + 6];
            double S[48];
            extract(P, level, iu, iv, S);
            ++ncell;
            double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
            for (int k = 0; k < 16; ++k)
                for (int c = 0; c < 3; ++c) {
                    lo[c] = fmin(lo[c], S[3 * k + c]);
                    hi[c] = fmax(hi[c], S[3 * k + c]);
                }
            if (ray_box(R, lo, hi)) {
                if (level >= kMaxLevel || (level >= flat_level && net_deviation(S) <= R.tau)) {
                    const unsigned last = (1u << level) - 1u;
                    bilinear_hits(R, S, (iu == 0 ? 1 : 0) | (iu == last ? 2 : 0) | (iv == 0 ? 4 : 0) |
                                            (iv == last ? 8 : 0));
                } else {
                    const unsigned long long nl = (unsigned long long)(level + 1) << 58;
                    const int slot = atomicAdd(&qpush, 4);
                    for (int c = 0; c < 4; ++c) {
                        const unsigned long long cu = 2ull * iu + (c & 1), cv = 2ull * iv + (c >> 1);
                        const unsigned long long child = nl | (cu << 29) | cv;
                        if (slot + 4 <= kCellQueue) {
                            queue[slot + c] = child;
                            qpatch[slot + c] = pi;
                        } else {   // no room: this lane alone
                            ncell += patch_ray(R, P, flat_level, child);
                        }
                    }
                }
            }
            if (R.amb) amb_any = 1;
        }
        __syncthreads();
        // slots are handed out 4 at a time from base: those below the last
        // multiple of 4 that fits were all written
        if (tid == 0) qn = min(qpush, base + ((kCellQueue - base) & ~3));
        __syncthreads();
    }
    __syncthreads();
    const bool amb = amb_any != 0;
    const int nh = min(hn, kMaxHits);
    const long long base = col * g.nz;
    for (long long k = tid; k < g.nz; k += kColThreads) {
        const double pz = cell_coord(g.o[2], g.s[2], k);
        int chi = 0;
        bool on = amb;
        for (int h = 0; h < nh && !on; ++h) {
            const double t = hz[h] - pz;
            if (fabs(t) <= 1e-12 * (1.0 + fabs(t))) on = true;
            else if (t > 0.0) chi += hs[h];
        }
        chi_out[base + k] = on ? 0 : chi;
        dir_out[base + k] = on ? kPending : 0;
    }
    if constexpr (STATS) atomicAdd(&stats[1], (unsigned long long)ncell);
}

// The boundary integrand (without 1 / 4 pi) at one point of a curve, from the
// point's coordinates relative to the query in the ray's frame (x, y along e1,
// e2; z along the ray) and the derivatives dx, dy along the curve's parameter:
// (y dx - x dy) / (l s), s = l - z, written for z > 0 through s = rho^2 / (l + z)
// so that neither side cancels.  1 / l and the other reciprocal come from the
// hardware estimates refined by one Newton step each (the step squares the
// estimate's relative error); against correctly rounded operations the
// quadrature's intervals and results move only in the last digits, far below
// its tolerance.  A zero length or denominator gives a non-finite value as a
// division would.
__device__ inline double area_rate_xyz(double x, double y, double z, double dx, double dy) {
    const double rho2 = x * x + y * y;
    const double l2 = rho2 + z * z, hl2 = 0.5 * l2;
    double ri = __builtin_amdgcn_rsq(l2);
    ri = ri * (1.5 - hl2 * (ri * ri));
    const double l = l2 * ri;
    const double num = y * dx - x * dy;
    const bool up = z > 0.0;
    const double den = up ? rho2 : l - z;
    double qi = __builtin_amdgcn_rcp(den);
    qi = qi * (2.0 - den * qi);
    return (up ? num * (l + z) : num) * ri * qi;
}

// GK15 of the integrand on the dyadic interval idx of 2^-level of curve C: K15
// and G7.  The curve is taken relative to the query in the ray's frame and
// expanded about the interval's centre in the local parameter s in [-1, 1]
// (t = centre + s h / 2), a cubic a0 + a1 s + a2 s^2 + a3 s^3 per coordinate;
// the nodes come in pairs +-x, whose points share the even and odd parts.  The
// integrand is homogeneous of degree 1 in the derivative, so with derivatives
// along s the rules' weights apply without the factor h / 2.
__device__ inline void gk15_interval(const double* __restrict__ C, int level, unsigned long long idx,
                                     const double* p, const Frame& F, double& K, double& G) {
    const double h = ldexp(1.0, -level);
    const double c = ((double)idx + 0.5) * h, hw = 0.5 * h;
    double a[3][4];
    for (int j = 0; j < 3; ++j) {
        const double* ax = j == 0 ? F.e1 : (j == 1 ? F.e2 : F.d);
        double q[4];
        for (int k = 0; k < 4; ++k)
            q[k] = (C[3 * k] - p[0]) * ax[0] + (C[3 * k + 1] - p[1]) * ax[1] + (C[3 * k + 2] - p[2]) * ax[2];
        // power basis in t
        const double b1 = 3.0 * (q[1] - q[0]), b2 = 3.0 * (q[0] - 2.0 * q[1] + q[2]);
        const double b3 = q[3] - q[0] + 3.0 * (q[1] - q[2]);
        // Taylor coefficients about c, scaled by powers of hw
        a[j][0] = q[0] + c * (b1 + c * (b2 + c * b3));
        a[j][1] = hw * (b1 + c * (2.0 * b2 + 3.0 * c * b3));
        a[j][2] = hw * hw * (b2 + 3.0 * c * b3);
        a[j][3] = hw * hw * hw * b3;
    }
    const double fc = area_rate_xyz(a[0][0], a[1][0], a[2][0], a[0][1], a[1][1]);
    K = c_gk_w[7] * fc;
    G = c_g7_w[3] * fc;
    for (int i = 0; i < 7; ++i) {
        const double x = c_gk_x[i], x2 = x * x;
        double ev[3], od[3];
        for (int j = 0; j < 3; ++j) {
            ev[j] = a[j][0] + a[j][2] * x2;
            od[j] = x * (a[j][1] + a[j][3] * x2);
        }
        // derivative a1 + 2 a2 s + 3 a3 s^2: even part a1 + 3 a3 x^2, odd part 2 a2 x
        const double dex = a[0][1] + 3.0 * a[0][3] * x2, dox = 2.0 * a[0][2] * x;
        const double dey = a[1][1] + 3.0 * a[1][3] * x2, doy = 2.0 * a[1][2] * x;
        const double f = area_rate_xyz(ev[0] - od[0], ev[1] - od[1], ev[2] - od[2], dex - dox, dey - doy) +
                         area_rate_xyz(ev[0] + od[0], ev[1] + od[1], ev[2] + od[2], dex + dox, dey + doy);
        K += c_gk_w[i] * f;
        if (i & 1) G += c_g7_w[i >> 1] * f;
    }
}

// The integral over interval idx of 2^-level of curve C by one lane alone:
// depth-first bisection with a private stack (for intervals that do not fit
// the wave's queue)
__device__ double interval_local(const double* __restrict__ C, int level0, unsigned long long idx0, const double* p,
                                 const Frame& F, double eps, int max_depth, long long& nint) {
    unsigned long long stk[2 * 32];
    int sp = 0;
    stk[sp++] = ((unsigned long long)level0 << 30) | idx0;
    double sum = 0.0;
    while (sp > 0) {
        const unsigned long long code = stk[--sp];
        const int level = (int)(code >> 30);
        const unsigned long long idx = code & ((1ull << 30) - 1);
        double K, G;
        gk15_interval(C, level, idx, p, F, K, G);
        ++nint;
        if (!(fabs(K - G) > eps) || level >= max_depth || sp + 2 > 2 * 32) {
            sum += K;
        } else {
            const unsigned long long nl = (unsigned long long)(level + 1) << 30;
            stk[sp++] = nl | (2ull * idx + 1);
            stk[sp++] = nl | (2ull * idx);
        }
    }
    return sum;
}

// Boundary term along the direction chosen for each query, and w.  The wave's
// 64 lanes share one queue of intervals in LDS (curve, level, index): each round
// the lanes take the 64 newest, accept those with |K15 - G7| <= eps (or at the
// maximum depth) and push both halves of the others; new curves enter as the
// queue drains.  Every lane stays busy whatever the curves' difficulty, and the
// order is fixed (pushes are placed by lane rank), so w is deterministic.  A
// lane whose halves find no room finishes that interval alone (interval_local).
constexpr int kQueue = 512;   // intervals per wave
constexpr int kQueueRefill = 192;   // new curves enter while fewer intervals wait

// MODE 0: the direction in dir[i], w = chi + S / 4 pi (NaN without a
// direction); MODE 1: the first direction for every query, w = S / 4 pi;
// MODE 2: after MODE 1, queries with dir[i] == 0 add chi, the others are
// computed as in MODE 0.
template <bool STATS, class Pts, int MODE = 0>
__global__ __launch_bounds__(64 * kParamWaves) void k_param_bdry(
    const double* __restrict__ curves, long long ncurves, Pts pts, long long nq, double eps, int max_depth,
    const int* __restrict__ chi, const int* __restrict__ dir, double* __restrict__ w,
    unsigned long long* __restrict__ stats) {
    __shared__ unsigned long long queue[kParamWaves][kQueue];
    const int wave = threadIdx.x >> 6;
    const long long i = blockIdx.x * (long long)kParamWaves + wave;
    if (i >= nq) return;
    const int lane = threadIdx.x & 63;
    unsigned long long* Qw = queue[wave];
    const int d = MODE == 1 ? 0 : dir[i];
    if (MODE == 2 && d == 0) {
        if (lane == 0) w[i] = (double)chi[i] + w[i];
        return;   // the whole wave
    }
    double p[3];
    pts.get(i, p);
    double S = 0.0;
    long long nint = 0;
    if (d >= 0) {
        const Frame F = make_frame(d);
        int n = 0;                 // queue length (the same in every lane)
        long long next = 0;        // next curve to enter
        long long done = 0;        // intervals taken so far by the wave
        while (true) {
            // curves enter while room for a full round of pushes remains
            while (next < ncurves && n < kQueueRefill) {
                const int take = (int)min((long long)min(64, kQueueRefill - n), ncurves - next);
                if (lane < take) Qw[n + lane] = (unsigned long long)(next + lane) << 36;   // level 0, index 0
                n += take;
                next += take;
            }
            // the take below reads slots other lanes wrote in the refill
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (n == 0) break;
            const int take = min(n, 64);
            n -= take;
            const unsigned long long code = lane < take ? Qw[n + lane] : 0ull;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            bool split = false;
            double K = 0.0;
            const long long cv = (long long)(code >> 36);
            const int level = (int)((code >> 30) & 63);
            const unsigned long long idx = code & ((1ull << 30) - 1);
            if (lane < take) {
                double G;
                gk15_interval(curves + 12 * cv, level, idx, p, F, K, G);
                split = fabs(K - G) > eps && level < max_depth && done < kMaxIntervals;   // NaN: accepted
                ++nint;
            }
            done += take;
            // halves go where the lane's rank among splitting lanes puts them; past
            // the queue's room the interval is accepted as it is
            const unsigned long long m = __builtin_amdgcn_ballot_w64(split);
            const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            const int room = (kQueue - n) / 2;
            if (split && rank >= room) {
                split = false;
                K = interval_local(curves + 12 * cv, level, idx, p, F, eps, max_depth, nint);
                --nint;   // the interval itself was counted above
            }
            if (lane < take && !split) S += K;
            if (split) {
                const unsigned long long nl = ((unsigned long long)cv << 36) | ((unsigned long long)(level + 1) << 30);
                Qw[n + 2 * rank] = nl | (2ull * idx + 1);
                Qw[n + 2 * rank + 1] = nl | (2ull * idx);
            }
            n += 2 * min(__builtin_popcountll(m), room);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    S = wave_sum(S);
    // the product rounded on its own in every mode, as MODE 1 + 2 split it
    const double b = __dmul_rn(S, kInv4Pi);
    if (lane == 0) w[i] = MODE == 1 ? b : (d >= 0 ? (double)chi[i] + b : NAN);
    if constexpr (STATS) atomicAdd(&stats[0], (unsigned long long)nint);
}

// both kernels for queries [0, n): chi and dir are device buffers of n
template <bool STATS>
hipError_t launch_param(const gwn_patches_s* h, const float* qx, const float* qy, const float* qz, long long qs,
                        long long n, double* w, int* chi, int* dir, unsigned long long* stats, hipStream_t st) {
    const unsigned blocks = (unsigned)((n + kParamWaves - 1) / kParamWaves);
    const BatchPts pts{qx, qy, qz, qs};
    k_param_chi<STATS, false><<<blocks, 64 * kParamWaves, 0, st>>>(h->patches, h->boxes, h->npatch, pts, n, h->tau,
                                                                   chi, dir, stats);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_param_bdry<STATS><<<blocks, 64 * kParamWaves, 0, st>>>(h->curves, h->ncurves, pts, n, h->eps, h->max_depth,
                                                             chi, dir, w, stats);
    return hipGetLastError();
}

// a grid: columns once, single rays for what they leave pending, then the boundary term
template <bool STATS>
// Without STATS the boundary term along the first direction runs on the
// handle's side stream while the columns are intersected (most queries take
// that direction); the rest is fixed up after both.  With STATS the kernels run
// in sequence, so each interval is counted once.
hipError_t launch_param_grid(gwn_patches_s* h, const GridPts& g, long long nx, double* w, int* chi, int* dir,
                             unsigned long long* stats, hipStream_t st) {
    const long long ncols = nx * g.ny, n = ncols * g.nz;
    const unsigned blocks = (unsigned)((n + kParamWaves - 1) / kParamWaves);
    std::unique_lock<std::mutex> lock(h->grid_mu, std::defer_lock);
    hipError_t e = hipSuccess;
    if constexpr (!STATS) {
        lock.lock();
        if (!h->side) {
            e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&h->fork, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&h->join, hipEventDisableTiming);
            if (e != hipSuccess) {   // leave none of the three half made
                if (h->side) (void)hipStreamDestroy(h->side);
                if (h->fork) (void)hipEventDestroy(h->fork);
                h->side = nullptr;
                h->fork = nullptr;
                return e;
            }
        }
        e = hipEventRecord(h->fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(h->side, h->fork, 0);
        if (e != hipSuccess) return e;
    }
    // after the fork every return joins the side stream back into st first, so
    // that work on st (and a caller synchronising st) also waits for the side
    // kernel, which may still be writing w
    bool joined = false;   // the join event has been recorded on the side stream
    auto rejoin = [&](hipError_t err) {
        if constexpr (!STATS) {
            if (!joined) (void)hipEventRecord(h->join, h->side);
            (void)hipStreamWaitEvent(st, h->join, 0);
        }
        return err;
    };
    k_param_cols<STATS><<<(unsigned)ncols, kColThreads, 0, st>>>(h->patches, h->boxes, h->npatch, g, ncols, h->tau,
                                                                 chi, dir, stats);
    e = hipGetLastError();
    if (e != hipSuccess) return rejoin(e);
    if constexpr (!STATS) {
        k_param_bdry<false, GridPts, 1><<<blocks, 64 * kParamWaves, 0, h->side>>>(
            h->curves, h->ncurves, g, n, h->eps, h->max_depth, chi, dir, w, nullptr);
        e = hipGetLastError();
        if (e == hipSuccess) {
            e = hipEventRecord(h->join, h->side);
            joined = e == hipSuccess;
        }
        if (e != hipSuccess) return rejoin(e);
    }
    k_param_chi<STATS, true><<<blocks, 64 * kParamWaves, 0, st>>>(h->patches, h->boxes, h->npatch, g, n, h->tau, chi,
                                                                  dir, stats);
    e = hipGetLastError();
    if (e != hipSuccess) return rejoin(e);
    if constexpr (STATS) {
        k_param_bdry<true><<<blocks, 64 * kParamWaves, 0, st>>>(h->curves, h->ncurves, g, n, h->eps, h->max_depth,
                                                                chi, dir, w, stats);
    } else {
        e = hipStreamWaitEvent(st, h->join, 0);
        if (e != hipSuccess) return e;
        k_param_bdry<false, GridPts, 2><<<blocks, 64 * kParamWaves, 0, st>>>(
            h->curves, h->ncurves, g, n, h->eps, h->max_depth, chi, dir, w, nullptr);
    }
    return hipGetLastError();
}

// host: the four boundary curves of patch k, counter-clockwise in (u, v)
void patch_curves(const double* P, double (*out)[12]) {
    auto cp = [&](int i, int j, double* o) {
        for (int c = 0; c < 3; ++c) o[c] = P[(4 * i + j) * 3 + c];
    };
    for (int k = 0; k < 4; ++k) {
        cp(k, 0, out[0] + 3 * k);        // v = 0, u 0 -> 1
        cp(3, k, out[1] + 3 * k);        // u = 1, v 0 -> 1
        cp(3 - k, 3, out[2] + 3 * k);    // v = 1, u 1 -> 0
        cp(0, 3 - k, out[3] + 3 * k);    // u = 0, v 1 -> 0
    }
}

struct CurveKey {
    uint64_t b[12];
    bool operator<(const CurveKey& o) const { return std::memcmp(b, o.b, sizeof b) < 0; }
};

CurveKey key_of(const double* c, bool reversed) {
    CurveKey k;
    for (int i = 0; i < 4; ++i) {
        const int src = reversed ? 3 - i : i;
        for (int x = 0; x < 3; ++x) {
            double v = c[3 * src + x];
            if (v == 0.0) v = 0.0;   // +0 and -0 are the same point
            std::memcpy(&k.b[3 * i + x], &v, 8);
        }
    }
    return k;
}

}  // namespace
}  // namespace gwn

using gwn::set_error;

extern "C" {

gwn_status gwn_patches_build(const double* cps, int64_t npatch, const gwn_patch_opts* opts, void* stream,
                             gwn_patches* out) {
    gwn::clear_error();
    if (!out || npatch < 0 || (npatch > 0 && !cps) || npatch > (1ll << 24)) {
        set_error("gwn_patches_build: null argument or npatch outside [0, 2^24]");
        return GWN_E_INVALID;
    }
    *out = nullptr;
    const double tau_rel = opts && opts->tau > 0.0 ? opts->tau : 1e-9;
    const double eps = opts && opts->eps > 0.0 ? opts->eps : 1e-11;
    const int max_depth = opts && opts->max_depth > 0 ? std::min(opts->max_depth, 30) : 30;
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> P((size_t)npatch * 48);
    if (npatch > 0) {
        GWN_HIP_TRY(hipMemcpyAsync(P.data(), cps, sizeof(double) * P.size(), hipMemcpyDeviceToHost, st));
        GWN_HIP_TRY(hipStreamSynchronize(st));
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    std::vector<double> boxes((size_t)npatch * 8);
    for (int64_t k = 0; k < npatch; ++k) {
        double* b = &boxes[8 * k];
        for (int c = 0; c < 3; ++c) {
            b[c] = 1e300;
            b[3 + c] = -1e300;
        }
        for (int j = 0; j < 16; ++j)
            for (int c = 0; c < 3; ++c) {
                const double v = P[48 * k + 3 * j + c];
                if (!std::isfinite(v)) {
                    set_error("gwn_patches_build: non-finite control point in patch %lld", (long long)k);
                    return GWN_E_INVALID;
                }
                b[c] = std::min(b[c], v);
                b[3 + c] = std::max(b[3 + c], v);
            }
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], b[c]);
            hi[c] = std::max(hi[c], b[3 + c]);
        }
    }
    // boundary: net multiplicity of each curve against its reverse
    std::map<gwn::CurveKey, long long> net;
    std::map<gwn::CurveKey, std::vector<double>> first;
    for (int64_t k = 0; k < npatch; ++k) {
        double cv[4][12];
        gwn::patch_curves(&P[48 * k], cv);
        for (int e = 0; e < 4; ++e) {
            const gwn::CurveKey f = gwn::key_of(cv[e], false), r = gwn::key_of(cv[e], true);
            auto it = net.find(r);
            if (it != net.end()) {
                it->second -= 1;
            } else {
                net[f] += 1;
                if (!first.count(f)) first[f] = std::vector<double>(cv[e], cv[e] + 12);
            }
        }
    }
    std::vector<double> curves;
    for (const auto& kv : net) {
        const std::vector<double>& c = first[kv.first];
        for (long long m = 0; m < std::llabs(kv.second); ++m)
            for (int i = 0; i < 4; ++i) {
                const int src = kv.second > 0 ? i : 3 - i;
                for (int x = 0; x < 3; ++x) curves.push_back(c[3 * src + x]);
            }
    }
    gwn_patches_s* h = new (std::nothrow) gwn_patches_s();
    if (!h) return GWN_E_OOM;
    GWN_HIP_TRY(hipGetDevice(&h->device));
    h->npatch = npatch;
    h->ncurves = (int64_t)(curves.size() / 12);
    double diag = 0.0;
    if (npatch > 0)
        diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                         (hi[2] - lo[2]) * (hi[2] - lo[2]));
    h->diag = diag;
    h->tau = tau_rel * std::max(diag, 1e-300);
    // first level worth the flatness test: the control net's distance from the
    // bilinear patch through its corners falls about 4x per subdivision level
    for (int64_t k = 0; k < npatch; ++k) {
        const double* Pk = &P[48 * k];
        double dev = 0.0;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                const double u = i / 3.0, v = j / 3.0;
                double e2 = 0.0;
                for (int c = 0; c < 3; ++c) {
                    const double b = (1.0 - u) * ((1.0 - v) * Pk[c] + v * Pk[9 + c]) +
                                     u * ((1.0 - v) * Pk[36 + c] + v * Pk[45 + c]);
                    e2 += (Pk[(4 * i + j) * 3 + c] - b) * (Pk[(4 * i + j) * 3 + c] - b);
                }
                dev = std::max(dev, std::sqrt(e2));
            }
        int lv = 0;
        if (dev > h->tau) lv = std::max(0, (int)std::floor(std::log(dev / h->tau) / std::log(4.0)) - 1);
        boxes[8 * k + 6] = (double)std::min(lv, 28);
        boxes[8 * k + 7] = 0.0;
    }
    h->eps = eps;
    h->max_depth = max_depth;
    auto up = [&](double** dst, const std::vector<double>& src) -> hipError_t {
        hipError_t e = gwn::dmalloc((void**)dst, sizeof(double) * std::max<size_t>(1, src.size()));
        if (e == hipSuccess && !src.empty())
            e = hipMemcpyAsync(*dst, src.data(), sizeof(double) * src.size(), hipMemcpyHostToDevice, st);
        return e;
    };
    hipError_t e = up(&h->patches, P);
    if (e == hipSuccess) e = up(&h->boxes, boxes);
    if (e == hipSuccess) e = up(&h->curves, curves);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(h->patches);
        (void)hipFree(h->boxes);
        (void)hipFree(h->curves);
        delete h;
        set_error("gwn_patches_build: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? GWN_E_OOM : GWN_E_HIP;
    }
    *out = h;
    return GWN_OK;
}

gwn_status gwn_patches_info_get(gwn_patches h, gwn_patches_info* out) {
    gwn::clear_error();
    if (!h || !out) {
        set_error("gwn_patches_info_get: null argument");
        return GWN_E_INVALID;
    }
    out->npatch = h->npatch;
    out->ncurves = h->ncurves;
    out->tau = h->tau;
    out->eps = h->eps;
    out->max_depth = h->max_depth;
    out->diag = h->diag;
    return GWN_OK;
}

gwn_status gwn_patches_query(gwn_patches h, const float* qx, const float* qy, const float* qz, int64_t qstride,
                             int64_t nq, double* w_out, int32_t* chi_out, int32_t* dir_out, void* stream) {
    gwn::clear_error();
    if (!h || nq < 0 || qstride < 1 || nq > (1ll << 40) || (nq > 0 && (!qx || !qy || !qz || !w_out))) {
        set_error("gwn_patches_query: null argument, nq < 0 or qstride < 1");
        return GWN_E_INVALID;
    }
    int dev = -1;
    GWN_HIP_TRY(hipGetDevice(&dev));
    if (dev != h->device) {
        set_error("gwn_patches_query: the patches were built on device %d, the current device is %d", h->device, dev);
        return GWN_E_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    const long long chunk = 1ll << 30;   // queries (workgroups of kParamWaves) per launch
    int *chi = nullptr, *dir = nullptr;
    hipError_t e = hipSuccess;
    if (!chi_out) e = gwn::dmalloc_async((void**)&chi, sizeof(int) * (size_t)std::min<long long>(std::max<long long>(nq, 1), chunk), st);
    if (e == hipSuccess && !dir_out)
        e = gwn::dmalloc_async((void**)&dir, sizeof(int) * (size_t)std::min<long long>(std::max<long long>(nq, 1), chunk), st);
    for (long long o = 0; o < nq && e == hipSuccess; o += chunk) {
        const long long n = std::min<long long>(chunk, nq - o);
        e = gwn::launch_param<false>(h, qx + o * qstride, qy + o * qstride, qz + o * qstride, qstride, n, w_out + o,
                                     chi_out ? chi_out + o : chi, dir_out ? dir_out + o : dir, nullptr, st);
    }
    if (chi) (void)hipFreeAsync(chi, st);
    if (dir) (void)hipFreeAsync(dir, st);
    GWN_HIP_TRY(e);
    return GWN_OK;
}

gwn_status gwn_patches_query_grid(gwn_patches h, const double* origin, const double* spacing, const int64_t* dims,
                                  double* w_out, int32_t* chi_out, int32_t* dir_out, int64_t* counts,
                                  void* stream) {
    gwn::clear_error();
    if (!h || !origin || !spacing || !dims || dims[0] < 0 || dims[1] < 0 || dims[2] < 0) {
        set_error("gwn_patches_query_grid: null argument or negative size");
        return GWN_E_INVALID;
    }
    const long long nx = dims[0], ny = dims[1], nz = dims[2];
    if (nx == 0 || ny == 0 || nz == 0) return GWN_OK;
    if (!w_out || nx > (1ll << 20) || ny > (1ll << 20) || nz > (1ll << 30) || nx * ny > (1ll << 30) ||
        (double)nx * (double)ny * (double)nz > 0x1p36) {
        set_error("gwn_patches_query_grid: null output or grid too large (at most 2^30 columns and 2^36 points)");
        return GWN_E_INVALID;
    }
    int dev = -1;
    GWN_HIP_TRY(hipGetDevice(&dev));
    if (dev != h->device) {
        set_error("gwn_patches_query_grid: the patches were built on device %d, the current device is %d", h->device,
                  dev);
        return GWN_E_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    const long long n = nx * ny * nz;
    if (n > (1ll << 30)) {
        set_error("gwn_patches_query_grid: at most 2^30 points per call");
        return GWN_E_INVALID;
    }
    int *chi = chi_out, *dir = dir_out;
    unsigned long long* d = nullptr;
    unsigned long long hc[2] = {0, 0};
    hipError_t e = hipSuccess;
    if (!chi) e = gwn::dmalloc_async((void**)&chi, sizeof(int) * (size_t)n, st);
    if (e == hipSuccess && !dir) e = gwn::dmalloc_async((void**)&dir, sizeof(int) * (size_t)n, st);
    if (e == hipSuccess && counts) e = gwn::dmalloc_async((void**)&d, sizeof hc, st);
    if (e == hipSuccess && counts) e = hipMemcpyAsync(d, hc, sizeof hc, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        gwn::GridPts g;
        for (int c = 0; c < 3; ++c) {
            g.o[c] = origin[c];
            g.s[c] = spacing[c];
        }
        g.ny = ny;
        g.nz = nz;
        e = counts ? gwn::launch_param_grid<true>(h, g, nx, w_out, chi, dir, d, st)
                   : gwn::launch_param_grid<false>(h, g, nx, w_out, chi, dir, nullptr, st);
    }
    if (e == hipSuccess && counts) e = hipMemcpyAsync(hc, d, sizeof hc, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && counts) e = hipStreamSynchronize(st);
    if (!chi_out && chi) (void)hipFreeAsync(chi, st);
    if (!dir_out && dir) (void)hipFreeAsync(dir, st);
    if (d) (void)hipFreeAsync(d, st);
    GWN_HIP_TRY(e);
    if (counts) {
        counts[0] = (int64_t)hc[0];
        counts[1] = (int64_t)hc[1];
    }
    return GWN_OK;
}

gwn_status gwn_patches_query_stats(gwn_patches h, const float* qx, const float* qy, const float* qz,
                                   int64_t qstride, int64_t nq, double* w_out, int64_t* counts, void* stream) {
    gwn::clear_error();
    if (!h || !counts || nq < 0 || qstride < 1 || nq > (1ll << 30) || (nq > 0 && (!qx || !qy || !qz || !w_out))) {
        set_error("gwn_patches_query_stats: null argument, nq outside [0, 2^30] or qstride < 1");
        return GWN_E_INVALID;
    }
    int dev = -1;
    GWN_HIP_TRY(hipGetDevice(&dev));
    if (dev != h->device) {
        set_error("gwn_patches_query_stats: the patches were built on device %d, the current device is %d", h->device,
                  dev);
        return GWN_E_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    unsigned long long* d = nullptr;
    GWN_HIP_TRY(gwn::dmalloc((void**)&d, 2 * sizeof(unsigned long long)));
    unsigned long long hc[2] = {0, 0};
    int* cd = nullptr;
    hipError_t e = hipMemcpyAsync(d, hc, sizeof hc, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = gwn::dmalloc_async((void**)&cd, sizeof(int) * 2 * (size_t)std::max<long long>(nq, 1), st);
    if (e == hipSuccess && nq > 0)
        e = gwn::launch_param<true>(h, qx, qy, qz, qstride, nq, w_out, cd, cd + nq, d, st);
    if (cd) (void)hipFreeAsync(cd, st);
    if (e == hipSuccess) e = hipMemcpyAsync(hc, d, sizeof hc, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    GWN_HIP_TRY(e);
    counts[0] = (int64_t)hc[0];
    counts[1] = (int64_t)hc[1];
    return GWN_OK;
}

gwn_status gwn_patches_destroy(gwn_patches h) {
    gwn::clear_error();
    if (!h) return GWN_OK;
    // the side stream's kernel reads the curves: drain it before they go, and
    // let work on the caller's streams finish with the patches too
    if (h->side) (void)hipStreamSynchronize(h->side);
    (void)hipDeviceSynchronize();
    (void)hipFree(h->patches);
    (void)hipFree(h->boxes);
    (void)hipFree(h->curves);
    if (h->side) {
        (void)hipStreamDestroy(h->side);
        (void)hipEventDestroy(h->fork);
        (void)hipEventDestroy(h->join);
    }
    delete h;
    return GWN_OK;
}

}  // extern "C"
