// gwn_kernels.h -- device routines of the query path shared by the single-mesh
// kernels (query.hip) and the persistent multi-mesh kernel (multi.hip).
//
// Boundary term of the antipodal method (Eq. 10, Alg. 1):
//
//   w(p) = chi(+z) + (1/2pi) * sum over boundary edges (a,b) of atan2(N, D)
//
// where, with r = v - p, rho^2 = r_x^2 + r_y^2, l = |r| and
// s = l - r_z = rho^2 / (l + r_z) (the second form for r_z > 0),
//
//   N = r_a,y r_b,x - r_a,x r_b,y          (= l_a l_b  A . (B x x1))
//   D = s_a s_b + r_a,x r_b,x + r_a,y r_b,y (= l_a l_b (1 + A.B + A.x1 + B.x1))
//
// for x1 = -z.  Scaling both atan2 arguments by l_a l_b > 0 and writing D
// through s (an exact algebraic rearrangement) keeps FP32 accurate when a
// boundary vertex is close to the ray above the query.  Offsets are in
// fixed-point cell units: x and y from the quantised grid (exact integers),
// z from the input scaled by 2^k.  The atan2 branch where an edge passes over
// the ray (D <= 0) takes the sign of N from the exact perturbed predicate
// that also decides ray crossings (Supp. Sec. 2.1), so the integer jumps of
// chi and of the boundary sum coincide.
#pragma once

#include <cmath>
#include <type_traits>

#include "gwn_internal.h"

namespace gwn {
namespace {

constexpr double kInv2Pi = 0.15915494309189533576888376337251;  // 1 / (2 pi)
constexpr double k2Pi = 6.283185307179586476925286766559;         // 2 pi

// atan(t) for |t| <= 1 as t + t x Q(x), x = t^2, Q of degree 7 fitted by the
// Remez exchange for minimax relative error (gen_atan_poly.py: 1.7e-8 in exact
// arithmetic, 9.2e-8 max / 2e-9 mean signed when evaluated in float32).
constexpr float kAtanQ[8] = {0.002920693f, -0.01636793f, 0.043211866f, -0.07552215f,
                             0.106660046f, -0.14211056f, 0.19993773f, -0.33333153f};
// atan(t) for |t| <= tan(pi/8) in double: Q of degree 9 interpolated at the
// Chebyshev nodes of [0, tan^2(pi/8)] (gen_atan_poly.py 9 double: |Q - h| <=
// 1e-15, relative error of atan <= 2e-16).
constexpr double kAtanQd[10] = {0.02277211404923737,  -0.044850509519182694, 0.05736903901999104,
                                -0.06649717364503759, 0.0769106629901103,    -0.09090853283150221,
                                0.11111109664858296,  -0.14285714266729652,  0.19999999999905727,
                                -0.33333333333333276};
// For |t| <= tan(pi/8) (the edge-pair path) atan(t) = t P(t^2), P of degree 4
// fitted to atan(sqrt x)/sqrt x by the Remez exchange (gen_atan_poly.py 4 pform:
// 1.8e-8 relative in exact arithmetic, 1.2e-7 max when evaluated in float32),
// so that a pair's arctangent accumulates in its final FMA.
constexpr float kAtanP[5] = {0.07986737f, -0.13852088f, 0.1997447f, -0.33332798f, 1.0f};
constexpr float kPi = 3.14159265358979f;
constexpr float kPi2 = 1.57079632679490f;

__device__ __forceinline__ float atan_unit(float t) {
    const float x = t * t;
    float q = kAtanQ[0];
#pragma unroll
    for (int k = 1; k < 8; ++k) q = fmaf(q, x, kAtanQ[k]);
    return fmaf(t * x, q, t);
}

// acc + atan(t) for |t| <= tan(pi/8) as fma(t, P(t^2), acc)
__device__ __forceinline__ float atan_pair_acc(float t, float acc) {
    const float x = t * t;
    float p = kAtanP[0];
#pragma unroll
    for (int k = 1; k < 5; ++k) p = fmaf(p, x, kAtanP[k]);
    return fmaf(t, p, acc);
}

// full-range atan2 built on atan_unit (octant reduction by min/max)
__device__ __forceinline__ float atan2_full(float y, float x) {
    const float ay = fabsf(y), ax = fabsf(x);
    const float mx = fmaxf(ay, ax), mn = fminf(ay, ax);
    const float t = mx > 0.f ? mn * __builtin_amdgcn_rcpf(mx) : 0.f;
    float a = atan_unit(t);
    a = ay > ax ? kPi2 - a : a;
    a = x < 0.f ? kPi - a : a;
    return copysignf(a, y);
}

// Arithmetic of the boundary loop per type.  kFast bounds |N|/D on the fast
// path (the range of the small-argument arctangent).
template <class T>
struct Arith;

template <>
struct Arith<float> {
    static constexpr float kFast = 1.0f;
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float atan_small(float t) { return atan_unit(t); }
    static __device__ __forceinline__ float atan2(float y, float x) { return atan2_full(y, x); }
};

template <>
struct Arith<double> {
    static constexpr double kFast = 0.41421356237;   // just below tan(pi/8)
    // hardware reciprocal square root, then one coupled Goldschmidt step on
    // (y ~ sqrt x, h ~ 1/(2 sqrt x)) and a final correction: correctly rounded on
    // 2^20 log-uniform arguments in [1e-12, 1e12], about half the cost of the
    // library square root; x = 0 gives 0
    static __device__ __forceinline__ double sqrt(double x) {
        const double r = __builtin_amdgcn_rsq(x);
        const double y0 = x * r, h0 = 0.5 * r;
        const double g = fma(-y0, h0, 0.5);
        const double y = fma(y0, g, y0), h = fma(h0, g, h0);
        const double s = fma(fma(-y, y, x), h, y);
        return x > 0.0 ? s : 0.0;
    }
    // hardware reciprocal refined by two Newton steps
    static __device__ __forceinline__ double rcp(double x) {
        double r = __builtin_amdgcn_rcp(x);
        double e = fma(-x, r, 1.0);
        r = fma(r, e, r);
        e = fma(-x, r, 1.0);
        return fma(r, e, r);
    }
    static __device__ __forceinline__ double atan_small(double t) {
        const double x = t * t;
        double q = kAtanQd[0];
#pragma unroll
        for (int k = 1; k < 10; ++k) q = fma(q, x, kAtanQd[k]);
        return fma(t * x, q, t);
    }
    // where the fast path would apply, its own expression, so that a lane gets
    // the same bits whichever path its wave takes (the FP32 full-range atan2
    // reduces to the same polynomial by construction)
    static __device__ __forceinline__ double atan2(double y, double x) {
        if (x > 0.0 && fabs(y) < kFast * x) return atan_small(y * rcp(x));
        return ::atan2(y, x);
    }
};

// ---------------------------------------------------------------- boundary loop
// x/y quantities of one boundary vertex relative to the query column (shared by
// all samples of a grid column; per lane in the batch kernels).
template <class T>
struct ColV {
    int dx, dy;
    T rx, ry, rho2;
};

// Offsets of a query outside the fixed-point box are taken in units of 2^e
// cells, e >= 0 chosen per query so that they stay below about 2^41: atan2(N, D)
// does not change under a common positive scale of all offsets, and FP32 would
// otherwise overflow N, D and rho^2 for queries ~1e10 mesh sizes away.  f = 2^-e
// scales the boundary vertices (exactly), scf = 2^(k-e) the query.
template <class T>
struct FarScale {
    T scf, f;
};

template <class T>
__device__ __forceinline__ FarScale<T> far_scale(float px, float py, float pz_abs_max, double scale) {
    const double M = fmax(fmax(fabs((double)px), fabs((double)py)), (double)pz_abs_max) * scale;
    const int e = M > 0x1p40 ? ilogb(M) - 40 : 0;
    FarScale<T> s;
    s.scf = (T)ldexp(scale, -e);
    s.f = (T)ldexp(1.0, -e);
    return s;
}

// value of x in lane l (uniform result)
template <class T>
__device__ __forceinline__ T wave_lane(T x, int l) {
    if constexpr (sizeof(T) == 4) {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
    } else {
        const long long v = __double_as_longlong(x);
        const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), l);
        const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    }
}

// Edge pairs.  Inside the fixed-point box two consecutive edges with
// |N| < tan(pi/16) D each (a wave-uniform test) are summed by one arctangent:
// (D1 + i N1)(D2 + i N2) has argument atan(N1/D1) + atan(N2/D2) in
// (-pi/8, pi/8), so its real part is positive and atan(Im/Re) needs no branch
// fix-up and only the short-range polynomial.  Where ZB samples share one
// column's x/y (grids), N1 N2 is the column's and the product costs three
// operations per sample instead of a second reciprocal and arctangent.  FP32
// offsets are in units of 2^16 cells (an exact scale that keeps products of two
// D below 2^68), and D <= 2^-50 of those units takes the single-edge path
// (products stay normal).
template <class T, int ZB, bool FAR>
struct EdgePairs {
    static constexpr bool on = !FAR;
    static constexpr bool f32 = std::is_same<T, float>::value;
    static constexpr float kUnit = on && f32 ? 0x1p-16f : 1.0f;   // cell units per offset unit
    static constexpr float kInvTan = 5.02734f;                     // 1 / tan(pi/16), rounded up
    static constexpr float kMinD = 0x1p-50f;
};

template <class T, int ZB, bool FAR>
__device__ __forceinline__ ColV<T> col_vtx(const BVert& b, int qqx, int qqy, T pxs, T pys, T f) {
    ColV<T> c;
    c.dx = b.qx - qqx;
    c.dy = b.qy - qqy;
    if (FAR) {
        c.rx = fma((T)b.x, f, -pxs);
        c.ry = fma((T)b.y, f, -pys);
    } else {
        c.rx = (T)c.dx * (T)EdgePairs<T, ZB, FAR>::kUnit;
        c.ry = (T)c.dy * (T)EdgePairs<T, ZB, FAR>::kUnit;
    }
    c.rho2 = c.rx * c.rx + c.ry * c.ry;
    return c;
}

// s = l - r_z without cancellation
template <class T>
__device__ __forceinline__ T samp_s(T rho2, T rz) {
    const T l = Arith<T>::sqrt(rz * rz + rho2);
    const T t = l + fabs(rz);
    return rz > (T)0 ? rho2 * Arith<T>::rcp(t) : t;
}

// Rare path of one (sample, edge): exact atan2 branch where D <= 0 (sign of N from
// the perturbed predicate, or the perturbation limit for an endpoint on the ray),
// then the full-range atan2.  An endpoint on the sample's vertical line
// (dx = dy = 0, so rho = 0 exactly) lies on the ray above it exactly when its
// s = rho^2 / (l + r_z) is 0 (below it s = 2 |r_z| > 0); s = 0 with r_z = 0 is a
// vertex at the sample itself, on the surface, where w is undefined.
template <class T>
__device__ __forceinline__ T edge_slow(const ColV<T>& a, const ColV<T>& b, T sa, T sb, T N, T D, bool exact) {
    if (exact && D <= (T)0) {
        const bool aon = (a.dx == 0) & (a.dy == 0) & (sa == (T)0);
        const bool bon = (b.dx == 0) & (b.dy == 0) & (sb == (T)0);
        if (aon && bon) {
            N = (T)0;
            D = (T)1;
        } else if (aon) {        // N ~ e1 rb_y - e2 rb_x,  D ~ -e1 rb_x - e2 rb_y
            if (b.ry != (T)0) { N = b.ry; D = -b.rx; }
            else if (b.rx > (T)0) { N = -(T)0; D = (T)-1; }
            else { N = (T)0; D = (T)1; }
        } else if (bon) {        // N ~ -e1 ra_y + e2 ra_x, D ~ -e1 ra_x - e2 ra_y
            if (a.ry != (T)0) { N = -a.ry; D = -a.rx; }
            else if (a.rx > (T)0) { N = (T)0; D = (T)-1; }
            else { N = (T)0; D = (T)1; }
        } else {
            const int o = orient_sos(a.dx, a.dy, b.dx, b.dy);   // N = -orient2d(a, b, q_eps)
            if (o > 0) N = -fabs(N);
            else if (o < 0) N = fabs(N);
        }
    }
    return Arith<T>::atan2(N, D);
}

// One boundary edge for ZB samples given N and D.  Fast path (wave-uniform):
// every sample has |N| < kFast D, so atan2(N, D) = atan(N/D) with no branch
// fix-up.
template <class T, int ZB, bool FAR>
__device__ __forceinline__ void edge_finish(const ColV<T>& a, const ColV<T>& b, const T* sa, const T* sb, T N,
                                            const T* D, T* acc) {
    const T aN = fabs(N);
    bool slow = false;
#pragma unroll
    for (int r = 0; r < ZB; ++r) slow |= !(aN < Arith<T>::kFast * D[r]);
    if (__builtin_amdgcn_ballot_w64(slow) == 0ull) {
#pragma unroll
        for (int r = 0; r < ZB; ++r) acc[r] += Arith<T>::atan_small(N * Arith<T>::rcp(D[r]));
    } else {
#pragma unroll
        for (int r = 0; r < ZB; ++r) acc[r] += edge_slow<T>(a, b, sa[r], sb[r], N, D[r], !FAR);
    }
}

template <class T, int ZB, bool FAR>
__device__ __forceinline__ void edge_step(const ColV<T>& a, const ColV<T>& b, const T* sa, const T* sb, T* acc) {
    const T N = a.ry * b.rx - a.rx * b.ry;
    const T dot = a.rx * b.rx + a.ry * b.ry;
    T D[ZB];
#pragma unroll
    for (int r = 0; r < ZB; ++r) D[r] = sa[r] * sb[r] + dot;
    edge_finish<T, ZB, FAR>(a, b, sa, sb, N, D, acc);
}

// Inside the box x and y are within 2^31 cells of every boundary vertex but z
// is not bounded: a sample more than 2^40 cells above or below the box takes
// single edges (its offsets may even be infinite in FP32, which the single-edge
// form turns into the right limit), so an edge pair's product stays below 2^101
// in its units.
__device__ __forceinline__ bool near_z(float pz, const QGrid& g) {
    return fabs(((double)pz - g.lo[2]) * g.scale) <= 0x1p40;
}

// Edges a -> b -> c for ZB samples: as one pair where allowed, else one by one.
// Each lane chooses for its own point, so a point's result does not depend on
// which points share its wave (the single-edge fast and exact forms agree bit
// for bit where |N| < D, so their wave-uniform choice never mattered).
template <class T, int ZB, bool FAR>
__device__ __forceinline__ void edge_pair(const ColV<T>& a, const ColV<T>& b, const ColV<T>& c, const T* sa,
                                          const T* sb, const T* sc, T* acc,
                                          bool pairs) {
    using P = EdgePairs<T, ZB, FAR>;
    if constexpr (!P::on) {
        edge_step<T, ZB, FAR>(a, b, sa, sb, acc);
        edge_step<T, ZB, FAR>(b, c, sb, sc, acc);
    } else {
        const T N1 = a.ry * b.rx - a.rx * b.ry, dot1 = a.rx * b.rx + a.ry * b.ry;
        const T N2 = b.ry * c.rx - b.rx * c.ry, dot2 = b.rx * c.rx + b.ry * c.ry;
        const T m1 = fmax(fabs(N1) * (T)P::kInvTan, (T)P::kMinD);
        const T m2 = fmax(fabs(N2) * (T)P::kInvTan, (T)P::kMinD);
        T D1[ZB], D2[ZB];
#pragma unroll
        for (int r = 0; r < ZB; ++r) {
            D1[r] = fma(sa[r], sb[r], dot1);
            D2[r] = fma(sb[r], sc[r], dot2);
        }
        bool slow = !pairs;
#pragma unroll
        for (int r = 0; r < ZB; ++r) slow |= !(m1 < D1[r]) | !(m2 < D2[r]);
        if (!slow) {
            const T N12 = N1 * N2;
#pragma unroll
            for (int r = 0; r < ZB; ++r) {
                const T re = fma(D1[r], D2[r], -N12);
                const T im = fma(D1[r], N2, N1 * D2[r]);
                const T t = im * Arith<T>::rcp(re);
                if constexpr (P::f32) acc[r] = atan_pair_acc(t, acc[r]);
                else acc[r] += Arith<T>::atan_small(t);   // |t| < tan(pi/8)
            }
        } else {
            edge_finish<T, ZB, FAR>(a, b, sa, sb, N1, D1, acc);
            edge_finish<T, ZB, FAR>(b, c, sb, sc, N2, D2, acc);
        }
    }
}

// s per block given R, the number of blocks with a sample below the vertex
// (r_z > 0).  With z ascending in r (and in the lane) blocks 0..R-2 lie wholly
// below the vertex (s = rho^2 / t, no select), block R-1 may straddle it (the
// two-sided form) and blocks R.. lie wholly at or above it (s = t).  R > ZB:
// no order known, the two-sided form everywhere.
//
// FARV: every sample below the vertex has r_z^2 <= 3 rho^2.  There
// s = l - r_z = t - 2 max(r_z, 0) loses at most ~16 ulps to cancellation (its
// rounding error is ~2 u l, and s = rho^2 / (l + r_z) >= l / 8 there), so the
// blocks take it without the reciprocal.
template <class T, int ZB, int R, bool FARV>
__device__ __forceinline__ void s_blocks(const T* rz, T rho2, T* sv) {
#pragma unroll
    for (int r = 0; r < ZB; ++r) {   // sv holds t = l + |r_z| on entry
        if (FARV && R <= ZB) {
            if (r < R - 1) sv[r] = fma((T)-2, rz[r], sv[r]);
            else if (r == R - 1) sv[r] = fma((T)-2, fmax(rz[r], (T)0), sv[r]);
        } else if (R > ZB || r == R - 1) {
            sv[r] = rz[r] > (T)0 ? rho2 * Arith<T>::rcp(sv[r]) : sv[r];
        } else if (r < R - 1) {
            sv[r] = rho2 * Arith<T>::rcp(sv[r]);
        }
    }
}

// R as above; farv: the FARV case (wave-uniform)
template <class T, int ZB>
__device__ __forceinline__ void s_prefix(int R, const T* rz, T rho2, T* sv, bool farv = false) {
#define GWN_S_CASE(K)                                                                          \
    case K:                                                                                    \
        if (farv) s_blocks<T, ZB, (K <= ZB ? K : ZB + 1), true>(rz, rho2, sv);                 \
        else s_blocks<T, ZB, (K <= ZB ? K : ZB + 1), false>(rz, rho2, sv);                     \
        break;
    switch (R) {
        case 0: break;
        GWN_S_CASE(1)
        GWN_S_CASE(2)
        GWN_S_CASE(3)
        GWN_S_CASE(4)
        GWN_S_CASE(5)
        GWN_S_CASE(6)
        GWN_S_CASE(7)
        GWN_S_CASE(8)
        default: s_blocks<T, ZB, ZB + 1, false>(rz, rho2, sv); break;
    }
#undef GWN_S_CASE
}

// Sample blocks.  Where the samples of a grid wave share a column, register r
// is a block of 64 consecutive samples and bminr[r] (the same in every lane)
// holds the block's smallest z.  A vertex at or below every sample of a block
// (r_z <= 0 in all its lanes) has s = l + |r_z| there with no reciprocal;
// fma(z, u, -bminr[r]) > 0 is exactly "some lane of block r has r_z > 0" (r_z
// is the same fma and falls as the sample's z rises).  When every block
// ascends in the lane and the blocks' smallest z do not fall with r (asc) the
// samples ascend through the whole column, so the blocks needing the
// reciprocal are a prefix, all but its last wholly below the vertex (their
// largest z is at most the next block's smallest).

// pzs: the samples' z in offset units (cells times EdgePairs' kUnit inside the box)
template <class T, int ZB, bool FAR>
__device__ __forceinline__ void load_vertex(const BVert& b, int qqx, int qqy, T pxs, T pys, const T* pzs, T f,
                                            ColV<T>& c, T* sv) {
    c = col_vtx<T, ZB, FAR>(b, qqx, qqy, pxs, pys, f);
    constexpr T u = (T)EdgePairs<T, ZB, FAR>::kUnit;
#pragma unroll
    for (int r = 0; r < ZB; ++r) {
        const T rz = FAR ? fma((T)b.z, f, -pzs[r]) : (u == (T)1 ? (T)b.z - pzs[r] : fma((T)b.z, u, -pzs[r]));
        sv[r] = samp_s<T>(c.rho2, rz);
    }
}

// Boundary sum S = sum of atan2 over the chained loops for ZB samples sharing one
// (x, y).  FP32 partials are flushed into the FP64 sum every 32 edges.  pzs in
// cells inside the box (FAR: in units of 2^e cells).  pairs: this lane's
// samples may take edge pairs (see near_z).  (Grid columns use column_loops.)
template <class T, int ZB, bool FAR>
__device__ __forceinline__ void boundary_loops(const MeshView& mv, int qqx, int qqy, T pxs, T pys, const T* pzs,
                                               double* S, T f = (T)1, bool pairs = true) {
    const BVert* __restrict__ bv = mv.bverts;
    T pz[ZB];
#pragma unroll
    for (int r = 0; r < ZB; ++r) pz[r] = FAR ? pzs[r] : pzs[r] * (T)EdgePairs<T, ZB, FAR>::kUnit;
    for (int l = 0; l < mv.nloops; ++l) {
        const int b0 = mv.loop_off[l], b1 = mv.loop_off[l + 1];
        ColV<T> cf, cp, cq, cr;
        T sf[ZB], sp[ZB], sq[ZB], sr[ZB];
        load_vertex<T, ZB, FAR>(bv[b0], qqx, qqy, pxs, pys, pz, f, cf, sf);
        cp = cf;
#pragma unroll
        for (int r = 0; r < ZB; ++r) {
            sp[r] = sf[r];
        }
        int j = b0 + 1;
        while (j < b1) {
            const int je = min(b1, j + 32);
            T acc[ZB];
#pragma unroll
            for (int r = 0; r < ZB; ++r) acc[r] = (T)0;
            // four vertices (two edge pairs) per trip: p-q-r, then r-q-p with q and p
            // reloaded, so the loop-carried vertex ends in the set it started in
            for (; j + 3 < je; j += 4) {
                load_vertex<T, ZB, FAR>(bv[j], qqx, qqy, pxs, pys, pz, f, cq, sq);
                load_vertex<T, ZB, FAR>(bv[j + 1], qqx, qqy, pxs, pys, pz, f, cr, sr);
                edge_pair<T, ZB, FAR>(cp, cq, cr, sp, sq, sr, acc, pairs);
                load_vertex<T, ZB, FAR>(bv[j + 2], qqx, qqy, pxs, pys, pz, f, cq, sq);
                load_vertex<T, ZB, FAR>(bv[j + 3], qqx, qqy, pxs, pys, pz, f, cp, sp);
                edge_pair<T, ZB, FAR>(cr, cq, cp, sr, sq, sp, acc, pairs);
            }
            if (j + 1 < je) {
                load_vertex<T, ZB, FAR>(bv[j], qqx, qqy, pxs, pys, pz, f, cq, sq);
                load_vertex<T, ZB, FAR>(bv[j + 1], qqx, qqy, pxs, pys, pz, f, cr, sr);
                edge_pair<T, ZB, FAR>(cp, cq, cr, sp, sq, sr, acc, pairs);
                cp = cr;
#pragma unroll
                for (int r = 0; r < ZB; ++r) {
                    sp[r] = sr[r];
                }
                j += 2;
            }
            if (j < je) {
                load_vertex<T, ZB, FAR>(bv[j], qqx, qqy, pxs, pys, pz, f, cq, sq);
                edge_step<T, ZB, FAR>(cp, cq, sp, sq, acc);
                cp = cq;
#pragma unroll
                for (int r = 0; r < ZB; ++r) {
                    sp[r] = sq[r];
                }
                ++j;
            }
#pragma unroll
            for (int r = 0; r < ZB; ++r) S[r] += (double)acc[r];
        }
        T acc[ZB];
#pragma unroll
        for (int r = 0; r < ZB; ++r) acc[r] = (T)0;
        edge_step<T, ZB, FAR>(cp, cf, sp, sf, acc);
#pragma unroll
        for (int r = 0; r < ZB; ++r) S[r] += (double)acc[r];
    }
}

// ---------------------------------------------------------------- grid columns
// In a grid column every sample shares x and y, so a boundary vertex's x/y
// terms (rho^2, and N, the x/y dot and the pair bound of its outgoing edge) are
// the same for the whole wave.  They are computed for 64 boundary vertices at a
// time, one vertex per lane, into a ring of records in LDS that every lane then
// reads at the same address (a broadcast): a wave instruction's worth of x/y
// work per vertex becomes one lane's.  The same pass counts each vertex's
// blocks with a sample below it (R, see the sample blocks note), and whether its outgoing
// edge pairs on its x/y terms alone becomes a bit of a wave mask.
template <class T>
struct alignas(4 * sizeof(T)) ColRec {
    T zu;     // vertex z in offset units
    T rho2;   // r_x^2 + r_y^2 from the column
    T N;      // N of the outgoing edge (to the next vertex of the loop)
    T dot;    // r_a,x r_b,x + r_a,y r_b,y of the outgoing edge
};

template <class T>
struct ColAux {   // read on the rare paths only
    T m;          // pair bound of the outgoing edge, max(|N| / tan(pi/16), kMinD)
    T rx, ry;
    int dx, dy;
};

constexpr int kColRing = 128;   // slots per wave; slot kColRing holds the loop's first vertex

template <class T>
struct ColRing {
    ColRec<T> rec[kColRing + 1];
    ColAux<T> aux[kColRing + 1];
    int R[kColRing + 1];   // block count R of the vertex, plus 256 in the FARV case (see the sample blocks note, s_blocks)
};

// Records of vertices v0 .. v0 + n - 1 (n <= 64) of the loop [b0, b1), into the
// ring slots (v0 - b0) mod kColRing; v0 - b0 is a multiple of 64, so they fill
// one half.  The first call of a loop (v0 == b0) also keeps its first vertex in
// slot kColRing.  bminr[r]: block r's smallest z in offset units (see the sample blocks note).
// Bit k of mk: the edge leaving the half's slot k pairs on its x/y terms alone.
template <class T, int ZB>
__device__ __forceinline__ void col_fill(const MeshView& mv, int v0, int n, int b0, int b1, int qqx, int qqy,
                                         const T* bminr, bool asc, bool pairs, ColRing<T>& ring,
                                         unsigned long long& mk) {
    using P = EdgePairs<T, ZB, false>;
    constexpr T u = (T)P::kUnit;
    int lane = (int)(threadIdx.x & 63);
    // Opaque to the optimiser (no instruction is emitted): the ring addresses
    // derived from the lane are then formed here, once per fill, instead of
    // being hoisted out of the boundary loops and held (or spilled) throughout.
    asm volatile("" : "+v"(lane));
    bool e = false;
    int R = 0;
    if (lane < n) {
        const int v = v0 + lane;
        const int vn = v + 1 < b1 ? v + 1 : b0;
        const BVert a = mv.bverts[v], b = mv.bverts[vn];
        const ColV<T> ca = col_vtx<T, ZB, false>(a, qqx, qqy, (T)0, (T)0, (T)1);
        const ColV<T> cb = col_vtx<T, ZB, false>(b, qqx, qqy, (T)0, (T)0, (T)1);
        ColRec<T> rc;
        rc.zu = u == (T)1 ? (T)a.z : (T)a.z * u;   // exact (u is a power of two)
        rc.rho2 = ca.rho2;
        rc.N = ca.ry * cb.rx - ca.rx * cb.ry;
        rc.dot = ca.rx * cb.rx + ca.ry * cb.ry;
        ColAux<T> ax;
        ax.m = fmax(fabs(rc.N) * (T)P::kInvTan, (T)P::kMinD);
        ax.rx = ca.rx;
        ax.ry = ca.ry;
        ax.dx = ca.dx;
        ax.dy = ca.dy;
        if (asc) {
            bool farv = true;   // every sample below the vertex has r_z^2 <= 3 rho^2
#pragma unroll
            for (int r = 0; r < ZB; ++r) {
                const T zr = u == (T)1 ? (T)a.z - bminr[r] : fma((T)a.z, u, -bminr[r]);
                R += zr > (T)0;
                farv &= !((zr > (T)0) & (zr * zr > (T)3 * rc.rho2));   // zr: the block's largest r_z
            }
            R |= farv ? 256 : 0;
        } else {
            R = ZB + 1;
        }
        e = ax.m < rc.dot;
        const int s = (v - b0) & (kColRing - 1);
        ring.rec[s] = rc;
        ring.aux[s] = ax;
        ring.R[s] = R;
        if (v == b0) {
            ring.rec[kColRing] = rc;
            ring.aux[kColRing] = ax;
            ring.R[kColRing] = R;
        }
    }
    mk = __builtin_amdgcn_ballot_w64(e && pairs);
    // the wave reads what its own lanes wrote; LDS operations of a wave complete in order
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bool col_e(unsigned long long m0, unsigned long long m1, int k) {
    return (((k & 64) ? m1 : m0) >> (k & 63)) & 1ull;
}

template <class T>
__device__ __forceinline__ int ring_R(const ColRing<T>& ring, int k) {
    return __builtin_amdgcn_readfirstlane(ring.R[k]);
}

// s of the vertex in slot k for the lane's ZB samples (pz in offset units),
// and its outgoing edge's N and x/y dot
template <class T, int ZB>
__device__ __forceinline__ void col_vertex(const ColRec<T>& c, int R, const T* pz, T* sv, T& N, T& dot) {
    T rz[ZB];
#pragma unroll
    for (int r = 0; r < ZB; ++r) {
        rz[r] = c.zu - pz[r];
        sv[r] = Arith<T>::sqrt(rz[r] * rz[r] + c.rho2) + fabs(rz[r]);   // t, made s in place
    }
    s_prefix<T, ZB>(R & 0xff, rz, c.rho2, sv, R >= 256);
    N = c.N;
    dot = c.dot;
}

template <class T>
__device__ __forceinline__ ColV<T> col_aux(const ColRing<T>& ring, int k) {
    const ColAux<T> a = ring.aux[k];
    ColV<T> c;
    c.dx = a.dx;
    c.dy = a.dy;
    c.rx = a.rx;
    c.ry = a.ry;
    c.rho2 = (T)0;   // not used by edge_slow
    return c;
}

// One edge (slot ka to slot kb) given its D per sample: the fast form where
// every sample allows it, else the exact and full-range forms (edge_slow).
template <class T, int ZB>
__device__ __forceinline__ void col_finish(const ColRing<T>& ring, int ka, int kb, const T* sa, const T* sb, T N,
                                           const T* D, T* acc) {
    const T aN = fabs(N);
    bool slow = false;
#pragma unroll
    for (int r = 0; r < ZB; ++r) slow |= !(aN < Arith<T>::kFast * D[r]);
    if (__builtin_amdgcn_ballot_w64(slow) == 0ull) {
#pragma unroll
        for (int r = 0; r < ZB; ++r) acc[r] += Arith<T>::atan_small(N * Arith<T>::rcp(D[r]));
    } else {
        const ColV<T> a = col_aux<T>(ring, ka), b = col_aux<T>(ring, kb);
#pragma unroll
        for (int r = 0; r < ZB; ++r) acc[r] += edge_slow<T>(a, b, sa[r], sb[r], N, D[r], true);
    }
}

// Edges slot ka -> kb -> kc: one arctangent for the pair where every sample of
// the wave allows it (decided by the x/y terms alone when ok, else per sample),
// else one by one.
template <class T, int ZB>
__device__ __forceinline__ void col_pair(const ColRing<T>& ring, int ka, int kb, int kc, T N1, T dot1, T N2,
                                         T dot2, bool ok, bool pairs, const T* sa, const T* sb, const T* sc,
                                         T* acc) {
    using P = EdgePairs<T, ZB, false>;
    T D1[ZB], D2[ZB];
#pragma unroll
    for (int r = 0; r < ZB; ++r) {
        D1[r] = fma(sa[r], sb[r], dot1);
        D2[r] = fma(sb[r], sc[r], dot2);
    }
    bool pair = ok;
    if (!ok && pairs) {
        const T m1 = ring.aux[ka].m, m2 = ring.aux[kb].m;
        bool slow = false;
#pragma unroll
        for (int r = 0; r < ZB; ++r) slow |= !(m1 < D1[r]) | !(m2 < D2[r]);
        pair = __builtin_amdgcn_ballot_w64(slow) == 0ull;
    }
    if (pair) {
        const T N12 = N1 * N2;
#pragma unroll
        for (int r = 0; r < ZB; ++r) {
            const T re = fma(D1[r], D2[r], -N12);
            const T im = fma(D1[r], N2, N1 * D2[r]);
            const T t = im * Arith<T>::rcp(re);
            if constexpr (P::f32) acc[r] = atan_pair_acc(t, acc[r]);
            else acc[r] += Arith<T>::atan_small(t);   // |t| < tan(pi/8)
        }
    } else {
        col_finish<T, ZB>(ring, ka, kb, sa, sb, N1, D1, acc);
        col_finish<T, ZB>(ring, kb, kc, sb, sc, N2, D2, acc);
    }
}

// Edges a -> b -> c known to pair on their x/y terms: one arctangent, no test.
template <class T, int ZB>
__device__ __forceinline__ void col_pair_xy(T N1, T dot1, T N2, T dot2, const T* sa, const T* sb, const T* sc,
                                            T* acc) {
    const T N12 = N1 * N2;
#pragma unroll
    for (int r = 0; r < ZB; ++r) {
        const T D1 = fma(sa[r], sb[r], dot1), D2 = fma(sb[r], sc[r], dot2);
        const T re = fma(D1, D2, -N12);
        const T im = fma(D1, N2, N1 * D2);
        const T t = im * Arith<T>::rcp(re);
        if constexpr (EdgePairs<T, ZB, false>::f32) acc[r] = atan_pair_acc(t, acc[r]);
        else acc[r] += Arith<T>::atan_small(t);
    }
}

// single edge slot ka -> kb
template <class T, int ZB>
__device__ __forceinline__ void col_edge(const ColRing<T>& ring, int ka, int kb, T N, T dot, const T* sa,
                                         const T* sb, T* acc) {
    T D[ZB];
#pragma unroll
    for (int r = 0; r < ZB; ++r) D[r] = fma(sa[r], sb[r], dot);
    col_finish<T, ZB>(ring, ka, kb, sa, sb, N, D, acc);
}

// Boundary sum S for the ZB samples of each lane of a grid column inside the
// fixed-point box (qqx, qqy: the column's quantised x, y; pzs: the samples' z in
// cells).  Register r of the wave is a block of 64 consecutive samples, z
// monotone in the lane.  pairs: edge pairs allowed (see near_z).  Same sums as
// boundary_loops, in the same order: FP32 partials flushed to FP64 every 32 edges.
template <class T, int ZB>
__device__ __forceinline__ void column_loops(const MeshView& mv, int qqx, int qqy, const T* pzs, double* S,
                                             bool pairs, ColRing<T>& ring) {
    constexpr T u = (T)EdgePairs<T, ZB, false>::kUnit;
    T pz[ZB];
#pragma unroll
    for (int r = 0; r < ZB; ++r) pz[r] = pzs[r] * u;
    // the samples of a block are monotone in the lane, so its smallest z is in
    // lane 0 or lane 63.  The column ascends (asc) when every block ascends and
    // the blocks' smallest z do not fall: the minima alone do not show it, as a
    // descending column's last block and the blocks of clamped copies of its
    // last sample after it share their smallest z.
    T bminr[ZB];
    bool asc = true;
    T prev = -(T)INFINITY;
#pragma unroll
    for (int r = 0; r < ZB; ++r) {
        const T z0 = wave_lane<T>(pz[r], 0), z63 = wave_lane<T>(pz[r], 63);
        bminr[r] = fmin(z0, z63);
        asc &= !(bminr[r] < prev) & !(z63 < z0);
        prev = bminr[r];
    }
    for (int l = 0; l < mv.nloops; ++l) {
        const int b0 = mv.loop_off[l], nv = mv.loop_off[l + 1] - b0;
        unsigned long long m0, m1;   // pair bits of the ring's two halves
        int done = min(64, nv);
        col_fill<T, ZB>(mv, b0, done, b0, b0 + nv, qqx, qqy, bminr, asc, pairs, ring, m0);
        m1 = m0;
        T sp[ZB], sq[ZB], sr[ZB];
        T Np, dotp, Nq, dotq, Nr, dotr;
        // the first vertex's s is computed again for the closing edge (from its
        // copy in slot kColRing) rather than held in registers through the loop
        const int R0 = ring_R(ring, 0);
        col_vertex<T, ZB>(ring.rec[0], R0, pz, sp, Np, dotp);
        int j = 1;   // vertices are counted from b0; slot of vertex j is j mod kColRing
        while (j < nv) {
            const int je = min(nv, j + 32);
            if (je > done) {   // one fill covers it: j <= done, je <= j + 32
                const int n = min(64, nv - done);
                if (done & 64) col_fill<T, ZB>(mv, b0 + done, n, b0, b0 + nv, qqx, qqy, bminr, asc, pairs, ring, m1);
                else col_fill<T, ZB>(mv, b0 + done, n, b0, b0 + nv, qqx, qqy, bminr, asc, pairs, ring, m0);
                done += n;
            }
            T acc[ZB];
#pragma unroll
            for (int r = 0; r < ZB; ++r) acc[r] = (T)0;
            // four vertices (two edge pairs) per trip: p-q-r, then r-q-p
            while (j + 3 < je) {
                // trips whose four edges all pair on their x/y terms alone
                for (; j + 3 < je && col_e(m0, m1, (j - 1) & (kColRing - 1)) &&
                       col_e(m0, m1, j & (kColRing - 1)) && col_e(m0, m1, (j + 1) & (kColRing - 1)) &&
                       col_e(m0, m1, (j + 2) & (kColRing - 1));
                     j += 4) {
                    const int kq = j & (kColRing - 1), kr = (j + 1) & (kColRing - 1);
                    const int kq2 = (j + 2) & (kColRing - 1), kp2 = (j + 3) & (kColRing - 1);
                    const ColRec<T> cq = ring.rec[kq], cr = ring.rec[kr], cq2 = ring.rec[kq2], cp2 = ring.rec[kp2];
                    col_vertex<T, ZB>(cq, ring_R(ring, kq), pz, sq, Nq, dotq);
                    col_vertex<T, ZB>(cr, ring_R(ring, kr), pz, sr, Nr, dotr);
                    col_pair_xy<T, ZB>(Np, dotp, Nq, dotq, sp, sq, sr, acc);
                    col_vertex<T, ZB>(cq2, ring_R(ring, kq2), pz, sq, Nq, dotq);
                    col_vertex<T, ZB>(cp2, ring_R(ring, kp2), pz, sp, Np, dotp);
                    col_pair_xy<T, ZB>(Nr, dotr, Nq, dotq, sr, sq, sp, acc);
                }
                if (j + 3 >= je) break;
                const int kp = (j - 1) & (kColRing - 1), kq = j & (kColRing - 1);
                const int kr = (j + 1) & (kColRing - 1), kq2 = (j + 2) & (kColRing - 1);
                const int kp2 = (j + 3) & (kColRing - 1);
                // the trip's four records are read up front (LDS latency)
                const ColRec<T> cq = ring.rec[kq], cr = ring.rec[kr], cq2 = ring.rec[kq2], cp2 = ring.rec[kp2];
                col_vertex<T, ZB>(cq, ring_R(ring, kq), pz, sq, Nq, dotq);
                col_vertex<T, ZB>(cr, ring_R(ring, kr), pz, sr, Nr, dotr);
                col_pair<T, ZB>(ring, kp, kq, kr, Np, dotp, Nq, dotq, col_e(m0, m1, kp) & col_e(m0, m1, kq),
                                pairs, sp, sq, sr, acc);
                col_vertex<T, ZB>(cq2, ring_R(ring, kq2), pz, sq, Nq, dotq);
                col_vertex<T, ZB>(cp2, ring_R(ring, kp2), pz, sp, Np, dotp);
                col_pair<T, ZB>(ring, kr, kq2, kp2, Nr, dotr, Nq, dotq,
                                col_e(m0, m1, kr) & col_e(m0, m1, kq2), pairs, sr, sq, sp, acc);
                j += 4;
            }
            if (j + 1 < je) {
                const int kp = (j - 1) & (kColRing - 1), kq = j & (kColRing - 1);
                const int kr = (j + 1) & (kColRing - 1);
                const ColRec<T> cq = ring.rec[kq], cr = ring.rec[kr];
                col_vertex<T, ZB>(cq, ring_R(ring, kq), pz, sq, Nq, dotq);
                col_vertex<T, ZB>(cr, ring_R(ring, kr), pz, sr, Nr, dotr);
                col_pair<T, ZB>(ring, kp, kq, kr, Np, dotp, Nq, dotq, col_e(m0, m1, kp) & col_e(m0, m1, kq),
                                pairs, sp, sq, sr, acc);
                Np = Nr;
                dotp = dotr;
#pragma unroll
                for (int r = 0; r < ZB; ++r) sp[r] = sr[r];
                j += 2;
            }
            if (j < je) {
                const int kp = (j - 1) & (kColRing - 1), kq = j & (kColRing - 1);
                col_vertex<T, ZB>(ring.rec[kq], ring_R(ring, kq), pz, sq, Nq, dotq);
                col_edge<T, ZB>(ring, kp, kq, Np, dotp, sp, sq, acc);
                Np = Nq;
                dotp = dotq;
#pragma unroll
                for (int r = 0; r < ZB; ++r) sp[r] = sq[r];
                ++j;
            }
#pragma unroll
            for (int r = 0; r < ZB; ++r) S[r] += (double)acc[r];
        }
        // closing edge, last vertex -> first (kept in slot kColRing)
        T acc[ZB], sf[ZB], Nf, dotf;
        col_vertex<T, ZB>(ring.rec[kColRing], R0, pz, sf, Nf, dotf);
#pragma unroll
        for (int r = 0; r < ZB; ++r) acc[r] = (T)0;
        col_edge<T, ZB>(ring, (nv - 1) & (kColRing - 1), kColRing, Np, dotp, sp, sf, acc);
#pragma unroll
        for (int r = 0; r < ZB; ++r) S[r] += (double)acc[r];
    }
}

// ---------------------------------------------------------------- grids

constexpr int kGridWaves = 4;  // waves per block in the wave-per-task kernels

// A cell-centred grid in the mesh frame; one wave per (column, z-chunk).
struct GridArgs {
    double o[3], s[3];
    long long nx, ny, nz;
    long long nchunks;   // z-chunks per column
    long long nwaves;    // columns * nchunks
    long long wave0;     // first wave of this launch (large grids take several)
    long long st[3];     // output strides of the frame's x, y, z indices (world z fastest)
};

// The grid in the frame of a mesh built along `axis`: frame axis c is world
// axis (c + axis) % 3; the output keeps the world layout (x slowest, z fastest).
inline GridArgs frame_grid(int axis, const double* origin, const double* spacing, const int64_t* dims) {
    GridArgs ga;
    const long long wst[3] = {dims[1] * dims[2], dims[2], 1};
    long long n[3];
    for (int c = 0; c < 3; ++c) {
        const int a = (c + axis) % 3;
        ga.o[c] = origin[a];
        ga.s[c] = spacing[a];
        n[c] = dims[a];
        ga.st[c] = wst[a];
    }
    ga.nx = n[0];
    ga.ny = n[1];
    ga.nz = n[2];
    ga.nchunks = ga.nwaves = ga.wave0 = 0;
    return ga;
}

// grid coordinate origin + (i + 0.5) * spacing in FP64, the product and the
// sum each rounded (no fused multiply-add: the pragma keeps the compiler from
// contracting them, which near a float32 rounding tie moves the sample by an
// ulp), then rounded to float32
__device__ __forceinline__ float grid_coord(double o, double s, long long i) {
#pragma clang fp contract(off)
    const double t = ((double)i + 0.5) * s;
    return (float)(o + t);
}

// ---------------------------------------------------------------- chi, batch

constexpr int kChiBlock = 64;

__device__ __forceinline__ int leaf_up(const MeshView& mv, int t, const QPoint& q) {
    return ray_up_hit(mv.tris[t], q.x, q.y, q.z);
}

// signed crossings of the +z ray from q: depth-first over the BVH with a
// per-lane stack in LDS (the radix tree over 62-bit keys is at most 63 deep)
__device__ int chi_up(const MeshView& mv, const QPoint& q, int* stk) {
    int node = mv.root;
    if (node == kNoRoot) return 0;
    if (node < 0) return leaf_up(mv, ~node, q);
    int c = 0, sp = 0;
    while (true) {
        const Node nd = mv.nodes[node];
        bool hl = box_has_xy(nd.lxy.x, nd.lxy.y, nd.lxy.z, nd.lxy.w, q.x, q.y) & (q.z <= nd.z.y);
        bool hr = box_has_xy(nd.rxy.x, nd.rxy.y, nd.rxy.z, nd.rxy.w, q.x, q.y) & (q.z <= nd.z.w);
        const int L = nd.link.x, R = nd.link.y;
        if (hl && L < 0) {
            c += leaf_up(mv, ~L, q);
            hl = false;
        }
        if (hr && R < 0) {
            c += leaf_up(mv, ~R, q);
            hr = false;
        }
        if (hl && hr) {
            stk[sp * kChiBlock] = R;
            ++sp;
            node = L;
        } else if (hl) {
            node = L;
        } else if (hr) {
            node = R;
        } else {
            if (sp == 0) break;
            --sp;
            node = stk[sp * kChiBlock];
        }
    }
    return c;
}

// Signed crossings of the whole vertical line through q, split at q: up = the
// sum of s over crossings above q (chi along +z), down = minus the sum over
// crossings below it (chi along -z).  Same traversal as chi_up without the
// z pruning.
__device__ void chi_line(const MeshView& mv, const QPoint& q, int* stk, int& up, int& down) {
    up = down = 0;
    int node = mv.root;
    if (node == kNoRoot) return;
    auto leaf = [&](int t) {
        const TriQ tr = mv.tris[t];
        const int s = tri_xy_sign(tr, q.x, q.y);
        if (s == 0) return;
        if (plane_above(plane_of(tr, q.x, q.y), q.z)) up += s;
        else down -= s;
    };
    if (node < 0) {
        leaf(~node);
        return;
    }
    int sp = 0;
    while (true) {
        const Node nd = mv.nodes[node];
        bool hl = box_has_xy(nd.lxy.x, nd.lxy.y, nd.lxy.z, nd.lxy.w, q.x, q.y);
        bool hr = box_has_xy(nd.rxy.x, nd.rxy.y, nd.rxy.z, nd.rxy.w, q.x, q.y);
        const int L = nd.link.x, R = nd.link.y;
        if (hl && L < 0) {
            leaf(~L);
            hl = false;
        }
        if (hr && R < 0) {
            leaf(~R);
            hr = false;
        }
        if (hl && hr) {
            stk[sp * kChiBlock] = R;
            ++sp;
            node = L;
        } else if (hl) {
            node = L;
        } else if (hr) {
            node = R;
        } else {
            if (sp == 0) break;
            --sp;
            node = stk[sp * kChiBlock];
        }
    }
}

// Signed crossings of the lines of a wave's lanes, the wave walking the BVH
// together: it descends into a child when the line of ANY active lane meets
// the child's box (ballot), nodes and triangles arrive by scalar loads, and each
// active lane applies its own exact leaf test (u: crossings above q, d: minus
// those below).  UP: the +z ray only, the walk pruned by z (d then holds only
// the leaves it visited); otherwise the whole line.  Every lane of the wave
// calls it together; stk is the wave's LDS stack of kLdsStack entries (a
// child is pushed only where both are taken, so it never holds more entries
// than the tree is deep).
template <bool UP>
__device__ __forceinline__ void chi_wave_walk(const MeshView& mv, const QPoint& q, bool act, int* stk, int& u,
                                              int& d) {
    u = d = 0;
    auto leaf = [&](int t) {
        const TriQ tr = mv.tris[t];
        const int s = tri_xy_sign(tr, q.x, q.y);
        if (s == 0) return;
        if (plane_above(plane_of(tr, q.x, q.y), q.z)) u += s;
        else d -= s;
    };
    int node = mv.root;
    if (__builtin_amdgcn_ballot_w64(act) == 0ull || node == kNoRoot) return;
    if (node < 0) {
        if (act) leaf(~node);
        return;
    }
    int sp = 0;
    while (true) {
        const Node nd = mv.nodes[node];
        const bool ml = act && box_has_xy(nd.lxy.x, nd.lxy.y, nd.lxy.z, nd.lxy.w, q.x, q.y) && (!UP || q.z <= nd.z.y);
        const bool mr = act && box_has_xy(nd.rxy.x, nd.rxy.y, nd.rxy.z, nd.rxy.w, q.x, q.y) && (!UP || q.z <= nd.z.w);
        bool hl = __builtin_amdgcn_ballot_w64(ml) != 0ull;
        bool hr = __builtin_amdgcn_ballot_w64(mr) != 0ull;
        const int L = nd.link.x, R = nd.link.y;
        if (hl && L < 0) {
            if (ml) leaf(~L);
            hl = false;
        }
        if (hr && R < 0) {
            if (mr) leaf(~R);
            hr = false;
        }
        if (hl && hr) {
            stk[sp++] = R;   // every lane stores the same value
            node = L;
        } else if (hl) {
            node = L;
        } else if (hr) {
            node = R;
        } else {
            if (sp == 0) break;
            --sp;
            node = stk[sp];
        }
        node = __builtin_amdgcn_readfirstlane(node);
    }
}

}  // namespace
}  // namespace gwn
