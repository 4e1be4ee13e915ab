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

template <class T>
struct Vtx {
    T rx, ry, rz, s;
    int dx, dy;
};

__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }
__device__ __forceinline__ double fatan2(double y, double x) { return atan2(y, x); }

// atan(t) for |t| <= 1 as t + t x Q(x), x = t^2, Q of degree 7 fitted by the
// Remez exchange for minimax relative error (gen_atan_poly.py: 1.7e-8 in exact
// arithmetic, 9.2e-8 max / 2e-9 mean signed when evaluated in float32).
constexpr float kAtanQ[8] = {0.002920693f, -0.01636793f, 0.043211866f, -0.07552215f,
                             0.106660046f, -0.14211056f, 0.19993773f, -0.33333153f};
constexpr float kPi = 3.14159265358979f;
constexpr float kPi2 = 1.57079632679490f;

__device__ __forceinline__ float atan_unit(float t) {
    const float x = t * t;
    float q = kAtanQ[0];
#pragma unroll
    for (int k = 1; k < 8; ++k) q = fmaf(q, x, kAtanQ[k]);
    return fmaf(t * x, q, t);
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
__device__ __forceinline__ float fatan2(float y, float x) { return atan2_full(y, x); }

// s = l - r_z, evaluated without cancellation
template <class T>
__device__ __forceinline__ T stereo_s(T rho2, T rz) {
    T l = fsqrt(rho2 + rz * rz);
    T t = l + fabs(rz);
    return rz > (T)0 ? fdiv(rho2, t) : t;
}

// FAR = the query's quantised x or y is outside the grid: raw offsets, and no
// exact decision is needed (no ray crossings; every edge has D > 0 there).
template <class T, bool FAR>
__device__ __forceinline__ Vtx<T> make_vtx(const BVert& b, int qqx, int qqy, T pxs, T pys, T pzs) {
    Vtx<T> v;
    v.dx = b.qx - qqx;
    v.dy = b.qy - qqy;
    if (FAR) {
        v.rx = (T)b.x - pxs;
        v.ry = (T)b.y - pys;
    } else {
        v.rx = (T)v.dx;
        v.ry = (T)v.dy;
    }
    v.rz = (T)b.z - pzs;
    v.s = stereo_s<T>(v.rx * v.rx + v.ry * v.ry, v.rz);
    return v;
}

// Rare path for D <= 0: fix the sign of N from the exact predicate, or take the
// limit under the perturbation when an endpoint lies on the +z ray (its x/y
// offset becomes (-e1, -e2)).
template <class T>
__device__ __forceinline__ void exact_branch(const Vtx<T>& a, const Vtx<T>& b, T& N, T& D) {
    const bool aon = (a.dx == 0) & (a.dy == 0) & (a.rz > (T)0);
    const bool bon = (b.dx == 0) & (b.dy == 0) & (b.rz > (T)0);
    if (aon && bon) {
        N = (T)0;
        D = (T)1;
    } else if (aon) {          // N ~ e1 rb_y - e2 rb_x,  D ~ -e1 rb_x - e2 rb_y
        if (b.ry != (T)0) {
            N = b.ry;
            D = -b.rx;
        } else if (b.rx > (T)0) {
            N = -(T)0;
            D = (T)-1;
        } else {
            N = (T)0;
            D = (T)1;
        }
    } else if (bon) {          // N ~ -e1 ra_y + e2 ra_x, D ~ -e1 ra_x - e2 ra_y
        if (a.ry != (T)0) {
            N = -a.ry;
            D = -a.rx;
        } else if (a.rx > (T)0) {
            N = (T)0;
            D = (T)-1;
        } else {
            N = (T)0;
            D = (T)1;
        }
    } else {
        const int o = orient_sos(a.dx, a.dy, b.dx, b.dy);   // N = -orient2d(a, b, q_eps)
        if (o > 0) N = -fabs(N);
        else if (o < 0) N = fabs(N);
    }
}

template <class T, bool FAR>
__device__ __forceinline__ T edge_angle(const Vtx<T>& a, const Vtx<T>& b) {
    T N = a.ry * b.rx - a.rx * b.ry;
    T D = a.s * b.s + (a.rx * b.rx + a.ry * b.ry);
    if (!FAR && D <= (T)0) exact_branch<T>(a, b, N, D);
    return fatan2(N, D);
}

// ---------------------------------------------------------------- FP32 loop
// x/y quantities of one boundary vertex relative to the query column (shared by
// all samples of a grid column; per lane in the batch kernel).
struct ColV {
    int dx, dy;
    float rx, ry, rho2;
};

template <bool FAR>
__device__ __forceinline__ ColV col_vtx(const BVert& b, int qqx, int qqy, float pxs, float pys) {
    ColV c;
    c.dx = b.qx - qqx;
    c.dy = b.qy - qqy;
    if (FAR) {
        c.rx = b.x - pxs;
        c.ry = b.y - pys;
    } else {
        c.rx = (float)c.dx;
        c.ry = (float)c.dy;
    }
    c.rho2 = fmaf(c.rx, c.rx, c.ry * c.ry);
    return c;
}

// s = l - r_z without cancellation
__device__ __forceinline__ float samp_s(float rho2, float rz) {
    const float l = __builtin_amdgcn_sqrtf(fmaf(rz, rz, rho2));
    const float t = l + fabsf(rz);
    return rz > 0.f ? rho2 * __builtin_amdgcn_rcpf(t) : t;
}

// Rare path of one (sample, edge): exact atan2 branch where D <= 0 (sign of N from
// the perturbed predicate, or the perturbation limit for an endpoint on the ray),
// then the full-range atan2.
__device__ __forceinline__ float edge_slow(const ColV& a, const ColV& b, float rza, float rzb, float N, float D,
                                           bool exact) {
    if (exact && D <= 0.f) {
        const bool aon = (a.dx == 0) & (a.dy == 0) & (rza > 0.f);
        const bool bon = (b.dx == 0) & (b.dy == 0) & (rzb > 0.f);
        if (aon && bon) {
            N = 0.f;
            D = 1.f;
        } else if (aon) {        // N ~ e1 rb_y - e2 rb_x,  D ~ -e1 rb_x - e2 rb_y
            if (b.ry != 0.f) { N = b.ry; D = -b.rx; }
            else if (b.rx > 0.f) { N = -0.f; D = -1.f; }
            else { N = 0.f; D = 1.f; }
        } else if (bon) {        // N ~ -e1 ra_y + e2 ra_x, D ~ -e1 ra_x - e2 ra_y
            if (a.ry != 0.f) { N = -a.ry; D = -a.rx; }
            else if (a.rx > 0.f) { N = 0.f; D = -1.f; }
            else { N = 0.f; D = 1.f; }
        } else {
            const int o = orient_sos(a.dx, a.dy, b.dx, b.dy);   // N = -orient2d(a, b, q_eps)
            if (o > 0) N = -fabsf(N);
            else if (o < 0) N = fabsf(N);
        }
    }
    return atan2_full(N, D);
}

// One boundary edge for ZB samples.  Fast path (wave-uniform): every sample has
// |N| < D, so atan2(N, D) = atan(N/D) with |N/D| < 1 and no branch fix-up.
template <int ZB, bool FAR>
__device__ __forceinline__ void edge_f32(const ColV& a, const ColV& b, const float* sa, const float* sb,
                                         const float* rza, const float* rzb, float* acc) {
    const float N = fmaf(a.ry, b.rx, -a.rx * b.ry);
    const float dot = fmaf(a.rx, b.rx, a.ry * b.ry);
    const float aN = fabsf(N);
    float D[ZB];
    bool slow = false;
#pragma unroll
    for (int r = 0; r < ZB; ++r) {
        D[r] = fmaf(sa[r], sb[r], dot);
        slow |= !(aN < D[r]);
    }
    if (__builtin_amdgcn_ballot_w64(slow) == 0ull) {
#pragma unroll
        for (int r = 0; r < ZB; ++r) acc[r] += atan_unit(N * __builtin_amdgcn_rcpf(D[r]));
    } else {
#pragma unroll
        for (int r = 0; r < ZB; ++r) acc[r] += edge_slow(a, b, rza[r], rzb[r], N, D[r], !FAR);
    }
}

// Boundary sum for ZB samples sharing one (x, y): loops of the chain, FP32
// partials flushed into FP64 every 32 edges.
template <int ZB, bool FAR>
__device__ __forceinline__ void loops_f32(const MeshView& mv, int qqx, int qqy, float pxs, float pys, const float* pzs,
                                          double* S) {
    const BVert* __restrict__ bv = mv.bverts;
    for (int l = 0; l < mv.nloops; ++l) {
        const int b0 = mv.loop_off[l], b1 = mv.loop_off[l + 1];
        ColV cf, cp;
        float rzf[ZB], sf[ZB], rzp[ZB], sp[ZB];
        {
            const BVert b = bv[b0];
            cf = col_vtx<FAR>(b, qqx, qqy, pxs, pys);
#pragma unroll
            for (int r = 0; r < ZB; ++r) {
                rzf[r] = b.z - pzs[r];
                sf[r] = samp_s(cf.rho2, rzf[r]);
                rzp[r] = rzf[r];
                sp[r] = sf[r];
            }
            cp = cf;
        }
        int j = b0 + 1;
        while (j < b1) {
            const int je = min(b1, j + 32);
            float acc[ZB];
#pragma unroll
            for (int r = 0; r < ZB; ++r) acc[r] = 0.f;
            // two vertices per trip: the loop-carried vertex alternates between
            // two register sets instead of being copied every edge
            for (; j + 1 < je; j += 2) {
                const BVert b1v = bv[j];
                const ColV c1 = col_vtx<FAR>(b1v, qqx, qqy, pxs, pys);
                float rz1[ZB], s1[ZB];
#pragma unroll
                for (int r = 0; r < ZB; ++r) {
                    rz1[r] = b1v.z - pzs[r];
                    s1[r] = samp_s(c1.rho2, rz1[r]);
                }
                edge_f32<ZB, FAR>(cp, c1, sp, s1, rzp, rz1, acc);
                const BVert b2v = bv[j + 1];
                cp = col_vtx<FAR>(b2v, qqx, qqy, pxs, pys);
#pragma unroll
                for (int r = 0; r < ZB; ++r) {
                    rzp[r] = b2v.z - pzs[r];
                    sp[r] = samp_s(cp.rho2, rzp[r]);
                }
                edge_f32<ZB, FAR>(c1, cp, s1, sp, rz1, rzp, acc);
            }
            if (j < je) {
                const BVert b = bv[j];
                const ColV cc = col_vtx<FAR>(b, qqx, qqy, pxs, pys);
                float rzc[ZB], sc[ZB];
#pragma unroll
                for (int r = 0; r < ZB; ++r) {
                    rzc[r] = b.z - pzs[r];
                    sc[r] = samp_s(cc.rho2, rzc[r]);
                }
                edge_f32<ZB, FAR>(cp, cc, sp, sc, rzp, rzc, acc);
                cp = cc;
#pragma unroll
                for (int r = 0; r < ZB; ++r) {
                    rzp[r] = rzc[r];
                    sp[r] = sc[r];
                }
                ++j;
            }
#pragma unroll
            for (int r = 0; r < ZB; ++r) S[r] += (double)acc[r];
        }
        float acc[ZB];
#pragma unroll
        for (int r = 0; r < ZB; ++r) acc[r] = 0.f;
        edge_f32<ZB, FAR>(cp, cf, sp, sf, rzp, rzf, acc);
#pragma unroll
        for (int r = 0; r < ZB; ++r) S[r] += (double)acc[r];
    }
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

}  // namespace
}  // namespace gwn
