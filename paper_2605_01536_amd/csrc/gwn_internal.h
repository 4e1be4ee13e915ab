// gwn_internal.h -- device data layouts and exact predicates shared by the
// library's HIP sources (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gwn {

constexpr long long kQMax = (1LL << 30) - 1;   // fixed-point coordinates live in [0, 2^30)
constexpr int kLdsStack = 64;  // per-lane BVH stack depth in LDS (a radix tree over 62-bit keys is <= 63 deep)

// Internal BVH node: boxes of both children (integer, fixed-point coords)
// plus the child links, 64 bytes = one fetch per visited node.
// link.x/.y: child >= 0 internal node, child < 0 leaf ~t (sorted triangle t);
// link.z: parent (-1 at the root).
struct alignas(16) Node {
    int4 lxy;   // left child  xlo, xhi, ylo, yhi
    int4 rxy;   // right child xlo, xhi, ylo, yhi
    int4 z;     // left zlo, left zhi, right zlo, right zhi
    int4 link;  // left, right, parent, unused
};

// Quantised triangle corners in Morton order (w unused).
struct alignas(16) TriQ {
    int4 a, b, c;
};

// One boundary-loop vertex, 32 bytes so a wave can fetch it with one scalar load.
// x, y, z: the input position times 2^k (an exact power-of-two scaling), i.e. in
// fixed-point cell units; qx, qy: the quantised x and y; loop: the loop it
// belongs to (its edge leads to the next vertex, or back to the loop's first).
struct alignas(32) BVert {
    float x, y, z;
    int qx, qy;
    int pad0, pad1;
    int loop;
};

// Fixed-point grid parameters: q = rint((x - lo) * scale), scale = 2^k.
struct QGrid {
    double lo[3];
    double scale;
    float scalef;  // 2^k as float (cell units for the boundary term)
    int k;
};

// Read-only view of a built mesh handed to query kernels.
struct MeshView {
    const Node* nodes;
    const TriQ* tris;
    const BVert* bverts;
    const int* loop_off;   // nloops + 1 offsets into bverts
    int nloops;
    int nf;
    int root;              // >= 0 internal node, < 0 leaf ~t, INT_MIN when nf == 0
    int axis;              // ray axis of the mesh frame: 0 = z, 1 = x, 2 = y (see axis_ptrs)
    QGrid g;
};

constexpr int kNoRoot = (int)0x80000000;

// A mesh built along axis a works in the frame (X, Y, Z) = (x, y, z), (y, z, x)
// or (z, x, y) for a = 0 (z), 1 (x), 2 (y): a cyclic permutation, i.e. a
// rotation, so orientations and w are unchanged and the ray +Z is the chosen
// world axis.  Frame component c is world component (c + a) % 3.
__host__ __device__ inline void axis_ptrs(int a, const float*& x, const float*& y, const float*& z) {
    const float* t = x;
    if (a == 1) {
        x = y;
        y = z;
        z = t;
    } else if (a == 2) {
        x = z;
        z = y;
        y = t;
    }
}

// Fixed-point coordinate of one input value, evaluated in FP64 exactly as the
// rule states: rint((x - lo) * 2^k).  The multiply by a power of two is exact,
// so no contraction can change the result.
__device__ __forceinline__ double qround(float x, double lo, double scale) {
    return rint(((double)x - lo) * scale);
}

struct QPoint {
    int x, y, z;   // x, y valid when inbox; z clamped to [-1, 2^30]
    bool inbox;
};

__device__ __forceinline__ QPoint quantize_point(float px, float py, float pz, const QGrid& g) {
    QPoint q;
    double tx = qround(px, g.lo[0], g.scale);
    double ty = qround(py, g.lo[1], g.scale);
    double tz = qround(pz, g.lo[2], g.scale);
    q.inbox = (tx >= 0.0) && (tx <= (double)kQMax) && (ty >= 0.0) && (ty <= (double)kQMax);
    q.x = q.inbox ? (int)tx : 0;
    q.y = q.inbox ? (int)ty : 0;
    tz = fmin(fmax(tz, -1.0), (double)(kQMax + 1));   // NaN -> -1 via fmax
    q.z = (int)tz;
    return q;
}

__device__ __forceinline__ int sgnll(long long v) { return (v > 0) - (v < 0); }
__device__ __forceinline__ int sgni(int v) { return (v > 0) - (v < 0); }

// Sign of orient2d(a, b, q_eps) = cross(a - q_eps, b - q_eps) with the query
// perturbed by (e1, e2), 0 < e2 << e1.  In offsets d = vertex - q the value is
// cross(da, db) + e1 (da.y - db.y) + e2 (db.x - da.x): exactly linear in e.
__device__ __forceinline__ int orient_sos(int dax, int day, int dbx, int dby) {
    long long o = (long long)dax * dby - (long long)day * dbx;
    if (o != 0) return sgnll(o);
    if (day != dby) return day > dby ? 1 : -1;
    return sgni(dbx - dax);
}

// x/y part of the crossing of the vertical line through q_eps with one
// quantised triangle: 0 for a miss, else the common sign s of the three
// perturbed edge tests (= sign of the projected area).
__device__ __forceinline__ int tri_xy_sign(const TriQ& t, int qx, int qy) {
    const int ax = t.a.x - qx, ay = t.a.y - qy;
    const int bx = t.b.x - qx, by = t.b.y - qy;
    const int cx = t.c.x - qx, cy = t.c.y - qy;
    const int e0 = orient_sos(ax, ay, bx, by);
    const int e1 = orient_sos(bx, by, cx, cy);
    const int e2 = orient_sos(cx, cy, ax, ay);
    return (e0 != 0 && e0 == e1 && e0 == e2) ? e0 : 0;
}

// Supporting plane of a quantised triangle, prepared for many queries on one
// vertical line: f(qz) = n . (a - q) = f0 - n_z qz with
// f0 = n . (a - (qx, qy, 0)), n = (b - a) x (c - a).
struct PlaneQ {
    __int128 f0;
    long long nx, ny, nz;
};

__device__ __forceinline__ PlaneQ plane_of(const TriQ& t, int qx, int qy) {
    const long long ux = t.b.x - t.a.x, uy = t.b.y - t.a.y, uz = t.b.z - t.a.z;
    const long long vx = t.c.x - t.a.x, vy = t.c.y - t.a.y, vz = t.c.z - t.a.z;
    PlaneQ p;
    p.nx = uy * vz - uz * vy;
    p.ny = uz * vx - ux * vz;
    p.nz = ux * vy - uy * vx;
    p.f0 = (__int128)p.nx * (long long)(t.a.x - qx) + (__int128)p.ny * (long long)(t.a.y - qy) +
           (__int128)p.nz * (long long)t.a.z;
    return p;
}

// Whether the crossing lies on the +z side of q_eps: the sign of
// f(q_eps) = f - n_x e1 - n_y e2 - n_z e3 (real part, then -n_x, -n_y, -n_z)
// equals the sign of n_z.
__device__ __forceinline__ bool plane_above(const PlaneQ& p, int qz) {
    const __int128 f = p.f0 - (__int128)p.nz * qz;
    int side;
    if (f != 0) side = f > 0 ? 1 : -1;
    else if (p.nx != 0) side = -sgnll(p.nx);
    else if (p.ny != 0) side = -sgnll(p.ny);
    else side = -sgnll(p.nz);
    return side == sgnll(p.nz);
}

// Signed crossing of the +z ray from q_eps with one triangle: 0 if the line
// misses it or the crossing is below the query, else s.
__device__ __forceinline__ int ray_up_hit(const TriQ& t, int qx, int qy, int qz) {
    const int s = tri_xy_sign(t, qx, qy);
    if (s == 0) return 0;
    return plane_above(plane_of(t, qx, qy), qz) ? s : 0;
}

__device__ __forceinline__ bool box_has_xy(int xlo, int xhi, int ylo, int yhi, int qx, int qy) {
    return (qx >= xlo) & (qx <= xhi) & (qy >= ylo) & (qy <= yhi);
}

}  // namespace gwn
