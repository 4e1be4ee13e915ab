// grad.hip -- gradient of w with respect to the query point (Supp. Sec. 4, Alg. 3).
//
// The crossing count is locally constant, so only the boundary term is
// differentiated: per boundary edge (a, b), with r0 = a - p, r1 = b - p and the
// same N, D as the value path (x1 = -z),
//     grad 2 atan2(N, D) = 2 (D grad N - N grad D) / (N^2 + D^2),
//     grad N = (r1y - r0y, r0x - r1x, 0),
//     grad D = -((1 + s1/l0) r0 + (1 + s0/l1) r1) + (l0 + l1) z^,
// whose z part simplifies to s0 s1 (1/l0 + 1/l1) (no cancellation).  N and D are
// scaled by 1/(l0 l1) before squaring so nothing overflows in cell units.  No
// exact predicate is needed: the derivative of atan2 is the same on both sides
// of its branch cut, so every query uses raw offsets.
//
// A boundary vertex exactly above the query (on the +z ray) makes N = D = 0 for
// its two edges; their divergent terms cancel in the sum but their values are
// 0/0.  Such a query is summed again with the opposite axis (x0 = -z): the
// gradient does not depend on the axis, and mirroring z maps that sum onto the
// same code with r_z negated and the x, y components negated.  A query with
// boundary vertices both above and below it takes a third pass with a general
// axis (grad_run_axis, in kernels of its own).  Grids share the x/y quantities (N, grad N, the x/y
// dot) of a column among its samples.
#include <algorithm>

#include "gwn_kernels.h"
#include "gwn_mesh.h"

namespace gwn {
namespace {

// x/y part of one boundary vertex relative to the query column, shared by all
// samples of a grid column.  Offsets are in units of 2^e cells (f = 2^-e, see
// far_scale): each edge term is homogeneous of degree -1 in the offsets, so the
// sum is rescaled at the end.
template <class T>
struct GCol {
    T rx, ry, rho2;
};

template <class T>
__device__ __forceinline__ GCol<T> gcol(const BVert& b, T pxs, T pys, T f) {
    GCol<T> c;
    c.rx = fma((T)b.x, f, -pxs);
    c.ry = fma((T)b.y, f, -pys);
    c.rho2 = c.rx * c.rx + c.ry * c.ry;
    return c;
}

// per-sample part of one vertex: u = 1/l and s = l - r_z (r_z negated for FLIP)
template <class T, bool FLIP>
__device__ __forceinline__ void gsamp(const BVert& b, const GCol<T>& c, T pzs, T f, T& u, T& s) {
    const T rz0 = fma((T)b.z, f, -pzs);
    const T rz = FLIP ? -rz0 : rz0;
    const T l = Arith<T>::sqrt(rz * rz + c.rho2);
    u = Arith<T>::rcp(l);
    const T t = l + fabs(rz);
    s = rz > (T)0 ? c.rho2 * Arith<T>::rcp(t) : t;
}

// one edge (a -> b) for one sample; N, dot and grad N come from x/y only
template <class T>
__device__ __forceinline__ void gedge(const GCol<T>& a, const GCol<T>& b, T N, T dot, T gNx, T gNy, T ua, T sa,
                                      T ub, T sb, T* g) {
    const T k = ua * ub;
    const T n = N * k;
    const T d = fma(sa, sb, dot) * k;
    const T c0 = (T)1 + sb * ua, c1 = (T)1 + sa * ub;
    const T dDx = -(c0 * a.rx + c1 * b.rx);
    const T dDy = -(c0 * a.ry + c1 * b.ry);
    const T dDz = sa * sb * (ua + ub);
    const T fr = k * Arith<T>::rcp(n * n + d * d);
    g[0] += (d * gNx - n * dDx) * fr;
    g[1] += (d * gNy - n * dDy) * fr;
    g[2] += (-n * dDz) * fr;
}

// Sum over all loops of the edge terms for ZB samples on one vertical line, in
// cell units (FP32 partials flushed into FP64 every 32 edges).  FLIP: the
// mirrored sum for the axis x0 = -z.
template <class T, int ZB, bool FLIP>
__device__ void grad_loops(const MeshView& mv, T pxs, T pys, const T* pzs, T f, double (*G)[3]) {
    const BVert* __restrict__ bv = mv.bverts;
#pragma unroll
    for (int r = 0; r < ZB; ++r) G[r][0] = G[r][1] = G[r][2] = 0.0;
    for (int lp = 0; lp < mv.nloops; ++lp) {
        const int b0 = mv.loop_off[lp], b1 = mv.loop_off[lp + 1];
        const GCol<T> cf = gcol<T>(bv[b0], pxs, pys, f);
        T uf[ZB], sf[ZB];
#pragma unroll
        for (int r = 0; r < ZB; ++r) gsamp<T, FLIP>(bv[b0], cf, pzs[r], f, uf[r], sf[r]);
        GCol<T> cp = cf;
        T up[ZB], sp[ZB];
#pragma unroll
        for (int r = 0; r < ZB; ++r) {
            up[r] = uf[r];
            sp[r] = sf[r];
        }
        for (int j = b0 + 1; j <= b1; j += 32) {
            const int je = min(b1 + 1, j + 32);
            T acc[ZB][3];
#pragma unroll
            for (int r = 0; r < ZB; ++r) acc[r][0] = acc[r][1] = acc[r][2] = (T)0;
            for (int jj = j; jj < je; ++jj) {
                // index b1 closes the loop back to its first vertex
                GCol<T> cc = cf;
                T uc[ZB], sc[ZB];
#pragma unroll
                for (int r = 0; r < ZB; ++r) {
                    uc[r] = uf[r];
                    sc[r] = sf[r];
                }
                if (jj < b1) {
                    cc = gcol<T>(bv[jj], pxs, pys, f);
#pragma unroll
                    for (int r = 0; r < ZB; ++r) gsamp<T, FLIP>(bv[jj], cc, pzs[r], f, uc[r], sc[r]);
                }
                const T N = cp.ry * cc.rx - cp.rx * cc.ry;
                const T dot = cp.rx * cc.rx + cp.ry * cc.ry;
                const T gNx = cc.ry - cp.ry, gNy = cp.rx - cc.rx;
#pragma unroll
                for (int r = 0; r < ZB; ++r) gedge<T>(cp, cc, N, dot, gNx, gNy, up[r], sp[r], uc[r], sc[r], acc[r]);
                cp = cc;
#pragma unroll
                for (int r = 0; r < ZB; ++r) {
                    up[r] = uc[r];
                    sp[r] = sc[r];
                }
            }
#pragma unroll
            for (int r = 0; r < ZB; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) G[r][c] += (double)acc[r][c];
        }
    }
    if (FLIP) {
#pragma unroll
        for (int r = 0; r < ZB; ++r) {
            G[r][0] = -G[r][0];
            G[r][1] = -G[r][1];
        }
    }
}

// Grid columns: a boundary vertex's x/y terms (its offsets, rho^2, and N, the
// x/y dot and grad N of its outgoing edge) are the same for every sample of a
// column's wave, so they are computed for 64 vertices at a time, one per lane,
// into a ring of records in LDS that the whole wave reads back (as for w; the
// ring's slots, fills and closing slot follow column_loops).
template <class T>
struct alignas(4 * sizeof(T)) GRec {
    T z;      // vertex z as stored (offset units once times f)
    T rho2;
    T rx, ry;
};

template <class T>
struct alignas(4 * sizeof(T)) GEdge {   // the vertex's outgoing edge
    T N, dot, gNx, gNy;
};

template <class T>
struct GRing {
    GRec<T> v[kColRing + 1];
    GEdge<T> e[kColRing + 1];
    int R[kColRing + 1];   // blocks of the column with a sample below the vertex (see the sample blocks note in gwn_kernels.h), plus 256
                           // when the vertex is far (s_blocks)
};

template <class T, int ZB>
__device__ __forceinline__ void grad_fill(const MeshView& mv, int v0, int n, int b0, int b1, T pxs, T pys, T f,
                                          const T* bminr, bool asc, GRing<T>& ring) {
    const int lane = (int)(threadIdx.x & 63);
    if (lane < n) {
        const int v = v0 + lane;
        const int vn = v + 1 < b1 ? v + 1 : b0;
        const BVert a = mv.bverts[v], b = mv.bverts[vn];
        const GCol<T> ca = gcol<T>(a, pxs, pys, f), cb = gcol<T>(b, pxs, pys, f);
        GRec<T> rv;
        rv.z = (T)a.z;
        rv.rho2 = ca.rho2;
        rv.rx = ca.rx;
        rv.ry = ca.ry;
        GEdge<T> re;
        re.N = ca.ry * cb.rx - ca.rx * cb.ry;
        re.dot = ca.rx * cb.rx + ca.ry * cb.ry;
        re.gNx = cb.ry - ca.ry;
        re.gNy = ca.rx - cb.rx;
        int R = ZB + 1;
        if (asc) {
            R = 0;
            bool farv = true;   // every sample below the vertex has r_z^2 <= 3 rho^2 (see s_blocks)
#pragma unroll
            for (int r = 0; r < ZB; ++r) {
                const T zr = fma((T)a.z, f, -bminr[r]);   // the block's largest r_z
                R += zr > (T)0;
                farv &= !((zr > (T)0) & (zr * zr > (T)3 * rv.rho2));
            }
            R |= farv ? 256 : 0;
        }
        const int k = (v - b0) & (kColRing - 1);
        ring.v[k] = rv;
        ring.e[k] = re;
        ring.R[k] = R;
        if (v == b0) {
            ring.v[kColRing] = rv;
            ring.e[kColRing] = re;
            ring.R[kColRing] = R;
        }
    }
    // the wave reads what its own lanes wrote; LDS operations of a wave complete in order
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// u = 1/l and s of one ring vertex for the ZB samples: blocks wholly at or above
// the vertex take s = l + |r_z|, blocks wholly below it s = rho^2 / (l + r_z),
// the block the vertex's height falls in the two-sided form, and a far vertex
// l - r_z in every block (the block count and the far test are the w kernel's;
// r_z is the same fma in both)
template <class T, int ZB>
__device__ __forceinline__ void grad_vertex(const GRec<T>& c, int R, const T* pzs, T f, T* u, T* s) {
    T rz[ZB];
#pragma unroll
    for (int r = 0; r < ZB; ++r) {
        rz[r] = fma(c.z, f, -pzs[r]);
        const T l = Arith<T>::sqrt(rz[r] * rz[r] + c.rho2);
        u[r] = Arith<T>::rcp(l);
        s[r] = l + fabs(rz[r]);   // t, made s in place
    }
    s_prefix<T, ZB>(R & 0xff, rz, c.rho2, s, R >= 256);
}

// grad_loops for a grid column (x0 = +z), register r of the wave a block of 64
// consecutive samples with z monotone in the lane; same sums in the same order.
template <class T, int ZB>
__device__ void grad_column_loops(const MeshView& mv, T pxs, T pys, const T* pzs, T f, double (*G)[3],
                                  GRing<T>& ring) {
    T bminr[ZB];
    bool asc = true;
    T prev = -(T)INFINITY;
#pragma unroll
    for (int r = 0; r < ZB; ++r) {   // ascending blocks with non-falling minima, as for w (column_loops)
        const T z0 = wave_lane<T>(pzs[r], 0), z63 = wave_lane<T>(pzs[r], 63);
        bminr[r] = fmin(z0, z63);
        asc &= !(bminr[r] < prev) & !(z63 < z0);
        prev = bminr[r];
    }
#pragma unroll
    for (int r = 0; r < ZB; ++r) G[r][0] = G[r][1] = G[r][2] = 0.0;
    for (int lp = 0; lp < mv.nloops; ++lp) {
        const int b0 = mv.loop_off[lp], nv = mv.loop_off[lp + 1] - b0;
        int done = min(64, nv);
        grad_fill<T, ZB>(mv, b0, done, b0, b0 + nv, pxs, pys, f, bminr, asc, ring);
        T up[ZB], sp[ZB];
        grad_vertex<T, ZB>(ring.v[0], __builtin_amdgcn_readfirstlane(ring.R[0]), pzs, f, up, sp);
        T prx = ring.v[0].rx, pry = ring.v[0].ry;
        // edge j leads from vertex j - 1 to vertex j; j = nv closes the loop
        for (int j = 1; j <= nv; j += 32) {
            const int je = min(nv + 1, j + 32);
            if (min(je, nv) > done) {   // one fill covers it: j <= done, je <= j + 32
                const int n = min(64, nv - done);
                grad_fill<T, ZB>(mv, b0 + done, n, b0, b0 + nv, pxs, pys, f, bminr, asc, ring);
                done += n;
            }
            T acc[ZB][3];
#pragma unroll
            for (int r = 0; r < ZB; ++r) acc[r][0] = acc[r][1] = acc[r][2] = (T)0;
            for (int jj = j; jj < je; ++jj) {
                const int kp = (jj - 1) & (kColRing - 1), kc = jj < nv ? (jj & (kColRing - 1)) : kColRing;
                const GRec<T> c = ring.v[kc];
                const GEdge<T> e = ring.e[kp];
                T uc[ZB], sc[ZB];
                grad_vertex<T, ZB>(c, __builtin_amdgcn_readfirstlane(ring.R[kc]), pzs, f, uc, sc);
                GCol<T> ga, gb;
                ga.rx = prx;
                ga.ry = pry;
                gb.rx = c.rx;
                gb.ry = c.ry;
                ga.rho2 = gb.rho2 = (T)0;   // not used by gedge
#pragma unroll
                for (int r = 0; r < ZB; ++r) gedge<T>(ga, gb, e.N, e.dot, e.gNx, e.gNy, up[r], sp[r], uc[r], sc[r], acc[r]);
                prx = c.rx;
                pry = c.ry;
#pragma unroll
                for (int r = 0; r < ZB; ++r) {
                    up[r] = uc[r];
                    sp[r] = sc[r];
                }
            }
#pragma unroll
            for (int r = 0; r < ZB; ++r)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) G[r][cc] += (double)acc[r][cc];
        }
    }
}

// Third pass, for samples whose lines along +z and -z both meet a boundary
// vertex (vertical stacks of boundary vertices), where both folded forms above
// are 0/0: the edge term of Alg. 3 for a general axis x0 = u, x1 = -u, in FP64
// on the same offsets.  u is fixed and in no special relation to the grid or
// the coordinate axes, so a sample whose line along u also meets a vertex is
// left as 0/0, as with the paper's random choice of axis.  Per edge, with
// r0 = a - p, r1 = b - p, l = |r|, v = r / l:
//     n = x1.(r0 x r1),   d = l0 l1 + l1 x1.r0 + l0 x1.r1 + r0.r1,
//     grad n = -(r1 x x1 + x1 x r0),
//     grad d = -(l1 (x1 + v1 + (1 + x1.v1) v0) + l0 (x1 + v0 + (1 + x1.v0) v1)),
// and the term (d grad n - n grad d) / (n^2 + d^2) is the gradient of
// atan2(n, d), as the folded forms sum it.
__device__ __forceinline__ void grad_axis_x1(double* x1) {
    const double a = 0.5381966011250105, b = 0.4142135623730950, c = 0.7320508075688772;
    const double k = -1.0 / sqrt(a * a + b * b + c * c);
    x1[0] = a * k;
    x1[1] = b * k;
    x1[2] = c * k;
}

__device__ __forceinline__ void cross3(const double* u, const double* v, double* w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
}

__device__ __forceinline__ double dot3(const double* u, const double* v) {
    return u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
}

__device__ __forceinline__ void grad_axis_edge(const double* r0, const double* r1, const double* x1, double* g) {
    const double l0 = sqrt(dot3(r0, r0)), l1 = sqrt(dot3(r1, r1));
    double v0[3], v1[3], c[3], c1[3], c0[3];
    for (int k = 0; k < 3; ++k) {
        v0[k] = r0[k] / l0;
        v1[k] = r1[k] / l1;
    }
    cross3(r0, r1, c);
    const double n = dot3(x1, c);
    const double d = l0 * l1 + l1 * dot3(x1, r0) + l0 * dot3(x1, r1) + dot3(r0, r1);
    cross3(r1, x1, c1);
    cross3(x1, r0, c0);
    const double e1 = 1.0 + dot3(x1, v1), e0 = 1.0 + dot3(x1, v0);
    const double inv = 1.0 / (n * n + d * d);
    for (int k = 0; k < 3; ++k) {
        const double gn = -(c1[k] + c0[k]);
        const double gd = -(l1 * (x1[k] + v1[k] + e1 * v0[k]) + l0 * (x1[k] + v0[k] + e0 * v1[k]));
        g[k] += (d * gn - n * gd) * inv;
    }
}

// the third pass over boundary vertices [a, e) (edge j leads to the next vertex
// of its loop) for ZB samples on one vertical line
template <int ZB>
__device__ void grad_run_axis(const MeshView& mv, int a, int e, double pxs, double pys, const double* pzs, double f,
                              double (*G)[3]) {
    double x1[3];
    grad_axis_x1(x1);
#pragma unroll
    for (int r = 0; r < ZB; ++r) G[r][0] = G[r][1] = G[r][2] = 0.0;
    const BVert* __restrict__ bv = mv.bverts;
    for (int j = a; j < e; ++j) {
        const int lp = min(max(bv[j].loop, 0), mv.nloops - 1);   // in range for any stored value
        const int nx = j + 1 < mv.loop_off[lp + 1] ? j + 1 : mv.loop_off[lp];
        const BVert A = bv[j], B = bv[nx];
        const double ax = fma((double)A.x, f, -pxs), ay = fma((double)A.y, f, -pys);
        const double bx = fma((double)B.x, f, -pxs), by = fma((double)B.y, f, -pys);
#pragma unroll
        for (int r = 0; r < ZB; ++r) {
            const double r0[3] = {ax, ay, fma((double)A.z, f, -pzs[r])};
            const double r1[3] = {bx, by, fma((double)B.z, f, -pzs[r])};
            grad_axis_edge(r0, r1, x1, G[r]);
        }
    }
}

__device__ __forceinline__ bool finite3(const double* g) { return isfinite(g[0]) && isfinite(g[1]) && isfinite(g[2]); }

template <class T>
__global__ __launch_bounds__(256) void k_grad_batch(MeshView mv, const float* __restrict__ qx,
                                                    const float* __restrict__ qy, const float* __restrict__ qz,
                                                    long long qs, long long nq, int axis, T* __restrict__ g) {
    const long long i = blockIdx.x * 256ll + threadIdx.x;
    if (blockIdx.x * 256ll >= nq) return;
    const long long ii = i < nq ? i : nq - 1;
    const float px = qx[ii * qs], py = qy[ii * qs], pz = qz[ii * qs];
    const FarScale<T> fs = far_scale<T>(px, py, fabsf(pz), mv.g.scale);
    const T pxs = (T)px * fs.scf, pys = (T)py * fs.scf, pzs = (T)pz * fs.scf;
    double G[1][3];
    grad_loops<T, 1, false>(mv, pxs, pys, &pzs, fs.f, G);
    if (!finite3(G[0])) grad_loops<T, 1, true>(mv, pxs, pys, &pzs, fs.f, G);
    if (i < nq) {
        // sum of 2 atan2 terms over 4 pi, and the chain rule through p * 2^(k-e)
        const double f = kInv2Pi * (double)fs.scf;
        // frame component c is world component (c + axis) % 3
        for (int c = 0; c < 3; ++c) g[3 * i + (c + axis) % 3] = (T)(G[0][c] * f);
    }
}

// Few points against many boundary edges: one workgroup per point, each lane a
// contiguous run of boundary vertices (edge j leads to the next vertex of its
// loop), reduced by wave shuffles and LDS in a fixed order.  FLIP as above.
constexpr int kSplitThreads = 256;

template <class T, bool FLIP>
__device__ void grad_run(const MeshView& mv, int a, int e, T pxs, T pys, T pzs, T f, double* G) {
    G[0] = G[1] = G[2] = 0.0;
    if (a >= e) return;
    const BVert* __restrict__ bv = mv.bverts;
    GCol<T> cp = gcol<T>(bv[a], pxs, pys, f);
    T up, sp;
    gsamp<T, FLIP>(bv[a], cp, pzs, f, up, sp);
    T acc[3] = {(T)0, (T)0, (T)0};
    int cnt = 0;
    for (int j = a; j < e; ++j) {
        const int lp = min(max(bv[j].loop, 0), mv.nloops - 1);   // in range for any stored value
        const int nx = j + 1 < mv.loop_off[lp + 1] ? j + 1 : mv.loop_off[lp];
        const GCol<T> cn = gcol<T>(bv[nx], pxs, pys, f);
        T un, sn;
        gsamp<T, FLIP>(bv[nx], cn, pzs, f, un, sn);
        const T N = cp.ry * cn.rx - cp.rx * cn.ry;
        const T dot = cp.rx * cn.rx + cp.ry * cn.ry;
        gedge<T>(cp, cn, N, dot, cn.ry - cp.ry, cp.rx - cn.rx, up, sp, un, sn, acc);
        if (++cnt == 32) {
            for (int c = 0; c < 3; ++c) {
                G[c] += (double)acc[c];
                acc[c] = (T)0;
            }
            cnt = 0;
        }
        if (j + 1 < e) {
            if (nx == j + 1) {
                cp = cn;
                up = un;
                sp = sn;
            } else {   // the next edge starts a new loop
                cp = gcol<T>(bv[j + 1], pxs, pys, f);
                gsamp<T, FLIP>(bv[j + 1], cp, pzs, f, up, sp);
            }
        }
    }
    for (int c = 0; c < 3; ++c) G[c] += (double)acc[c];
    if (FLIP) {
        G[0] = -G[0];
        G[1] = -G[1];
    }
}

// sum of the workgroup's per-lane vectors, the same in every lane afterwards
__device__ void block_sum3(double* G, double (*red)[3]) {
    for (int c = 0; c < 3; ++c)
        for (int o = 32; o > 0; o >>= 1) G[c] += __shfl_xor(G[c], o);
    __syncthreads();   // red may still be read from a previous call
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < 3; ++c) red[threadIdx.x >> 6][c] = G[c];
    __syncthreads();
    for (int c = 0; c < 3; ++c) {
        double t = 0.0;
        for (int k = 0; k < kSplitThreads / 64; ++k) t += red[k][c];
        G[c] = t;
    }
}

template <class T>
__global__ __launch_bounds__(kSplitThreads) void k_grad_split(MeshView mv, const float* __restrict__ qx,
                                                             const float* __restrict__ qy,
                                                             const float* __restrict__ qz, long long qs, long long nq,
                                                             int axis, T* __restrict__ g) {
    __shared__ double red[kSplitThreads / 64][3];
    const long long i = blockIdx.x;   // one point per workgroup
    if (i >= nq) return;
    const float px = qx[i * qs], py = qy[i * qs], pz = qz[i * qs];
    const FarScale<T> fs = far_scale<T>(px, py, fabsf(pz), mv.g.scale);
    const T pxs = (T)px * fs.scf, pys = (T)py * fs.scf, pzs = (T)pz * fs.scf;
    const int nb = mv.loop_off[mv.nloops];
    const int per = (nb + kSplitThreads - 1) / kSplitThreads;
    const int a = (int)threadIdx.x * per, e = min(nb, a + per);
    double G[3];
    grad_run<T, false>(mv, a, e, pxs, pys, pzs, fs.f, G);
    block_sum3(G, red);
    if (!finite3(G)) {   // uniform: every lane holds the same sum
        grad_run<T, true>(mv, a, e, pxs, pys, pzs, fs.f, G);
        block_sum3(G, red);
    }
    if (threadIdx.x == 0) {
        const double f = kInv2Pi * (double)fs.scf;
        for (int c = 0; c < 3; ++c) g[3 * i + (c + axis) % 3] = (T)(G[c] * f);
    }
}

// Gradient on a grid: one wave per (column, z-chunk) as for w, ZB samples per
// lane (lane l holds samples l + 64 r of the chunk) sharing the column's x/y
// terms.  A column through a boundary vertex
// makes the samples below it 0/0 on the +z axis; if any lane has such a sample,
// the wave sums the mirrored axis too and those samples take that sum.
template <class T, int ZB>
__global__ __launch_bounds__(64 * kGridWaves) void k_grad_grid(MeshView mv, GridArgs ga, int axis,
                                                               T* __restrict__ g) {
    __shared__ GRing<T> ring[kGridWaves];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const long long gw = ga.wave0 + (long long)blockIdx.x * kGridWaves + wave;
    if (gw >= ga.nwaves) return;
    const long long col = gw / ga.nchunks;
    const long long chunk = gw - col * ga.nchunks;
    const long long ci = col / ga.ny, cj = col - ci * ga.ny;
    const float px = grid_coord(ga.o[0], ga.s[0], ci);
    const float py = grid_coord(ga.o[1], ga.s[1], cj);
    const long long k0 = chunk * 64 * ZB + lane;   // sample r is k0 + 64 r
    float pz[ZB], pzm = 0.f;
#pragma unroll
    for (int r = 0; r < ZB; ++r) {
        pz[r] = grid_coord(ga.o[2], ga.s[2], min(k0 + 64 * r, ga.nz - 1));
        pzm = fmaxf(pzm, fabsf(pz[r]));
    }
    const FarScale<T> fs = far_scale<T>(px, py, pzm, mv.g.scale);
    T pzs[ZB];
#pragma unroll
    for (int r = 0; r < ZB; ++r) pzs[r] = (T)pz[r] * fs.scf;
    const T pxs = (T)px * fs.scf, pys = (T)py * fs.scf;
    double G[ZB][3];
    grad_column_loops<T, ZB>(mv, pxs, pys, pzs, fs.f, G, ring[wave]);
    bool bad = false;
#pragma unroll
    for (int r = 0; r < ZB; ++r) bad |= !finite3(G[r]);
    if (__builtin_amdgcn_ballot_w64(bad) != 0ull) {
        double H[ZB][3];
        grad_loops<T, ZB, true>(mv, pxs, pys, pzs, fs.f, H);
#pragma unroll
        for (int r = 0; r < ZB; ++r)
            if (!finite3(G[r]))
                for (int c = 0; c < 3; ++c) G[r][c] = H[r][c];
    }
    const double f = kInv2Pi * (double)fs.scf;
    const long long base = ci * ga.st[0] + cj * ga.st[1];
#pragma unroll
    for (int r = 0; r < ZB; ++r) {
        const long long k = k0 + 64 * r;
        if (k < ga.nz)
            for (int c = 0; c < 3; ++c) g[3 * (base + k * ga.st[2]) + (c + axis) % 3] = (T)(G[r][c] * f);
    }
}

// The third pass (grad_run_axis) as kernels of its own, so that the main
// kernels keep their register budgets: every output with a component that is
// not finite (both folded forms 0/0; also a query on the boundary itself, which
// stays 0/0) is summed again with the general axis.  Arbitrary points:
template <class T>
__global__ __launch_bounds__(256) void k_grad_fix_points(MeshView mv, const float* __restrict__ qx,
                                                         const float* __restrict__ qy, const float* __restrict__ qz,
                                                         long long qs, long long nq, int axis, T* __restrict__ g) {
    const long long i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= nq) return;
    T* gi = g + 3 * i;
    if (isfinite(gi[0]) && isfinite(gi[1]) && isfinite(gi[2])) return;
    const float px = qx[i * qs], py = qy[i * qs], pz = qz[i * qs];
    const FarScale<T> fs = far_scale<T>(px, py, fabsf(pz), mv.g.scale);
    const double pzd = (double)((T)pz * fs.scf);
    double G[1][3];
    grad_run_axis<1>(mv, 0, mv.loop_off[mv.nloops], (double)((T)px * fs.scf), (double)((T)py * fs.scf), &pzd,
                     (double)fs.f, G);
    const double f = kInv2Pi * (double)fs.scf;
    for (int c = 0; c < 3; ++c) gi[(c + axis) % 3] = (T)(G[0][c] * f);
}

// ... and grid samples, t = n0 + thread in the frame's order (z fastest)
template <class T>
__global__ __launch_bounds__(256) void k_grad_fix_grid(MeshView mv, GridArgs ga, long long n0, long long n, int axis,
                                                       T* __restrict__ g) {
    const long long t = n0 + blockIdx.x * 256ll + threadIdx.x;
    if (t >= n) return;
    const long long k = t % ga.nz, col = t / ga.nz;
    const long long ci = col / ga.ny, cj = col - ci * ga.ny;
    T* gi = g + 3 * (ci * ga.st[0] + cj * ga.st[1] + k * ga.st[2]);
    if (isfinite(gi[0]) && isfinite(gi[1]) && isfinite(gi[2])) return;
    const float px = grid_coord(ga.o[0], ga.s[0], ci), py = grid_coord(ga.o[1], ga.s[1], cj);
    const float pz = grid_coord(ga.o[2], ga.s[2], k);
    const FarScale<T> fs = far_scale<T>(px, py, fabsf(pz), mv.g.scale);
    const double pzd = (double)((T)pz * fs.scf);
    double G[1][3];
    grad_run_axis<1>(mv, 0, mv.loop_off[mv.nloops], (double)((T)px * fs.scf), (double)((T)py * fs.scf), &pzd,
                     (double)fs.f, G);
    const double f = kInv2Pi * (double)fs.scf;
    for (int c = 0; c < 3; ++c) gi[(c + axis) % 3] = (T)(G[0][c] * f);
}

template <class T, int ZB>
gwn_status launch_grad_grid(const gwn_mesh_s* m, GridArgs ga, T* g, hipStream_t st) {
    ga.nchunks = (ga.nz + 64 * ZB - 1) / (64 * ZB);
    ga.nwaves = ga.nx * ga.ny * ga.nchunks;
    const long long kMaxWaves = max_launch_queries() / 64;   // 2^30 work-items per launch
    for (long long w0 = 0; w0 < ga.nwaves; w0 += kMaxWaves) {
        ga.wave0 = w0;
        const long long blocks = (std::min(kMaxWaves, ga.nwaves - w0) + kGridWaves - 1) / kGridWaves;
        k_grad_grid<T, ZB><<<(unsigned)blocks, 64 * kGridWaves, 0, st>>>(m->view(), ga, m->axis, g);
        GWN_HIP_TRY(hipGetLastError());
    }
    const long long ns = ga.nx * ga.ny * ga.nz, chunk = max_launch_queries();
    for (long long n0 = 0; n0 < ns; n0 += chunk) {
        const long long n = std::min(chunk, ns - n0);
        k_grad_fix_grid<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(m->view(), ga, n0, n0 + n, m->axis, g);
        GWN_HIP_TRY(hipGetLastError());
    }
    return GWN_OK;
}

}  // namespace

gwn_status query_grid_gradient(const gwn_mesh_s* m, const double* origin, const double* spacing, const int64_t* dims,
                               int prec, void* g, hipStream_t st) {
    GridArgs ga = frame_grid(m->axis, origin, spacing, dims);
    if (ga.nx == 0 || ga.ny == 0 || ga.nz == 0) return GWN_OK;
    // four samples per lane (two in FP64) share the column's x/y work
    if (prec == GWN_PREC_FP64) return launch_grad_grid<double, 2>(m, ga, (double*)g, st);
    return launch_grad_grid<float, 4>(m, ga, (float*)g, st);
}

gwn_status query_gradient(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qs,
                          int64_t nq, int prec, void* g, hipStream_t st) {
    const MeshView mv = m->view();
    axis_ptrs(m->axis, qx, qy, qz);
    const int64_t chunk = max_launch_queries();
    for (int64_t o = 0; o < nq; o += chunk) {
        const int64_t n = std::min<int64_t>(chunk, nq - o);
        const unsigned blocks = (unsigned)((n + 255) / 256);
        const float *x = qx + o * qs, *y = qy + o * qs, *z = qz + o * qs;
        if (want_split(m, n, -1)) {   // few points, many edges: a workgroup per point
            if (prec == GWN_PREC_FP64)
                k_grad_split<double><<<(unsigned)n, kSplitThreads, 0, st>>>(mv, x, y, z, qs, n, m->axis,
                                                                             (double*)g + 3 * o);
            else
                k_grad_split<float><<<(unsigned)n, kSplitThreads, 0, st>>>(mv, x, y, z, qs, n, m->axis,
                                                                            (float*)g + 3 * o);
        } else if (prec == GWN_PREC_FP64) {
            k_grad_batch<double><<<blocks, 256, 0, st>>>(mv, x, y, z, qs, n, m->axis, (double*)g + 3 * o);
        } else {
            k_grad_batch<float><<<blocks, 256, 0, st>>>(mv, x, y, z, qs, n, m->axis, (float*)g + 3 * o);
        }
        GWN_HIP_TRY(hipGetLastError());
        if (prec == GWN_PREC_FP64)
            k_grad_fix_points<double><<<blocks, 256, 0, st>>>(mv, x, y, z, qs, n, m->axis, (double*)g + 3 * o);
        else
            k_grad_fix_points<float><<<blocks, 256, 0, st>>>(mv, x, y, z, qs, n, m->axis, (float*)g + 3 * o);
        GWN_HIP_TRY(hipGetLastError());
    }
    return GWN_OK;
}

}  // namespace gwn
