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
// same code with r_z negated and the x, y components negated.
#include <algorithm>

#include "gwn_kernels.h"
#include "gwn_mesh.h"

namespace gwn {
namespace {

template <class T>
struct GVtx {
    T rx, ry, rz, l, u, s;   // offset from p, length, 1/length, l - r_z
};

// offsets in units of 2^e cells (f = 2^-e, see far_scale): each edge term is
// homogeneous of degree -1 in the offsets, so the sum is rescaled at the end
template <class T, bool FLIP>
__device__ __forceinline__ GVtx<T> gvtx(const BVert& b, T pxs, T pys, T pzs, T f) {
    GVtx<T> v;
    v.rx = fma((T)b.x, f, -pxs);
    v.ry = fma((T)b.y, f, -pys);
    v.rz = FLIP ? -fma((T)b.z, f, -pzs) : fma((T)b.z, f, -pzs);
    const T rho2 = v.rx * v.rx + v.ry * v.ry;
    v.l = Arith<T>::sqrt(v.rz * v.rz + rho2);
    v.u = Arith<T>::rcp(v.l);
    const T t = v.l + fabs(v.rz);
    v.s = v.rz > (T)0 ? rho2 * Arith<T>::rcp(t) : t;
    return v;
}

template <class T>
__device__ __forceinline__ void gedge(const GVtx<T>& a, const GVtx<T>& b, T& gx, T& gy, T& gz) {
    const T k = a.u * b.u;
    const T n = (a.ry * b.rx - a.rx * b.ry) * k;
    const T d = (a.s * b.s + a.rx * b.rx + a.ry * b.ry) * k;
    const T c0 = (T)1 + b.s * a.u, c1 = (T)1 + a.s * b.u;
    const T dDx = -(c0 * a.rx + c1 * b.rx);
    const T dDy = -(c0 * a.ry + c1 * b.ry);
    const T dDz = a.s * b.s * (a.u + b.u);
    const T f = k * Arith<T>::rcp(n * n + d * d);
    gx += (d * (b.ry - a.ry) - n * dDx) * f;
    gy += (d * (a.rx - b.rx) - n * dDy) * f;
    gz += (-n * dDz) * f;
}

// Sum over all loops of the edge terms, in cell units (FP32 partials flushed
// into FP64 every 32 edges).  FLIP: the mirrored sum for the axis x0 = -z.
template <class T, bool FLIP>
__device__ void grad_loops(const MeshView& mv, T pxs, T pys, T pzs, T f, double* G) {
    const BVert* __restrict__ bv = mv.bverts;
    G[0] = G[1] = G[2] = 0.0;
    for (int l = 0; l < mv.nloops; ++l) {
        const int b0 = mv.loop_off[l], b1 = mv.loop_off[l + 1];
        const GVtx<T> first = gvtx<T, FLIP>(bv[b0], pxs, pys, pzs, f);
        GVtx<T> prev = first;
        for (int j = b0 + 1; j <= b1; j += 32) {
            const int je = min(b1 + 1, j + 32);
            T gx = (T)0, gy = (T)0, gz = (T)0;
            for (int jj = j; jj < je; ++jj) {
                // index b1 closes the loop back to its first vertex
                const GVtx<T> cur = jj < b1 ? gvtx<T, FLIP>(bv[jj], pxs, pys, pzs, f) : first;
                gedge<T>(prev, cur, gx, gy, gz);
                prev = cur;
            }
            G[0] += (double)gx;
            G[1] += (double)gy;
            G[2] += (double)gz;
        }
    }
    if (FLIP) {
        G[0] = -G[0];
        G[1] = -G[1];
    }
}

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
    double G[3];
    grad_loops<T, false>(mv, pxs, pys, pzs, fs.f, G);
    if (!(isfinite(G[0]) && isfinite(G[1]) && isfinite(G[2]))) grad_loops<T, true>(mv, pxs, pys, pzs, fs.f, G);
    if (i < nq) {
        // sum of 2 atan2 terms over 4 pi, and the chain rule through p * 2^(k-e)
        const double f = kInv2Pi * (double)fs.scf;
        // frame component c is world component (c + axis) % 3
        for (int c = 0; c < 3; ++c) g[3 * i + (c + axis) % 3] = (T)(G[c] * f);
    }
}

}  // namespace

gwn_status query_gradient(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qs,
                          int64_t nq, int prec, void* g, hipStream_t st) {
    const MeshView mv = m->view();
    axis_ptrs(m->axis, qx, qy, qz);
    const int64_t chunk = max_launch_queries();
    for (int64_t o = 0; o < nq; o += chunk) {
        const int64_t n = std::min<int64_t>(chunk, nq - o);
        const unsigned blocks = (unsigned)((n + 255) / 256);
        const float *x = qx + o * qs, *y = qy + o * qs, *z = qz + o * qs;
        if (prec == GWN_PREC_FP64) k_grad_batch<double><<<blocks, 256, 0, st>>>(mv, x, y, z, qs, n, m->axis, (double*)g + 3 * o);
        else k_grad_batch<float><<<blocks, 256, 0, st>>>(mv, x, y, z, qs, n, m->axis, (float*)g + 3 * o);
        GWN_HIP_TRY(hipGetLastError());
    }
    return GWN_OK;
}

}  // namespace gwn
