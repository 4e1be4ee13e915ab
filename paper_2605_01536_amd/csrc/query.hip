// query.hip -- single-mesh query kernels for arbitrary points: crossing counts
// and the boundary term per point (the arithmetic lives in gwn_kernels.h; the
// grid kernel with one ray per column is in grid.hip).
#include <cmath>
#include <cstdlib>
#include <type_traits>

#include <algorithm>

#include "gwn_alloc.h"
#include "gwn_kernels.h"
#include "gwn_mesh.h"

namespace gwn {
namespace {

// crossing counts of arbitrary points (per-lane LDS traversal stack)
__global__ __launch_bounds__(kChiBlock) void k_chi_batch(MeshView mv, const float* __restrict__ qx,
                                                         const float* __restrict__ qy, const float* __restrict__ qz,
                                                         long long qs, long long nq, int* __restrict__ chi) {
    __shared__ int stk[kLdsStack * kChiBlock];
    const long long i = blockIdx.x * (long long)kChiBlock + threadIdx.x;
    if (i >= nq) return;
    const QPoint q = quantize_point(qx[i * qs], qy[i * qs], qz[i * qs], mv.g);
    chi[i] = q.inbox ? chi_up(mv, q, stk + threadIdx.x) : 0;
}


// Crossing counts of Morton-ordered points, one wave-uniform traversal per wave
// (chi_wave_walk): neighbouring lines share almost their whole path, so the
// wave walks about one path instead of 64 divergent ones.  UP: the +z ray only
// (z-pruned); otherwise both directions of the whole line.
template <bool UP>
__global__ __launch_bounds__(64 * kGridWaves) void k_chi_wave(MeshView mv, const float* __restrict__ qx,
                                                             const float* __restrict__ qy,
                                                             const float* __restrict__ qz, long long qs, long long nq,
                                                             const int* __restrict__ perm, int* __restrict__ up,
                                                             int* __restrict__ down) {
    __shared__ int wstack[kGridWaves][kLdsStack];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const long long j = ((long long)blockIdx.x * kGridWaves + wave) * 64 + (threadIdx.x & 63);
    if ((long long)(blockIdx.x * kGridWaves + wave) * 64 >= nq) return;   // whole wave past the end
    const bool valid = j < nq;
    const long long i = perm[valid ? j : nq - 1];
    const QPoint q = quantize_point(qx[i * qs], qy[i * qs], qz[i * qs], mv.g);
    const bool act = valid && q.inbox;
    int u, d;
    chi_wave_walk<UP>(mv, q, act, wstack[wave], u, d);
    if (valid) {
        if (up) up[i] = u;
        if (down) down[i] = d;
    }
}

// both crossing counts of arbitrary points (the whole vertical line)
__global__ __launch_bounds__(kChiBlock) void k_chi_line(MeshView mv, const float* __restrict__ qx,
                                                        const float* __restrict__ qy, const float* __restrict__ qz,
                                                        long long qs, long long nq, int* __restrict__ up,
                                                        int* __restrict__ down) {
    __shared__ int stk[kLdsStack * kChiBlock];
    const long long i = blockIdx.x * (long long)kChiBlock + threadIdx.x;
    if (i >= nq) return;
    const QPoint q = quantize_point(qx[i * qs], qy[i * qs], qz[i * qs], mv.g);
    int u = 0, d = 0;
    if (q.inbox) chi_line(mv, q, stk + threadIdx.x, u, d);
    if (up) up[i] = u;
    if (down) down[i] = d;
}

// ---------------------------------------------------------------- boundary, batch

template <class T>
__global__ __launch_bounds__(256) void k_bdry_batch(MeshView mv, const float* __restrict__ qx, const float* __restrict__ qy,
                                                    const float* __restrict__ qz, long long qs, long long nq,
                                                    const int* __restrict__ perm, const int* __restrict__ chi,
                                                    T* __restrict__ w) {
    const long long j = blockIdx.x * 256ll + threadIdx.x;
    if (nq <= 0 || blockIdx.x * 256ll >= nq) return;
    const long long jj = j < nq ? j : nq - 1;
    // with a traversal order, lane j takes point perm[j]: the lanes of a wave are
    // neighbours in x/y, so an edge's pair test passes or fails for all of them
    const long long i = j < nq ? (perm ? (long long)perm[j] : j) : nq;
    const long long ii = perm ? (long long)perm[jj] : jj;
    const float px = qx[ii * qs], py = qy[ii * qs], pz = qz[ii * qs];
    const QPoint q = quantize_point(px, py, pz, mv.g);
    // lanes outside the fixed-point grid (rare) take the raw-offset loop
    double S = 0.0;
    if (q.inbox) {
        const T pzs = (T)pz * (T)mv.g.scale;
        boundary_loops<T, 1, false>(mv, q.x, q.y, (T)0, (T)0, &pzs, &S, (T)1, near_z(pz, mv.g));
    } else {
        const FarScale<T> fs = far_scale<T>(px, py, fabsf(pz), mv.g.scale);
        const T pzs = (T)pz * fs.scf;
        boundary_loops<T, 1, true>(mv, 0, 0, (T)px * fs.scf, (T)py * fs.scf, &pzs, &S, fs.f);
    }
    if (i < nq) w[i] = (T)((double)chi[i] + S * kInv2Pi);
}

// ---------------------------------------------------------------- boundary, split
// Few points against many boundary edges: one workgroup per point, each lane
// a contiguous run of boundary vertices (edge j leads from vertex j to the next
// vertex of its loop), the partial sums reduced across the wave by shuffles and
// across the workgroup in LDS, in a fixed order.  Fills the GPU where one lane
// per point would leave most of it idle.

constexpr int kSplitThreads = 256;

template <class T, bool FAR>
__device__ void split_run(const MeshView& mv, int a, int e, int qqx, int qqy, T pxs, T pys, T pzs, T f,
                          double* S) {
    if (a >= e) return;
    const BVert* __restrict__ bv = mv.bverts;
    ColV<T> cp;
    T sp;
    load_vertex<T, 1, FAR>(bv[a], qqx, qqy, pxs, pys, &pzs, f, cp, &sp);
    T acc = (T)0;
    int cnt = 0;
    for (int j = a; j < e; ++j) {
        const int lp = min(max(bv[j].loop, 0), mv.nloops - 1);   // in range for any stored value
        const int nx = j + 1 < mv.loop_off[lp + 1] ? j + 1 : mv.loop_off[lp];
        ColV<T> cn;
        T sn;
        load_vertex<T, 1, FAR>(bv[nx], qqx, qqy, pxs, pys, &pzs, f, cn, &sn);
        edge_step<T, 1, FAR>(cp, cn, &sp, &sn, &acc);
        if (++cnt == 32) {   // FP32 partials flushed into the FP64 sum every 32 edges
            *S += (double)acc;
            acc = (T)0;
            cnt = 0;
        }
        if (j + 1 < e) {
            if (nx == j + 1) {
                cp = cn;
                sp = sn;
            } else {   // the next edge starts a new loop
                load_vertex<T, 1, FAR>(bv[j + 1], qqx, qqy, pxs, pys, &pzs, f, cp, &sp);
            }
        }
    }
    *S += (double)acc;
}

template <class T>
__global__ __launch_bounds__(kSplitThreads) void k_bdry_split(MeshView mv, const float* __restrict__ qx,
                                                             const float* __restrict__ qy,
                                                             const float* __restrict__ qz, long long qs, long long nq,
                                                             const int* __restrict__ chi, T* __restrict__ w) {
    __shared__ double red[kSplitThreads / 64];
    const long long i = blockIdx.x;   // one point per workgroup
    if (i >= nq) return;
    const float px = qx[i * qs], py = qy[i * qs], pz = qz[i * qs];
    const QPoint q = quantize_point(px, py, pz, mv.g);
    const int nb = mv.loop_off[mv.nloops];
    const int per = (nb + kSplitThreads - 1) / kSplitThreads;
    const int a = (int)threadIdx.x * per, e = min(nb, a + per);
    double S = 0.0;
    if (q.inbox) {
        split_run<T, false>(mv, a, e, q.x, q.y, (T)0, (T)0,
                            (T)pz * (T)mv.g.scale * (T)EdgePairs<T, 1, false>::kUnit, (T)1, &S);
    } else {
        const FarScale<T> fs = far_scale<T>(px, py, fabsf(pz), mv.g.scale);
        split_run<T, true>(mv, a, e, 0, 0, (T)px * fs.scf, (T)py * fs.scf, (T)pz * fs.scf, fs.f, &S);
    }
    for (int o = 32; o > 0; o >>= 1) S += __shfl_xor(S, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = S;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kSplitThreads / 64; ++k) t += red[k];
        w[i] = (T)((double)chi[i] + t * kInv2Pi);
    }
}

// ws (nullable): caller memory for the temporaries -- a crossing-count buffer
// when chi_out is null, the traversal order and its sort's scratch -- for at
// most one launch's worth of points; without it they are stream-ordered
// allocations.
template <class T>
gwn_status launch_batch(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qs, int64_t nq,
                        T* w, int32_t* chi_out, const BatchWorkspace* ws, hipStream_t st) {
    int* chi = chi_out;
    if (!chi) {
        if (ws) chi = ws->chi;
        else GWN_HIP_TRY(gwn::dmalloc_async((void**)&chi, sizeof(int) * (size_t)nq, st));
    }
    const bool own_chi = !chi_out && !ws;
    const MeshView mv = m->view();
    hipError_t e = hipSuccess;
    // one launch covers at most max_launch_queries() points (the 32-bit grid size)
    const int64_t chunk = max_launch_queries();
    for (int64_t o = 0; o < nq && e == hipSuccess; o += chunk) {
        const int64_t n = std::min<int64_t>(chunk, nq - o);
        const float *x = qx + o * qs, *y = qy + o * qs, *z = qz + o * qs;
        int* perm = nullptr;
        if (want_xy_order(m, n)) {
            const gwn_status so = ws ? xy_order_into(m, x, y, z, qs, n, ws->perm, ws->order_temp, st)
                                     : xy_order(m, x, y, z, qs, n, &perm, st);
            if (so != GWN_OK) {
                if (own_chi) (void)hipFreeAsync(chi, st);
                return so;   // the order has set the message
            }
            if (ws) perm = ws->perm;
        }
        if (perm) {
            k_chi_wave<true><<<(unsigned)((n + 64 * kGridWaves - 1) / (64 * kGridWaves)), 64 * kGridWaves, 0, st>>>(
                mv, x, y, z, qs, n, perm, chi + o, nullptr);
        } else {
            k_chi_batch<<<(unsigned)((n + kChiBlock - 1) / kChiBlock), kChiBlock, 0, st>>>(mv, x, y, z, qs, n,
                                                                                           chi + o);
        }
        e = hipGetLastError();
        if (e == hipSuccess) {
            if (want_split(m, n, sizeof(T) == 8 ? GWN_PREC_FP64 : GWN_PREC_FP32))
                k_bdry_split<T><<<(unsigned)n, kSplitThreads, 0, st>>>(mv, x, y, z, qs, n, chi + o, w + o);
            else
                k_bdry_batch<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(mv, x, y, z, qs, n, perm, chi + o,
                                                                             w + o);
            e = hipGetLastError();
        }
        if (perm && !ws) (void)hipFreeAsync(perm, st);
    }
    if (own_chi) (void)hipFreeAsync(chi, st);
    GWN_HIP_TRY(e);
    return GWN_OK;
}

}  // namespace

gwn_status query_crossings(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qs,
                           int64_t nq, int32_t* up, int32_t* down, hipStream_t st) {
    axis_ptrs(m->axis, qx, qy, qz);
    const MeshView mv = m->view();
    const int64_t chunk = max_launch_queries();
    for (int64_t o = 0; o < nq; o += chunk) {
        const int64_t n = std::min<int64_t>(chunk, nq - o);
        const float *x = qx + o * qs, *y = qy + o * qs, *z = qz + o * qs;
        int* perm = nullptr;
        if (want_xy_order(m, n)) {
            const gwn_status so = xy_order(m, x, y, z, qs, n, &perm, st);
            if (so != GWN_OK) return so;
        }
        if (perm) {
            k_chi_wave<false><<<(unsigned)((n + 64 * kGridWaves - 1) / (64 * kGridWaves)), 64 * kGridWaves, 0, st>>>(
                mv, x, y, z, qs, n, perm, up ? up + o : nullptr, down ? down + o : nullptr);
        } else {
            k_chi_line<<<(unsigned)((n + kChiBlock - 1) / kChiBlock), kChiBlock, 0, st>>>(
                mv, x, y, z, qs, n, up ? up + o : nullptr, down ? down + o : nullptr);
        }
        const hipError_t e = hipGetLastError();
        if (perm) (void)hipFreeAsync(perm, st);
        GWN_HIP_TRY(e);
    }
    return GWN_OK;
}

bool want_split(const gwn_mesh_s* m, int64_t n, int prec) {
    if (const char* e = std::getenv("GWN_SPLIT_BOUNDARY")) return std::atoi(e) != 0 && m->nb > 0;
    if (prec >= 0 && prec < 2 && m->split_max[prec] != 0) return m->split_max[prec] > 0 && n <= m->split_max[prec] && m->nb > 0;
    return n <= 8192 && m->nb >= 16 * 256;
}

int64_t max_launch_queries() {
    int64_t n = int64_t(1) << 30;
    if (const char* e = std::getenv("GWN_MAX_LAUNCH_QUERIES")) {
        const long long v = std::atoll(e);
        if (v >= 256 && v < n && v % 256 == 0) n = v;
    }
    return n;
}

gwn_status query_batch(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qs, int64_t nq,
                       int prec, void* w, int32_t* chi_out, hipStream_t st) {
    return query_batch_ws(m, qx, qy, qz, qs, nq, prec, w, chi_out, nullptr, st);
}

gwn_status query_batch_ws(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qs,
                          int64_t nq, int prec, void* w, int32_t* chi_out, const BatchWorkspace* ws, hipStream_t st) {
    if (nq == 0) return GWN_OK;
    if (ws && nq > max_launch_queries()) {
        set_error("query_batch: a workspace covers one launch of at most %lld points", (long long)max_launch_queries());
        return GWN_E_INVALID;
    }
    axis_ptrs(m->axis, qx, qy, qz);
    if (prec == GWN_PREC_FP64) return launch_batch<double>(m, qx, qy, qz, qs, nq, (double*)w, chi_out, ws, st);
    return launch_batch<float>(m, qx, qy, qz, qs, nq, (float*)w, chi_out, ws, st);
}

}  // namespace gwn
