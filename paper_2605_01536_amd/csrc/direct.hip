// direct.hip -- the direct sum of per-triangle signed solid angles (Eq. 2, with
// the triangle's area by Eq. 6 scaled by |a||b||c| > 0).  O(F) per query: the
// baseline the antipodal method is measured against (Sec. 5.1 compares with a
// GPU parallelisation of this sum), and an independent GPU cross-check of w.
//
// One lane per query; each 256-lane block walks one slice of the triangles in
// tiles of 256 staged through LDS (one coalesced load per lane, then broadcast
// reads).  When the queries alone cannot fill the chip, the triangle range is cut
// into slices whose per-query partial sums land in a workspace and are added in
// slice order by a second kernel (deterministic).
#include <algorithm>
#include <cmath>

#include "gwn_alloc.h"
#include "gwn_kernels.h"
#include "gwn_mesh.h"

namespace gwn {
namespace {

constexpr int kDirBlock = 256;

template <class T>
__device__ __forceinline__ T len3(T x, T y, T z) {
    return Arith<T>::sqrt(x * x + y * y + z * z);
}

// 2 atan2(num, den) / 2 of one triangle seen from p (half its signed solid angle)
template <class T>
__device__ __forceinline__ T half_omega(const float* t, T px, T py, T pz) {
    const T ax = (T)t[0] - px, ay = (T)t[1] - py, az = (T)t[2] - pz;
    const T bx = (T)t[3] - px, by = (T)t[4] - py, bz = (T)t[5] - pz;
    const T cx = (T)t[6] - px, cy = (T)t[7] - py, cz = (T)t[8] - pz;
    const T la = len3(ax, ay, az), lb = len3(bx, by, bz), lc = len3(cx, cy, cz);
    const T num = ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx);
    const T den = la * lb * lc + (ax * bx + ay * by + az * bz) * lc + (ax * cx + ay * cy + az * cz) * lb +
                  (bx * cx + by * cy + bz * cz) * la;
    // the small-argument polynomial when every lane of the wave allows it
    const bool slow = !(fabs(num) < Arith<T>::kFast * den);
    if (__builtin_amdgcn_ballot_w64(slow) == 0ull) return Arith<T>::atan_small(num * Arith<T>::rcp(den));
    return Arith<T>::atan2(num, den);
}

// block (bx, s): queries bx*256 .. +255, triangles [s*per, min(nf, (s+1)*per))
template <class T>
__global__ __launch_bounds__(kDirBlock) void k_direct(const float4* __restrict__ trif, long long nf, long long per,
                                                      const float* __restrict__ qx, const float* __restrict__ qy,
                                                      const float* __restrict__ qz, long long qs, long long nq,
                                                      T* __restrict__ w, double* __restrict__ part) {
    __shared__ float tile[kDirBlock * 9];
    const long long i = blockIdx.x * (long long)kDirBlock + threadIdx.x;
    const long long ii = i < nq ? i : nq - 1;
    const T px = (T)qx[ii * qs], py = (T)qy[ii * qs], pz = (T)qz[ii * qs];
    const long long t0 = (long long)blockIdx.y * per, t1 = min(nf, t0 + per);
    double S = 0.0;
    for (long long b = t0; b < t1; b += kDirBlock) {
        const int nt = (int)min((long long)kDirBlock, t1 - b);
        __syncthreads();
        if ((int)threadIdx.x < nt) {
            const long long t = b + threadIdx.x;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float4 v = trif[3 * t + c];
                tile[threadIdx.x * 9 + 3 * c] = v.x;
                tile[threadIdx.x * 9 + 3 * c + 1] = v.y;
                tile[threadIdx.x * 9 + 3 * c + 2] = v.z;
            }
        }
        __syncthreads();
        for (int k0 = 0; k0 < nt; k0 += 64) {   // FP32 partials of at most 64 terms
            const int k1 = min(nt, k0 + 64);
            T acc = (T)0;
            for (int k = k0; k < k1; ++k) acc += half_omega<T>(&tile[9 * k], px, py, pz);
            S += (double)acc;
        }
    }
    if (i < nq) {
        if (part) part[(long long)blockIdx.y * nq + i] = S;
        else w[i] = (T)(S * kInv2Pi);   // sum Omega / (4 pi), Omega = 2 atan2
    }
}

template <class T>
__global__ void k_direct_reduce(const double* __restrict__ part, int nslice, long long nq, T* __restrict__ w) {
    const long long i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= nq) return;
    double S = 0.0;
    for (int s = 0; s < nslice; ++s) S += part[(long long)s * nq + i];
    w[i] = (T)(S * kInv2Pi);
}

template <class T>
gwn_status launch_direct(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qs,
                         int64_t nq, T* w, hipStream_t st) {
    const long long qblocks = (nq + kDirBlock - 1) / kDirBlock;
    // aim for 8 waves per SIMD (256 CUs x 4 SIMDs x 8 = 2048 blocks of 4 waves),
    // with no slice shorter than 4 tiles
    const long long want = (2048 + qblocks - 1) / qblocks;
    const long long maxs = std::max<long long>(1, m->nf / (4 * kDirBlock));
    const int nslice = (int)std::min<long long>(std::min(want, maxs), 64);
    const long long per = ((m->nf + nslice - 1) / nslice + kDirBlock - 1) / kDirBlock * kDirBlock;
    double* part = nullptr;
    if (nslice > 1) GWN_HIP_TRY(gwn::dmalloc_async((void**)&part, sizeof(double) * (size_t)nslice * (size_t)nq, st));
    dim3 grid((unsigned)qblocks, (unsigned)nslice);
    k_direct<T><<<grid, kDirBlock, 0, st>>>(m->trif, m->nf, per, qx, qy, qz, qs, nq, w, part);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && part) {
        k_direct_reduce<T><<<(unsigned)((nq + 255) / 256), 256, 0, st>>>(part, nslice, nq, w);
        e = hipGetLastError();
    }
    if (part) (void)hipFreeAsync(part, st);
    GWN_HIP_TRY(e);
    return GWN_OK;
}

}  // namespace

gwn_status query_direct(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qs, int64_t nq,
                        int prec, void* w, hipStream_t st) {
    axis_ptrs(m->axis, qx, qy, qz);
    const int64_t chunk = max_launch_queries();
    for (int64_t o = 0; o < nq; o += chunk) {
        const int64_t n = std::min<int64_t>(chunk, nq - o);
        const float *x = qx + o * qs, *y = qy + o * qs, *z = qz + o * qs;
        const gwn_status s = prec == GWN_PREC_FP64 ? launch_direct<double>(m, x, y, z, qs, n, (double*)w + o, st)
                                                   : launch_direct<float>(m, x, y, z, qs, n, (float*)w + o, st);
        if (s != GWN_OK) return s;
    }
    return GWN_OK;
}

}  // namespace gwn
