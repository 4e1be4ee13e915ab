// direct.hip -- the direct sum of per-triangle signed solid angles (Eq. 2, with
// the triangle's area by Eq. 6 scaled by |a||b||c| > 0), one query per lane and
// every triangle streamed through scalar loads.  O(F) per query: the baseline
// the antipodal method is measured against (Sec. 6.1 compares with a GPU
// parallelisation of this sum), and an independent GPU cross-check of w.
#include <cmath>

#include <algorithm>

#include "gwn_kernels.h"
#include "gwn_mesh.h"

namespace gwn {
namespace {

template <class T>
__device__ __forceinline__ T len3(T x, T y, T z) {
    return Arith<T>::sqrt(x * x + y * y + z * z);
}

template <class T>
__global__ __launch_bounds__(256) void k_direct(const float4* __restrict__ trif, long long nf,
                                                const float* __restrict__ qx, const float* __restrict__ qy,
                                                const float* __restrict__ qz, long long qs, long long nq,
                                                T* __restrict__ w) {
    const long long i = blockIdx.x * 256ll + threadIdx.x;
    if (blockIdx.x * 256ll >= nq) return;
    const long long ii = i < nq ? i : nq - 1;
    const T px = (T)qx[ii * qs], py = (T)qy[ii * qs], pz = (T)qz[ii * qs];
    double S = 0.0;
    for (long long t0 = 0; t0 < nf; t0 += 64) {
        const long long t1 = min(nf, t0 + 64);
        T acc = (T)0;
        for (long long t = t0; t < t1; ++t) {
            const float4 A = trif[3 * t], B = trif[3 * t + 1], C = trif[3 * t + 2];
            const T ax = (T)A.x - px, ay = (T)A.y - py, az = (T)A.z - pz;
            const T bx = (T)B.x - px, by = (T)B.y - py, bz = (T)B.z - pz;
            const T cx = (T)C.x - px, cy = (T)C.y - py, cz = (T)C.z - pz;
            const T la = len3(ax, ay, az), lb = len3(bx, by, bz), lc = len3(cx, cy, cz);
            const T num = ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx);
            const T den = la * lb * lc + (ax * bx + ay * by + az * bz) * lc + (ax * cx + ay * cy + az * cz) * lb +
                          (bx * cx + by * cy + bz * cz) * la;
            // Omega/2 = atan2(num, den); the small-argument polynomial when every lane allows it
            const bool slow = !(fabs(num) < Arith<T>::kFast * den);
            if (__builtin_amdgcn_ballot_w64(slow) == 0ull) acc += Arith<T>::atan_small(num * Arith<T>::rcp(den));
            else acc += Arith<T>::atan2(num, den);
        }
        S += (double)acc;
    }
    if (i < nq) w[i] = (T)(S * (1.0 / 6.283185307179586476925));   // sum Omega / (4 pi), Omega = 2 atan2
}

}  // namespace

gwn_status query_direct(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qs, int64_t nq,
                        int prec, void* w, hipStream_t st) {
    const int64_t chunk = max_launch_queries();
    for (int64_t o = 0; o < nq; o += chunk) {
        const int64_t n = std::min<int64_t>(chunk, nq - o);
        const unsigned blocks = (unsigned)((n + 255) / 256);
        const float *x = qx + o * qs, *y = qy + o * qs, *z = qz + o * qs;
        if (prec == GWN_PREC_FP64) k_direct<double><<<blocks, 256, 0, st>>>(m->trif, m->nf, x, y, z, qs, n, (double*)w + o);
        else k_direct<float><<<blocks, 256, 0, st>>>(m->trif, m->nf, x, y, z, qs, n, (float*)w + o);
        GWN_HIP_TRY(hipGetLastError());
    }
    return GWN_OK;
}

}  // namespace gwn
