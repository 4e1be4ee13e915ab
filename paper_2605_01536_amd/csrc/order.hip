// order.hip -- a traversal order for batches of arbitrary points.
//
// Lanes of one wave that trace nearby vertical lines visit the same BVH nodes.
// Visiting the points in Morton order of their quantised x, y (the ray is
// vertical: z does not matter) lets a wave walk the tree once, uniformly, for
// all its lanes (k_chi_wave).  The order only permutes which lane handles which
// point; every result is written to the point's own slot.
#include <hipcub/hipcub.hpp>

#include <cstdlib>

#include "gwn_internal.h"
#include "gwn_mesh.h"

namespace gwn {
namespace {

// 16 high bits of each quantised coordinate, interleaved (x in the even bits)
__device__ __forceinline__ uint32_t spread16(uint32_t v) {
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__global__ void k_xy_keys(const float* __restrict__ qx, const float* __restrict__ qy, const float* __restrict__ qz,
                          long long qs, long long n, QGrid g, uint32_t* __restrict__ key, int* __restrict__ idx) {
    const long long i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= n) return;
    const QPoint q = quantize_point(qx[i * qs], qy[i * qs], qz[i * qs], g);
    key[i] = q.inbox ? (spread16((uint32_t)q.x >> 14) | (spread16((uint32_t)q.y >> 14) << 1)) : 0xffffffffu;
    idx[i] = (int)i;
}

}  // namespace

// Worth it when the points are dense enough that a wave's 64 neighbours in
// Morton order trace nearly the same path: measured on the 1.05M-triangle soup,
// 2^20 random grid points go 3.4x faster, 2^16 (16x sparser) 25% slower.
bool want_xy_order(const gwn_mesh_s* m, int64_t n) {
    if (const char* e = std::getenv("GWN_ORDER_QUERIES")) return std::atoi(e) != 0 && n > 1;
    return n >= (1 << 18) && m->nf >= (1 << 15);
}

gwn_status xy_order(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qs, int64_t n,
                    int** perm_out, hipStream_t st) {
    *perm_out = nullptr;
    uint32_t *k0 = nullptr, *k1 = nullptr;
    int *i0 = nullptr, *i1 = nullptr;
    void* tmp = nullptr;
    size_t bytes = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, k0, k1, i0, i1, (int)n, 0, 32, st);
    if (e == hipSuccess) e = hipMallocAsync((void**)&k0, sizeof(uint32_t) * (size_t)n, st);
    if (e == hipSuccess) e = hipMallocAsync((void**)&k1, sizeof(uint32_t) * (size_t)n, st);
    if (e == hipSuccess) e = hipMallocAsync((void**)&i0, sizeof(int) * (size_t)n, st);
    if (e == hipSuccess) e = hipMallocAsync((void**)&i1, sizeof(int) * (size_t)n, st);
    if (e == hipSuccess) e = hipMallocAsync(&tmp, bytes, st);
    if (e == hipSuccess) {
        k_xy_keys<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(qx, qy, qz, qs, n, m->g, k0, i0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipcub::DeviceRadixSort::SortPairs(tmp, bytes, k0, k1, i0, i1, (int)n, 0, 32, st);
    if (tmp) (void)hipFreeAsync(tmp, st);
    if (k0) (void)hipFreeAsync(k0, st);
    if (k1) (void)hipFreeAsync(k1, st);
    if (i0) (void)hipFreeAsync(i0, st);
    if (e != hipSuccess) {
        if (i1) (void)hipFreeAsync(i1, st);
        GWN_HIP_TRY(e);
    }
    *perm_out = i1;
    return GWN_OK;
}

}  // namespace gwn
