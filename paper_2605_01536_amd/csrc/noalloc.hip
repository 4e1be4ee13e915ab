// noalloc.hip -- gwn_query_batch_noalloc: the batch query with every
// temporary in one file-scope device array, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).
//
// The array `scratch` exists once per GPU the library is loaded on and lives
// until the process ends.  Host code never passes its name to a kernel (on the
// host it is only a stand-in for the symbol): the first call on each device
// looks up that device's address with hipGetSymbolAddress, with the device
// current, and every later call on it uses the stored address.
#include <mutex>

#include "gwn_mesh.h"

namespace {

// the largest batch the scratch serves, and the scratch: crossing counts, the
// traversal order and its sort's temporaries for that many points (28.3 MiB)
constexpr int64_t kMaxPoints = GWN_NOALLOC_MAX_POINTS;
constexpr size_t kScratchBytes = (size_t)29 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// byte layout of the scratch for n points: chi, perm, the order's temporaries
size_t layout(int64_t n, size_t* off_perm, size_t* off_order) {
    const size_t ints = round256(sizeof(int) * (size_t)n);
    *off_perm = ints;
    *off_order = 2 * ints;
    return 2 * ints + gwn::xy_order_temp_bytes(n);
}

// this device's copy of `scratch` (the current device; looked up once)
gwn_status scratch_of(int dev, unsigned char** out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (dev < 0 || dev >= kMaxDevices) {
        gwn::set_error("gwn_query_batch_noalloc: device %d beyond the %d the scratch table holds", dev, kMaxDevices);
        return GWN_E_UNSUPPORTED;
    }
    if (!g_scratch[dev]) {
        size_t a, b;
        if (layout(kMaxPoints, &a, &b) > kScratchBytes) {
            gwn::set_error("gwn_query_batch_noalloc: the scratch array is too small for %lld points",
                           (long long)kMaxPoints);
            return GWN_E_UNSUPPORTED;
        }
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            gwn::set_error("gwn_query_batch_noalloc: hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                           hipGetErrorString(e));
            return GWN_E_HIP;
        }
        g_scratch[dev] = p;
    }
    *out = (unsigned char*)g_scratch[dev];
    return GWN_OK;
}

}  // namespace

extern "C" gwn_status gwn_query_batch_noalloc(gwn_mesh m, const float* qx, const float* qy, const float* qz,
                                              int64_t qstride, int64_t nq, int32_t prec, void* w_out,
                                              int32_t* chi_out, void* stream) {
    gwn::clear_error();
    if (!m) {
        gwn::set_error("gwn_query_batch_noalloc: null mesh handle");
        return GWN_E_INVALID;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m->device) {
        gwn::set_error("gwn_query_batch_noalloc: mesh was built on device %d, current device is %d", m->device, dev);
        return GWN_E_INVALID;
    }
    if (nq < 0 || qstride < 1 || (prec != GWN_PREC_FP32 && prec != GWN_PREC_FP64)) {
        gwn::set_error("gwn_query_batch_noalloc: bad nq=%lld, qstride=%lld or precision %d", (long long)nq,
                       (long long)qstride, (int)prec);
        return GWN_E_INVALID;
    }
    if (nq > kMaxPoints) {
        gwn::set_error("gwn_query_batch_noalloc: %lld points exceed the maximum of %lld per call (split the batch, "
                       "or use gwn_query_batch)", (long long)nq, (long long)kMaxPoints);
        return GWN_E_INVALID;
    }
    if (nq == 0) return GWN_OK;
    if (!qx || !qy || !qz || !w_out) {
        gwn::set_error("gwn_query_batch_noalloc: null query or output array");
        return GWN_E_INVALID;
    }
    unsigned char* base = nullptr;
    gwn_status s = scratch_of(dev, &base);
    if (s != GWN_OK) return s;
    size_t off_perm, off_order;
    layout(nq, &off_perm, &off_order);
    gwn::BatchWorkspace ws;
    ws.chi = (int*)base;
    ws.perm = (int*)(base + off_perm);
    ws.order_temp = base + off_order;
    return gwn::query_batch_ws(m, qx, qy, qz, qstride, nq, prec, w_out, chi_out, &ws, (hipStream_t)stream);
}
