// api.hip -- extern "C" entry points declared in include/gwn.h: argument
// validation, handle lifetime and thread-local error reporting.  All compute
// happens in the kernels of the other sources (build, query, grad, direct,
// order, multi, mlp).
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cmath>
#include <new>

#include "../../include/gwn_test.h"
#include "gwn_alloc.h"
#include "gwn_mesh.h"

namespace gwn {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

// ---- device allocations and the allocation-failure hook (include/gwn_test.h)
namespace {
std::atomic<long long> g_alloc_budget{-1};   // < 0: no failures; else allocations left before they fail
std::atomic<long long> g_alloc_count{0};

bool take_alloc() {
    g_alloc_count.fetch_add(1, std::memory_order_relaxed);
    long long b = g_alloc_budget.load(std::memory_order_relaxed);
    while (b >= 0) {
        if (b == 0) return false;
        if (g_alloc_budget.compare_exchange_weak(b, b - 1, std::memory_order_relaxed)) return true;
    }
    return true;
}
}  // namespace

hipError_t dmalloc(void** p, size_t bytes) {
    if (!take_alloc()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

hipError_t dmalloc_async(void** p, size_t bytes, hipStream_t st) {
    if (!take_alloc()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMallocAsync(p, bytes, st);
}

}  // namespace gwn

namespace {

void release(gwn_mesh_s* m) {
    if (!m) return;
    (void)hipFree(m->nodes);
    (void)hipFree(m->tris);
    (void)hipFree(m->trif);
    (void)hipFree(m->bverts);
    (void)hipFree(m->loop_off);
    delete m;
}

gwn_status check_mesh(gwn_mesh m, const char* fn) {
    if (!m) {
        gwn::set_error("%s: null mesh handle", fn);
        return GWN_E_INVALID;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m->device) {
        gwn::set_error("%s: mesh was built on device %d, current device is %d", fn, m->device, dev);
        return GWN_E_INVALID;
    }
    return GWN_OK;
}

}  // namespace

extern "C" {

int64_t gwn_test_fail_alloc_after(int64_t n) {
    gwn::g_alloc_budget.store(n < 0 ? -1 : n);
    return gwn::g_alloc_count.exchange(0);
}

gwn_status gwn_build_mesh(const float* vx, const float* vy, const float* vz, int64_t vstride, int64_t nv,
                          const int32_t* tri, int64_t nf, void* stream, gwn_mesh* out) {
    return gwn_build_mesh_opts(vx, vy, vz, vstride, nv, tri, nf, nullptr, stream, out);
}

gwn_status gwn_build_mesh_opts(const float* vx, const float* vy, const float* vz, int64_t vstride, int64_t nv,
                               const int32_t* tri, int64_t nf, const gwn_build_opts* opts, void* stream,
                               gwn_mesh* out) {
    gwn::clear_error();
    if (!out) {
        gwn::set_error("gwn_build_mesh: out is null");
        return GWN_E_INVALID;
    }
    *out = nullptr;
    if (nv < 0 || nf < 0 || vstride < 1 || nv >= (1ll << 31) || nf >= (1ll << 29)) {
        gwn::set_error("gwn_build_mesh: bad sizes nv=%lld nf=%lld vstride=%lld", (long long)nv, (long long)nf,
                       (long long)vstride);
        return GWN_E_INVALID;
    }
    if ((nv > 0 && (!vx || !vy || !vz)) || (nf > 0 && !tri)) {
        gwn::set_error("gwn_build_mesh: null array with nonzero size");
        return GWN_E_INVALID;
    }
    if (nf > 0 && nv == 0) {
        gwn::set_error("gwn_build_mesh: triangles given without vertices");
        return GWN_E_INVALID;
    }
    const bool weld = opts && opts->weld_positions;
    // public codes: 0 = z, 1 = x, 2 = y, -1 = choose; the same as the internal ones
    const int axis = opts ? opts->axis : 0;
    if (axis < -1 || axis > 2) {
        gwn::set_error("gwn_build_mesh_opts: axis must be -1, 0 (z), 1 (x) or 2 (y), got %d", axis);
        return GWN_E_INVALID;
    }
    gwn_mesh_s* m = new (std::nothrow) gwn_mesh_s();
    if (!m) {
        gwn::set_error("gwn_build_mesh: host allocation failed");
        return GWN_E_OOM;
    }
    gwn_status s = gwn::build_mesh(vx, vy, vz, vstride, nv, tri, nf, weld, axis, (hipStream_t)stream, m);
    if (s == GWN_OK && m->depth > gwn::kLdsStack - 1) {
        gwn::set_error("gwn_build_mesh: BVH depth %d exceeds the traversal stack", m->depth);
        s = GWN_E_UNSUPPORTED;
    }
    if (s != GWN_OK) {
        release(m);
        return s;
    }
    *out = m;
    return GWN_OK;
}

gwn_status gwn_mesh_info_get(gwn_mesh m, gwn_mesh_info* out) {
    gwn::clear_error();
    if (!m || !out) {
        gwn::set_error("gwn_mesh_info_get: null argument");
        return GWN_E_INVALID;
    }
    out->nv = m->nv;
    out->nf = m->nf;
    out->nboundary = m->nb;
    out->nloops = m->nloops;
    out->nnodes = m->nnodes;
    out->bvh_depth = m->depth;
    out->qshift = m->g.k;
    // the mesh keeps its data in its axis frame: frame component c is world (c + axis) % 3
    for (int c = 0; c < 3; ++c) {
        const int a = (c + m->axis) % 3;
        out->bbox[a] = m->bbox[c];
        out->bbox[3 + a] = m->bbox[3 + c];
        out->qlo[a] = m->g.lo[c];
    }
    out->build_ms = m->build_ms;
    out->nunique = m->nunique;
    out->axis = m->axis;
    for (int a = 0; a < 3; ++a) out->proj_area[a] = m->proj_area[a];
    return GWN_OK;
}

gwn_status gwn_mesh_destroy(gwn_mesh m) {
    gwn::clear_error();
    release(m);
    return GWN_OK;
}

gwn_status gwn_query_batch(gwn_mesh m, const float* qx, const float* qy, const float* qz, int64_t qstride, int64_t nq,
                           int32_t prec, void* w_out, int32_t* chi_out, void* stream) {
    gwn::clear_error();
    gwn_status s = check_mesh(m, "gwn_query_batch");
    if (s != GWN_OK) return s;
    if (nq < 0 || qstride < 1 || (prec != GWN_PREC_FP32 && prec != GWN_PREC_FP64)) {
        gwn::set_error("gwn_query_batch: bad nq=%lld, qstride=%lld or precision %d", (long long)nq,
                       (long long)qstride, (int)prec);
        return GWN_E_INVALID;
    }
    if (nq == 0) return GWN_OK;
    if (!qx || !qy || !qz || !w_out) {
        gwn::set_error("gwn_query_batch: null query or output array");
        return GWN_E_INVALID;
    }
    if (nq > (1ll << 40)) {
        gwn::set_error("gwn_query_batch: nq too large");
        return GWN_E_INVALID;
    }
    return gwn::query_batch(m, qx, qy, qz, qstride, nq, prec, w_out, chi_out, (hipStream_t)stream);
}

// shared checks of the grid entry points; *empty is set for a zero-size grid
static gwn_status check_grid(const char* who, const double* origin, const double* spacing, const int64_t* dims,
                             int32_t prec, const void* out, bool* empty) {
    if (!origin || !spacing || !dims || (prec != GWN_PREC_FP32 && prec != GWN_PREC_FP64)) {
        gwn::set_error("%s: null grid description or bad precision", who);
        return GWN_E_INVALID;
    }
    for (int a = 0; a < 3; ++a) {
        if (dims[a] < 0 || dims[a] > (1ll << 20) || !std::isfinite(origin[a]) || !std::isfinite(spacing[a])) {
            gwn::set_error("%s: bad dims/origin/spacing on axis %d", who, a);
            return GWN_E_INVALID;
        }
    }
    *empty = dims[0] * dims[1] * dims[2] == 0;
    if (!*empty && !out) {
        gwn::set_error("%s: null output array", who);
        return GWN_E_INVALID;
    }
    return GWN_OK;
}

gwn_status gwn_query_grid(gwn_mesh m, const double* origin, const double* spacing, const int64_t* dims, int32_t prec,
                          void* w_out, int32_t* chi_out, void* stream) {
    gwn::clear_error();
    gwn_status s = check_mesh(m, "gwn_query_grid");
    if (s != GWN_OK) return s;
    bool empty = false;
    s = check_grid("gwn_query_grid", origin, spacing, dims, prec, w_out, &empty);
    if (s != GWN_OK || empty) return s;
    return gwn::query_grid(m, origin, spacing, dims, prec, w_out, chi_out, (hipStream_t)stream);
}

gwn_status gwn_query_grid_gradient(gwn_mesh m, const double* origin, const double* spacing, const int64_t* dims,
                                   int32_t prec, void* grad_out, void* stream) {
    gwn::clear_error();
    gwn_status s = check_mesh(m, "gwn_query_grid_gradient");
    if (s != GWN_OK) return s;
    bool empty = false;
    s = check_grid("gwn_query_grid_gradient", origin, spacing, dims, prec, grad_out, &empty);
    if (s != GWN_OK || empty) return s;
    return gwn::query_grid_gradient(m, origin, spacing, dims, prec, grad_out, (hipStream_t)stream);
}

gwn_status gwn_query_crossings(gwn_mesh m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                               int64_t nq, int32_t* chi_up_out, int32_t* chi_down_out, void* stream) {
    gwn::clear_error();
    gwn_status s = check_mesh(m, "gwn_query_crossings");
    if (s != GWN_OK) return s;
    if (nq < 0 || qstride < 1) {
        gwn::set_error("gwn_query_crossings: bad nq or stride");
        return GWN_E_INVALID;
    }
    if (nq == 0) return GWN_OK;
    if (!qx || !qy || !qz || (!chi_up_out && !chi_down_out) || nq > (1ll << 40)) {
        gwn::set_error("gwn_query_crossings: null array (one output may be null, not both) or nq too large");
        return GWN_E_INVALID;
    }
    return gwn::query_crossings(m, qx, qy, qz, qstride, nq, chi_up_out, chi_down_out, (hipStream_t)stream);
}

gwn_status gwn_query_gradient(gwn_mesh m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                              int64_t nq, int32_t prec, void* grad_out, void* stream) {
    gwn::clear_error();
    gwn_status s = check_mesh(m, "gwn_query_gradient");
    if (s != GWN_OK) return s;
    if (nq < 0 || qstride < 1 || (prec != GWN_PREC_FP32 && prec != GWN_PREC_FP64)) {
        gwn::set_error("gwn_query_gradient: bad nq, stride or precision");
        return GWN_E_INVALID;
    }
    if (nq == 0) return GWN_OK;
    if (!qx || !qy || !qz || !grad_out || nq > (1ll << 40)) {
        gwn::set_error("gwn_query_gradient: null array or nq too large");
        return GWN_E_INVALID;
    }
    return gwn::query_gradient(m, qx, qy, qz, qstride, nq, prec, grad_out, (hipStream_t)stream);
}

gwn_status gwn_query_direct(gwn_mesh m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                            int64_t nq, int32_t prec, void* w_out, void* stream) {
    gwn::clear_error();
    gwn_status s = check_mesh(m, "gwn_query_direct");
    if (s != GWN_OK) return s;
    if (nq < 0 || qstride < 1 || (prec != GWN_PREC_FP32 && prec != GWN_PREC_FP64)) {
        gwn::set_error("gwn_query_direct: bad nq, stride or precision");
        return GWN_E_INVALID;
    }
    if (nq == 0) return GWN_OK;
    if (!qx || !qy || !qz || !w_out || nq > (1ll << 40)) {
        gwn::set_error("gwn_query_direct: null array or nq too large");
        return GWN_E_INVALID;
    }
    return gwn::query_direct(m, qx, qy, qz, qstride, nq, prec, w_out, (hipStream_t)stream);
}

gwn_status gwn_multi_create(const gwn_mesh* meshes, int32_t nmesh, const float* qx, const float* qy,
                            const float* qz, int64_t qstride, const int64_t* q_offsets, int32_t prec, void* w_out,
                            int32_t* chi_out, const gwn_multi_opts* opts, void* stream, gwn_multi* out) {
    gwn::clear_error();
    if (!out || !meshes || !q_offsets || nmesh < 1 || qstride < 1 ||
        (prec != GWN_PREC_FP32 && prec != GWN_PREC_FP64)) {
        gwn::set_error("gwn_multi_create: null argument, nmesh < 1, qstride < 1 or unknown prec");
        return GWN_E_INVALID;
    }
    *out = nullptr;
    if (q_offsets[0] != 0) {
        gwn::set_error("gwn_multi_create: q_offsets[0] must be 0");
        return GWN_E_INVALID;
    }
    for (int m = 0; m < nmesh; ++m) {
        gwn_status s = check_mesh(meshes[m], "gwn_multi_create");
        if (s != GWN_OK) return s;
        if (q_offsets[m + 1] < q_offsets[m]) {
            gwn::set_error("gwn_multi_create: q_offsets must be non-decreasing (at mesh %d)", m);
            return GWN_E_INVALID;
        }
    }
    if (q_offsets[nmesh] > 0 && (!qx || !qy || !qz || !w_out)) {
        gwn::set_error("gwn_multi_create: null query or output array");
        return GWN_E_INVALID;
    }
    if (q_offsets[nmesh] > (1ll << 40)) {
        gwn::set_error("gwn_multi_create: too many queries");
        return GWN_E_INVALID;
    }
    if (opts && (opts->order < 0 || opts->order > 3)) {
        gwn::set_error("gwn_multi_create: opts->order must be 0, 1, 2 or 3");
        return GWN_E_INVALID;
    }
    return gwn::multi_create(meshes, nmesh, qx, qy, qz, qstride, q_offsets, prec, w_out, chi_out, opts,
                             (hipStream_t)stream, out);
}

gwn_status gwn_multi_run(gwn_multi plan, void* stream) {
    gwn::clear_error();
    if (!plan) {
        gwn::set_error("gwn_multi_run: null plan");
        return GWN_E_INVALID;
    }
    return gwn::multi_run(plan, (hipStream_t)stream);
}

gwn_status gwn_multi_info_get(gwn_multi plan, gwn_multi_info* out) {
    gwn::clear_error();
    if (!plan || !out) {
        gwn::set_error("gwn_multi_info_get: null argument");
        return GWN_E_INVALID;
    }
    gwn::multi_info(plan, out);
    return GWN_OK;
}

gwn_status gwn_multi_destroy(gwn_multi plan) {
    gwn::clear_error();
    gwn::multi_destroy(plan);
    return GWN_OK;
}

static gwn_status check_points(const char* fn, const float* qx, const float* qy, const float* qz, int64_t qs,
                               int64_t n, const void* out) {
    if (n < 0 || n >= (1ll << 31) || qs < 1) {
        gwn::set_error("%s: bad n=%lld or stride=%lld", fn, (long long)n, (long long)qs);
        return GWN_E_INVALID;
    }
    if (n > 0 && (!qx || !qy || !qz || !out)) {
        gwn::set_error("%s: null point or output array", fn);
        return GWN_E_INVALID;
    }
    return GWN_OK;
}

static gwn_status check_mlp(gwn_mlp h, const char* fn) {
    if (!h) {
        gwn::set_error("%s: null handle", fn);
        return GWN_E_INVALID;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != gwn::mlp_device(h)) {
        gwn::set_error("%s: the network was created on device %d, current device is %d", fn, gwn::mlp_device(h), dev);
        return GWN_E_INVALID;
    }
    return GWN_OK;
}

gwn_status gwn_mlp_create(uint64_t seed, double fourier_sigma, gwn_mlp* out) {
    gwn::clear_error();
    if (!out || !(fourier_sigma > 0.0) || !std::isfinite(fourier_sigma)) {
        gwn::set_error("gwn_mlp_create: null out or bad sigma");
        return GWN_E_INVALID;
    }
    *out = nullptr;
    return gwn::mlp_create(seed, fourier_sigma, out);
}

gwn_status gwn_mlp_destroy(gwn_mlp h) {
    gwn::clear_error();
    gwn::mlp_release(h);
    return GWN_OK;
}

gwn_status gwn_mlp_get_state(gwn_mlp h, float* theta, float* m, float* v, float* G, int64_t* step) {
    gwn::clear_error();
    gwn_status s = check_mlp(h, "gwn_mlp_get_state");
    return s != GWN_OK ? s : gwn::mlp_get_state(h, theta, m, v, G, step);
}

gwn_status gwn_mlp_set_state(gwn_mlp h, const float* theta, const float* m, const float* v, const float* G,
                             int64_t step) {
    gwn::clear_error();
    gwn_status s = check_mlp(h, "gwn_mlp_set_state");
    return s != GWN_OK ? s : gwn::mlp_set_state(h, theta, m, v, G, step);
}

gwn_status gwn_mlp_forward(gwn_mlp h, const float* qx, const float* qy, const float* qz, int64_t qs, int64_t n,
                           float* y, void* stream) {
    gwn::clear_error();
    gwn_status s = check_mlp(h, "gwn_mlp_forward");
    if (s == GWN_OK) s = check_points("gwn_mlp_forward", qx, qy, qz, qs, n, y);
    return s != GWN_OK ? s : gwn::mlp_forward(h, qx, qy, qz, qs, n, y, (hipStream_t)stream);
}

gwn_status gwn_mlp_loss_grad(gwn_mlp h, const float* qx, const float* qy, const float* qz, int64_t qs,
                             const float* target, int64_t n, float* grad_out, float* loss_out, void* stream) {
    gwn::clear_error();
    gwn_status s = check_mlp(h, "gwn_mlp_loss_grad");
    if (s == GWN_OK) s = check_points("gwn_mlp_loss_grad", qx, qy, qz, qs, n, target);
    if (s == GWN_OK && n == 0) {
        gwn::set_error("gwn_mlp_loss_grad: empty batch");
        s = GWN_E_INVALID;
    }
    return s != GWN_OK ? s : gwn::mlp_loss_grad(h, qx, qy, qz, qs, target, n, grad_out, loss_out, (hipStream_t)stream);
}

gwn_status gwn_mlp_train_step(gwn_mlp h, const float* qx, const float* qy, const float* qz, int64_t qs,
                              const float* target, int64_t n, float lr, float* loss_out, void* stream) {
    gwn::clear_error();
    gwn_status s = check_mlp(h, "gwn_mlp_train_step");
    if (s == GWN_OK) s = check_points("gwn_mlp_train_step", qx, qy, qz, qs, n, target);
    if (s == GWN_OK && (n == 0 || !(lr >= 0.f))) {
        gwn::set_error("gwn_mlp_train_step: empty batch or bad learning rate");
        s = GWN_E_INVALID;
    }
    return s != GWN_OK ? s : gwn::mlp_train_step(h, qx, qy, qz, qs, target, n, lr, loss_out, (hipStream_t)stream);
}

gwn_status gwn_surrogate_query(gwn_mlp h, gwn_mesh mesh, const float* qx, const float* qy, const float* qz, int64_t qs,
                               int64_t n, float band, int32_t rule, float* w_out, uint8_t* fallback_out,
                               int64_t* nfallback_out, void* stream) {
    gwn::clear_error();
    gwn_status s = check_mlp(h, "gwn_surrogate_query");
    if (s == GWN_OK) s = check_mesh(mesh, "gwn_surrogate_query");
    if (s == GWN_OK) s = check_points("gwn_surrogate_query", qx, qy, qz, qs, n, w_out);
    if (s == GWN_OK && (!(band >= 0.f) || (rule != GWN_BAND_HALF && rule != GWN_BAND_FRAC))) {
        gwn::set_error("gwn_surrogate_query: band must be >= 0 and rule 0 or 1 (got %g, %d)", (double)band, rule);
        s = GWN_E_INVALID;
    }
    return s != GWN_OK ? s
                       : gwn::surrogate_query(h, mesh, qx, qy, qz, qs, n, band, rule, w_out, fallback_out,
                                              nfallback_out, (hipStream_t)stream);
}

gwn_status gwn_surrogate_train(gwn_surrogate h, gwn_mesh mesh, const gwn_surrogate_cfg* cfg, const float* X,
                               const float* T, int64_t n, float* epoch_loss, int64_t* epochs_run, void* stream) {
    gwn::clear_error();
    if (epochs_run) *epochs_run = 0;
    gwn_status s = check_mlp(h, "gwn_surrogate_train");
    if (s != GWN_OK) return s;
    if (!cfg) {
        gwn::set_error("gwn_surrogate_train: null cfg");
        return GWN_E_INVALID;
    }
    const gwn_surrogate_cfg& c = *cfg;
    const int64_t npts = X ? n : c.n_train;
    if (npts < 1 || npts >= (1ll << 31) || c.batch < 1 || c.epochs < 1 || c.stop_epoch < 0 ||
        !(c.lr >= 0.f) || !std::isfinite(c.lr) || !(c.lr_final >= 0.f) || !std::isfinite(c.lr_final)) {
        gwn::set_error("gwn_surrogate_train: bad configuration (points %lld, batch %d, epochs %d, stop %d, lr %g, "
                       "lr_final %g)", (long long)npts, c.batch, c.epochs, c.stop_epoch, (double)c.lr,
                       (double)c.lr_final);
        return GWN_E_INVALID;
    }
    if (!X) {
        const bool dflt = c.box_lo[0] == 0 && c.box_lo[1] == 0 && c.box_lo[2] == 0 && c.box_hi[0] == 0 &&
                          c.box_hi[1] == 0 && c.box_hi[2] == 0;
        for (int a = 0; a < 3 && !dflt; ++a)
            if (!(c.box_hi[a] > c.box_lo[a]) || !std::isfinite(c.box_lo[a]) || !std::isfinite(c.box_hi[a])) {
                gwn::set_error("gwn_surrogate_train: the box must have lo < hi on every axis");
                return GWN_E_INVALID;
            }
    }
    if (!X || !T) {
        s = check_mesh(mesh, "gwn_surrogate_train");
        if (s != GWN_OK) return s;
    }
    return gwn::surrogate_train(h, mesh, c, X, T, npts, epoch_loss, epochs_run, (hipStream_t)stream);
}

gwn_status gwn_surrogate_save(gwn_surrogate h, const char* path) {
    gwn::clear_error();
    gwn_status s = check_mlp(h, "gwn_surrogate_save");
    if (s == GWN_OK && !path) {
        gwn::set_error("gwn_surrogate_save: null path");
        s = GWN_E_INVALID;
    }
    return s != GWN_OK ? s : gwn::surrogate_save(h, path);
}

gwn_status gwn_surrogate_load(const char* path, gwn_surrogate* out) {
    gwn::clear_error();
    if (!path || !out) {
        gwn::set_error("gwn_surrogate_load: null argument");
        return GWN_E_INVALID;
    }
    *out = nullptr;
    return gwn::surrogate_load(path, out);
}

gwn_status gwn_surrogate_destroy(gwn_surrogate h) {
    gwn::clear_error();
    gwn::mlp_release(h);
    return GWN_OK;
}

const char* gwn_status_str(gwn_status s) {
    switch (s) {
        case GWN_OK: return "ok";
        case GWN_E_INVALID: return "invalid argument";
        case GWN_E_OOM: return "out of device memory";
        case GWN_E_HIP: return "HIP runtime error";
        case GWN_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* gwn_last_error(void) { return gwn::g_err; }

}  // extern "C"
