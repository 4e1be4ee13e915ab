// tune.hip -- per-mesh query tuning: gwn_mesh_set_tuning / _get_tuning and the
// autotuner gwn_mesh_autotune.
//
// Three choices of the single-mesh paths depend on the mesh and the device
// rather than on the arithmetic (none changes a crossing count; the first
// changes w's summation order, the other two none of its bits):
//   * the largest batch that gives each point a workgroup with the boundary
//     edges split among its lanes (few points against many edges), per
//     precision;
//   * the smallest batch worth a Morton order of the points for the crossing
//     walk (dense points share BVH paths, sparse ones pay for the sort);
//   * the grid kernel's samples per lane (more share more x/y work, fewer leave
//     registers for more resident waves), per precision.
// The tuner sets the mesh's tuning to each candidate in turn and times the
// ordinary query calls on points it draws uniformly in the mesh's bounding box
// (and on a 64 x 64 x nz grid over it), keeping the fastest; the choice can be
// stored in and read from a JSON-lines cache keyed by the device architecture,
// the mesh's triangle and boundary-edge counts (powers of two) and the
// precision.  Environment overrides (GWN_SPLIT_BOUNDARY, GWN_ORDER_QUERIES,
// GWN_GRID_SAMPLES_PER_LANE) take precedence over any tuning.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "gwn_alloc.h"
#include "gwn_mesh.h"

namespace gwn {
namespace {

__global__ void k_tune_points(unsigned long long seed, long long n, double lx, double ly, double lz, double ex,
                              double ey, double ez, float* __restrict__ X) {
    const long long i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= n) return;
    const double lo[3] = {lx, ly, lz}, ext[3] = {ex, ey, ez};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        unsigned long long z = seed + (unsigned long long)(3 * i + c + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        X[3 * i + c] = (float)(lo[c] + (double)(z >> 11) * (1.0 / 9007199254740992.0) * ext[c]);
    }
}

struct Tuning {
    int split_max, order_min, grid_zb;
};

std::string arch_of(int device) {
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    return arch;
}

int log2_bucket(double x) { return (int)std::lround(std::log2(std::max(1.0, x))); }

std::string cache_key(const gwn_mesh_s* m, int prec, int nz) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s|mesh|F=2^%d|B=2^%d|prec=%d|nz=%d", arch_of(m->device).c_str(),
                  log2_bucket((double)m->nf), log2_bucket((double)m->nb), prec, nz);
    return buf;
}

bool valid(const Tuning& t, int prec) {
    const bool zb_ok = t.grid_zb == 0 || t.grid_zb == 1 || t.grid_zb == 2 || t.grid_zb == 4 ||
                       (t.grid_zb == 8 && prec == GWN_PREC_FP32);
    return t.split_max >= -1 && t.order_min >= -1 && zb_ok;
}

bool cache_lookup(const char* path, const std::string& key, int prec, Tuning* out) {
    if (!path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char k[256];
        Tuning t;
        if (std::sscanf(line, " {\"key\": \"%255[^\"]\", \"split_max_points\": %d, \"order_min_points\": %d, "
                              "\"grid_samples_per_lane\": %d",
                        k, &t.split_max, &t.order_min, &t.grid_zb) == 4 &&
            key == k && valid(t, prec)) {
            *out = t;
            found = true;   // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, const Tuning& t) {
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%s\", \"split_max_points\": %d, \"order_min_points\": %d, "
                    "\"grid_samples_per_lane\": %d}\n",
                 key.c_str(), t.split_max, t.order_min, t.grid_zb);
    std::fclose(f);
}

// the smallest of `reps` timings of fn() (after one untimed call), in ms
template <class F>
gwn_status time_ms(F&& fn, int reps, hipStream_t st, float* out) {
    hipEvent_t a = nullptr, b = nullptr;
    GWN_HIP_TRY(hipEventCreate(&a));
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        GWN_HIP_TRY(e);
    }
    gwn_status s = fn();
    float best = 1e30f;
    for (int r = 0; r < reps && s == GWN_OK; ++r) {
        e = hipEventRecord(a, st);
        if (e == hipSuccess) s = fn();
        if (s == GWN_OK && e == hipSuccess) e = hipEventRecord(b, st);
        if (s == GWN_OK && e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (s == GWN_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e != hipSuccess) break;
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (s != GWN_OK) return s;
    GWN_HIP_TRY(e);
    *out = best;
    return GWN_OK;
}

// world-frame bounding box of the mesh's vertices (the handle keeps it in its ray frame)
void world_box(const gwn_mesh_s* m, double lo[3], double hi[3]) {
    for (int c = 0; c < 3; ++c) {
        const int a = (c + m->axis) % 3;
        lo[a] = m->bbox[c];
        hi[a] = m->bbox[3 + c];
    }
}

gwn_status autotune(gwn_mesh_s* m, int prec, int nz, int reps, hipStream_t st, Tuning* best) {
    constexpr long long kMaxPts = 1 << 20;
    double lo[3], hi[3];
    world_box(m, lo, hi);
    for (int a = 0; a < 3; ++a)
        if (!(hi[a] > lo[a])) hi[a] = lo[a] + 1.0;   // flat meshes: a unit-thick box
    float* X = nullptr;
    void* W = nullptr;
    int* C = nullptr;
    const size_t wbytes = (prec == GWN_PREC_FP64 ? 8 : 4);
    const long long ngrid = nz > 0 ? 64ll * 64 * nz : 0;
    const long long nout = std::max(kMaxPts, ngrid);
    struct Bufs {
        float*& X;
        void*& W;
        int*& C;
        hipStream_t st;
        ~Bufs() {
            (void)hipStreamSynchronize(st);
            (void)hipFree(X);
            (void)hipFree(W);
            (void)hipFree(C);
        }
    } bufs{X, W, C, st};
    GWN_HIP_TRY(dmalloc((void**)&X, sizeof(float) * 3 * (size_t)kMaxPts));
    GWN_HIP_TRY(dmalloc(&W, wbytes * (size_t)nout));
    GWN_HIP_TRY(dmalloc((void**)&C, sizeof(int) * (size_t)nout));
    k_tune_points<<<(unsigned)((kMaxPts + 255) / 256), 256, 0, st>>>(0x5EEDull + (unsigned long long)m->nf, kMaxPts,
                                                                     lo[0], lo[1], lo[2], hi[0] - lo[0],
                                                                     hi[1] - lo[1], hi[2] - lo[2], X);
    GWN_HIP_TRY(hipGetLastError());
    auto batch = [&](long long n) {
        return [&, n]() { return query_batch(m, X, X + 1, X + 2, 3, n, prec, W, C, st); };
    };
    // 1. split threshold: scan up while the split form is at least as fast
    int split = -1;
    if (m->nb > 0) {
        for (long long n = 256; n <= 32768; n *= 2) {
            float ts = 0.f, tl = 0.f;
            m->split_max[prec] = (int)n;
            gwn_status s = time_ms(batch(n), reps, st, &ts);
            m->split_max[prec] = -1;
            if (s == GWN_OK) s = time_ms(batch(n), reps, st, &tl);
            if (s != GWN_OK) return s;
            if (ts <= tl) split = (int)n;
            else break;
        }
    }
    m->split_max[prec] = split;
    // 2. order threshold: the smallest batch from which ordering stays ahead
    int order = -1;
    for (long long n = kMaxPts; n >= (1 << 14); n /= 2) {
        float to = 0.f, tp = 0.f;
        m->order_min = (int)n;
        gwn_status s = time_ms(batch(n), reps, st, &to);
        m->order_min = -1;
        if (s == GWN_OK) s = time_ms(batch(n), reps, st, &tp);
        if (s != GWN_OK) return s;
        if (to < tp) order = (int)n;
        else break;
    }
    m->order_min = order;
    // 3. grid samples per lane on a 64 x 64 x nz grid over the box
    int zb = 0;
    if (nz > 0) {
        const double org[3] = {lo[0], lo[1], lo[2]};
        const double sp[3] = {(hi[0] - lo[0]) / 64, (hi[1] - lo[1]) / 64, (hi[2] - lo[2]) / nz};
        const int64_t dims[3] = {64, 64, nz};
        float bt = 1e30f;
        for (int cand : {1, 2, 4, 8}) {
            if (cand == 8 && prec == GWN_PREC_FP64) continue;
            float t = 0.f;
            m->grid_zb[prec] = cand;
            const gwn_status s = time_ms([&]() { return query_grid(m, org, sp, dims, prec, W, nullptr, st); }, reps,
                                         st, &t);
            if (s != GWN_OK) return s;
            if (t < bt) {
                bt = t;
                zb = cand;
            }
        }
    }
    m->grid_zb[prec] = zb;
    best->split_max = split;
    best->order_min = order;
    best->grid_zb = zb;
    return GWN_OK;
}

gwn_status check(gwn_mesh m, const char* fn) {
    if (!m) {
        set_error("%s: null mesh handle", fn);
        return GWN_E_INVALID;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m->device) {
        set_error("%s: mesh was built on device %d, current device is %d", fn, m->device, dev);
        return GWN_E_INVALID;
    }
    return GWN_OK;
}

}  // namespace
}  // namespace gwn

extern "C" {

gwn_status gwn_mesh_get_tuning(gwn_mesh m, gwn_query_tuning* out) {
    gwn::clear_error();
    if (!m || !out) {
        gwn::set_error("gwn_mesh_get_tuning: null argument");
        return GWN_E_INVALID;
    }
    for (int p = 0; p < 2; ++p) {
        out->split_max_points[p] = m->split_max[p];
        out->grid_samples_per_lane[p] = m->grid_zb[p];
    }
    out->order_min_points = m->order_min;
    out->tuned = m->tuned;
    return GWN_OK;
}

gwn_status gwn_mesh_set_tuning(gwn_mesh m, const gwn_query_tuning* t) {
    gwn::clear_error();
    if (!m || !t) {
        gwn::set_error("gwn_mesh_set_tuning: null argument");
        return GWN_E_INVALID;
    }
    for (int p = 0; p < 2; ++p) {
        const gwn::Tuning c{t->split_max_points[p], t->order_min_points, t->grid_samples_per_lane[p]};
        if (!gwn::valid(c, p)) {
            gwn::set_error("gwn_mesh_set_tuning: split/order thresholds must be >= -1 and samples per lane 0, 1, 2, 4 "
                           "or 8 (FP64: at most 4)");
            return GWN_E_INVALID;
        }
    }
    for (int p = 0; p < 2; ++p) {
        m->split_max[p] = t->split_max_points[p];
        m->grid_zb[p] = t->grid_samples_per_lane[p];
    }
    m->order_min = t->order_min_points;
    m->tuned = 0;
    return GWN_OK;
}

gwn_status gwn_mesh_autotune(gwn_mesh m, const gwn_autotune_opts* opts, void* stream) {
    gwn::clear_error();
    gwn_status s = gwn::check(m, "gwn_mesh_autotune");
    if (s != GWN_OK) return s;
    const int prec = opts ? opts->prec : GWN_PREC_FP32;
    const int nz = opts ? opts->grid_nz : 0;
    const int reps = opts && opts->reps > 0 ? opts->reps : 3;
    if ((prec != GWN_PREC_FP32 && prec != GWN_PREC_FP64) || nz < 0 || nz > (1 << 20) || reps > 100) {
        gwn::set_error("gwn_mesh_autotune: bad precision %d, grid_nz %d or reps %d", prec, nz, reps);
        return GWN_E_INVALID;
    }
    const char* cache = opts ? opts->cache : nullptr;
    const std::string key = gwn::cache_key(m, prec, nz);
    gwn::Tuning t;
    if (gwn::cache_lookup(cache, key, prec, &t)) {
        m->split_max[prec] = t.split_max;
        m->order_min = t.order_min;
        m->grid_zb[prec] = t.grid_zb;
        m->tuned |= 1 << prec;
        return GWN_OK;
    }
    // time with the mesh's current tuning restored if anything fails
    const int keep_split = m->split_max[prec], keep_order = m->order_min, keep_zb = m->grid_zb[prec];
    s = gwn::autotune(m, prec, nz, reps, (hipStream_t)stream, &t);
    if (s != GWN_OK) {
        m->split_max[prec] = keep_split;
        m->order_min = keep_order;
        m->grid_zb[prec] = keep_zb;
        return s;
    }
    m->tuned |= 1 << prec;
    gwn::cache_store(cache, key, t);
    return GWN_OK;
}

}  // extern "C"
