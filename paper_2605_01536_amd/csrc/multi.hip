// multi.hip -- many meshes with uneven sizes and query counts in one captured
// HIP graph: [reset work counter] -> [crossing counts for every query of every
// mesh] -> [persistent boundary-term kernel].  The persistent kernel keeps
// waves resident and hands out (mesh, query tile) work items through an atomic
// counter, largest estimated cost first, so meshes whose cost spans orders of
// magnitude share the GPU without a long tail.  The schedule (tile size, item
// order, resident waves) is chosen by timing candidates (autotune) and can be
// cached in a JSON-lines file keyed by device and problem size.  Optionally the
// queries of each mesh are taken in Morton order of their quantised x, y (an
// index permutation made once at creation), so that the 64 queries of a wave
// lie close together and take the same branches of the boundary loop.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gwn_alloc.h"
#include "gwn_kernels.h"
#include "gwn_mesh.h"

namespace gwn {
namespace {

struct alignas(16) Item {
    long long q0;   // first query (global index)
    int mesh;
    int nq;         // queries in this item
};

__global__ void k_reset_counter(int* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
}

// Crossing counts along +z for every query, one wave per work item: the item's
// queries (in Morton order within their mesh when perm is given, as the
// boundary-term kernel takes them) walk the mesh's BVH together
// (chi_wave_walk), so a wave follows about one path.  Out-of-box queries get 0.
__global__ __launch_bounds__(64 * kGridWaves) void k_chi_items(const MeshView* __restrict__ table,
                                                              const Item* __restrict__ items, int nitems,
                                                              const float* __restrict__ qx,
                                                              const float* __restrict__ qy,
                                                              const float* __restrict__ qz, long long qs,
                                                              const int* __restrict__ perm, int* __restrict__ chi) {
    __shared__ int wstack[kGridWaves][kLdsStack];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const long long it = (long long)blockIdx.x * kGridWaves + wave;
    if (it >= nitems) return;   // the whole wave
    const Item I = items[it];
    const MeshView mv = table[I.mesh];
    const float *x = qx, *y = qy, *z = qz;
    axis_ptrs(mv.axis, x, y, z);   // the mesh's frame
    for (int sub = 0; sub < I.nq; sub += 64) {
        const int k = sub + lane;
        const long long i0 = I.q0 + min(k, I.nq - 1);
        const long long i = perm ? (long long)perm[i0] : i0;
        const QPoint q = quantize_point(x[i * qs], y[i * qs], z[i * qs], mv.g);
        int u, d;
        chi_wave_walk<true>(mv, q, k < I.nq && q.inbox, wstack[wave], u, d);
        if (k < I.nq) chi[i] = u;
    }
}

// global query index i0 + perm_local[i - i0] for i in [i0, i0 + n)
__global__ void k_perm_offset(const int* __restrict__ local, long long i0, int n, int* __restrict__ perm) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < n) perm[i0 + k] = (int)(i0 + (local ? local[k] : k));
}

// Persistent boundary-term kernel: every wave claims items until none are left
// (the counter only grows, so every wave reaches the exit).  perm (nullable):
// position i of the work list is query perm[i], a permutation within each mesh.
// T is the geometry precision; per query it takes the same steps, in the same
// order, as the one-lane-per-point batch kernel, so the results are the same bits.
// FP32 is held to 64 VGPRs, so the 8 resident waves per SIMD the schedules ask
// for all fit (68 unconstrained, i.e. 7).
template <class T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 1)))
void k_bdry_persistent(const MeshView* __restrict__ table, const Item* __restrict__ items, int nitems,
                       int* __restrict__ counter, const float* __restrict__ qx, const float* __restrict__ qy,
                       const float* __restrict__ qz, long long qs, const int* __restrict__ perm,
                       const int* __restrict__ chi, T* __restrict__ w) {
    const int lane = threadIdx.x & 63;
    while (true) {
        int it = 0;
        if (lane == 0) it = atomicAdd(counter, 1);
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
        if (it >= nitems) break;
        const Item I = items[it];
        const MeshView mv = table[I.mesh];
        const float *x = qx, *y = qy, *z = qz;
        axis_ptrs(mv.axis, x, y, z);   // the mesh's frame
        for (int sub = 0; sub < I.nq; sub += 64) {
            const int k = sub + lane;
            const long long i0 = I.q0 + min(k, I.nq - 1);
            const long long i = perm ? (long long)perm[i0] : i0;
            const float px = x[i * qs], py = y[i * qs], pz = z[i * qs];
            const QPoint q = quantize_point(px, py, pz, mv.g);
            double S = 0.0;
            if (q.inbox) {
                const T pzs = (T)pz * (T)mv.g.scale;
                boundary_loops<T, 1, false>(mv, q.x, q.y, (T)0, (T)0, &pzs, &S, (T)1, near_z(pz, mv.g));
            } else {
                const FarScale<T> fs = far_scale<T>(px, py, fabsf(pz), mv.g.scale);
                const T pzs = (T)pz * fs.scf;
                boundary_loops<T, 1, true>(mv, 0, 0, (T)px * fs.scf, (T)py * fs.scf, &pzs, &S, fs.f);
            }
            if (k < I.nq) w[i] = (T)((double)chi[i] + S * kInv2Pi);
        }
    }
}

struct Schedule {
    int item_queries = 128;   // multiple of 64
    int waves_per_simd = 8;   // resident persistent waves per SIMD
    int order = 0;            // bit 0: mesh order (else largest cost first); bit 1: queries in Morton order
};

constexpr int kOrderMesh = 1, kOrderSorted = 2;

}  // namespace
}  // namespace gwn

struct gwn_multi_s {
    int device = 0;
    int nmesh = 0;
    long long nq = 0;
    double est_pairs = 0.0;
    gwn::Schedule sched;
    bool tuned = false;
    double tuned_ms = 0.0;
    std::vector<gwn_mesh_s*> meshes;
    std::vector<long long> qoff_h;
    const float *qx = nullptr, *qy = nullptr, *qz = nullptr;
    long long qs = 1;
    int prec = GWN_PREC_FP32;
    void* w = nullptr;   // float (GWN_PREC_FP32) or double (GWN_PREC_FP64)
    int* chi = nullptr;
    bool own_chi = false;
    gwn::MeshView* table = nullptr;
    gwn::Item* items = nullptr;
    int nitems = 0;
    int* perm = nullptr;   // Morton order of each mesh's queries (made when a schedule asks for it)
    int* counter = nullptr;
    int grid = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace gwn {
namespace {

void drop_graph(gwn_multi_s* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

void release(gwn_multi_s* p) {
    if (!p) return;
    drop_graph(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    (void)hipFree(p->table);
    (void)hipFree(p->items);
    (void)hipFree(p->perm);
    (void)hipFree(p->counter);
    if (p->own_chi) (void)hipFree(p->chi);
    delete p;
}

// Work list for a schedule: tiles of item_queries queries, ordered by estimated
// cost (queries x (boundary edges + a traversal allowance)) or by mesh.
gwn_status build_items(gwn_multi_s* p, const Schedule& s, hipStream_t st) {
    std::vector<Item> h;
    std::vector<double> cost;
    for (int m = 0; m < p->nmesh; ++m) {
        const long long q0 = p->qoff_h[m], q1 = p->qoff_h[m + 1];
        const double per_q = (double)p->meshes[m]->nb + 16.0;
        for (long long a = q0; a < q1; a += s.item_queries) {
            Item it;
            it.q0 = a;
            it.mesh = m;
            it.nq = (int)std::min<long long>(s.item_queries, q1 - a);
            h.push_back(it);
            cost.push_back(per_q * it.nq);
        }
    }
    if (!(s.order & kOrderMesh)) {
        std::vector<size_t> idx(h.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
        std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
        std::vector<Item> s2(h.size());
        for (size_t i = 0; i < idx.size(); ++i) s2[i] = h[idx[i]];
        h.swap(s2);
    }
    (void)hipFree(p->items);
    p->items = nullptr;
    p->nitems = (int)h.size();
    GWN_HIP_TRY(gwn::dmalloc((void**)&p->items, sizeof(Item) * std::max<size_t>(1, h.size())));
    if (!h.empty())
        GWN_HIP_TRY(hipMemcpyAsync(p->items, h.data(), sizeof(Item) * h.size(), hipMemcpyHostToDevice, st));
    GWN_HIP_TRY(hipStreamSynchronize(st));
    return GWN_OK;
}

// Each mesh's queries in Morton order of their quantised x, y in the mesh's
// frame (the batch path's traversal order), as one permutation of all queries.
gwn_status build_perm(gwn_multi_s* p, hipStream_t st) {
    if (p->perm) return GWN_OK;
    GWN_HIP_TRY(gwn::dmalloc((void**)&p->perm, sizeof(int) * (size_t)std::max<long long>(1, p->nq)));
    for (int m = 0; m < p->nmesh; ++m) {
        const long long q0 = p->qoff_h[m], n = p->qoff_h[m + 1] - q0;
        if (n <= 0) continue;
        const float *x = p->qx, *y = p->qy, *z = p->qz;
        axis_ptrs(p->meshes[m]->axis, x, y, z);
        int* local = nullptr;
        if (n > 1) {
            const gwn_status r = xy_order(p->meshes[m], x + q0 * p->qs, y + q0 * p->qs, z + q0 * p->qs, p->qs, n,
                                          &local, st);
            if (r != GWN_OK) return r;
        }
        k_perm_offset<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(local, q0, (int)n, p->perm);
        const hipError_t e = hipGetLastError();
        if (local) (void)hipFreeAsync(local, st);
        GWN_HIP_TRY(e);
    }
    GWN_HIP_TRY(hipStreamSynchronize(st));
    return GWN_OK;
}

gwn_status capture(gwn_multi_s* p, const Schedule& s) {
    drop_graph(p);
    int ncu = 0;
    GWN_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device));
    const long long waves = (long long)ncu * 4 * s.waves_per_simd;
    const long long need = ((long long)p->nitems + 3) / 4;   // no more blocks than 4-wave groups of items
    p->grid = (int)std::max<long long>(1, std::min<long long>(waves / 4, std::max<long long>(need, 1)));
    GWN_HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    k_reset_counter<<<1, 64, 0, p->cap>>>(p->counter);
    if (p->nq > 0) {
        const int* perm = (s.order & kOrderSorted) ? p->perm : nullptr;
        k_chi_items<<<(unsigned)((p->nitems + kGridWaves - 1) / kGridWaves), 64 * kGridWaves, 0, p->cap>>>(
            p->table, p->items, p->nitems, p->qx, p->qy, p->qz, p->qs, perm, p->chi);
        if (p->prec == GWN_PREC_FP64)
            k_bdry_persistent<double><<<p->grid, 256, 0, p->cap>>>(p->table, p->items, p->nitems, p->counter, p->qx,
                                                                   p->qy, p->qz, p->qs, perm, p->chi,
                                                                   (double*)p->w);
        else
            k_bdry_persistent<float><<<p->grid, 256, 0, p->cap>>>(p->table, p->items, p->nitems, p->counter, p->qx,
                                                                  p->qy, p->qz, p->qs, perm, p->chi, (float*)p->w);
    }
    hipError_t e = hipStreamEndCapture(p->cap, &p->graph);
    GWN_HIP_TRY(e);
    GWN_HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return GWN_OK;
}

gwn_status apply(gwn_multi_s* p, Schedule s, hipStream_t st) {
    if (p->nq > 0x7fffffffll) s.order &= ~kOrderSorted;   // the permutation holds 32-bit indices
    gwn_status r = (s.order & kOrderSorted) ? build_perm(p, st) : GWN_OK;
    if (r != GWN_OK) return r;
    r = build_items(p, s, st);
    if (r != GWN_OK) return r;
    r = capture(p, s);
    if (r != GWN_OK) return r;
    p->sched = s;
    return GWN_OK;
}

gwn_status time_replay(gwn_multi_s* p, hipStream_t st, double* ms) {
    hipEvent_t a, b;
    GWN_HIP_TRY(hipEventCreate(&a));
    GWN_HIP_TRY(hipEventCreate(&b));
    GWN_HIP_TRY(hipGraphLaunch(p->exec, st));           // warm-up
    GWN_HIP_TRY(hipEventRecord(a, st));
    GWN_HIP_TRY(hipGraphLaunch(p->exec, st));
    GWN_HIP_TRY(hipEventRecord(b, st));
    GWN_HIP_TRY(hipEventSynchronize(b));
    float f = 0.f;
    GWN_HIP_TRY(hipEventElapsedTime(&f, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = f;
    return GWN_OK;
}

std::string cache_key(const gwn_multi_s* p) {
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s|%s|meshes=%d|q=2^%d|pairs=2^%d", arch.c_str(),
                  p->prec == GWN_PREC_FP64 ? "fp64" : "fp32", p->nmesh,
                  (int)std::lround(std::log2(std::max(1.0, (double)p->nq))),
                  (int)std::lround(std::log2(std::max(1.0, p->est_pairs))));
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, Schedule* s) {
    if (!path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char k[256];
        Schedule t;
        if (std::sscanf(line, " {\"key\": \"%255[^\"]\", \"item_queries\": %d, \"waves_per_simd\": %d, \"order\": %d",
                        k, &t.item_queries, &t.waves_per_simd, &t.order) == 4 &&
            key == k && t.item_queries >= 64 && t.item_queries % 64 == 0 && t.waves_per_simd >= 1 &&
            t.waves_per_simd <= 8 && t.order >= 0 && t.order <= 3) {
            *s = t;
            found = true;   // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, const Schedule& s, double ms) {
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%s\", \"item_queries\": %d, \"waves_per_simd\": %d, \"order\": %d, \"ms\": %.4f}\n",
                 key.c_str(), s.item_queries, s.waves_per_simd, s.order, ms);
    std::fclose(f);
}

}  // namespace

gwn_status multi_create(const gwn_mesh* meshes, int nmesh, const float* qx, const float* qy, const float* qz,
                        int64_t qs, const int64_t* q_offsets, int prec, void* w_out, int32_t* chi_out,
                        const gwn_multi_opts* opts, hipStream_t st, gwn_multi_s** out) {
    gwn_multi_s* p = new (std::nothrow) gwn_multi_s();
    if (!p) return GWN_E_OOM;
    struct Guard {
        gwn_multi_s* p;
        ~Guard() { if (p) release(p); }
    } guard{p};
    GWN_HIP_TRY(hipGetDevice(&p->device));
    p->nmesh = nmesh;
    p->meshes.assign(meshes, meshes + nmesh);
    p->qoff_h.assign(q_offsets, q_offsets + nmesh + 1);
    p->nq = p->qoff_h[nmesh];
    for (int m = 0; m < nmesh; ++m)
        p->est_pairs += (double)(p->qoff_h[m + 1] - p->qoff_h[m]) * (double)p->meshes[m]->nb;
    p->qx = qx;
    p->qy = qy;
    p->qz = qz;
    p->qs = qs;
    p->prec = prec;
    p->w = w_out;
    p->chi = chi_out;
    if (!p->chi) {
        GWN_HIP_TRY(gwn::dmalloc((void**)&p->chi, sizeof(int) * (size_t)std::max<long long>(1, p->nq)));
        p->own_chi = true;
    }
    std::vector<MeshView> tab(nmesh);
    for (int m = 0; m < nmesh; ++m) tab[m] = p->meshes[m]->view();
    GWN_HIP_TRY(gwn::dmalloc((void**)&p->table, sizeof(MeshView) * (size_t)nmesh));
    GWN_HIP_TRY(gwn::dmalloc((void**)&p->counter, sizeof(int)));
    GWN_HIP_TRY(hipMemcpyAsync(p->table, tab.data(), sizeof(MeshView) * nmesh, hipMemcpyHostToDevice, st));
    GWN_HIP_TRY(hipStreamSynchronize(st));
    GWN_HIP_TRY(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));

    Schedule s;
    const bool explicit_sched = opts && (opts->item_queries > 0 || opts->waves_per_simd > 0 || opts->order > 0);
    if (opts && opts->item_queries > 0) s.item_queries = ((opts->item_queries + 63) / 64) * 64;
    if (opts && opts->waves_per_simd > 0) s.waves_per_simd = std::min(8, opts->waves_per_simd);
    if (opts && opts->order > 0) s.order = opts->order & 3;
    const char* cache = opts ? opts->tune_cache : nullptr;
    const std::string key = cache_key(p);
    Schedule cached;
    if (!explicit_sched && cache_lookup(cache, key, &cached)) {
        s = cached;
        p->tuned = true;
    } else if (!explicit_sched && opts && opts->autotune && p->nq > 0) {
        static const int tiles[] = {64, 128, 256, 512};
        static const int wps[] = {4, 8};
        static const int orders[] = {0, 1};
        double best = 1e300;
        Schedule bs = s;
        for (int o : orders)
            for (int wv : wps)
                for (int t : tiles) {
                    Schedule c;
                    c.item_queries = t;
                    c.waves_per_simd = wv;
                    c.order = o;
                    gwn_status r = apply(p, c, st);
                    if (r != GWN_OK) return r;
                    double ms = 0.0;
                    r = time_replay(p, st, &ms);
                    if (r != GWN_OK) return r;
                    if (ms < best) {
                        best = ms;
                        bs = c;
                    }
                }
        // the best schedule again with each mesh's queries in Morton order
        Schedule c = bs;
        c.order |= kOrderSorted;
        gwn_status r = apply(p, c, st);
        if (r != GWN_OK) return r;
        double ms = 0.0;
        r = time_replay(p, st, &ms);
        if (r != GWN_OK) return r;
        if (ms < best) {
            best = ms;
            bs = c;
        }
        s = bs;
        p->tuned = true;
        p->tuned_ms = best;
        cache_store(cache, key, s, best);
    }
    gwn_status r = apply(p, s, st);
    if (r != GWN_OK) return r;
    guard.p = nullptr;
    *out = p;
    return GWN_OK;
}

gwn_status multi_run(gwn_multi_s* p, hipStream_t st) {
    GWN_HIP_TRY(hipGraphLaunch(p->exec, st));
    return GWN_OK;
}

void multi_destroy(gwn_multi_s* p) { release(p); }

void multi_info(const gwn_multi_s* p, gwn_multi_info* o) {
    o->nmesh = p->nmesh;
    o->nqueries = p->nq;
    o->nitems = p->nitems;
    o->item_queries = p->sched.item_queries;
    o->waves_per_simd = p->sched.waves_per_simd;
    o->order = p->sched.order;
    o->grid_blocks = p->grid;
    o->tuned = p->tuned ? 1 : 0;
    o->est_pairs = p->est_pairs;
    o->tuned_ms = p->tuned_ms;
}

}  // namespace gwn
