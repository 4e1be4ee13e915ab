// gwn_mesh.h -- host-side mesh handle and internal entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <new>
#include <string>

#include "../../include/gwn.h"
#include "gwn_internal.h"

struct gwn_mesh_s {
    int device = 0;
    int64_t nv = 0, nf = 0, nb = 0, nloops = 0, nnodes = 0;
    int64_t nunique = 0;           // distinct positions after welding (nv without it)
    int axis = 0;                  // ray axis (0 = z, 1 = x, 2 = y); all device data is in its frame
    double proj_area[3] = {0, 0, 0};   // 2 x projected area on the planes normal to x, y, z (when chosen)
    int depth = 0;
    double build_ms = 0.0;
    double bbox[6] = {0, 0, 0, 0, 0, 0};
    gwn::QGrid g{};
    int root = gwn::kNoRoot;
    // device memory owned by the handle
    gwn::Node* nodes = nullptr;
    gwn::TriQ* tris = nullptr;
    float4* trif = nullptr;        // float corners in Morton order (direct sum)
    gwn::BVert* bverts = nullptr;
    int* loop_off = nullptr;
    // query tuning (gwn_mesh_set_tuning / gwn_mesh_autotune); 0 = the built-in rule
    int split_max[2] = {0, 0};     // per precision: batches of at most this many points split their edges
    int order_min = 0;             // batches of at least this many points are Morton-ordered
    int grid_zb[2] = {0, 0};       // per precision: grid samples per lane
    int tuned = 0;                 // bit p: precision p was tuned

    gwn::MeshView view() const {
        gwn::MeshView v;
        v.nodes = nodes;
        v.tris = tris;
        v.bverts = bverts;
        v.loop_off = loop_off;
        v.nloops = (int)nloops;
        v.nf = (int)nf;
        v.root = root;
        v.axis = axis;
        v.g = g;
        return v;
    }
};

namespace gwn {

// thread-local error reporting shared by all translation units
void set_error(const char* fmt, ...);
void clear_error();

// axis: 0 = z, 1 = x, 2 = y, -1 = the one with the least projected triangle area
gwn_status build_mesh(const float* vx, const float* vy, const float* vz, int64_t vstride, int64_t nv,
                      const int32_t* tri, int64_t nf, bool weld, int axis, hipStream_t stream, gwn_mesh_s* m);

gwn_status query_batch(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                       int64_t nq, int prec, void* w_out, int32_t* chi_out, hipStream_t stream);

// Caller memory for the temporaries of one batch launch (see query_batch_ws).
struct BatchWorkspace {
    int* chi;           // nq ints: crossing counts when the caller passes no chi_out
    int* perm;          // nq ints: the traversal order
    void* order_temp;   // xy_order_temp_bytes(nq) bytes
};

// query_batch with its temporaries in ws (nullable: stream-ordered allocations);
// with ws, nq must fit one launch (max_launch_queries()).
gwn_status query_batch_ws(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                          int64_t nq, int prec, void* w_out, int32_t* chi_out, const BatchWorkspace* ws,
                          hipStream_t stream);

gwn_status query_grid(const gwn_mesh_s* m, const double* origin, const double* spacing, const int64_t* dims,
                      int prec, void* w_out, int32_t* chi_out, hipStream_t stream);

// queries per kernel launch in the one-lane-per-query paths (keeps the launch
// within the 32-bit work-item count); larger batches take several launches.
// GWN_MAX_LAUNCH_QUERIES (a positive multiple of 256) lowers it, for tests.
int64_t max_launch_queries();

// Few points against many boundary edges take a workgroup per point with the
// edges split among its lanes: batches of at most 8,192 points on meshes with at
// least 16 boundary edges per lane of a 256-lane workgroup.
// GWN_SPLIT_BOUNDARY=0/1 overrides.
// prec: the precision whose tuning applies (-1: the built-in rule only).
bool want_split(const gwn_mesh_s* m, int64_t n, int prec);

// Morton order of the points' quantised x, y for the crossing traversal (perm is
// stream-ordered device memory the caller frees with hipFreeAsync).
// GWN_ORDER_QUERIES=0/1 overrides the size heuristic.
bool want_xy_order(const gwn_mesh_s* m, int64_t n);
gwn_status xy_order(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qstride, int64_t n,
                    int** perm, hipStream_t stream);
// the same into caller memory: perm (n ints) and temp (xy_order_temp_bytes(n))
size_t xy_order_temp_bytes(int64_t n);
gwn_status xy_order_into(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                         int64_t n, int* perm, void* temp, hipStream_t stream);

gwn_status query_grid_gradient(const gwn_mesh_s* m, const double* origin, const double* spacing, const int64_t* dims,
                               int prec, void* g_out, hipStream_t stream);

gwn_status query_crossings(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                           int64_t nq, int32_t* up, int32_t* down, hipStream_t stream);

gwn_status query_gradient(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                          int64_t nq, int prec, void* g_out, hipStream_t stream);

gwn_status query_direct(const gwn_mesh_s* m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                        int64_t nq, int prec, void* w_out, hipStream_t stream);

gwn_status multi_create(const gwn_mesh* meshes, int nmesh, const float* qx, const float* qy, const float* qz,
                        int64_t qs, const int64_t* q_offsets, int prec, void* w_out, int32_t* chi_out,
                        const gwn_multi_opts* opts, hipStream_t stream, gwn_multi_s** out);
gwn_status multi_run(gwn_multi_s* p, hipStream_t stream);
void multi_destroy(gwn_multi_s* p);
void multi_info(const gwn_multi_s* p, gwn_multi_info* out);

gwn_status mlp_create(uint64_t seed, double sigma, gwn_mlp_s** out);
void mlp_release(gwn_mlp_s* h);
int mlp_device(const gwn_mlp_s* h);
gwn_status mlp_get_state(gwn_mlp_s* h, float* theta, float* m, float* v, float* G, int64_t* step);
gwn_status mlp_set_state(gwn_mlp_s* h, const float* theta, const float* m, const float* v, const float* G,
                         int64_t step);
gwn_status mlp_forward(gwn_mlp_s* h, const float* qx, const float* qy, const float* qz, int64_t qs, int64_t n,
                       float* y, hipStream_t st);
gwn_status mlp_loss_grad(gwn_mlp_s* h, const float* qx, const float* qy, const float* qz, int64_t qs,
                         const float* tgt, int64_t n, float* grad_out, float* loss_out, hipStream_t st);
gwn_status mlp_train_step(gwn_mlp_s* h, const float* qx, const float* qy, const float* qz, int64_t qs,
                          const float* tgt, int64_t n, float lr, float* loss_out, hipStream_t st);
gwn_status surrogate_query(gwn_mlp_s* h, const gwn_mesh_s* mesh, const float* qx, const float* qy, const float* qz,
                           int64_t qs, int64_t n, float band, int rule, float* w, unsigned char* mask,
                           int64_t* nfallback, hipStream_t st);
gwn_status surrogate_train(gwn_mlp_s* h, const gwn_mesh_s* mesh, const gwn_surrogate_cfg& cfg, const float* X,
                           const float* T, int64_t n, float* epoch_loss, int64_t* epochs_run, hipStream_t st);
gwn_status surrogate_save(gwn_mlp_s* h, const char* path);
gwn_status surrogate_load(const char* path, gwn_mlp_s** out);

// Fixed-point grid rule (host, FP64): origin = bbox_lo - 0.75 e, scale 2^k with
// k the largest integer such that 2.5 e 2^k <= 2^30 - 1 (e = max extent, 1 if 0).
QGrid make_qgrid(const double bbox[6]);

}  // namespace gwn

#define GWN_HIP_TRY(expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            gwn::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                           __LINE__);                                                      \
            return e_ == hipErrorOutOfMemory ? GWN_E_OOM : GWN_E_HIP;                      \
        }                                                                                  \
    } while (0)
