/*
 * gwn.h -- C ABI of the MI355X (gfx950) generalized-winding-number library.
 *
 * Computes w_M(p), the generalized winding number of a triangle soup M at
 * query points p (Eq. 1: the signed solid angle of M seen from p over 4 pi),
 * by the antipodal method (Eq. 10, Alg. 1):
 *
 *     w(p) = chi(x0) + (1/4pi) * sum_{(a,b) in dM} Area_{S^2}(a^, b^, x1)
 *
 * with ray direction x0 = +z and its antipode x1 = -z.  chi(x0) is the signed
 * number of crossings of the ray from p along +z with the soup, +1 where the
 * ray has positive dot product with the triangle normal (Sec. 3.2); dM is the
 * directed boundary chain left after interior edges cancel (Sec. 4.1).
 *
 * Robustness (Supp. Sec. 2.1): every decision that can change w by an
 * integer -- whether the ray crosses a triangle, on which side of the
 * triangle's plane the query lies, and the branch of atan2 where a boundary
 * edge passes over the ray -- is taken with exact integer predicates on a
 * 30-bit fixed-point copy of the input, with the query symbolically
 * perturbed to q + (e1, e2, e3), 0 < e3 << e2 << e1.  The crossing counts
 * are therefore exact and deterministic for every query, including queries
 * on the surface.
 *
 * Conventions shared by all calls
 *   - All array pointers are DEVICE pointers on the current HIP device,
 *     owned by the caller.  The library owns mesh handles and their device
 *     memory.  `stream` is a hipStream_t (NULL = default stream); query calls
 *     are asynchronous on it.
 *   - Triangle (v0, v1, v2) has normal (v1 - v0) x (v2 - v0); w > 0 on the
 *     side opposite the normal, so w = +1 inside a closed mesh whose normals
 *     point outward.
 *   - Strided coordinates: element i of a coordinate array X is X[i*stride]
 *     (stride 1 for separate arrays; stride 3 with x = P, y = P+1, z = P+2
 *     for an interleaved (n, 3) array).
 *   - Errors never cross the ABI as exceptions; every call returns a
 *     gwn_status and gwn_last_error() gives a message for the calling thread.
 */
#ifndef GWN_H
#define GWN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GWN_OK = 0,
    GWN_E_INVALID = 1,     /* bad argument, out-of-range index, non-finite coordinate */
    GWN_E_OOM = 2,         /* device allocation failed */
    GWN_E_HIP = 3,         /* a HIP runtime call failed */
    GWN_E_UNSUPPORTED = 4  /* valid request the library does not implement */
} gwn_status;

typedef enum {
    GWN_PREC_FP32 = 0,     /* FP32 geometry arithmetic, exact predicates, FP64 accumulation; float output */
    GWN_PREC_FP64 = 1      /* FP64 geometry arithmetic, exact predicates; double output */
} gwn_precision;

typedef struct gwn_mesh_s* gwn_mesh;

typedef struct {
    int64_t nv, nf;          /* vertices and triangles given to gwn_build_mesh */
    int64_t nboundary;       /* directed boundary edges after cancellation (B) */
    int64_t nloops;          /* closed boundary loops the edges were chained into */
    int64_t nnodes;          /* internal BVH nodes (nf - 1, or 0) */
    int32_t bvh_depth;       /* deepest leaf of the BVH (root = 0) */
    int32_t qshift;          /* fixed-point scale is 2^qshift */
    double bbox[6];          /* min xyz, max xyz of the vertices */
    double qlo[3];           /* fixed-point origin: q = rint((x - qlo) * 2^qshift) */
    double build_ms;         /* wall time of the build */
    int64_t nunique;         /* distinct vertex positions after welding (nv without welding) */
    int32_t axis;            /* ray axis the mesh was built for: 0 = z, 1 = x, 2 = y */
    int32_t pad;
    double proj_area[3];     /* twice the total |projected area| on the planes normal to x, y, z
                                (filled when the axis was chosen automatically, else 0) */
} gwn_mesh_info;

typedef struct {
    int32_t weld_positions;  /* nonzero: vertices with equal float coordinates (+0 == -0) become one
                                index before the boundary is extracted, so a soup whose triangles
                                carry their own vertex copies (as in STL files) still cancels its
                                interior edges (Sec. 4.1); w is unchanged, B shrinks */
    int32_t axis;            /* direction of the crossing ray x0 (Sec. 3.2; any direction gives the
                                same w, Prop. 4.2): 0 = +z (default), 1 = +x, 2 = +y, -1 = the axis
                                with the least total projected triangle area (fewest expected
                                crossings).  The mesh is stored in the cyclically permuted frame
                                whose third axis is the ray; every query call accepts and returns
                                world coordinates, chi counts crossings along the chosen axis, and
                                grids keep the world layout (z fastest). */
    int32_t reserved[2];     /* zero */
} gwn_build_opts;

/*
 * gwn_build_mesh -- ingest a soup, quantise it, extract and chain the boundary,
 * and build the BVH, all on the device (precomputation; Sec. 5.1 excludes it
 * from query timings).
 *
 *   vx, vy, vz, vstride, nv : vertex coordinates (float32), strided as above.
 *   tri                     : nf*3 int32 vertex indices, row-major.
 *   stream                  : work is enqueued on it; the call synchronises it
 *                             before returning (it reads back sizes).
 *   out                     : receives the new handle (NULL on failure).
 *
 * Fixed-point grid: with bbox [lo, hi] and e = max extent (1 if zero), the
 * origin is lo - 0.75 e per axis and the scale 2^k with k the largest integer
 * such that 2.5 e 2^k <= 2^30 - 1; q = rint((x - origin) 2^k) in FP64.
 * Boundary chain by vertex index: net multiplicity m(u,v) = #(u->v) - #(v->u),
 * emitted |m| times; triangles with a repeated index contribute nothing.
 * Errors: GWN_E_INVALID for nv < 0, nf < 0, null pointers with n > 0,
 * indices outside [0, nv), non-finite coordinates or nv >= 2^31.
 */
gwn_status gwn_build_mesh(const float* vx, const float* vy, const float* vz, int64_t vstride, int64_t nv,
                          const int32_t* tri, int64_t nf, void* stream, gwn_mesh* out);

/* gwn_build_mesh with options (opts may be NULL: the defaults of gwn_build_mesh). */
gwn_status gwn_build_mesh_opts(const float* vx, const float* vy, const float* vz, int64_t vstride, int64_t nv,
                               const int32_t* tri, int64_t nf, const gwn_build_opts* opts, void* stream,
                               gwn_mesh* out);

/* Host-side copy of the mesh's sizes and fixed-point parameters. */
gwn_status gwn_mesh_info_get(gwn_mesh m, gwn_mesh_info* out);

/* Release the handle and its device memory (NULL is a no-op). */
gwn_status gwn_mesh_destroy(gwn_mesh m);

/*
 * Per-mesh query tuning.  Three choices of the query paths depend on the mesh
 * and the device, not on the arithmetic: the largest batch that gives each
 * point a workgroup with the boundary edges split among its lanes (per
 * precision; this changes the summation order of w, i.e. its last bits), the
 * smallest batch worth a Morton order of the points for the crossing walk (no
 * result changes), and the grid kernel's samples per lane (per precision;
 * w's last bits).  Crossing counts never change.  A field of 0 takes the
 * built-in rule (split: at most 8,192 points on meshes with at least 4,096
 * boundary edges; order: at least 2^18 points on meshes of at least 2^15
 * triangles; samples: the largest of 8 (FP32) or 4 (FP64), 4, 2, 1 that the
 * column length fills), -1 never (split, order).  The environment variables
 * GWN_SPLIT_BOUNDARY, GWN_ORDER_QUERIES and GWN_GRID_SAMPLES_PER_LANE override
 * any tuning.
 *
 * gwn_mesh_set_tuning / gwn_mesh_get_tuning: host-side, no device work.
 *   Errors: GWN_E_INVALID for thresholds below -1 or samples per lane other
 *   than 0, 1, 2, 4, 8 (FP64: at most 4).
 * gwn_mesh_autotune: for opts->prec, times each candidate on the device with
 *   points drawn uniformly in the mesh's bounding box -- split against one
 *   lane per point for 256 .. 32,768 points, ordered against unordered for
 *   2^20 down to 2^14 points, and, when opts->grid_nz > 0, samples per lane on
 *   a 64 x 64 x grid_nz grid over the box -- keeping the fastest (the smallest
 *   of opts->reps timings, default 3), and sets the mesh's tuning.  With
 *   opts->cache (a JSON-lines file), a choice stored for the same device
 *   architecture, triangle and boundary-edge counts (as powers of two),
 *   precision and grid_nz is applied without timing, and a new one is
 *   appended.  Allocates about 16 MB (more for large grid_nz) and synchronises
 *   `stream`.  opts may be NULL (FP32, no grid, no cache).
 */
typedef struct {
    int32_t split_max_points[2];       /* per precision (index GWN_PREC_FP32, GWN_PREC_FP64) */
    int32_t order_min_points;
    int32_t grid_samples_per_lane[2];  /* per precision */
    int32_t tuned;                     /* get only: bit p set when precision p was tuned by gwn_mesh_autotune */
} gwn_query_tuning;

typedef struct {
    int32_t prec;            /* GWN_PREC_FP32 or GWN_PREC_FP64 */
    int32_t grid_nz;         /* column length of the grids to tune for; 0 = leave the grid choice */
    int32_t reps;            /* timings per candidate; 0 = 3 */
    int32_t reserved;        /* zero */
    const char* cache;       /* nullable JSON-lines cache file */
} gwn_autotune_opts;

gwn_status gwn_mesh_set_tuning(gwn_mesh m, const gwn_query_tuning* t);
gwn_status gwn_mesh_get_tuning(gwn_mesh m, gwn_query_tuning* out);
gwn_status gwn_mesh_autotune(gwn_mesh m, const gwn_autotune_opts* opts, void* stream);

/*
 * gwn_query_batch -- w for nq arbitrary points (Alg. 1 per point).
 *
 *   qx, qy, qz, qstride, nq : query coordinates (float32), strided.
 *   prec                    : GWN_PREC_FP32 (w_out is float*) or GWN_PREC_FP64 (double*).
 *   w_out                   : nq results.
 *   chi_out                 : nullable; nq int32 crossing counts along +z.
 * nq == 0 is a no-op.  Queries on the surface get a well-defined chi; their w is
 * not meaningful (w is undefined on M).  A point's w does not depend on the
 * other points of the call or their order, and repeated calls give the same
 * bits; gwn_query_multi gives the same bits too.  The one exception is the
 * summation order: small batches (at most 8,192 points on meshes with at least
 * 4,096 boundary edges, or the mesh's tuning, see gwn_mesh_set_tuning) give
 * each point a workgroup that splits its edges among lanes (GWN_SPLIT_BOUNDARY=
 * 0/1 overrides), which agrees with the other form to rounding.
 */
gwn_status gwn_query_batch(gwn_mesh m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                           int64_t nq, int32_t prec, void* w_out, int32_t* chi_out, void* stream);

/*
 * gwn_query_batch_noalloc -- gwn_query_batch for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  The same kernels and the same results, bit for bit,
 * as gwn_query_batch on the same points; no hipMalloc, hipFree or allocating
 * call is made.  Its temporaries (a crossing-count buffer when chi_out is
 * NULL, the traversal order of dense batches and that order's sort scratch)
 * live in one fixed array of 29 MiB per GPU, held by the library on every GPU
 * it runs on until the process ends.  That array is shared by every call on
 * the GPU and keeps the last call's contents: calls that overlap on one GPU
 * (other streams, other host threads) race and must be serialised by the
 * caller.  At most GWN_NOALLOC_MAX_POINTS points per call; larger nq returns
 * GWN_E_INVALID (split the batch).  Arguments and other errors as for
 * gwn_query_batch.
 */
#define GWN_NOALLOC_MAX_POINTS 1048576
gwn_status gwn_query_batch_noalloc(gwn_mesh m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                                   int64_t nq, int32_t prec, void* w_out, int32_t* chi_out, void* stream);

/*
 * gwn_query_grid -- w on a cell-centred regular grid, reusing one ray per
 * (x, y) column for all its points (Sec. 4.3.1, ray reuse).
 *
 *   origin, spacing, dims : host arrays of 3; point (i,j,k) is
 *                           float(origin + (idx + 0.5) * spacing) per axis,
 *                           evaluated in FP64 then rounded once.
 *   w_out, chi_out        : dims[0]*dims[1]*dims[2] results at (i*ny + j)*nz + k.
 * chi equals gwn_query_batch's at the same points bit for bit; w agrees with it
 * to rounding (the boundary sum of a column is formed in a different order),
 * and is itself deterministic for a given grid.
 */
gwn_status gwn_query_grid(gwn_mesh m, const double* origin, const double* spacing, const int64_t* dims,
                          int32_t prec, void* w_out, int32_t* chi_out, void* stream);

/*
 * gwn_query_crossings -- both signed crossing counts of each query's vertical
 * line (Sec. 3.2 with the perturbed exact predicates of Supp. Sec. 2.1):
 * chi_up = chi along x0 = +z (the count gwn_query_batch uses), chi_down = chi
 * along the antipode -z, i.e. minus the signed crossings below the query.  For
 * a closed mesh the two are equal; in general chi_up - chi_down is the signed
 * count over the whole line.  Either output (device int32[nq]) may be NULL, not
 * both.  Queries and errors as in gwn_query_batch.
 */
gwn_status gwn_query_crossings(gwn_mesh m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                               int64_t nq, int32_t* chi_up_out, int32_t* chi_down_out, void* stream);

/*
 * gwn_query_gradient -- the gradient of w with respect to the query point
 * (Supp. Sec. 4, Alg. 3): the crossing count is locally constant, so only the
 * boundary-edge term is differentiated (x0 = +z; the gradient does not depend
 * on the axis).  grad_out: device array of 3 * nq values, (dw/dx, dw/dy, dw/dz)
 * per query, float for GWN_PREC_FP32 and double for GWN_PREC_FP64.  Queries and
 * errors as in gwn_query_batch.  Undefined (may be inf/nan) on the boundary
 * curve and where w is undefined.
 */
gwn_status gwn_query_gradient(gwn_mesh m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                              int64_t nq, int32_t prec, void* grad_out, void* stream);

/*
 * gwn_query_grid_gradient -- grad w (as gwn_query_gradient) at the points of the
 * grid of gwn_query_grid, sharing each column's x/y work among its samples.
 * grad_out: 3 * nx * ny * nz values, (dw/dx, dw/dy, dw/dz) for point (i, j, k)
 * at 3 * ((i * ny + j) * nz + k); float or double by prec.  Errors as in
 * gwn_query_grid.
 */
gwn_status gwn_query_grid_gradient(gwn_mesh m, const double* origin, const double* spacing, const int64_t* dims,
                                   int32_t prec, void* grad_out, void* stream);

/*
 * gwn_query_direct -- w as the direct sum of per-triangle signed solid angles
 * (Eq. 2, each triangle's area by Eq. 6), O(F) per query, from the float
 * vertex positions given to gwn_build_mesh.  The baseline the antipodal method
 * is measured against, and an independent cross-check.  Arguments as in
 * gwn_query_batch (no crossing counts).
 */
gwn_status gwn_query_direct(gwn_mesh m, const float* qx, const float* qy, const float* qz, int64_t qstride,
                            int64_t nq, int32_t prec, void* w_out, void* stream);

/*
 * Many meshes in one launch (batched workloads of uneven size).
 *
 * gwn_multi_create prepares a plan for nmesh built meshes whose queries are
 * concatenated: mesh m owns queries [q_offsets[m], q_offsets[m+1]) of the
 * strided arrays qx, qy, qz (q_offsets: host array of nmesh+1 non-decreasing
 * values, q_offsets[0] = 0).  It splits the queries into work items (mesh,
 * query tile), orders them (largest estimated cost first by default), and
 * captures one HIP graph: reset of a work counter, crossing counts for every
 * query, and a persistent kernel whose waves claim items from the counter.
 * With opts->autotune the candidate schedules (tile size, item order, resident
 * waves, and the best of those with each mesh's queries in Morton order) are
 * timed on the real inputs and the fastest is kept; with
 * opts->tune_cache a previously stored choice for the same device and problem
 * size class is reused (and a new choice is appended).  Tuning runs the plan,
 * so it writes w_out / chi_out.
 *
 * gwn_multi_run replays the graph on `stream` (asynchronous).  The plan keeps
 * the pointers it was created with: the caller keeps the query arrays, w_out
 * (float for GWN_PREC_FP32, double for GWN_PREC_FP64) and chi_out (nullable;
 * the plan then owns a scratch buffer) alive and unchanged in size until
 * gwn_multi_destroy.  The meshes must outlive the plan.  Per query the result
 * is the same bits as gwn_query_batch at the same precision on that mesh alone
 * (one lane per query; see the split-path exception above).  Errors:
 * GWN_E_INVALID for bad arguments, an unknown prec, meshes from another device
 * or an order outside 0..3.
 */
typedef struct gwn_multi_s* gwn_multi;

typedef struct {
    int32_t item_queries;     /* queries per work item, rounded up to a multiple of 64; 0 = default or tuned */
    int32_t waves_per_simd;   /* resident persistent waves per SIMD, 1..8; 0 = default or tuned */
    int32_t order;            /* 0 = largest estimated cost first, 1 = mesh order; +2: each mesh's queries
                                 taken in Morton order of their quantised x, y (a permutation made once at
                                 creation from the query values then; results are the same bits either way) */
    int32_t autotune;         /* nonzero: time candidate schedules at creation and keep the fastest */
    const char* tune_cache;   /* nullable JSON-lines file read before tuning and appended after */
} gwn_multi_opts;

typedef struct {
    int32_t nmesh;
    int64_t nqueries;
    int32_t nitems, item_queries, waves_per_simd, order, grid_blocks, tuned;
    double est_pairs;         /* sum over meshes of queries x boundary edges */
    double tuned_ms;          /* best replay time seen by the tuner (0 if not tuned here) */
} gwn_multi_info;

gwn_status gwn_multi_create(const gwn_mesh* meshes, int32_t nmesh, const float* qx, const float* qy,
                            const float* qz, int64_t qstride, const int64_t* q_offsets, int32_t prec, void* w_out,
                            int32_t* chi_out, const gwn_multi_opts* opts, void* stream, gwn_multi* out);
gwn_status gwn_multi_run(gwn_multi plan, void* stream);
gwn_status gwn_multi_info_get(gwn_multi plan, gwn_multi_info* out);
gwn_status gwn_multi_destroy(gwn_multi plan);

/*
 * Parametric surfaces (Sec. 4.4, Alg. 2): a surface made of tensor-product
 * cubic Bezier patches, FP64 throughout.
 *
 * gwn_patches_build: cps is a DEVICE array of npatch * 16 * 3 doubles, patch k's
 *   control point P[i][j] (i along u, j along v) at ((16 k + 4 i + j) * 3); it
 *   is copied, the caller keeps ownership.  The patch's normal is S_u x S_v and
 *   its boundary runs counter-clockwise in (u, v), so w = +1 inside a closed
 *   surface whose normals point out.  The surface's boundary is the patches'
 *   boundary curves after each curve cancels the same curve traversed
 *   backwards (equal control points, +0 = -0), kept with net multiplicity.
 *   opts (nullable; zero fields take the default): tau, the tolerance of the
 *   "approximately bilinear" test of the ray-patch subdivision, relative to
 *   the control points' bounding-box diagonal (default 1e-9); eps, the
 *   absolute tolerance |K15 - G7| of each accepted quadrature interval
 *   (default 1e-11); max_depth, the deepest interval bisection (default and
 *   at most 30).  Synchronises `stream`.  Errors: GWN_E_INVALID for a null
 *   argument, npatch outside [0, 2^24] or a non-finite control point.
 * gwn_patches_query: w (double, nq) per query point (FP32 strided input, as for
 *   meshes): w = chi(x0) + (1 / 4 pi) * sum over boundary curves of the
 *   integral of the area rate of the geodesic triangle (-x0, Gamma(t),
 *   Gamma(t + dt)) (Alg. 1's edge term in the limit of short edges), by
 *   adaptive 15-point Gauss-Kronrod.  chi counts the signed crossings of the
 *   ray p + t x0, t > 0 (+1 where the ray has positive dot product with the
 *   normal).  x0 is the first of +z, (0.36, 0.48, 0.8), (-0.48, 0.6, 0.64),
 *   (0.6, -0.64, 0.48) whose ray has no tangent hit, no hit at the query, no
 *   hit within 1e-9 (in a leaf's parameters) of a subdivision leaf's edge and
 *   no hit or near miss within 4 tau of a leaf edge on a patch's boundary
 *   (Sec. 4.4.1 shoots another ray in such cases); dir_out (nullable) receives
 *   its index, or -1 with w = NaN when all four are ambiguous; chi_out
 *   (nullable) the crossing count along it.  w is independent of the choice
 *   (Prop. 4.2); chi is not.  Asynchronous on `stream`; nq = 0 is a no-op.
 *   Errors: GWN_E_INVALID for null arguments, nq < 0, qstride < 1 or another
 *   current device than the build's.
 */
typedef struct gwn_patches_s* gwn_patches;

typedef struct {
    double tau;          /* bilinear tolerance, relative to the bounding-box diagonal; 0 = 1e-9 */
    double eps;          /* |K15 - G7| per accepted interval; 0 = 1e-11 */
    int32_t max_depth;   /* deepest interval bisection; 0 = 30 */
} gwn_patch_opts;

typedef struct {
    int64_t npatch, ncurves;   /* patches; boundary curves left after cancellation */
    double tau;                /* absolute bilinear tolerance */
    double eps;
    int32_t max_depth;
    double diag;               /* bounding-box diagonal of the control points */
} gwn_patches_info;

gwn_status gwn_patches_build(const double* cps, int64_t npatch, const gwn_patch_opts* opts, void* stream,
                             gwn_patches* out);
gwn_status gwn_patches_info_get(gwn_patches h, gwn_patches_info* out);
gwn_status gwn_patches_query(gwn_patches h, const float* qx, const float* qy, const float* qz, int64_t qstride,
                             int64_t nq, double* w_out, int32_t* chi_out, int32_t* dir_out, void* stream);
/* gwn_patches_query_grid: the same on the cell-centred grid point (i, j, k) =
 * float(origin + (idx + 0.5) * spacing) (each coordinate rounded once from
 * double), outputs at (i * ny + j) * nz + k.  Each (i, j) column's vertical line
 * is intersected with the patches once and every sample counts the crossings
 * above it (ray reuse, Sec. 4.3.1); a column with an ambiguous hit, and a
 * sample within the on-surface margin of a crossing, take single rays as in
 * gwn_patches_query.  Crossing counts and directions equal
 * gwn_patches_query's at the same points; w agrees to the last bits of FP64
 * (the two paths' kernels contract their products differently).
 * counts (nullable HOST array of 2): when given, the work is also counted as
 * for gwn_patches_query_stats and the call synchronises `stream`.  Without
 * counts the boundary term along the first direction runs on a stream the
 * handle creates at its first grid call (released by gwn_patches_destroy),
 * forked from and joined back into `stream` by events, beside the column
 * kernel; calls on one handle from several host threads take turns enqueuing.
 * Errors: GWN_E_INVALID for null arguments, negative sizes, or more than 2^30
 * points or columns. */
gwn_status gwn_patches_query_grid(gwn_patches h, const double* origin, const double* spacing, const int64_t* dims,
                                  double* w_out, int32_t* chi_out, int32_t* dir_out, int64_t* counts,
                                  void* stream);
/* The same evaluation (w only) that also counts its work: counts[0] = quadrature
 * intervals (15 integrand evaluations each), counts[1] = sub-patch cells
 * extracted by the ray subdivision, summed over the queries (nq <= 2^30).
 * counts is a HOST array of 2; synchronises `stream`; for measurement. */
gwn_status gwn_patches_query_stats(gwn_patches h, const float* qx, const float* qy, const float* qz,
                                   int64_t qstride, int64_t nq, double* w_out, int64_t* counts, void* stream);
gwn_status gwn_patches_destroy(gwn_patches h);

/*
 * Learned surrogate (a Fourier-feature MLP standing in for far-field queries;
 * not part of the paper's method, whose nearest item is its closing remark on
 * approximating the fractional part of w quickly, Sec. 6).
 *
 * Network: gamma(p) = [sin 2piGp, cos 2piGp] with G (32x3) ~ N(0, sigma^2)
 * fixed at creation; four GELU layers 64->128->128->128->128; linear output
 * 128->1.  Training's matrix products use bf16 MFMA with fp32 accumulation
 * and the erf form of GELU; gwn_mlp_forward uses half-precision operands (the
 * bf16 weights carried over exactly, activations rounded to half, fp32
 * accumulation) and a polynomial GELU in packed half arithmetic (within
 * 2.9e-3 |z|), or the training arithmetic when the environment variable
 * GWN_INFER_GELU is "erf".  Adam updates fp32 master weights.  Parameters form one flat vector of GWN_MLP_NPARAMS
 * floats: W1 (64x128, row-major [in][out]), b1, W2, b2, W3, b3, W4, b4, W5
 * (128), b5.  Loss: mean squared error.  A handle (gwn_mlp, also called
 * gwn_surrogate) is bound to the device current at its creation.
 *
 *   gwn_mlp_create: a new network; G and the weights are drawn from `seed`
 *     (splitmix64 stream; Box-Muller normals for G, uniform +-sqrt(6/fan_in)
 *     weights, zero biases).
 *   gwn_mlp_get_state / gwn_mlp_set_state copy the state between the device and
 *     HOST arrays (each nullable: theta and the Adam moments m, v of
 *     GWN_MLP_NPARAMS floats, G of 96 floats, the step counter; step < 0 keeps
 *     it).  They synchronise the device.
 *   gwn_mlp_forward: y_out[i] = network(q_i) for n device points (pre-
 *     activations beyond the half range, |z| > 65504, overflow there).
 *   gwn_mlp_loss_grad: gradient of the loss over the n points with targets
 *     `target` into grad_out (device, nullable) and the loss (host, nullable).
 *   gwn_mlp_train_step: the same, then one Adam step (lr; beta1 0.9, beta2
 *     0.999, eps 1e-8, bias-corrected by the handle's step count).
 * The training scratch is owned by the handle and sized to the largest batch;
 * n must be < 2^31.
 */
#define GWN_MLP_NPARAMS 57985

typedef struct gwn_mlp_s* gwn_mlp;
typedef gwn_mlp gwn_surrogate;

gwn_status gwn_mlp_create(uint64_t seed, double fourier_sigma, gwn_mlp* out);
gwn_status gwn_mlp_destroy(gwn_mlp h);
gwn_status gwn_mlp_get_state(gwn_mlp h, float* theta, float* adam_m, float* adam_v, float* G, int64_t* step);
gwn_status gwn_mlp_set_state(gwn_mlp h, const float* theta, const float* adam_m, const float* adam_v,
                             const float* G, int64_t step);
gwn_status gwn_mlp_forward(gwn_mlp h, const float* qx, const float* qy, const float* qz, int64_t qstride,
                           int64_t n, float* y_out, void* stream);
gwn_status gwn_mlp_loss_grad(gwn_mlp h, const float* qx, const float* qy, const float* qz, int64_t qstride,
                             const float* target, int64_t n, float* grad_out, float* loss_out, void* stream);
gwn_status gwn_mlp_train_step(gwn_mlp h, const float* qx, const float* qy, const float* qz, int64_t qstride,
                              const float* target, int64_t n, float lr, float* loss_out, void* stream);

/*
 * gwn_surrogate_train -- fit the network to w on `mesh`, labels generated by the
 * method itself (the exact FP32 path of gwn_query_batch).
 *
 * Data: with X == NULL the library draws cfg->n_train points uniformly in the
 *   box [box_lo, box_hi] (both all zero: the mesh's bounding box) from
 *   cfg->seed -- coordinate c of point i is lo_c + u (hi_c - lo_c), u the top 53
 *   bits of splitmix64 at counter 3 i + c + 1 over 2^53, rounded once to float --
 *   labels them, and keeps points and labels in the handle (16 bytes per
 *   point).  Otherwise X is a DEVICE (n, 3) float array of the caller's points
 *   (interleaved, stride 3) with labels T (device, n floats), or T == NULL to
 *   have them labelled on `mesh` (kept in the handle).  `mesh` may be NULL only
 *   when both X and T are given.
 * Schedule: cfg->epochs passes over the data in mini-batches of cfg->batch
 *   points (the last batch of a pass may be smaller); every pass visits the
 *   points in a new random order, a keyed permutation that is a pure function
 *   of (cfg->seed, pass number), evaluated on the device; the learning rate of
 *   step k of the K-step schedule is lr_final + (lr - lr_final)(1 + cos(pi k /
 *   (K - 1)))/2; one Adam step per batch.
 * Resumption: the handle records the schedule and the data recipe it trains
 *   under and how many passes are done; a call trains up to pass
 *   cfg->stop_epoch (0 = cfg->epochs) and returns.  A later call -- on the same
 *   handle, or on one made by gwn_surrogate_load -- with the same cfg and mesh
 *   continues where it stopped, with the same bits as an uninterrupted run (the
 *   shuffle and the learning rate depend only on the pass and step numbers, and
 *   generated data are re-made identically).  A call with another schedule or
 *   recipe on a handle that has trained passes returns GWN_E_INVALID.
 * epoch_loss (HOST, nullable): one float per pass trained by this call, the
 *   mean of its batches' losses; *epochs_run (HOST, nullable) receives the
 *   number of passes trained.  Synchronises `stream` at the end.
 * Errors: GWN_E_INVALID for a null handle, n_train or n outside [1, 2^31),
 *   batch < 1, epochs < 1, lr or lr_final negative or not finite, an empty or
 *   inverted box, or a mesh from another device.
 */
typedef struct {
    uint64_t seed;           /* training points and the per-pass shuffles */
    int64_t n_train;         /* generated points (when X is NULL) */
    double box_lo[3];        /* box of the generated points; lo = hi = 0: the mesh's bounding box */
    double box_hi[3];
    int32_t epochs;          /* passes in the schedule */
    int32_t batch;           /* points per Adam step */
    float lr;                /* learning rate at the first step */
    float lr_final;          /* ... at the last step of the schedule */
    int32_t stop_epoch;      /* train until this many passes are done (0 = epochs) */
    int32_t reserved;        /* zero */
} gwn_surrogate_cfg;

gwn_status gwn_surrogate_train(gwn_surrogate h, gwn_mesh mesh, const gwn_surrogate_cfg* cfg, const float* X,
                               const float* T, int64_t n, float* epoch_loss, int64_t* epochs_run, void* stream);

/*
 * gwn_surrogate_save -- write the handle's complete state to `path` (a host
 * file, replaced atomically): a fixed header (magic "GWNSURR1", format
 * version 2, sizes, Adam step count, passes done, sigma, the seeds, the data
 * recipe and the schedule of the run in progress, the labelling mesh's
 * triangle and boundary-edge counts), then G, the fp32 master weights, the
 * Adam moments m and v, the three bf16 copies the kernels read (the half copy
 * of inference is not stored: loading re-derives it), and an FNV-1a
 * 64-bit checksum of everything before it; little-endian.  Synchronises the
 * device.  GWN_E_INVALID if the file cannot be written.
 *
 * gwn_surrogate_load -- a new handle on the current device from such a file.
 * The bf16 copies are re-derived from the fp32 masters and must equal the
 * stored ones.  GWN_E_INVALID for a missing, truncated, corrupted (checksum)
 * or foreign file.  Training data are not stored: a resumed gwn_surrogate_train
 * re-makes them from the recorded recipe.
 *
 * gwn_surrogate_destroy -- release the handle (NULL is a no-op); the same as
 * gwn_mlp_destroy.
 */
gwn_status gwn_surrogate_save(gwn_surrogate h, const char* path);
gwn_status gwn_surrogate_load(const char* path, gwn_surrogate* out);
gwn_status gwn_surrogate_destroy(gwn_surrogate h);

/*
 * gwn_surrogate_query -- w_out = network prediction, except for points the
 * fallback rule marks, which are re-evaluated by the exact FP32 path
 * (gwn_query_batch) on `mesh`:
 *   rule GWN_BAND_HALF (0): |prediction - 1/2| < band (uncertain between
 *     outside, w = 0, and inside, w = 1);
 *   rule GWN_BAND_FRAC (1): |frac(prediction) - 1/2| < band, i.e. the
 *     prediction lies within band of a half-integer (uncertain between any two
 *     consecutive winding levels, as where surfaces overlap).
 * band > 1/2 under rule 1 re-evaluates every point (at 1/2 a prediction that is
 * exactly an integer keeps its value).  fallback_out (device,
 * nullable) flags the re-evaluated points and *nfallback_out (host, nullable)
 * counts them.  The exact values are bit-identical to gwn_query_batch's at the
 * same points.  The call synchronises the stream once, to size the exact
 * evaluation by that count.  Errors: GWN_E_INVALID for band < 0, a rule other
 * than 0 or 1, and as for gwn_query_batch.
 */
#define GWN_BAND_HALF 0
#define GWN_BAND_FRAC 1
gwn_status gwn_surrogate_query(gwn_surrogate h, gwn_mesh mesh, const float* qx, const float* qy, const float* qz,
                               int64_t qstride, int64_t n, float band, int32_t rule, float* w_out,
                               uint8_t* fallback_out, int64_t* nfallback_out, void* stream);

const char* gwn_status_str(gwn_status s);
const char* gwn_last_error(void);   /* thread-local; "" if none */

#ifdef __cplusplus
}
#endif

#endif /* GWN_H */
