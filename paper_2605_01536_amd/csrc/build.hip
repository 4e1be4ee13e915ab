// build.hip -- device-side mesh ingest (gwn_build_mesh):
//   vertex statistics and validation, fixed-point quantisation, Morton-ordered
//   LBVH with integer boxes (Karras-style split search, bottom-up refit), and
//   the directed boundary chain of the soup (Sec. 4.1: interior edges cancel),
//   chained into closed loops so that the query kernels visit every boundary
//   vertex once.  Sorting and scans use the library's radix sort and scan
//   (sort.hip); everything else is below.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "gwn_alloc.h"
#include "gwn_mesh.h"
#include "gwn_sort.h"

namespace gwn {
namespace {

constexpr int kThreads = 256;

inline int nblocks(int64_t n, int t = kThreads) {
    int64_t b = (n + t - 1) / t;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 20));
}

// ------------------------------------------------------------------ helpers

// Build temporaries, released when the build returns -- also on an error path,
// where kernels enqueued before the failure may still be running: the stream is
// drained first.
struct Scratch {
    std::vector<void*> ptrs;
    hipStream_t st = nullptr;
    ~Scratch() {
        if (!ptrs.empty()) (void)hipStreamSynchronize(st);
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <class T>
    hipError_t alloc(T** p, int64_t n) {
        *p = nullptr;
        hipError_t e = gwn::dmalloc((void**)p, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
};

// ------------------------------------------------------------------ kernels

__global__ void k_vertex_stats(const float* __restrict__ vx, const float* __restrict__ vy, const float* __restrict__ vz,
                               int64_t vs, int64_t nv, float* __restrict__ part, int* __restrict__ flags) {
    __shared__ float sm[6][kThreads];
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        float p[3] = {vx[i * vs], vy[i * vs], vz[i * vs]};
        for (int a = 0; a < 3; ++a) {
            bad |= !isfinite(p[a]);
            mn[a] = fminf(mn[a], p[a]);
            mx[a] = fmaxf(mx[a], p[a]);
        }
    }
    if (bad) atomicOr(flags, 1);
    for (int a = 0; a < 3; ++a) {
        sm[a][threadIdx.x] = mn[a];
        sm[3 + a][threadIdx.x] = mx[a];
    }
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int a = 0; a < 3; ++a) {
                sm[a][threadIdx.x] = fminf(sm[a][threadIdx.x], sm[a][threadIdx.x + s]);
                sm[3 + a][threadIdx.x] = fmaxf(sm[3 + a][threadIdx.x], sm[3 + a][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 6; ++a) part[blockIdx.x * 6 + a] = sm[a][0];
}

__global__ void k_tri_check(const int32_t* __restrict__ tri, int64_t n3, int64_t nv, int* __restrict__ flags) {
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = tri[i];
        bad |= (v < 0) | ((int64_t)v >= nv);
    }
    if (bad) atomicOr(flags, 2);
}

__global__ void k_quantize_vertices(const float* __restrict__ vx, const float* __restrict__ vy,
                                    const float* __restrict__ vz, int64_t vs, int64_t nv, QGrid g,
                                    int4* __restrict__ qv) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nv) return;
    int4 q;
    q.x = (int)qround(vx[i * vs], g.lo[0], g.scale);
    q.y = (int)qround(vy[i * vs], g.lo[1], g.scale);
    q.z = (int)qround(vz[i * vs], g.lo[2], g.scale);
    q.w = 0;
    qv[i] = q;
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 1023u;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void k_tri_setup(const int32_t* __restrict__ tri, int64_t nf, const int4* __restrict__ qv, int4 qlo,
                            int4 qspan, TriQ* __restrict__ tq, uint64_t* __restrict__ keys) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nf) return;
    int4 a = qv[tri[3 * t]], b = qv[tri[3 * t + 1]], c = qv[tri[3 * t + 2]];
    TriQ r;
    r.a = a;
    r.b = b;
    r.c = c;
    tq[t] = r;
    long long cx = ((long long)a.x + b.x + c.x) / 3 - qlo.x;
    long long cy = ((long long)a.y + b.y + c.y) / 3 - qlo.y;
    long long cz = ((long long)a.z + b.z + c.z) / 3 - qlo.z;
    uint32_t mx = (uint32_t)((cx * 1024) / ((long long)qspan.x + 1));
    uint32_t my = (uint32_t)((cy * 1024) / ((long long)qspan.y + 1));
    uint32_t mz = (uint32_t)((cz * 1024) / ((long long)qspan.z + 1));
    uint32_t m = (spread10(mx) << 2) | (spread10(my) << 1) | spread10(mz);
    keys[t] = ((uint64_t)m << 32) | (uint64_t)t;
}

__global__ void k_permute_tris(const uint64_t* __restrict__ keys, int64_t nf, const TriQ* __restrict__ src,
                               TriQ* __restrict__ dst, const int32_t* __restrict__ tri, const float* __restrict__ vx,
                               const float* __restrict__ vy, const float* __restrict__ vz, int64_t vs,
                               float4* __restrict__ trif) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int64_t t = (int64_t)(keys[i] & 0xffffffffull);
    dst[i] = src[t];
    for (int c = 0; c < 3; ++c) {
        const int64_t v = tri[3 * t + c];
        trif[3 * i + c] = make_float4(vx[v * vs], vy[v * vs], vz[v * vs], 0.f);
    }
}

__device__ __forceinline__ int prefix_len(const uint64_t* __restrict__ keys, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    return __clzll((long long)(keys[i] ^ keys[j]));   // keys are unique (index in the low bits)
}

// Karras (2012) radix-tree construction over the sorted unique keys: node i
// spans a key range found by exponential + binary search on the common-prefix
// length; its split is where the prefix length drops.
__global__ void k_karras(const uint64_t* __restrict__ keys, int n, Node* __restrict__ nodes, int* __restrict__ leaf_parent) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = (prefix_len(keys, n, i, i + 1) - prefix_len(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = prefix_len(keys, n, i, i - d);
    int lmax = 2;
    while (prefix_len(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(keys, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = prefix_len(keys, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix_len(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int gamma = i + s * d + min(d, 0);
    int left = (min(i, j) == gamma) ? ~gamma : gamma;
    int right = (max(i, j) == gamma + 1) ? ~(gamma + 1) : gamma + 1;
    nodes[i].link.x = left;
    nodes[i].link.y = right;
    if (left >= 0) nodes[left].link.z = i;
    else leaf_parent[~left] = i;
    if (right >= 0) nodes[right].link.z = i;
    else leaf_parent[~right] = i;
}

__device__ __forceinline__ int ld_acq(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void write_slot(Node* nodes, int parent, int child, const int b[6]) {
    Node* p = nodes + parent;
    if (p->link.x == child) {
        p->lxy = make_int4(b[0], b[1], b[2], b[3]);
        p->z.x = b[4];
        p->z.y = b[5];
    } else {
        p->rxy = make_int4(b[0], b[1], b[2], b[3]);
        p->z.z = b[4];
        p->z.w = b[5];
    }
}

// Bottom-up refit: each leaf writes its box into its parent's child slot; the
// second thread to reach a node merges both slots and continues upward.
__global__ void k_refit(const TriQ* __restrict__ tris, int n, Node* nodes, const int* __restrict__ leaf_parent,
                        int* flags) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n || n < 2) return;
    TriQ q = tris[t];
    int b[6] = {min(q.a.x, min(q.b.x, q.c.x)), max(q.a.x, max(q.b.x, q.c.x)),
                min(q.a.y, min(q.b.y, q.c.y)), max(q.a.y, max(q.b.y, q.c.y)),
                min(q.a.z, min(q.b.z, q.c.z)), max(q.a.z, max(q.b.z, q.c.z))};
    int child = ~t;
    int parent = leaf_parent[t];
    for (int guard = 0; parent >= 0; ++guard) {
        if (guard > 70) {           // a radix tree over 62-bit keys is at most 63 deep
            atomicOr(flags + n, 4);
            return;
        }
        write_slot(nodes, parent, child, b);
        __threadfence();
        if (atomicAdd(flags + parent, 1) == 0) return;
        __threadfence();
        const int* L = &nodes[parent].lxy.x;
        const int* R = &nodes[parent].rxy.x;
        const int* Z = &nodes[parent].z.x;
        b[0] = min(ld_acq(L + 0), ld_acq(R + 0));
        b[1] = max(ld_acq(L + 1), ld_acq(R + 1));
        b[2] = min(ld_acq(L + 2), ld_acq(R + 2));
        b[3] = max(ld_acq(L + 3), ld_acq(R + 3));
        b[4] = min(ld_acq(Z + 0), ld_acq(Z + 2));
        b[5] = max(ld_acq(Z + 1), ld_acq(Z + 3));
        child = parent;
        parent = ld_acq(&nodes[parent].link.z);
    }
}

__global__ void k_depth(int n, const Node* __restrict__ nodes, const int* __restrict__ leaf_parent, int* depth) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n || n < 2) return;
    int d = 0;
    for (int p = leaf_parent[t]; p >= 0 && d < 1000; p = nodes[p].link.z) ++d;
    atomicMax(depth, d);
}

// ---- boundary chain

__global__ void k_edge_keys(const int32_t* __restrict__ tri, int64_t nf, uint64_t* __restrict__ keys,
                            int* __restrict__ sgn) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= 3 * nf) return;
    int64_t t = i / 3;
    int c = (int)(i - 3 * t);
    uint32_t u = (uint32_t)tri[3 * t + c];
    uint32_t v = (uint32_t)tri[3 * t + (c + 1) % 3];
    if (u == v) {
        keys[i] = ~0ull;
        sgn[i] = 0;
    } else {
        keys[i] = ((uint64_t)min(u, v) << 32) | (uint64_t)max(u, v);
        sgn[i] = u < v ? 1 : -1;
    }
}

// net multiplicity per unordered vertex pair, stored at the first entry of its run
__global__ void k_edge_runs(const uint64_t* __restrict__ keys, const int* __restrict__ sgn, int64_t n,
                            int* __restrict__ net, int* __restrict__ cnt) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t k = keys[i];
    bool head = (k != ~0ull) && (i == 0 || keys[i - 1] != k);
    int m = 0;
    if (head)
        for (int64_t j = i; j < n && keys[j] == k; ++j) m += sgn[j];
    net[i] = m;
    cnt[i] = head ? abs(m) : 0;
}

__global__ void k_edge_emit(const uint64_t* __restrict__ keys, const int* __restrict__ net, const int* __restrict__ cnt,
                            const int* __restrict__ off, int64_t n, int* __restrict__ efrom, int* __restrict__ eto) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n || cnt[i] == 0) return;
    int lo = (int)(keys[i] >> 32), hi = (int)(keys[i] & 0xffffffffull);
    int m = net[i];
    for (int r = 0; r < cnt[i]; ++r) {
        efrom[off[i] + r] = m > 0 ? lo : hi;
        eto[off[i] + r] = m > 0 ? hi : lo;
    }
}

__global__ void k_iota(int* __restrict__ a, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) a[i] = (int)i;
}

// in-degree == out-degree at every vertex, so the k-th edge sorted by target
// and the k-th edge sorted by source meet at the same vertex
__global__ void k_link(const int* __restrict__ in_by_to, const int* __restrict__ out_by_from, int64_t n,
                       int* __restrict__ succ) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) succ[in_by_to[k]] = out_by_from[k];
}

__global__ void k_rep_round(const int* __restrict__ rep, const int* __restrict__ jmp, int64_t n, int* __restrict__ rep2,
                            int* __restrict__ jmp2) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int j = jmp[i];
    rep2[i] = min(rep[i], rep[j]);
    jmp2[i] = jmp[j];
}

__global__ void k_rank_init(const int* __restrict__ succ, const int* __restrict__ rep, int64_t n, int* __restrict__ nxt,
                            int* __restrict__ dist) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int s = succ[i];
    nxt[i] = (s == rep[i]) ? -1 : s;
    dist[i] = (s == rep[i]) ? 0 : 1;
}

__global__ void k_rank_round(const int* __restrict__ nxt, const int* __restrict__ dist, int64_t n, int* __restrict__ nxt2,
                             int* __restrict__ dist2) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int j = nxt[i];
    if (j < 0) {
        nxt2[i] = -1;
        dist2[i] = dist[i];
    } else {
        nxt2[i] = nxt[j];
        dist2[i] = dist[i] + dist[j];
    }
}

__global__ void k_loop_counts(const int* __restrict__ rep, const int* __restrict__ dist, int64_t n, int* __restrict__ len,
                              int* __restrict__ head) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool h = rep[i] == (int)i;
    len[i] = h ? dist[i] + 1 : 0;
    head[i] = h ? 1 : 0;
}

__global__ void k_emit_loops(const int* __restrict__ efrom, const int* __restrict__ rep, const int* __restrict__ dist,
                             const int* __restrict__ voff, const int* __restrict__ lid, int64_t n, const float* __restrict__ vx,
                             const float* __restrict__ vy, const float* __restrict__ vz, int64_t vs,
                             const int4* __restrict__ qv, float scalef, BVert* __restrict__ bv, int* __restrict__ loop_off) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int r = rep[i];
    int pos = dist[r] - dist[i];
    int slot = voff[r] + pos;
    if (r < 0 || r >= n || pos < 0 || slot < 0 || slot >= n) return;   // unreachable for a balanced chain
    int v = efrom[i];
    BVert b;
    b.x = vx[(int64_t)v * vs] * scalef;
    b.y = vy[(int64_t)v * vs] * scalef;
    b.z = vz[(int64_t)v * vs] * scalef;
    int4 q = qv[v];
    b.qx = q.x;
    b.qy = q.y;
    b.pad0 = v;
    b.pad1 = 0;
    b.loop = lid[r];   // lid is the loop index at each loop's representative only
    bv[slot] = b;
    if (r == (int)i) loop_off[lid[i]] = voff[i];
}

// ---------------------------------------------------------------- ray axis
// Twice the triangles' total |projected area| on the planes normal to x, y, z:
// the expected number of crossings of a random line along that axis scales
// with it.  Per-block partial sums, written by one lane each.
__global__ __launch_bounds__(kThreads) void k_proj_area(const float* __restrict__ vx, const float* __restrict__ vy,
                                                         const float* __restrict__ vz, int64_t vs,
                                                         const int32_t* __restrict__ tri, int64_t nf,
                                                         double* __restrict__ part) {
    __shared__ double sm[3][kThreads];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < nf; t += (int64_t)gridDim.x * kThreads) {
        double p[3][3];
        for (int c = 0; c < 3; ++c) {
            const int64_t v = tri[3 * t + c];
            p[c][0] = vx[v * vs];
            p[c][1] = vy[v * vs];
            p[c][2] = vz[v * vs];
        }
        const double ux = p[1][0] - p[0][0], uy = p[1][1] - p[0][1], uz = p[1][2] - p[0][2];
        const double wx = p[2][0] - p[0][0], wy = p[2][1] - p[0][1], wz = p[2][2] - p[0][2];
        acc[0] += fabs(uy * wz - uz * wy);
        acc[1] += fabs(uz * wx - ux * wz);
        acc[2] += fabs(ux * wy - uy * wx);
    }
    for (int a = 0; a < 3; ++a) sm[a][threadIdx.x] = acc[a];
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int a = 0; a < 3; ++a) sm[a][threadIdx.x] += sm[a][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) part[blockIdx.x * 3 + a] = sm[a][0];
}

// ---------------------------------------------------------------- welding
// Vertices with equal float coordinates (+0 and -0 equal) become one index, the
// smallest: sort by (x, y, z) bit patterns (stable LSD passes), find runs, map.

__device__ __forceinline__ uint32_t weld_bits(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x7fffffffu) == 0u ? 0u : b;
}

__global__ void k_weld_zkeys(const float* __restrict__ vz, int64_t vs, int64_t nv, uint32_t* __restrict__ kz,
                             int* __restrict__ idx) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nv) return;
    kz[i] = weld_bits(vz[i * vs]);
    idx[i] = (int)i;
}

__global__ void k_weld_xykeys(const float* __restrict__ vx, const float* __restrict__ vy, int64_t vs, int64_t nv,
                              const int* __restrict__ idx, uint64_t* __restrict__ kxy) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nv) return;
    const int64_t v = idx[j];
    kxy[j] = ((uint64_t)weld_bits(vx[v * vs]) << 32) | weld_bits(vy[v * vs]);
}

// run start of each sorted position (0 where the position continues a run)
__global__ void k_weld_heads(const float* __restrict__ vz, int64_t vs, int64_t nv, const uint64_t* __restrict__ kxy,
                             const int* __restrict__ idx, int* __restrict__ head) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nv) return;
    bool h = j == 0;
    if (!h) h = kxy[j] != kxy[j - 1] || weld_bits(vz[(int64_t)idx[j] * vs]) != weld_bits(vz[(int64_t)idx[j - 1] * vs]);
    head[j] = h ? (int)j : 0;
}

__global__ void k_weld_map(const int* __restrict__ idx, const int* __restrict__ start, int64_t nv,
                           int* __restrict__ remap, int* __restrict__ nunique) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nv) return;
    const int s = start[j];
    remap[idx[j]] = idx[s];   // the stable sort keeps the smallest index first in a run
    if (s == (int)j) atomicAdd(nunique, 1);
}

__global__ void k_weld_tris(const int32_t* __restrict__ tri, int64_t n3, const int* __restrict__ remap,
                            int32_t* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n3) return;
    out[i] = remap[tri[i]];
}

// runs f(temp) with `bytes` of build scratch
template <class F>
hipError_t with_temp(Scratch& S, size_t bytes, F&& f) {
    char* tmp = nullptr;
    hipError_t e = S.alloc(&tmp, (int64_t)bytes);
    if (e != hipSuccess) return e;
    return f((void*)tmp);
}

int bits_for(int64_t n) {
    int b = 1;
    while ((1ll << b) < n) ++b;
    return b;
}

}  // namespace

QGrid make_qgrid(const double bbox[6]) {
    QGrid g;
    double e = 0.0;
    for (int a = 0; a < 3; ++a) e = std::max(e, bbox[3 + a] - bbox[a]);
    if (!(e > 0.0)) e = 1.0;
    for (int a = 0; a < 3; ++a) g.lo[a] = bbox[a] - 0.75 * e;
    const double ext = 2.5 * e;
    const double qmax = (double)kQMax;
    int k = 0;
    if (std::ldexp(ext, 0) <= qmax) {
        while (std::ldexp(ext, k + 1) <= qmax) ++k;
    } else {
        while (std::ldexp(ext, k) > qmax) --k;
    }
    g.k = k;
    g.scale = std::ldexp(1.0, k);
    g.scalef = std::ldexp(1.0f, k);
    return g;
}

gwn_status build_mesh(const float* vx, const float* vy, const float* vz, int64_t vs, int64_t nv, const int32_t* tri,
                      int64_t nf, bool weld, int axis, hipStream_t st, gwn_mesh_s* m) {
    auto t0 = std::chrono::steady_clock::now();
    Scratch S;
    S.st = st;
    int loop_tail = 0;
    m->nv = nv;
    m->nf = nf;
    GWN_HIP_TRY(hipGetDevice(&m->device));

    // ---- vertex statistics and validation
    int* flags = nullptr;
    GWN_HIP_TRY(S.alloc(&flags, 1));
    GWN_HIP_TRY(hipMemsetAsync(flags, 0, sizeof(int), st));
    const int sb = 256;
    float* part = nullptr;
    GWN_HIP_TRY(S.alloc(&part, sb * 6));
    if (nv > 0) {
        k_vertex_stats<<<sb, kThreads, 0, st>>>(vx, vy, vz, vs, nv, part, flags);
        GWN_HIP_TRY(hipGetLastError());
    }
    if (nf > 0) {
        k_tri_check<<<std::min(nblocks(3 * nf), 4096), kThreads, 0, st>>>(tri, 3 * nf, nv, flags);
        GWN_HIP_TRY(hipGetLastError());
    }
    std::vector<float> hpart(sb * 6);
    int hflags = 0;
    if (nv > 0) GWN_HIP_TRY(hipMemcpyAsync(hpart.data(), part, sizeof(float) * sb * 6, hipMemcpyDeviceToHost, st));
    GWN_HIP_TRY(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, st));
    GWN_HIP_TRY(hipStreamSynchronize(st));
    if (hflags & 1) {
        set_error("gwn_build_mesh: non-finite vertex coordinate");
        return GWN_E_INVALID;
    }
    if (hflags & 2) {
        set_error("gwn_build_mesh: triangle index outside [0, %lld)", (long long)nv);
        return GWN_E_INVALID;
    }
    // ---- ray axis: least total projected area (fewest expected crossings) when asked
    if (axis < 0) {
        axis = 0;
        if (nf > 0) {
            const int pb = 256;
            double* pa = nullptr;
            GWN_HIP_TRY(S.alloc(&pa, 3 * pb));
            k_proj_area<<<pb, kThreads, 0, st>>>(vx, vy, vz, vs, tri, nf, pa);
            GWN_HIP_TRY(hipGetLastError());
            std::vector<double> h(3 * pb);
            GWN_HIP_TRY(hipMemcpyAsync(h.data(), pa, sizeof(double) * 3 * pb, hipMemcpyDeviceToHost, st));
            GWN_HIP_TRY(hipStreamSynchronize(st));
            double A[3] = {0, 0, 0};
            for (int b = 0; b < pb; ++b)
                for (int a = 0; a < 3; ++a) A[a] += h[3 * b + a];
            // world x, y, z -> axis codes 1, 2, 0; z wins ties
            if (A[0] < A[2] && A[0] <= A[1]) axis = 1;
            else if (A[1] < A[2] && A[1] < A[0]) axis = 2;
            m->proj_area[0] = A[0];
            m->proj_area[1] = A[1];
            m->proj_area[2] = A[2];
        }
    }
    m->axis = axis;
    axis_ptrs(axis, vx, vy, vz);   // from here on every coordinate is in the mesh frame

    // ---- optional welding of equal positions (the boundary is extracted by index)
    m->nunique = nv;
    if (weld && nv > 1 && nf > 0) {
        uint32_t *kz = nullptr, *kz2 = nullptr;
        uint64_t *kxy = nullptr, *kxy2 = nullptr;
        int *idx = nullptr, *idx2 = nullptr, *idx3 = nullptr, *head = nullptr, *start = nullptr, *remap = nullptr,
            *nuq = nullptr;
        int32_t* triw = nullptr;
        GWN_HIP_TRY(S.alloc(&kz, nv));
        GWN_HIP_TRY(S.alloc(&kz2, nv));
        GWN_HIP_TRY(S.alloc(&kxy, nv));
        GWN_HIP_TRY(S.alloc(&kxy2, nv));
        GWN_HIP_TRY(S.alloc(&idx, nv));
        GWN_HIP_TRY(S.alloc(&idx2, nv));
        GWN_HIP_TRY(S.alloc(&idx3, nv));
        GWN_HIP_TRY(S.alloc(&head, nv));
        GWN_HIP_TRY(S.alloc(&start, nv));
        GWN_HIP_TRY(S.alloc(&remap, nv));
        GWN_HIP_TRY(S.alloc(&nuq, 1));
        GWN_HIP_TRY(S.alloc(&triw, 3 * nf));
        GWN_HIP_TRY(hipMemsetAsync(nuq, 0, sizeof(int), st));
        k_weld_zkeys<<<nblocks(nv), kThreads, 0, st>>>(vz, vs, nv, kz, idx);
        GWN_HIP_TRY(hipGetLastError());
        GWN_HIP_TRY(with_temp(S, sort_temp_bytes(nv, 4, true), [&](void* tmp) {
            return radix_sort_u32(kz, kz2, idx, idx2, nv, 0, 32, tmp, st);
        }));
        k_weld_xykeys<<<nblocks(nv), kThreads, 0, st>>>(vx, vy, vs, nv, idx2, kxy);
        GWN_HIP_TRY(hipGetLastError());
        GWN_HIP_TRY(with_temp(S, sort_temp_bytes(nv, 8, true), [&](void* tmp) {
            return radix_sort_u64(kxy, kxy2, idx2, idx3, nv, 0, 64, tmp, st);
        }));
        k_weld_heads<<<nblocks(nv), kThreads, 0, st>>>(vz, vs, nv, kxy2, idx3, head);
        GWN_HIP_TRY(hipGetLastError());
        GWN_HIP_TRY(with_temp(S, scan_temp_bytes(nv), [&](void* tmp) {
            return scan_inclusive_max(head, start, nv, tmp, st);
        }));
        k_weld_map<<<nblocks(nv), kThreads, 0, st>>>(idx3, start, nv, remap, nuq);
        GWN_HIP_TRY(hipGetLastError());
        k_weld_tris<<<nblocks(3 * nf), kThreads, 0, st>>>(tri, 3 * nf, remap, triw);
        GWN_HIP_TRY(hipGetLastError());
        int hn = 0;
        GWN_HIP_TRY(hipMemcpyAsync(&hn, nuq, sizeof(int), hipMemcpyDeviceToHost, st));
        GWN_HIP_TRY(hipStreamSynchronize(st));
        m->nunique = hn;
        tri = triw;   // the rest of the build sees welded indices
    }

    double bbox[6] = {0, 0, 0, 0, 0, 0};
    if (nv > 0) {
        for (int a = 0; a < 3; ++a) {
            float mn = INFINITY, mx = -INFINITY;
            for (int b = 0; b < sb; ++b) {
                mn = std::min(mn, hpart[b * 6 + a]);
                mx = std::max(mx, hpart[b * 6 + 3 + a]);
            }
            bbox[a] = (double)mn;
            bbox[3 + a] = (double)mx;
        }
        // the statistics ran on the world axes: frame component c is world (c + axis) % 3
        double bw[6];
        std::memcpy(bw, bbox, sizeof(bw));
        for (int c = 0; c < 3; ++c) {
            bbox[c] = bw[(c + axis) % 3];
            bbox[3 + c] = bw[3 + (c + axis) % 3];
        }
    }
    std::memcpy(m->bbox, bbox, sizeof(bbox));
    m->g = make_qgrid(bbox);
    const QGrid g = m->g;

    int4* qv = nullptr;
    GWN_HIP_TRY(S.alloc(&qv, nv));
    if (nv > 0) {
        k_quantize_vertices<<<nblocks(nv), kThreads, 0, st>>>(vx, vy, vz, vs, nv, g, qv);
        GWN_HIP_TRY(hipGetLastError());
    }

    // ---- triangles, Morton order, LBVH
    if (nf > 0) {
        int4 qlo, qspan;
        auto qc = [&](double x, int a) { return (int)std::rint((x - g.lo[a]) * g.scale); };
        qlo = make_int4(qc(bbox[0], 0), qc(bbox[1], 1), qc(bbox[2], 2), 0);
        qspan = make_int4(qc(bbox[3], 0) - qlo.x, qc(bbox[4], 1) - qlo.y, qc(bbox[5], 2) - qlo.z, 0);
        TriQ* tq = nullptr;
        uint64_t *keys = nullptr, *keys2 = nullptr;
        GWN_HIP_TRY(S.alloc(&tq, nf));
        GWN_HIP_TRY(S.alloc(&keys, nf));
        GWN_HIP_TRY(S.alloc(&keys2, nf));
        k_tri_setup<<<nblocks(nf), kThreads, 0, st>>>(tri, nf, qv, qlo, qspan, tq, keys);
        GWN_HIP_TRY(hipGetLastError());
        // the low 32 bits of a key are its triangle's index, i.e. its input
        // position: a stable sort by the Morton code (bits 32..61) alone gives
        // the order of a sort by the whole key
        GWN_HIP_TRY(with_temp(S, sort_temp_bytes(nf, 8, false), [&](void* tmp) {
            return radix_sort_u64(keys, keys2, nullptr, nullptr, nf, 32, 62, tmp, st);
        }));
        GWN_HIP_TRY(gwn::dmalloc((void**)&m->tris, sizeof(TriQ) * (size_t)nf));
        GWN_HIP_TRY(gwn::dmalloc((void**)&m->trif, sizeof(float4) * 3 * (size_t)nf));
        k_permute_tris<<<nblocks(nf), kThreads, 0, st>>>(keys2, nf, tq, m->tris, tri, vx, vy, vz, vs, m->trif);
        GWN_HIP_TRY(hipGetLastError());
        if (nf >= 2) {
            m->nnodes = nf - 1;
            GWN_HIP_TRY(gwn::dmalloc((void**)&m->nodes, sizeof(Node) * (size_t)(nf - 1)));
            GWN_HIP_TRY(hipMemsetAsync(m->nodes, 0xff, sizeof(Node) * (size_t)(nf - 1), st));
            int *leaf_parent = nullptr, *rflags = nullptr, *depth = nullptr;
            GWN_HIP_TRY(S.alloc(&leaf_parent, nf));
            GWN_HIP_TRY(S.alloc(&rflags, nf + 1));
            GWN_HIP_TRY(S.alloc(&depth, 1));
            GWN_HIP_TRY(hipMemsetAsync(rflags, 0, sizeof(int) * (size_t)(nf + 1), st));
            GWN_HIP_TRY(hipMemsetAsync(depth, 0, sizeof(int), st));
            k_karras<<<nblocks(nf - 1), kThreads, 0, st>>>(keys2, (int)nf, m->nodes, leaf_parent);
            GWN_HIP_TRY(hipGetLastError());
            k_refit<<<nblocks(nf), kThreads, 0, st>>>(m->tris, (int)nf, m->nodes, leaf_parent, rflags);
            GWN_HIP_TRY(hipGetLastError());
            k_depth<<<nblocks(nf), kThreads, 0, st>>>((int)nf, m->nodes, leaf_parent, depth);
            GWN_HIP_TRY(hipGetLastError());
            int hd = 0, rf = 0;
            GWN_HIP_TRY(hipMemcpyAsync(&hd, depth, sizeof(int), hipMemcpyDeviceToHost, st));
            GWN_HIP_TRY(hipMemcpyAsync(&rf, rflags + nf, sizeof(int), hipMemcpyDeviceToHost, st));
            GWN_HIP_TRY(hipStreamSynchronize(st));
            if (rf != 0) {
                set_error("gwn_build_mesh: malformed BVH (refit did not reach the root)");
                return GWN_E_HIP;
            }
            m->depth = hd;
            m->root = 0;
        } else {
            m->root = ~0;
            m->depth = 0;
        }
    }

    // ---- boundary chain
    if (nf > 0) {
        const int64_t ne = 3 * nf;
        uint64_t *ek = nullptr, *ek2 = nullptr;
        int *es = nullptr, *es2 = nullptr, *net = nullptr, *cnt = nullptr, *off = nullptr;
        GWN_HIP_TRY(S.alloc(&ek, ne));
        GWN_HIP_TRY(S.alloc(&ek2, ne));
        GWN_HIP_TRY(S.alloc(&es, ne));
        GWN_HIP_TRY(S.alloc(&es2, ne));
        GWN_HIP_TRY(S.alloc(&net, ne));
        GWN_HIP_TRY(S.alloc(&cnt, ne));
        GWN_HIP_TRY(S.alloc(&off, ne));
        k_edge_keys<<<nblocks(ne), kThreads, 0, st>>>(tri, nf, ek, es);
        GWN_HIP_TRY(hipGetLastError());
        GWN_HIP_TRY(with_temp(S, sort_temp_bytes(ne, 8, true), [&](void* tmp) {
            return radix_sort_u64(ek, ek2, es, es2, ne, 0, 64, tmp, st);
        }));
        k_edge_runs<<<nblocks(ne), kThreads, 0, st>>>(ek2, es2, ne, net, cnt);
        GWN_HIP_TRY(hipGetLastError());
        GWN_HIP_TRY(with_temp(S, scan_temp_bytes(ne), [&](void* tmp) {
            return scan_exclusive_sum(cnt, off, ne, tmp, st);
        }));
        int last_off = 0, last_cnt = 0;
        GWN_HIP_TRY(hipMemcpyAsync(&last_off, off + ne - 1, sizeof(int), hipMemcpyDeviceToHost, st));
        GWN_HIP_TRY(hipMemcpyAsync(&last_cnt, cnt + ne - 1, sizeof(int), hipMemcpyDeviceToHost, st));
        GWN_HIP_TRY(hipStreamSynchronize(st));
        const int64_t nb = (int64_t)last_off + last_cnt;
        m->nb = nb;
        if (nb > 0) {
            int *efrom = nullptr, *eto = nullptr, *ids = nullptr, *kk = nullptr, *in_by_to = nullptr,
                *out_by_from = nullptr, *succ = nullptr;
            int *repA = nullptr, *repB = nullptr, *jA = nullptr, *jB = nullptr, *dA = nullptr, *dB = nullptr;
            int *len = nullptr, *head = nullptr, *voff = nullptr, *lid = nullptr;
            for (int** p : {&efrom, &eto, &ids, &kk, &in_by_to, &out_by_from, &succ, &repA, &repB, &jA, &jB, &dA, &dB,
                            &len, &head, &voff, &lid})
                GWN_HIP_TRY(S.alloc(p, nb));
            k_edge_emit<<<nblocks(ne), kThreads, 0, st>>>(ek2, net, cnt, off, ne, efrom, eto);
            GWN_HIP_TRY(hipGetLastError());
            k_iota<<<nblocks(nb), kThreads, 0, st>>>(ids, nb);
            const int vb = bits_for(nv);
            GWN_HIP_TRY(with_temp(S, sort_temp_bytes(nb, 4, true), [&](void* tmp) {
                return radix_sort_u32((const uint32_t*)eto, (uint32_t*)kk, ids, in_by_to, nb, 0, vb, tmp, st);
            }));
            GWN_HIP_TRY(with_temp(S, sort_temp_bytes(nb, 4, true), [&](void* tmp) {
                return radix_sort_u32((const uint32_t*)efrom, (uint32_t*)kk, ids, out_by_from, nb, 0, vb, tmp, st);
            }));
            k_link<<<nblocks(nb), kThreads, 0, st>>>(in_by_to, out_by_from, nb, succ);
            GWN_HIP_TRY(hipGetLastError());
            // cycle representative = smallest edge id on the cycle (pointer jumping)
            GWN_HIP_TRY(hipMemcpyAsync(jA, succ, sizeof(int) * nb, hipMemcpyDeviceToDevice, st));
            k_iota<<<nblocks(nb), kThreads, 0, st>>>(repA, nb);
            const int rounds = bits_for(nb) + 1;
            for (int r = 0; r < rounds; ++r) {
                k_rep_round<<<nblocks(nb), kThreads, 0, st>>>(repA, jA, nb, repB, jB);
                std::swap(repA, repB);
                std::swap(jA, jB);
            }
            GWN_HIP_TRY(hipGetLastError());
            // distance to the end of the cycle opened at its representative (list ranking)
            k_rank_init<<<nblocks(nb), kThreads, 0, st>>>(succ, repA, nb, jA, dA);
            for (int r = 0; r < rounds; ++r) {
                k_rank_round<<<nblocks(nb), kThreads, 0, st>>>(jA, dA, nb, jB, dB);
                std::swap(jA, jB);
                std::swap(dA, dB);
            }
            GWN_HIP_TRY(hipGetLastError());
            k_loop_counts<<<nblocks(nb), kThreads, 0, st>>>(repA, dA, nb, len, head);
            GWN_HIP_TRY(with_temp(S, scan_temp_bytes(nb), [&](void* tmp) {
                return scan_exclusive_sum(len, voff, nb, tmp, st);
            }));
            GWN_HIP_TRY(with_temp(S, scan_temp_bytes(nb), [&](void* tmp) {
                return scan_exclusive_sum(head, lid, nb, tmp, st);
            }));
            int last_lid = 0, last_head = 0;
            GWN_HIP_TRY(hipMemcpyAsync(&last_lid, lid + nb - 1, sizeof(int), hipMemcpyDeviceToHost, st));
            GWN_HIP_TRY(hipMemcpyAsync(&last_head, head + nb - 1, sizeof(int), hipMemcpyDeviceToHost, st));
            GWN_HIP_TRY(hipStreamSynchronize(st));
            m->nloops = (int64_t)last_lid + last_head;
            GWN_HIP_TRY(gwn::dmalloc((void**)&m->bverts, sizeof(BVert) * (size_t)nb));
            GWN_HIP_TRY(gwn::dmalloc((void**)&m->loop_off, sizeof(int) * (size_t)(m->nloops + 1)));
            k_emit_loops<<<nblocks(nb), kThreads, 0, st>>>(efrom, repA, dA, voff, lid, nb, vx, vy, vz, vs, qv, g.scalef,
                                                          m->bverts, m->loop_off);
            GWN_HIP_TRY(hipGetLastError());
            loop_tail = (int)nb;   // function scope: the copy reads it after this block
            GWN_HIP_TRY(hipMemcpyAsync(m->loop_off + m->nloops, &loop_tail, sizeof(int), hipMemcpyHostToDevice, st));
        }
    }
    if (!m->loop_off) {
        GWN_HIP_TRY(gwn::dmalloc((void**)&m->loop_off, sizeof(int)));
        GWN_HIP_TRY(hipMemsetAsync(m->loop_off, 0, sizeof(int), st));
    }
    GWN_HIP_TRY(hipStreamSynchronize(st));
    m->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return GWN_OK;
}

}  // namespace gwn
