// grid.hip -- w on a regular grid with one ray per (x, y) column (Sec. 4.3.1,
// ray reuse): the column's vertical line is cast once and every crossing is
// classified against each sample; the boundary term shares the column's x/y
// work (the arithmetic lives in gwn_kernels.h).
//
// Built on its own with the max-ILP machine scheduler: the edge loops of the
// FP32 kernel, held to 128 VGPRs, issue the same instructions under either
// scheduler, but in an order that ran 7% faster on the 512^3 grid of the
// 1.05M-triangle soup (411 vs 440 ms), while that scheduler costs the FP64
// point kernels half their occupancy -- hence the separate source.
#include <cmath>
#include <cstdlib>

#include <algorithm>

#include "gwn_kernels.h"
#include "gwn_mesh.h"

namespace gwn {
namespace {

// FP32 with 8 samples per lane and FP64 with 4 are held to 128 VGPRs (4 waves
// per SIMD).  The FP32 kernel fits without spilling: the crossing counts ride
// in the boundary sums (which start at 2 pi chi), the output positions are
// recomputed from the wave-uniform column after the loops, and the ring's
// per-lane addresses are formed per fill.  The FP64 kernel spills; the fourth
// wave still gains more than the spill costs.
// One wave owns one (x, y) column and a chunk of 64*ZB consecutive z samples;
// lane l holds samples l, l+64, ..., l+64(ZB-1) of the chunk, so each of its ZB
// registers covers a block of 64 consecutive samples (most boundary vertices
// lie wholly above or below a block, see load_vertex).  The column's line is
// cast once (all lanes walk the same BVH path) and every crossing is classified
// against each sample with the exact plane predicate (Sec. 4.3.1, ray reuse).
template <class T, int ZB>
__global__ __launch_bounds__(64 * kGridWaves)
__attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 && ZB == 8) || (sizeof(T) == 8 && ZB == 4) ? 4 : 1))) void k_grid(MeshView mv, GridArgs ga, int* __restrict__ chi_out,
                                                          T* __restrict__ w) {
    __shared__ int wstack[kGridWaves][kLdsStack];
    __shared__ ColRing<T> ring[kGridWaves];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const long long gw = ga.wave0 + (long long)blockIdx.x * kGridWaves + wave;
    if (gw >= ga.nwaves) return;
    // column (ci, cj) and z chunk of this wave: every grid axis has at most 2^20
    // points, so they are 32-bit and wave-uniform (scalar registers)
    const long long col = gw / ga.nchunks;
    const int chunk = __builtin_amdgcn_readfirstlane((int)(gw - col * ga.nchunks));
    const int ci = __builtin_amdgcn_readfirstlane((int)(col / ga.ny));
    const int cj = __builtin_amdgcn_readfirstlane((int)(col - (long long)ci * ga.ny));
    const float px = grid_coord(ga.o[0], ga.s[0], ci);
    const float py = grid_coord(ga.o[1], ga.s[1], cj);
    const int nz = (int)ga.nz;
    const int k0 = chunk * 64 * ZB + lane;   // sample r is k0 + 64 r

    float pz[ZB];
    int qzr[ZB];
    int chi[ZB];
    const QPoint q0 = quantize_point(px, py, 0.0f, mv.g);
#pragma unroll
    for (int r = 0; r < ZB; ++r) {
        pz[r] = grid_coord(ga.o[2], ga.s[2], min(k0 + 64 * r, nz - 1));
        qzr[r] = quantize_point(px, py, pz[r], mv.g).z;
        chi[r] = 0;
    }

    // ---- crossings along the column's vertical line, classified per sample
    if (q0.inbox && mv.root != kNoRoot) {
        int* stk = wstack[wave];
        int node = mv.root;
        int sp = 0;
        const bool leaf_only = node < 0;
        while (true) {
            // up to two leaves reached at this node (the triangles to test); -1 = none
            int leaf0 = -1, leaf1 = -1;
            if (leaf_only) {
                leaf0 = ~node;
            } else {
                const Node nd = mv.nodes[node];
                bool hl = box_has_xy(nd.lxy.x, nd.lxy.y, nd.lxy.z, nd.lxy.w, q0.x, q0.y);
                bool hr = box_has_xy(nd.rxy.x, nd.rxy.y, nd.rxy.z, nd.rxy.w, q0.x, q0.y);
                const int L = nd.link.x, R = nd.link.y;
                if (hl && L < 0) { leaf0 = ~L; hl = false; }
                if (hr && R < 0) { leaf1 = ~R; hr = false; }
                if (hl && hr) { stk[sp++] = R; node = L; }
                else if (hl) node = L;
                else if (hr) node = R;
                else node = -1;
            }
            for (int h = 0; h < 2; ++h) {
                const int leaf = h == 0 ? leaf0 : leaf1;
                if (leaf < 0) continue;
                const TriQ t = mv.tris[leaf];
                const int s = tri_xy_sign(t, q0.x, q0.y);
                if (s == 0) continue;
                const PlaneQ pl = plane_of(t, q0.x, q0.y);
#pragma unroll
                for (int r = 0; r < ZB; ++r) chi[r] += plane_above(pl, qzr[r]) ? s : 0;
            }
            if (leaf_only) break;
            if (node < 0) {
                if (sp == 0) break;
                node = stk[--sp];
            }
        }
    }

    // The crossing counts are final here: store them, and start each sample's
    // boundary sum at 2 pi chi (w = S / 2 pi), so that no register holds the
    // counts through the boundary loops.
    if (chi_out) {
        const long long base = (long long)ci * ga.st[0] + (long long)cj * ga.st[1];
#pragma unroll
        for (int r = 0; r < ZB; ++r) {
            const int k = k0 + 64 * r;
            if (k < nz) chi_out[base + (long long)k * ga.st[2]] = chi[r];
        }
    }

    // ---- boundary term
    T pzs[ZB];
    double S[ZB];
    if (q0.inbox) {
        const T sc = (T)mv.g.scale;
        bool near = true;
#pragma unroll
        for (int r = 0; r < ZB; ++r) {
            pzs[r] = (T)pz[r] * sc;
            S[r] = (double)chi[r] * k2Pi;
            near &= near_z(pz[r], mv.g);
        }
        near = __builtin_amdgcn_ballot_w64(!near) == 0ull;   // one choice for the whole column
        column_loops<T, ZB>(mv, q0.x, q0.y, pzs, S, near, ring[wave]);
    } else {
        float pzm = 0.f;
#pragma unroll
        for (int r = 0; r < ZB; ++r) pzm = fmaxf(pzm, fabsf(pz[r]));
        const FarScale<T> fs = far_scale<T>(px, py, pzm, mv.g.scale);
#pragma unroll
        for (int r = 0; r < ZB; ++r) {
            pzs[r] = (T)pz[r] * fs.scf;
            S[r] = (double)chi[r] * k2Pi;
        }
        boundary_loops<T, ZB, true>(mv, 0, 0, (T)px * fs.scf, (T)py * fs.scf, pzs, S, fs.f);
    }

    // output positions from the wave-uniform column and the lane, recomputed
    // here rather than kept through the boundary loops
    const long long base = (long long)ci * ga.st[0] + (long long)cj * ga.st[1];
    const int k1 = chunk * 64 * ZB + (int)(threadIdx.x & 63);
#pragma unroll
    for (int r = 0; r < ZB; ++r) {
        const int k = k1 + 64 * r;
        if (k < nz) w[base + (long long)k * ga.st[2]] = (T)(S[r] * kInv2Pi);
    }
}

template <class T, int ZB>
gwn_status launch_grid_zb(const gwn_mesh_s* m, GridArgs ga, T* w, int32_t* chi_out, hipStream_t st) {
    ga.nchunks = (ga.nz + 64 * ZB - 1) / (64 * ZB);
    ga.nwaves = ga.nx * ga.ny * ga.nchunks;
    // at most 2^24 waves (2^30 work-items) per launch
    const long long kMaxWaves = max_launch_queries() / 64;
    for (long long w0 = 0; w0 < ga.nwaves; w0 += kMaxWaves) {
        ga.wave0 = w0;
        const long long blocks = (std::min(kMaxWaves, ga.nwaves - w0) + kGridWaves - 1) / kGridWaves;
        k_grid<T, ZB><<<(unsigned)blocks, 64 * kGridWaves, 0, st>>>(m->view(), ga, chi_out, w);
        GWN_HIP_TRY(hipGetLastError());
    }
    return GWN_OK;
}

// Samples per lane: more samples share more x/y work, fewer leave registers for
// more resident waves.  GWN_GRID_SAMPLES_PER_LANE (1, 2, 4 or 8) overrides
// everything; then the mesh's tuning for the precision (gwn_mesh_set_tuning,
// gwn_mesh_autotune); the built-in choice is the largest value the column fills.
template <class T>
gwn_status launch_grid(const gwn_mesh_s* m, GridArgs ga, T* w, int32_t* chi_out, hipStream_t st) {
    int zb = 0;
    if (const char* e = std::getenv("GWN_GRID_SAMPLES_PER_LANE")) zb = std::atoi(e);
    if (zb == 0) zb = m->grid_zb[sizeof(T) == 8 ? GWN_PREC_FP64 : GWN_PREC_FP32];
    switch (zb) {
        case 1: return launch_grid_zb<T, 1>(m, ga, w, chi_out, st);
        case 2: return launch_grid_zb<T, 2>(m, ga, w, chi_out, st);
        case 4: return launch_grid_zb<T, 4>(m, ga, w, chi_out, st);
        case 8: return launch_grid_zb<T, 8>(m, ga, w, chi_out, st);
        default: break;
    }
    // FP64 keeps at most 4 samples per lane (8 would need ~200 VGPRs)
    if (ga.nz >= 64 * 8 && sizeof(T) == 4) return launch_grid_zb<T, 8>(m, ga, w, chi_out, st);
    if (ga.nz >= 64 * 4) return launch_grid_zb<T, 4>(m, ga, w, chi_out, st);
    if (ga.nz >= 64 * 2) return launch_grid_zb<T, 2>(m, ga, w, chi_out, st);
    return launch_grid_zb<T, 1>(m, ga, w, chi_out, st);
}

}  // namespace

gwn_status query_grid(const gwn_mesh_s* m, const double* origin, const double* spacing, const int64_t* dims, int prec,
                      void* w, int32_t* chi_out, hipStream_t st) {
    GridArgs ga = frame_grid(m->axis, origin, spacing, dims);
    if (ga.nx == 0 || ga.ny == 0 || ga.nz == 0) return GWN_OK;
    if (prec == GWN_PREC_FP64) return launch_grid<double>(m, ga, (double*)w, chi_out, st);
    return launch_grid<float>(m, ga, (float*)w, chi_out, st);
}

}  // namespace gwn
