#!/usr/bin/env python3
"""Benchmark: GWN queries/s of the antipodal method on one MI355X.

Workload (default): the ~1.05M-triangle soup of 64 overlapping, randomly opened
spheres and ellipsoids in [-1,1]^3, queried on the 512^3 cell-centred grid
(134,217,728 points) through gwn_query_grid, FP32 geometry with exact
predicates and FP64 accumulation.  One step = one full grid evaluation (ray
reuse + boundary term + combine).  The mesh build is precomputation and is not
timed (Sec. 5.1 excludes it); its time is reported separately.

Prints ONE JSON line (see the keys below).  `roofline` prices the dominant
kernel (the fused grid kernel) against the VALU issue ceiling; `cpu_baseline`
times the CPU oracle on a bounded random sample of the same grid and also
reports the max |w_gpu - w_oracle| on that sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GWN queries/sec on 1M-tri open soup at max|err|≤1e-4 vs FP64; % roofline"

# VALU issue ceiling of MI355X, from the published FP32 vector peak of
# 157.3 TFLOP/s (an FMA counted as 2 FLOPs): 7.86e13 FP32 VALU instruction slots
# per second, i.e. 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz.  FP32 add/mul/fma,
# compares, selects and 32-bit integer ops take one slot each; sqrt and rcp were
# measured on the box at 3.0 slots each (profiles/valu_issue_rates_gfx950.md).
N_CU, SIMD_PER_CU, LANES_PER_CLK, CLOCK_HZ = 256, 4, 32, 2.4e9
PEAK_SLOTS = N_CU * SIMD_PER_CU * LANES_PER_CLK * CLOCK_HZ
TRANS_SLOTS = 3

# Minimal VALU slots per (query, boundary edge) pair on the grid path, with x/y
# work (N, N1 N2, the x/y dot) shared by the samples of a column and consecutive
# edges summed in pairs by one arctangent (one boundary vertex per edge):
#   per sample and vertex:    r_z (1), l^2 (1), sqrt, l+|r_z| (1), rcp, rho^2*rcp (1),
#                             compare + select (2)                 = 6 + 2 trans
#   per sample and edge:      D (1), fast-path test (1)            = 2
#   per sample and edge pair: Re (1), Im (2), rcp, Im*rcp (1), t^2 (1), 4 FMAs for
#                             P(t^2), accumulate as FMA(t, P, acc) (1)
#                                                                  = 10 + 1 trans
I_MIN_GRID = 6 + 2 * TRANS_SLOTS + 2 + (10 + TRANS_SLOTS) / 2      # = 20.5
# The single-edge form (reciprocal and degree-7 arctangent per edge) that the
# per-lane kernels use: 6 + 14 + 3 transcendentals = 29.
I_MIN_EDGE = 6 + 14 + 3 * TRANS_SLOTS      # = 29

# The all-FP64 grid path against the same issue ceiling, with FP64 add/mul/fma
# and compares at 1.5 FP32 slots and v_rcp_f64 / v_rsq_f64 at 5.4 (measured by
# the same probe).  The hardware reciprocal and reciprocal square root are only
# ~26-bit approximations (measured on the box: 2.4e8 ulp), so the refinement a
# double result needs is part of the minimum:
#   per sample and vertex: r_z, l^2 (2); sqrt = rsq + 7; l+|r_z| (1); rcp = rcp + 4;
#                          rho^2*rcp (1); compare (1)          = 16 FP64 + 2 trans + select (2)
#   per sample and edge:   D, fast-path test (2)                       = 2 FP64
#   per sample and pair:   Re, Im (3); rcp + 4; Im*rcp, t^2 (2); 9 polynomial
#                          FMAs; t*x, final FMA, accumulate (3)         = 21 FP64 + 1 trans
# Arbitrary points (one query per lane, edge pairs chosen per lane): the x/y
# quantities are no longer shared by a column.
#   per vertex:      dx, dy (2), their conversion (2) and scale to offset units (2),
#                    rho^2 (2), r_z (1), l^2 (1), sqrt, l+|r_z| (1), rcp,
#                    rho^2*rcp (1), compare + select (2)      = 14 + 2 trans
#   per edge:        N (2), x/y dot (2), pair bound (2), D (1), pair test (1) = 8
#   per edge pair:   N1 N2 (1), Re (1), Im (2), rcp, Im*rcp (1), t^2 (1),
#                    4 FMAs for P(t^2), FMA(t, P, acc) (1)    = 11 + 1 trans
I_MIN_BATCH = 14 + 2 * TRANS_SLOTS + 8 + (11 + TRANS_SLOTS) / 2      # = 35
# The gradient (Supp. Alg. 3) per pair: per vertex r (3), rho^2 (2), l^2 (1), sqrt,
# 1/l, l+|r_z| (1), rcp, rho^2*rcp (1), compare + select (2) = 10 + 3 trans; per
# edge l0 l1 (1), n (3), d (3), c0, c1 (2), grad D (6), n^2+d^2 (2), rcp, scale
# (1), the three components (8), accumulate (3) = 29 + 1 trans
I_MIN_GRAD = 10 + 29 + 4 * TRANS_SLOTS     # = 51
# Dense MFMA peak of MI355X (no sparsity), the same for bf16 (training) and
# fp16 (inference) operands
PEAK_BF16 = 2.5e15
PEAK_F16 = 2.5e15
# The network's VALU work per point at inference, in lane slots (a packed half
# instruction on two values is one slot, counted at the 2-clock FP32 rate,
# which it does not reach: rocprofv3 shows packed half instructions never
# dual-issued, so each takes the unpaired ~4 clocks): 512
# GELU activations at 5 slots (10 packed half instructions per pair: the
# conversion from the float32 accumulator, the clamp, 2t - 1, the square, 4 FMAs
# of the polynomial, the 1/2 term, the product; the bias enters through the
# matrix product's accumulator), 32 frequencies of the Fourier features at 12
# (the argument, 3; its fractional part, 1; the hardware sine and cosine, 3
# each; half a packed conversion per value, 1) and the 128-term output dot
# product on mixed-precision FMAs (128)
NET_VALU_SLOTS = 512 * 5 + 32 * 12 + 128     # = 3,072 per point
# HBM bytes moved per k_grid<float, 8> launch on the default workload (512^3 grid,
# 1.05M-triangle soup), from two rocprofv3 --pmc passes over this command:
# FETCH_SIZE 231,964.50 KiB and WRITE_SIZE 524,288.0 KiB per dispatch, scaled by
# what the same counters read for a plain 1 GiB device copy (bench.py
# --copy-probe: FETCH_SIZE shows 524,308.25 KiB -> x2.000, WRITE_SIZE
# 1,048,576 KiB -> x1.000).  Writes are exactly the w output (134,217,728 x 4 B);
# fetches are the BVH, triangles and boundary vertices read by the 8 XCD L2s.
# Measured on the kernel as it stands; re-take the counters after any change to
# k_grid or the workload.
K_GRID_TRAFFIC_BYTES = (231964.5 * 2.0 + 524288.0 * 1.0) * 1024
FP64_OP_SLOTS, FP64_TRANS_SLOTS = 1.5, 5.4
I_MIN_GRID_FP64 = (16 + 2 + 21 / 2) * FP64_OP_SLOTS + 2.5 * FP64_TRANS_SLOTS + 2   # = 58.25
# Parametric path (FP64), per unit of work the kernel reports, counted from its
# arithmetic (a division = one reciprocal at the transcendental cost plus 4 ops):
# one integrand evaluation from frame coordinates: rho^2, l^2, the numerator,
# the two-sided s and its selects, and one Newton step on each of the hardware
# estimates of 1 / l and of the other reciprocal, 19 ops and 2 estimates; a
# quadrature interval: the control points relative to the query projected onto
# the ray's frame (48), their power basis and Taylor coefficients about the
# interval's centre (66), the 7 node pairs' even and odd parts and their sums
# (196), 15 evaluations and 30 ops of the two rules; a sub-patch cell: 24 cubic
# interval extractions (24 ops and 1 division each), the control points' box
# (96), the slab test (24, 3 divisions) and the control net's distance to the
# bilinear patch (528, 1 square root).
PARAM_EVAL_SLOTS = 19 * FP64_OP_SLOTS + 2 * FP64_TRANS_SLOTS
PARAM_INTERVAL_SLOTS = 15 * PARAM_EVAL_SLOTS + (48 + 66 + 196 + 30) * FP64_OP_SLOTS
PARAM_CELL_SLOTS = (24 * 24 + 96 + 24 + 528 + 27 * 4) * FP64_OP_SLOTS + 28 * FP64_TRANS_SLOTS
# Per sample and boundary vertex the two-sided form of s (rcp, rho^2*rcp, the sign
# compare and the select) is skipped where the vertex lies at or below all 64
# samples of a grid block: 6 FP32 slots (11.4 + 1.5 + 1.5 + 2 in FP64); where it
# lies above all of them only the compare and select are: 2 slots (1.5 + 2).
SKIP_SLOTS = {"fp32": 6.0, "fp64": 16.4}
SKIP_SEL_SLOTS = {"fp32": 2.0, "fp64": 3.5}


def boundary_vertex_z(V, F):
    """z of the first vertex of every boundary edge (net multiplicity of the
    directed edge over its reverse, counted with multiplicity)."""
    nv = np.int64(V.shape[0])
    a = np.concatenate([F[:, 0], F[:, 1], F[:, 2]]).astype(np.int64)
    b = np.concatenate([F[:, 1], F[:, 2], F[:, 0]]).astype(np.int64)
    keys, cnt = np.unique(a * nv + b, return_counts=True)
    rev = (keys % nv) * nv + keys // nv
    pos = np.clip(np.searchsorted(keys, rev), 0, keys.size - 1)
    rcnt = np.where(keys[pos] == rev, cnt[pos], 0)
    net = cnt - rcnt
    sel = net > 0
    return np.repeat(V[keys[sel] // nv, 2].astype(np.float64), net[sel])


def grid_slots(soup, grid, prec):
    """Minimal VALU slots per (sample, edge) pair of the grid kernel on this
    workload, and the fractions of (vertex, sample) pairs whose block skips the
    reciprocal (the vertex at or below all its samples) and whose block skips
    only the select (one of the R blocks with a sample below the vertex other
    than the last).  Blocks are 64 consecutive samples of a column, z ascending."""
    zv = boundary_vertex_z(soup.V, soup.F)
    nz = int(grid.dims[2])
    kmin = np.arange(0, nz, 64)
    zmin = grid.origin[2] + (kmin + 0.5) * grid.spacing[2]
    sizes = np.minimum(64, nz - kmin)
    if zv.size == 0:
        return (I_MIN_GRID_FP64 if prec == "fp64" else I_MIN_GRID), 0.0, 0.0
    need = zv[:, None] > zmin[None, :]              # blocks with a sample below the vertex
    above = ((~need) * sizes[None, :]).sum(1).mean() / nz
    # of the R blocks that need the reciprocal, all but the last drop the select
    R = need.sum(1)
    first = np.arange(kmin.size)[None, :] < (R - 1)[:, None]
    below = (first * sizes[None, :]).sum(1).mean() / nz
    dense = I_MIN_GRID_FP64 if prec == "fp64" else I_MIN_GRID
    return dense - SKIP_SLOTS[prec] * above - SKIP_SEL_SLOTS[prec] * below, float(above), float(below)


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--n", type=int, default=512, help="grid points per axis")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["grid", "batch", "batched", "surrogate", "precision", "gradient",
                                                 "direct", "weld", "axis", "parametric"], default="grid",
                    help="grid: the headline 512^3 grid on the 1M-triangle soup (default); batch: 2M points on the "
                         "torus soup; batched: 256 soups in one persistent graph; surrogate: MLP + exact fallback; "
                         "parametric: 100 cubic Bezier patches on a 32^3 grid")
    ap.add_argument("--n-mesh", type=int, default=256, help="soups in the batched workload")
    ap.add_argument("--sample", type=int, default=20000, help="oracle sample size of the precision workload")
    ap.add_argument("--epochs", type=int, default=32, help="surrogate training epochs")
    ap.add_argument("--sigma", type=float, default=1.0, help="surrogate Fourier-feature scale")
    ap.add_argument("--lr", type=float, default=1e-3, help="surrogate peak learning rate")
    ap.add_argument("--train-batch", type=int, default=8192, help="surrogate training batch (points per Adam step)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (calibrates HBM counters) and exit")
    return ap.parse_args()


def copy_probe(nbytes: int):
    """A plain copy kernel of known size: reads and writes nbytes once each."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4}), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: queries and grid columns are independent, so more GPUs "
              "would each take a contiguous share of them with no communication; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2605_01536_amd import gwn, workloads as W

    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.workload != "grid":
        {"batch": bench_batch, "batched": bench_batched, "surrogate": bench_surrogate,
         "precision": bench_precision, "gradient": bench_gradient, "direct": bench_direct,
         "weld": bench_weld, "axis": bench_axis, "parametric": bench_parametric}[args.workload](args)
        return
    t0 = time.time()
    soup, grid = W.config4(n=args.n)
    gen_s = time.time() - t0
    mesh = gwn.Mesh(torch.from_numpy(soup.V).cuda(), torch.from_numpy(soup.F).cuda())
    info = mesh.info()
    n = grid.n
    B = info["nboundary"]
    dt = torch.float64 if args.prec == "fp64" else torch.float32
    w = torch.empty(n, device="cuda", dtype=dt)
    stream = torch.cuda.current_stream()

    def step():
        gwn.query_grid(mesh, grid.origin, grid.spacing, grid.dims, prec=args.prec, out=w, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1e3 / args.steps
    qps = n / (ms_per_step / 1e3)
    avg_kernel_s = float(np.mean(kern_ms)) / 1e3
    pairs = float(n) * B
    slots, skip_frac, below_frac = grid_slots(soup, grid, args.prec)
    achieved = pairs * slots / avg_kernel_s
    roof = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": PEAK_SLOTS / 1e12,
        "unit": "T FP32-VALU-slots/s",
        "frac": achieved / PEAK_SLOTS,
        # HBM bytes per launch (rocprofv3 counters); only measured for the default workload
        "traffic": K_GRID_TRAFFIC_BYTES if (args.n == 512 and args.prec == "fp32") else None,
        "traffic_unit": "bytes per launch",
        "kernel": "k_grid",
        "slots_per_pair": slots,
        "block_above_fraction": skip_frac,
        "block_below_fraction": below_frac,
        "pairs_per_launch": pairs,
        "avg_kernel_ms": avg_kernel_s * 1e3,
    }
    print(f"[bench] {n} queries, B={B}, {ms_per_step:.1f} ms/step, {qps:.3e} q/s, "
          f"{pairs / avg_kernel_s:.3e} pairs/s", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(12345)
        # size the sample to ~cpu_seconds of oracle work; the per-point cost is
        # calibrated on two sample sizes so the one-off setup of each call cancels
        t = time.perf_counter()
        oracle.antipodal(soup.V, soup.F, W.grid_points(grid, rng.choice(n, 500, replace=False)))
        t500 = time.perf_counter() - t
        t = time.perf_counter()
        oracle.antipodal(soup.V, soup.F, W.grid_points(grid, rng.choice(n, 4500, replace=False)))
        t4500 = time.perf_counter() - t
        per_q = max((t4500 - t500) / 4000.0, 1e-9)
        m = int(max(1000, min(5_000_000, args.cpu_seconds / per_q)))
        idx = rng.choice(n, m, replace=False)
        P = W.grid_points(grid, idx)
        t = time.perf_counter()
        w_o = oracle.antipodal(soup.V, soup.F, P)
        cpu_s = time.perf_counter() - t
        diag = float(np.linalg.norm(np.asarray(info["bbox"][3:]) - np.asarray(info["bbox"][:3])))
        mc = min(m, 200_000)   # error check on the first 200k sampled points
        far = oracle.distance(soup.V, soup.F, P[:mc], 2e-4 * diag) > 1e-4 * diag
        wg = w[torch.from_numpy(idx[:mc]).cuda()].double().cpu().numpy()
        err = float(np.abs(wg - w_o[:mc])[far].max())
        # the direct sum (O1: Eq. 2 with Eq. 6, double-double) on a subsample sized to
        # a few seconds, reported as triangle evaluations per second
        t = time.perf_counter()
        oracle.direct(soup.V, soup.F, W.grid_points(grid, idx[:64]))
        per_pt = max((time.perf_counter() - t) / 64, 1e-9)
        m1 = int(max(64, min(10_000, 0.5 * args.cpu_seconds / per_pt)))
        t = time.perf_counter()
        w_d = oracle.direct(soup.V, soup.F, P[:m1])
        o1_s = time.perf_counter() - t
        o1_far = far[:m1] if m1 <= mc else oracle.distance(soup.V, soup.F, P[:m1], 2e-4 * diag) > 1e-4 * diag
        cpu = {"value": m / cpu_s, "unit": "queries/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"{m} random points of the same grid, FP64 antipodal oracle, {cpu_s:.1f} s",
               "max_abs_err_vs_gpu": err, "n_compared": int(far.sum()),
               "nproc": os.cpu_count(), "cpu_model": cpu_model(),
               "direct_sum": {"kind": "oracle O1 (direct solid-angle sum, double-double)", "points": m1,
                              "seconds": o1_s, "triangle_evals_per_s": m1 * float(soup.F.shape[0]) / o1_s,
                              "queries_per_s": m1 / o1_s, "threads": oracle.num_threads(),
                              "max_abs_diff_vs_antipodal_oracle": float(np.abs(w_d - w_o[:m1])[o1_far].max())}}
        print(f"[bench] oracle {m / cpu_s:.3e} q/s on {cpu['cores']} threads of {cpu['nproc']} ({cpu['cpu_model']}); "
              f"max|err| {err:.2e}; direct sum {cpu['direct_sum']['triangle_evals_per_s']:.3e} triangle evals/s",
              file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"opened-spheres soup ({info['nf']} tris, {B} boundary edges, "
                               f"{info['nloops']} loops) on a {args.n}^3 grid over [-1,1]^3",
                   "queries": n, "boundary_edges": B, "triangles": info["nf"], "precision": args.prec,
                   "build_ms": info["build_ms"], "generate_s": gen_s},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _timed(fn, steps, warmup, stream):
    """Average ms of fn() over `steps` launches bracketed by HIP events on `stream`."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps, (time.perf_counter() - t0) * 1e3 / steps


def _alu_roof(pairs, slots, ms, kernel):
    a = pairs * slots / (ms / 1e3)
    return {"bound": "alu", "achieved": a / 1e12, "peak": PEAK_SLOTS / 1e12, "unit": "T FP32-VALU-slots/s",
            "frac": a / PEAK_SLOTS, "traffic": None, "kernel": kernel, "slots_per_pair": slots}


def _emit(metric, value, unit, args, ms, config, extra=None, dtype="f32"):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic", "config": config}
    if extra:
        out.update(extra)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """2M points (1M uniform in the bbox, 1M near the surface) on the ~85k-triangle torus soup."""
    import torch
    from paper_2605_01536_amd import gwn, workloads as W
    soup, Q = W.config2()
    mesh = gwn.Mesh(torch.from_numpy(soup.V).cuda(), torch.from_numpy(soup.F).cuda())
    info = mesh.info()
    Qd = torch.from_numpy(Q).cuda()
    w = torch.empty(Q.shape[0], device="cuda", dtype=torch.float64 if args.prec == "fp64" else torch.float32)
    st = torch.cuda.current_stream()
    ev_ms, wall_ms = _timed(lambda: gwn.query_batch(mesh, Qd, prec=args.prec, out=w, stream=st), args.steps,
                            args.warmup, st)
    pairs = Q.shape[0] * info["nboundary"]
    print(f"[bench] batch {Q.shape[0]} pts B={info['nboundary']}: {wall_ms:.1f} ms, {pairs / wall_ms * 1e3:.3e} pairs/s",
          file=sys.stderr, flush=True)
    # a small batch (4,096 points): one workgroup per point with the edges split
    # among its lanes (the default at this size) against one lane per point
    small = {}
    Qs = Qd[:4096].contiguous()
    ws = torch.empty(4096, device="cuda", dtype=w.dtype)
    for mode, flag in (("split", "1"), ("per_lane", "0")):
        os.environ["GWN_SPLIT_BOUNDARY"] = flag
        small[mode + "_ms"], _ = _timed(lambda: gwn.query_batch(mesh, Qs, prec=args.prec, out=ws, stream=st),
                                        args.steps, args.warmup, st)
    del os.environ["GWN_SPLIT_BOUNDARY"]
    print(f"[bench] 4096 points: split {small['split_ms']:.2f} ms, per-lane {small['per_lane_ms']:.2f} ms",
          file=sys.stderr, flush=True)
    _emit("GWN queries/sec, arbitrary points", Q.shape[0] / (wall_ms / 1e3), "queries/s", args, wall_ms,
          {"workload": f"torus soup ({info['nf']} tris, {info['nboundary']} boundary edges), 1M uniform + 1M "
                       f"near-surface points", "precision": args.prec, "pairs_per_s": pairs / (ev_ms / 1e3),
           "small_batch_4096": small},
          extra={"roofline": _alu_roof(pairs, I_MIN_BATCH, ev_ms, "k_chi_* + k_bdry_batch")}
          if args.prec == "fp32" else None, dtype="f32" if args.prec == "fp32" else "f64")


def bench_gradient(args):
    """grad w (Supp. Alg. 3) at the 2M torus-soup points, beside w at the same points."""
    import torch
    from paper_2605_01536_amd import gwn, workloads as W
    soup, Q = W.config2()
    mesh = gwn.Mesh(torch.from_numpy(soup.V).cuda(), torch.from_numpy(soup.F).cuda())
    info = mesh.info()
    Qd = torch.from_numpy(Q).cuda()
    dt = torch.float64 if args.prec == "fp64" else torch.float32
    g = torch.empty((Q.shape[0], 3), device="cuda", dtype=dt)
    w = torch.empty(Q.shape[0], device="cuda", dtype=dt)
    st = torch.cuda.current_stream()
    ev_g, wall_g = _timed(lambda: gwn.query_gradient(mesh, Qd, prec=args.prec, out=g, stream=st), args.steps,
                          args.warmup, st)
    ev_w, wall_w = _timed(lambda: gwn.query_batch(mesh, Qd, prec=args.prec, out=w, stream=st), args.steps,
                          args.warmup, st)
    pairs = Q.shape[0] * info["nboundary"]
    print(f"[bench] gradient {Q.shape[0]} pts B={info['nboundary']}: {wall_g:.1f} ms ({pairs / ev_g * 1e3:.3e} "
          f"edge terms/s); w at the same points {wall_w:.1f} ms", file=sys.stderr, flush=True)
    # a small batch (4,096 points): workgroup per point against lane per point
    small = {}
    Qs = Qd[:4096].contiguous()
    gs = torch.empty((4096, 3), device="cuda", dtype=dt)
    for mode, flag in (("split", "1"), ("per_lane", "0")):
        os.environ["GWN_SPLIT_BOUNDARY"] = flag
        small[mode + "_ms"], _ = _timed(lambda: gwn.query_gradient(mesh, Qs, prec=args.prec, out=gs, stream=st),
                                        args.steps, args.warmup, st)
    del os.environ["GWN_SPLIT_BOUNDARY"]
    print(f"[bench] gradient 4096 points: split {small['split_ms']:.2f} ms, per-lane {small['per_lane_ms']:.2f} ms",
          file=sys.stderr, flush=True)
    # the 512^3 grid on the 1.05M-triangle soup: column-shared gradient kernel
    soup4, grid = W.config4()
    m4 = gwn.Mesh(torch.from_numpy(soup4.V).cuda(), torch.from_numpy(soup4.F).cuda())
    g4 = torch.empty((grid.n, 3), device="cuda", dtype=dt)
    ev_gg, _ = _timed(lambda: gwn.query_grid_gradient(m4, grid.origin, grid.spacing, grid.dims, prec=args.prec,
                                                      out=g4, stream=st), max(1, args.steps // 5), 1, st)
    pairs4 = float(grid.n) * m4.info()["nboundary"]
    print(f"[bench] grid gradient 512^3: {ev_gg:.1f} ms ({pairs4 / ev_gg * 1e3:.3e} edge terms/s)",
          file=sys.stderr, flush=True)
    del g4, m4
    _emit("GWN gradients/sec, arbitrary points", Q.shape[0] / (wall_g / 1e3), "queries/s", args, wall_g,
          {"workload": f"torus soup ({info['nf']} tris, {info['nboundary']} boundary edges), 1M uniform + 1M "
                       f"near-surface points", "precision": args.prec, "pairs_per_s": pairs / (ev_g / 1e3),
           "w_ms_same_points": wall_w, "small_batch_4096": small, "grid_512_ms": ev_gg, "grid_512_pairs_per_s": pairs4 / (ev_gg / 1e3)},
          extra={"roofline": _alu_roof(pairs, I_MIN_GRAD, ev_g, "k_grad_batch")} if args.prec == "fp32" else None,
          dtype="f32" if args.prec == "fp32" else "f64")


def bench_direct(args):
    """The direct per-triangle sum (the O(F) baseline) against the antipodal path on the same
    points: a sample of the 512^3 grid on the 1M-triangle soup and of the torus-soup points."""
    import torch
    from paper_2605_01536_amd import gwn, workloads as W
    rows = []
    soup4, grid = W.config4()
    rng = np.random.default_rng(0)
    P4 = W.grid_points(grid, np.sort(rng.choice(grid.n, 65536, replace=False)))
    soup2, Q2 = W.config2()
    P2 = Q2[np.sort(rng.choice(Q2.shape[0], 131072, replace=False))]
    st = torch.cuda.current_stream()
    dt = torch.float64 if args.prec == "fp64" else torch.float32
    for name, soup, P in (("opened-spheres 512^3 grid sample", soup4, P4), ("torus soup points", soup2, P2)):
        mesh = gwn.Mesh(torch.from_numpy(soup.V).cuda(), torch.from_numpy(soup.F).cuda())
        info = mesh.info()
        Pd = torch.from_numpy(np.ascontiguousarray(P)).cuda()
        w = torch.empty(P.shape[0], device="cuda", dtype=dt)
        ev_d, wall_d = _timed(lambda: gwn.query_direct(mesh, Pd, prec=args.prec, out=w, stream=st),
                              max(1, args.steps // 5), 1, st)
        ev_a, wall_a = _timed(lambda: gwn.query_batch(mesh, Pd, prec=args.prec, out=w, stream=st), args.steps,
                              args.warmup, st)
        rows.append({"mesh": name, "tris": info["nf"], "boundary_edges": info["nboundary"], "points": P.shape[0],
                     "direct_qps": P.shape[0] / (ev_d / 1e3),
                     "direct_tri_pairs_per_s": P.shape[0] * info["nf"] / (ev_d / 1e3),
                     "antipodal_qps": P.shape[0] / (ev_a / 1e3), "speedup": ev_d / ev_a})
        print(f"[bench] direct {name}: direct {ev_d:.2f} ms, antipodal {ev_a:.2f} ms, speedup {ev_d / ev_a:.1f}x",
              file=sys.stderr, flush=True)
        del mesh
    _emit("GWN queries/sec, direct triangle sum (baseline)", rows[0]["direct_qps"], "queries/s", args,
          P4.shape[0] / rows[0]["direct_qps"] * 1e3,
          {"workload": "direct per-triangle sum vs antipodal on the same points", "precision": args.prec,
           "cases": rows}, dtype="f32" if args.prec == "fp32" else "f64")


def bench_parametric(args):
    """Surfaces of cubic Bezier patches (Sec. 4.4): 100 patches with control points uniform in
    the unit cube on a 32^3 cell-centred grid over [-0.2, 1.2]^3 (the paper's synthetic
    parametric benchmark in a voxelization setting), FP64."""
    import torch
    from paper_2605_01536_amd import gwn
    n_patch, n = 100, 32
    rng = np.random.default_rng(7)
    P = rng.uniform(0.0, 1.0, size=(n_patch, 16, 3))
    g = (-0.2 + (np.arange(n) + 0.5) * (1.4 / n)).astype(np.float32)   # the grid's own rounding
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    Q = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float32)
    pt = gwn.Patches(torch.from_numpy(P).cuda())
    info = pt.info()
    Qd = torch.from_numpy(Q).cuda()
    w = torch.empty(Q.shape[0], device="cuda", dtype=torch.float64)
    st = torch.cuda.current_stream()
    origin, spacing, dims = (-0.2, -0.2, -0.2), (1.4 / n, 1.4 / n, 1.4 / n), (n, n, n)
    counts = []
    pt.query_grid(origin, spacing, dims, out=w, stream=st, counts=counts)
    nint, ncell = counts
    # the grid with ray reuse (the timed path), then single rays at the same points for comparison
    ev_ms, wall_ms = _timed(lambda: pt.query_grid(origin, spacing, dims, out=w, stream=st), args.steps,
                            args.warmup, st)
    _, _, dirs = pt.query_grid(origin, spacing, dims, want_chi=True, stream=st)
    wb = torch.empty_like(w)
    ev_b, _ = _timed(lambda: pt.query(Qd, out=wb, stream=st), max(1, args.steps // 2), 1, st)
    torch.cuda.synchronize()
    same = float((w - wb).abs().max())
    dirs = dirs.cpu().numpy()
    slots = nint * PARAM_INTERVAL_SLOTS + ncell * PARAM_CELL_SLOTS
    achieved = slots / (ev_ms / 1e3)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12, "unit": "T FP32-VALU-slots/s",
            "frac": achieved / PEAK_SLOTS, "traffic": None, "kernel": "k_param",
            "quadrature_intervals_per_query": nint / Q.shape[0], "subpatch_cells_per_query": ncell / Q.shape[0],
            "slots_per_interval": PARAM_INTERVAL_SLOTS, "slots_per_cell": PARAM_CELL_SLOTS}
    print(f"[bench] parametric: {ev_ms:.2f} ms per {Q.shape[0]} points (single rays {ev_b:.2f} ms, max diff "
          f"{same:.1e}), {nint / Q.shape[0]:.0f} intervals and {ncell / Q.shape[0]:.0f} cells per point, "
          f"directions {np.bincount(dirs + 2).tolist()} (pending, none, 0..3)", file=sys.stderr, flush=True)
    extra = {"roofline": roof}
    if not args.no_cpu_baseline:
        import oracle as O
        idx = np.sort(np.random.default_rng(1).choice(Q.shape[0], 16384, replace=False))
        sample = Q[idx].astype(np.float64)
        t0 = time.perf_counter()
        wo, _, _ = O.parametric(P, sample)
        dt = time.perf_counter() - t0
        wg = w.cpu().numpy()
        ok = np.isfinite(wo) & np.isfinite(wg[idx])
        extra["cpu_baseline"] = {"value": sample.shape[0] / dt, "unit": "queries/s", "cores": O.num_threads(),
                                 "kind": "oracle", "sample": f"{sample.shape[0]} points of the same grid, Alg. 2 "
                                 f"oracle (GK15 at 1e-12, subdivision to 1e-9 of the diagonal), {dt:.1f} s",
                                 "max_abs_err_vs_gpu": float(np.abs(wo - wg[idx])[ok].max())}
    _emit("GWN queries/sec, cubic Bezier patches (Sec. 4.4)", Q.shape[0] / (ev_ms / 1e3), "queries/s", args, ev_ms,
          {"workload": f"{n_patch} cubic Bezier patches, control points U[0,1]^3 (seed 7), {n}^3 cell-centred grid "
                       "over [-0.2, 1.2]^3", "patches": n_patch, "boundary_curves": info["ncurves"],
           "queries": int(Q.shape[0]), "tau": info["tau"], "eps": info["eps"], "max_depth": info["max_depth"],
           "path": "gwn_patches_query_grid (one line per column)", "single_rays_ms": ev_b,
           "max_diff_vs_single_rays": same},
          extra, dtype="f64")


def bench_weld(args):
    """The 1.05M-triangle soup given STL-style (three private vertices per triangle): build with
    and without welding equal positions, and w at 1M grid points through each mesh."""
    import torch
    from paper_2605_01536_amd import gwn, workloads as W
    soup, grid = W.config4()
    ex = W.explode(soup, seed=4)
    P = torch.from_numpy(W.grid_points(grid, np.sort(np.random.default_rng(0).choice(grid.n, 1 << 20,
                                                                                       replace=False)))).cuda()
    Vd, Fd = torch.from_numpy(ex.V).cuda(), torch.from_numpy(ex.F).cuda()
    st = torch.cuda.current_stream()
    rows = {}
    for weld in (True, False):
        gwn.Mesh(Vd, Fd, weld=weld)          # warm-up build
        torch.cuda.synchronize()
        t = time.perf_counter()
        m = gwn.Mesh(Vd, Fd, weld=weld)
        build_ms = (time.perf_counter() - t) * 1e3
        info = m.info()
        w = torch.empty(P.shape[0], device="cuda")
        ev, wall = _timed(lambda: gwn.query_batch(m, P, out=w, stream=st), 2 if weld else 1, 1, st)
        rows["weld" if weld else "no_weld"] = {"build_ms": build_ms, "nunique": info["nunique"],
                                               "boundary_edges": info["nboundary"], "query_ms": ev,
                                               "queries_per_s": P.shape[0] / (ev / 1e3)}
        rows["w_" + ("weld" if weld else "no_weld")] = w
        print(f"[bench] weld={weld}: build {build_ms:.1f} ms, {info['nunique']} positions, "
              f"B={info['nboundary']}, 1M points {ev:.1f} ms", file=sys.stderr, flush=True)
        del m
    diff = float((rows.pop("w_weld") - rows.pop("w_no_weld")).abs().max())
    _emit("GWN queries/sec, STL-style soup with welding", rows["weld"]["queries_per_s"], "queries/s", args,
          rows["weld"]["query_ms"], {"workload": f"opened-spheres soup exploded to {ex.nv} private vertices "
                                                 f"({ex.nf} tris), 2^20 grid points", "cases": rows,
                                     "max_abs_diff_weld_vs_not": diff})


def bench_axis(args):
    """Ray-axis choice: 12 stacked wavy sheets (960k triangles) and 2M random points; the
    crossing ray along z (meets every sheet) against the automatically chosen axis."""
    import torch
    from paper_2605_01536_amd import gwn, workloads as W
    soup = W.wavy_sheets(seed=6, n_sheets=12, n=201)
    P = torch.from_numpy(W.uniform_box(np.random.default_rng(6), 2_000_000, (-1.05,) * 3, (1.05,) * 3)).cuda()
    Vd, Fd = torch.from_numpy(soup.V).cuda(), torch.from_numpy(soup.F).cuda()
    st = torch.cuda.current_stream()
    rows, outs = {}, {}
    for axis in ("z", "auto"):
        m = gwn.Mesh(Vd, Fd, axis=axis)
        info = m.info()
        w = torch.empty(P.shape[0], device="cuda")
        up = torch.empty(P.shape[0], device="cuda", dtype=torch.int32)
        ev, _ = _timed(lambda: gwn.query_batch(m, P, out=w, stream=st), args.steps, args.warmup, st)
        ev_c, _ = _timed(lambda: gwn.query_batch(m, P, out=w, chi_out=up, stream=st), args.steps, args.warmup, st)
        outs[axis] = w.clone()
        rows[axis] = {"axis": info["axis"], "proj_area": info["proj_area"], "boundary_edges": info["nboundary"],
                      "query_ms": ev, "queries_per_s": P.shape[0] / (ev / 1e3),
                      "mean_abs_chi": float(up.abs().float().mean())}
        print(f"[bench] axis {axis} -> {info['axis']}: {ev:.2f} ms, mean |chi| {rows[axis]['mean_abs_chi']:.2f}",
              file=sys.stderr, flush=True)
        del m
    rows["max_abs_diff"] = float((outs["z"] - outs["auto"]).abs().max())
    _emit("GWN queries/sec, automatic ray axis", rows["auto"]["queries_per_s"], "queries/s", args,
          rows["auto"]["query_ms"], {"workload": f"{soup.nf} triangles in 12 stacked wavy sheets, 2M uniform points",
                                     "cases": rows})


def bench_batched(args):
    """256 ellipsoid-union soups of uneven size in one captured persistent launch, against one
    gwn_query_batch launch pair per mesh."""
    import torch
    from paper_2605_01536_amd import gwn, workloads as W
    t0 = time.time()
    soups, queries = W.config3(n_mesh=args.n_mesh)
    print(f"[bench] generated {len(soups)} soups in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    meshes = [gwn.Mesh(torch.from_numpy(s.V).cuda(), torch.from_numpy(s.F).cuda()) for s in soups]
    offs = np.concatenate([[0], np.cumsum([q.shape[0] for q in queries])]).astype(np.int64)
    Q = torch.from_numpy(np.concatenate(queries)).cuda()
    nq = int(offs[-1])
    pairs = float(sum((offs[i + 1] - offs[i]) * meshes[i].info()["nboundary"] for i in range(len(meshes))))
    print(f"[bench] {len(meshes)} meshes built, {nq} queries, {pairs:.3e} pairs", file=sys.stderr, flush=True)
    st = torch.cuda.current_stream()
    t = time.time()
    plan = gwn.MultiPlan(meshes, Q, offs, autotune=True, stream=st)
    tune_s = time.time() - t
    inf = plan.info()
    print(f"[bench] autotune {tune_s:.1f} s -> {inf}", file=sys.stderr, flush=True)
    ev_ms, wall_ms = _timed(lambda: plan.run(stream=st), args.steps, args.warmup, st)
    w_ref = torch.empty(nq, device="cuda")

    def per_mesh():
        for i, m in enumerate(meshes):
            a, b = int(offs[i]), int(offs[i + 1])
            gwn.query_batch(m, Q[a:b], out=w_ref[a:b], stream=st)

    ev2, wall2 = _timed(per_mesh, max(1, args.steps // 2), 1, st)
    same = bool(torch.equal(plan.w, w_ref))
    print(f"[bench] graph replay {wall_ms:.1f} ms vs per-mesh launches {wall2:.1f} ms; identical={same}",
          file=sys.stderr, flush=True)
    _emit("GWN queries/sec, 256 soups in one persistent graph launch", nq / (wall_ms / 1e3), "queries/s", args,
          wall_ms, {"workload": f"{len(meshes)} ellipsoid-union soups, {nq} queries, {pairs:.3e} pairs",
                    "pairs_per_s": pairs / (ev_ms / 1e3), "schedule": inf, "autotune_s": tune_s,
                    "per_mesh_launches_ms": wall2, "graph_speedup_vs_per_mesh": wall2 / wall_ms,
                    "bitwise_equal_to_per_mesh": same},
          extra={"roofline": _alu_roof(pairs, I_MIN_BATCH, ev_ms, "graph: k_chi_items + k_bdry_persistent")})


def bench_surrogate(args):
    """Train the MLP through gwn_surrogate_train on 10M points the library draws in [-1,1]^3 and
    labels with the exact kernel (the ~500k-triangle opened-spheres soup), then evaluate 16M uniform
    points: the exact kernel against network + exact fallback, for both fallback rules over a sweep
    of band half-widths."""
    import torch
    from paper_2605_01536_amd import gwn, workloads as W
    soup, _, Xin = W.config5(n_train=0)
    mesh = gwn.Mesh(torch.from_numpy(soup.V).cuda(), torch.from_numpy(soup.F).cuda())
    info = mesh.info()
    st = torch.cuda.current_stream()
    Xi = torch.from_numpy(Xin).cuda()
    del Xin
    sur = gwn.Surrogate(seed=0, sigma=args.sigma)
    n_train, batch = 10_000_000, args.train_batch
    t = time.time()
    losses = sur.train(mesh, epochs=args.epochs, n_train=n_train, batch=batch, lr=args.lr, lr_final=5e-5, seed=1,
                       box=((-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)))
    torch.cuda.synchronize()
    train_s = time.time() - t
    steps = sur.state()["step"]
    print(f"[train] {args.epochs} epochs, {steps} steps in {train_s:.1f} s (labels included); "
          f"losses {[round(x, 5) for x in losses]}", file=sys.stderr, flush=True)
    n = Xi.shape[0]
    w_ex = torch.empty(n, device="cuda")
    ex_ev, ex_ms = _timed(lambda: gwn.query_batch(mesh, Xi, out=w_ex, stream=st), args.steps, args.warmup, st)
    y = torch.empty(n, device="cuda")
    nn_ev, nn_ms = _timed(lambda: sur.forward(Xi, out=y, stream=st), args.steps, args.warmup, st)
    err_nn = (y - w_ex).abs()
    # max|err| of the exact kernel itself on these points, judged by the FP64 path
    w64 = gwn.query_batch(mesh, Xi[:1 << 20], prec="fp64")
    exact_err = float((w_ex[:1 << 20].double() - w64).abs().max())
    del w64
    w_s = torch.empty(n, device="cuda")
    sweeps = {}
    for rule, bands in (("half", (0.1, 0.2, 0.3, 0.4, 0.45, 0.5, 0.6)),
                        ("frac", (0.1, 0.2, 0.3, 0.4, 0.45, 0.48, 0.49, 0.495, 0.5, 0.5001))):
        rows = []
        for band in bands:
            res = {}

            def run():
                _, res["nfb"] = sur.query(mesh, Xi, band, out=w_s, rule=rule, stream=st)

            ev, ms = _timed(run, args.steps, 1, st)
            e = (w_s - w_ex).abs()
            agree = float(((w_s >= 0.5) == (w_ex >= 0.5)).float().mean())
            rows.append({"band": band, "ms": ms, "queries_per_s": n / (ms / 1e3), "speedup_vs_exact": ex_ms / ms,
                         "fallback_frac": res["nfb"] / n, "max_abs_err": float(e.max()),
                         "p99_abs_err": float(torch.quantile(e[::16], 0.99)),
                         "rms_err": float(e.pow(2).mean().sqrt()), "inside_outside_agreement": agree})
            print(f"[bench] rule {rule} band {band}: {ms:.1f} ms ({ex_ms / ms:.2f}x exact), fallback "
                  f"{res['nfb'] / n:.3f}, max|err| {rows[-1]['max_abs_err']:.3e}, p99 {rows[-1]['p99_abs_err']:.3e},"
                  f" agree {agree:.5f}", file=sys.stderr, flush=True)
        sweeps[rule] = rows
    best = [r for r in sweeps["half"] if r["band"] == 0.3][0]
    identical = {"exact_max_abs_err_vs_fp64": exact_err}
    # every point re-evaluated (frac rule above 1/2): the exact path's bits, its max|err| and the
    # cost of the network and the compaction on top of it
    full = sweeps["frac"][-1]
    identical["all_fallback"] = {"queries_per_s": full["queries_per_s"], "speedup_vs_exact": full["speedup_vs_exact"],
                                 "max_abs_err": full["max_abs_err"]}
    for rule, rows in sweeps.items():
        same = [r for r in rows if r["max_abs_err"] <= exact_err and r["fallback_frac"] < 1.0]
        identical[f"{rule}_smallest_band_at_exact_max_err"] = same[0]["band"] if same else None
        for tgt in (1e-1, 1e-2, 1e-3):
            ok = [r for r in rows if r["max_abs_err"] <= tgt and r["fallback_frac"] < 1.0]
            identical[f"{rule}_band_for_max_err_{tgt:g}"] = (
                {"band": ok[0]["band"], "speedup_vs_exact": ok[0]["speedup_vs_exact"]} if ok else None)
    _emit("surrogate+fallback GWN queries/sec (band 0.3)", best["queries_per_s"], "queries/s", args, best["ms"],
          {"workload": f"opened-spheres soup ({info['nf']} tris, {info['nboundary']} boundary edges), "
                       f"train {n_train} generated points / infer {n} uniform points", "exact_ms": ex_ms,
           "exact_queries_per_s": n / (ex_ms / 1e3), "network_only_ms": nn_ms,
           "network_roofline": {"bound": "mfma", "unit": "TFLOP/s", "flop_per_query": 114944,
                                "operands": "f16, f32 accumulation",
                                "achieved": n * 114944 / (nn_ev / 1e3) / 1e12,
                                "peak": PEAK_F16 / 1e12,
                                "frac": n * 114944 / (nn_ev / 1e3) / PEAK_F16},
           "network_valu_roofline": {"bound": "alu", "unit": "T VALU-slots/s",
                                     "slots_per_query": NET_VALU_SLOTS,
                                     "achieved": n * NET_VALU_SLOTS / (nn_ev / 1e3) / 1e12,
                                     "peak": PEAK_SLOTS / 1e12,
                                     "frac": n * NET_VALU_SLOTS / (nn_ev / 1e3) / PEAK_SLOTS},
           "training": {"seconds": train_s, "steps": steps, "batch": batch, "epochs": args.epochs,
                        "points_per_s": n_train * args.epochs / train_s,
                        "flop_per_point": 3 * 114944,
                        "tflop_per_s": 3 * 114944 * n_train * args.epochs / train_s / 1e12,
                        "frac_of_bf16_peak": 3 * 114944 * n_train * args.epochs / train_s / PEAK_BF16,
                        "epoch_losses": losses},
           "network_max_abs_err": float(err_nn.max()),
           "network_rms_err": float(err_nn.pow(2).mean().sqrt()), "sigma": args.sigma,
           "bands": sweeps, "identical_max_err": identical})


def bench_precision(args):
    """The 512^3 grid on the 1M-triangle soup in FP32 and FP64; both compared with the FP64
    oracle on a random sample of grid points (queries closer than 1e-4 of the diagonal to the
    surface excluded, crossing counts compared on every sampled point)."""
    import torch

    import oracle
    from paper_2605_01536_amd import gwn, workloads as W
    soup, grid = W.config4(n=args.n)
    mesh = gwn.Mesh(torch.from_numpy(soup.V).cuda(), torch.from_numpy(soup.F).cuda())
    info = mesh.info()
    st = torch.cuda.current_stream()
    res = {}
    rng = np.random.default_rng(777)
    idx = np.sort(rng.choice(grid.n, min(args.sample, grid.n), replace=False))
    it = torch.from_numpy(idx).cuda()
    P = W.grid_points(grid, idx)
    t = time.perf_counter()
    w_o = np.empty(len(idx))
    chi_o = np.empty(len(idx), dtype=np.int32)
    chunk = 25000
    for a in range(0, len(idx), chunk):     # chunks, so that progress is printed
        wo, _, co, _ = oracle.antipodal(soup.V, soup.F, P[a:a + chunk], full=True)
        w_o[a:a + chunk] = wo
        chi_o[a:a + chunk] = co
        print(f"[oracle] {min(a + chunk, len(idx))}/{len(idx)} points, {time.perf_counter() - t:.0f} s",
              file=sys.stderr, flush=True)
    oracle_s = time.perf_counter() - t
    diag = float(np.linalg.norm(np.asarray(info["bbox"][3:]) - np.asarray(info["bbox"][:3])))
    far = oracle.distance(soup.V, soup.F, P, 2e-4 * diag) > 1e-4 * diag
    print(f"[bench] oracle on {len(idx)} points: {oracle_s:.1f} s", file=sys.stderr, flush=True)
    for prec in ("fp32", "fp64"):
        w = torch.empty(grid.n, device="cuda", dtype=torch.float64 if prec == "fp64" else torch.float32)
        chi = torch.empty(grid.n, device="cuda", dtype=torch.int32)
        ev, ms = _timed(lambda: gwn.query_grid(mesh, grid.origin, grid.spacing, grid.dims, prec=prec, out=w,
                                               chi_out=chi, stream=st), args.steps, args.warmup, st)
        e = np.abs(w[it].double().cpu().numpy() - w_o)[far]
        chi_ok = bool(np.array_equal(chi[it].cpu().numpy(), chi_o))
        pairs = float(grid.n) * info["nboundary"]
        slots, _, _ = grid_slots(soup, grid, prec)
        res[prec] = {"ms": ms, "queries_per_s": grid.n / (ms / 1e3), "max_abs_err": float(e.max()),
                     "p99_abs_err": float(np.quantile(e, 0.99)), "rms_err": float(np.sqrt(np.mean(e * e))),
                     "chi_bit_exact": chi_ok,
                     "roofline": {"bound": "alu", "slots_per_pair": slots, "unit": "T FP32-VALU-slots/s",
                                  "achieved": pairs * slots / (ev / 1e3) / 1e12, "peak": PEAK_SLOTS / 1e12,
                                  "frac": pairs * slots / (ev / 1e3) / PEAK_SLOTS}}
        print(f"[bench] {prec}: {ms:.1f} ms, max|err| {e.max():.3e}, chi exact {chi_ok}", file=sys.stderr, flush=True)
        del w, chi
        torch.cuda.empty_cache()
    _emit("GWN queries/sec on 1M-tri open soup, FP32 vs FP64", res["fp32"]["queries_per_s"], "queries/s", args,
          res["fp32"]["ms"], {"workload": f"opened-spheres soup ({info['nf']} tris, {info['nboundary']} boundary "
                                          f"edges) on a {args.n}^3 grid", "sample": len(idx),
                              "compared_off_surface": int(far.sum()), "oracle_s": oracle_s,
                              "oracle_threads": oracle.num_threads(), "fp32": res["fp32"], "fp64": res["fp64"]})


if __name__ == "__main__":
    main()
