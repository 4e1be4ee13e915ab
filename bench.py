#!/usr/bin/env python3
"""Benchmark: GWN queries/s of the antipodal method on one MI355X.

Workload (default): the ~1.05M-triangle soup of 64 overlapping, randomly opened
spheres and ellipsoids in [-1,1]^3, queried on the 512^3 cell-centred grid
(134,217,728 points) through gwn_query_grid, FP32 geometry with exact
predicates and FP64 accumulation.  One step = one full grid evaluation (ray
reuse + boundary term + combine).  The mesh build is precomputation and is not
timed (Sec. 6.1 excludes it); its time is reported separately.

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

# VALU issue ceiling of MI355X: FP32 add/mul/fma (and compares, selects,
# 32-bit integer ops) issue at 32 lanes per clock per SIMD, i.e. one wave64
# instruction per 2 clocks (measured on the box; this is the rate behind the
# 157.3 TFLOP/s FP32 vector figure, which counts an FMA as 2 FLOPs):
# 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 7.86e13 FP32 VALU slots/s.
# sqrt and rcp were measured at ~3.1 slots each.
N_CU, SIMD_PER_CU, LANES_PER_CLK, CLOCK_HZ = 256, 4, 32, 2.4e9
PEAK_SLOTS = N_CU * SIMD_PER_CU * LANES_PER_CLK * CLOCK_HZ
TRANS_SLOTS = 3

# Minimal VALU slots per (query, boundary edge) pair on the grid path, with x/y
# work shared by the samples of a column (one boundary vertex per edge):
#   per sample and vertex: r_z (1), l^2 (1), sqrt, l+|r_z| (1), rcp, rho^2*rcp (1),
#                          compare + select (2)                    = 6 + 2 trans
#   per sample and edge:   D (1), fast-path test (1), rcp, N*rcp (1), t^2 (1),
#                          7 polynomial FMAs, t*x (1), final FMA (1), accumulate (1)
#                                                                  = 14 + 1 trans
I_MIN_GRID = 6 + 14 + 3 * TRANS_SLOTS      # = 29
def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--n", type=int, default=512, help="grid points per axis")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
        print("bench.py: this build measures one GPU only (queries shard without communication; "
              "see the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2605_01536_amd import gwn, workloads as W

    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(args.copy_probe)
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
    achieved = pairs * I_MIN_GRID / avg_kernel_s
    roof = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": PEAK_SLOTS / 1e12,
        "unit": "T FP32-VALU-slots/s",
        "frac": achieved / PEAK_SLOTS,
        "traffic": None,
        "kernel": "k_grid",
        "slots_per_pair": I_MIN_GRID,
        "pairs_per_launch": pairs,
        "avg_kernel_ms": avg_kernel_s * 1e3,
    }
    print(f"[bench] {n} queries, B={B}, {ms_per_step:.1f} ms/step, {qps:.3e} q/s, "
          f"{pairs / avg_kernel_s:.3e} pairs/s", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(12345)
        # size the sample to ~cpu_seconds of oracle work (calibrated on a small sample)
        cal = rng.choice(n, 64, replace=False)
        t = time.perf_counter()
        oracle.antipodal(soup.V, soup.F, W.grid_points(grid, cal))
        per_q = (time.perf_counter() - t) / 64
        m = int(max(256, min(200_000, args.cpu_seconds / max(per_q, 1e-9))))
        idx = rng.choice(n, m, replace=False)
        P = W.grid_points(grid, idx)
        t = time.perf_counter()
        w_o = oracle.antipodal(soup.V, soup.F, P)
        cpu_s = time.perf_counter() - t
        diag = float(np.linalg.norm(np.asarray(info["bbox"][3:]) - np.asarray(info["bbox"][:3])))
        far = oracle.distance(soup.V, soup.F, P, 2e-4 * diag) > 1e-4 * diag
        wg = w[torch.from_numpy(idx).cuda()].double().cpu().numpy()
        err = float(np.abs(wg - w_o)[far].max())
        cpu = {"value": m / cpu_s, "unit": "queries/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"{m} random points of the same grid, FP64 antipodal oracle, {cpu_s:.1f} s",
               "max_abs_err_vs_gpu": err, "n_compared": int(far.sum())}
        print(f"[bench] oracle {m / cpu_s:.3e} q/s on {cpu['cores']} threads; max|err| {err:.2e}",
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


if __name__ == "__main__":
    main()
