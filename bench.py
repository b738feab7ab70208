"""Benchmark: TT multigroup transport solves on one MI355X.

Workload (the 2D configuration): 128 x 128 cells on [0,1]^2, 32 groups with
log-spaced edges on [0.01, 10], 8 polar x 8 azimuthal product quadrature,
seeded lognormal kappa0 (sigma 1, correlation length 0.1), kappa_g = kappa0 nu_g^-3,
medium T = 0.1, Planck T = 1 inflow on x = 0; FP32 contractions with FP64
QR / SVD / truncation, rank cap 32, tol 1e-6; one solve = 512 steps (t = L/c
at CFL 0.5) from the rank-1 Planck state.  A benchmark step is one full solve of a batch of B independent requests
of this workload (seeds 0..B-1) advanced together on B streams.

Prints one JSON line.  `value` = aggregate solves/s of the batch with inputs
resident on the device.  A second timed phase runs one solve alone with
HIP-event timing of every kernel class on the library's stream; `roofline`
reports the dominant class from it.  `cpu_baseline` times the dense FP64 CPU
oracle on this host for a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks, TFLOP/s
    "fp64": 78.6, "fp32": 157.3, "bf16": 2500.0,
}
HBM_PEAK_GBS = 8000.0

METRIC = "TT solves/s & TT apply+round GFLOP/s (% MFMA peak); p50/p99 solve latency"


def cpu_baseline(prob, budget_s: float = 12.0):
    """Dense FP64 oracle march on the host cores for a bounded number of steps
    of the same workload, scaled to solves/s."""
    from oracle import dense
    I = dense.initial_dense(prob)
    cores = len(os.sched_getaffinity(0))
    nthr = min(cores, 16)
    dense.march(prob, I, 1, n_threads=nthr)     # warm (page-in, thread pool)
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and steps < prob.n_steps:
        I = dense.march(prob, I, 4, n_threads=nthr)
        steps += 4
    dt = time.perf_counter() - t0
    per_step = dt / steps
    return {
        "value": 1.0 / (per_step * prob.n_steps),
        "unit": "solves/s",
        "cores": nthr,
        "kind": "oracle",
        "sample": f"dense FP64 upwind march (C/OpenMP), {steps} of {prob.n_steps} steps of the same workload "
                  f"({prob.dense_entries} entries), {per_step * 1e3:.1f} ms/step, "
                  f"{prob.dense_entries / per_step:.3e} DOF-updates/s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--round-method", default="auto", choices=["qr", "gram", "auto"])
    ap.add_argument("--timing", type=int, default=1, help="HIP-event timing of kernel classes")
    ap.add_argument("--batch", type=int, default=16, help="independent solves advanced together")
    ap.add_argument("--streams", type=int, default=16, help="HIP streams for the batch")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="GPU_MAX_HW_QUEUES for this process (0: keep the environment's)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    # one hardware queue per stream: with fewer queues than streams, independent
    # solves wait behind each other's latency-bound small-core kernels.  Must be
    # set before the HIP runtime initialises.
    if args.hw_queues > 0:
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, args.hw_queues))

    import numpy as np
    import torch

    import paper_2602_00290_amd as tt
    import tt_inputs as ti

    prob = ti.plane2d()
    method = {"qr": tt.TT_ROUND_QR, "gram": tt.TT_ROUND_GRAM, "auto": tt.TT_ROUND_AUTO}[args.round_method]
    dev = torch.device("cuda:0")
    K = prob.n_steps
    B = max(1, args.batch)

    # ---- phase 1: batched throughput (B independent solves, seeds 0..B-1) ----
    probs = [prob] + [ti.plane2d(seed=b) for b in range(1, B)]
    solvers = [tt.Solver(p, device=dev, round_method=method) for p in probs]
    streams = [torch.cuda.Stream(device=dev) for _ in range(min(B, args.streams))]
    for _ in range(args.warmup):
        for sv in solvers:
            sv.reset()
        tt.solve_batch(solvers, K, streams)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        for sv in solvers:
            sv.reset()
        stats = tt.solve_batch(solvers, K, streams)
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    last = stats[0]
    value = B * args.steps / elapsed
    batch_flops = sum(sum(st["flops"].values()) for st in stats)   # flops of the last batch solve

    # ---- phase 2: one solve alone, HIP-event timing of every kernel class ----
    single = solvers[0]
    single.reset()
    single.set_timing(bool(args.timing))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = single.solve(K)
    single_s = time.perf_counter() - t1
    single.set_timing(False)
    agg_ms, agg_n, agg_fl = st1["kernel_ms"], st1["kernel_launches"], st1["flops"]

    # dominant kernel class by measured time
    dom = max(agg_ms, key=lambda c: agg_ms[c])
    prec_of = {"project": "fp32", "output": "fp32", "factor": "fp64", "tree": "fp64", "svd": "fp64", "prep": "fp64"}
    bound_of = {"project": "mfma", "output": "mfma", "factor": "mfma", "tree": "hbm", "svd": "alu", "prep": "alu"}
    roof = None
    if agg_ms[dom] > 0 and agg_n[dom] > 0:
        fl = agg_fl.get(dom, 0.0)
        avg_ms = agg_ms[dom] / agg_n[dom]
        achieved = (fl / agg_n[dom]) / (avg_ms * 1e-3) / 1e12 if fl > 0 else None
        peak = PEAKS[prec_of.get(dom, "fp64")]
        roof = {"bound": bound_of.get(dom, "alu"), "kernel_class": dom, "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": (achieved / peak) if achieved else None, "traffic": None,
                "avg_launch_ms": avg_ms, "launches": agg_n[dom]}
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plane2d: 128x128 cells, 32 groups [0.01,10], 8x8 angles, lognormal kappa0 "
                               "(sigma 1, l 0.1), FP32 contractions + FP64 factorisation/SVD, rank cap 32, tol 1e-6, "
                               "512 steps per solve",
                   "batch": B, "streams": len(streams), "seeds": f"0..{B - 1}",
                   "round_method": args.round_method, "timesteps_per_solve": K},
        "gflops": batch_flops * args.steps / elapsed / 1e9,
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "single_solve": {"solves_per_s": 1.0 / single_s, "ms": single_s * 1e3,
                         "gflops": sum(agg_fl.values()) / single_s / 1e9},
        "ranks": [last["r1"], last["r2"]],
        "max_R": [last["max_R1"], last["max_R2"]],
        "compression": last["compression"],
        "kernel_ms_per_solve": {c: agg_ms[c] for c in tt.KERNEL_CLASSES if agg_n[c]},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
