"""Benchmark: TT multigroup transport solves on one MI355X.

Workload (the 2D configuration): 128 x 128 cells on [0,1]^2, 32 groups with
log-spaced edges on [0.01, 10], 8 polar x 8 azimuthal product quadrature,
seeded lognormal kappa0 (sigma 1, correlation length 0.1), kappa_g = kappa0 nu_g^-3,
medium T = 0.1, Planck T = 1 inflow on x = 0; FP32 contractions with FP64
Gram / SVD / truncation, rank cap 32, tol 1e-6; one solve = 512 steps (t = L/c
at CFL 0.5) from the rank-1 Planck state.  A benchmark step is one full solve
of a batch of B independent requests of this workload (seeds 0..B-1)
advanced together on B streams.

Prints one JSON line.  `value` = aggregate solves/s of the batch with inputs
resident on the device.  A second timed phase runs one solve alone with
HIP-event timing of every kernel class on the library's stream; `roofline`
reports the kernel that bounds the batched throughput (the fused projection +
FP64 Gram contraction) from it, and `traffic` its HBM bytes per launch from the
committed counter summary (null when the kernel source has changed since).
`cpu_baseline` times the dense FP64 CPU oracle on this host for a bounded
sample of the same workload.

Other modes (for profiling runs; they print one line and exit):
  --mode probe        one solve of `--probe-workload` (plane2d, clumps3d, plane2d_coupled, plane2d_rusanov_scatter,
                      plane2d_randomized)
                      for `--probe-steps` steps
  --mode c3           the 64^3 clump workload at steady state: ranks at the cap, then `--steps` timed steps
  --mode c5-slab      one GPU's z-slab of the 256^3 spike workload (cap 18), `--steps` timed steps
  --mode copy         a plain device-to-device copy of `--copy-mb` MiB (counter calibration)
  --mode served       only the served request mix (capacity, then Poisson arrivals)
  --mode pmc-summary  turn rocprofv3 counter CSVs (--pmc-dir) into profiles/traffic_plane2d.json
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
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
FUSED_KERNEL = "k_fused_f32<4, true>"
KERNEL_SOURCES = ["paper_2602_00290_amd/csrc/k_fused.hpp", "paper_2602_00290_amd/csrc/k_mfma.hpp",
                  "paper_2602_00290_amd/csrc/tt_common.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_plane2d.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


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
    # the same march on one host core, over a few steps
    t1 = time.perf_counter()
    dense.march(prob, I, 4, n_threads=1)
    one = (time.perf_counter() - t1) / 4
    return {
        "value": 1.0 / (per_step * prob.n_steps),
        "unit": "solves/s",
        "cores": nthr,
        "one_core": {"ms_per_step": one * 1e3, "solves_per_s": 1.0 / (one * prob.n_steps),
                     "dof_updates_per_s": prob.dense_entries / one, "sample": "4 steps, 1 thread"},
        "kind": "oracle",
        "sample": f"dense FP64 upwind march (C/OpenMP), {steps} of {prob.n_steps} steps of the same workload "
                  f"({prob.dense_entries} entries), {per_step * 1e3:.1f} ms/step, "
                  f"{prob.dense_entries / per_step:.3e} DOF-updates/s",
    }


def stored_traffic():
    """HBM bytes per launch of the fused kernel from the committed counter
    summary, or None if it is missing or was taken on different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t


def tt_rel_diff(x, y):
    """||X - Y|| / ||X|| of two TTs (Z, Theta, Phi) from TT inner products (no
    full tensor): <X, Y> = sum Phi_x Phi_y^T o (Theta_x^T (Z_x^T Z_y) Theta_y)."""
    import numpy as np

    def inner(a, b):
        Za, Ta, Pa = a
        Zb, Tb, Pb = b
        A = Za.T @ Zb                                        # r1a x r1b
        Bm = np.einsum("ij,ilp,jlq->pq", A, Ta, Tb)          # r2a x r2b
        return float(np.sum(Bm * (Pa @ Pb.T)))
    xx, yy, xy = inner(x, x), inner(y, y), inner(x, y)
    return float(np.sqrt(max(xx + yy - 2.0 * xy, 0.0) / xx))


def roofline(st1):
    """Roofline of the fused projection + FP64 Gram kernel from the single-solve
    event timing.  Its flops are FP32 MFMA (projection, 2 M R1 k1 per launch)
    plus FP64 MFMA (symmetric Gram, M k1 (k1 + 1)); the peak is the rate of
    that mix at the published dense peaks: (F32 + F64) / (F32 / P32 + F64 / P64)."""
    ms, n, fl = st1["kernel_ms"], st1["kernel_launches"], st1["flops"]
    if not n["project"] or not ms["project"]:
        return None
    f32, f64 = fl["project"], (fl["factor"] if n["factor"] == 0 else 0.0)
    sec = ms["project"] * 1e-3
    achieved = (f32 + f64) / sec / 1e12
    peak = (f32 + f64) / (f32 / PEAKS["fp32"] + f64 / PEAKS["fp64"]) if (f32 + f64) > 0 else PEAKS["fp32"]
    t = stored_traffic()
    out = {"bound": "mfma", "kernel": FUSED_KERNEL, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
           "frac": achieved / peak, "traffic": (t["fetch_bytes"] + t["write_bytes"]) if t else None,
           "avg_launch_ms": ms["project"] / n["project"], "launches": n["project"],
           "flops_per_launch": {"fp32": f32 / n["project"], "fp64": f64 / n["project"]}}
    if t:
        out["traffic_detail"] = {k: t[k] for k in ("fetch_bytes", "write_bytes", "algorithmic_bytes")}
    return out


def kernel_hbm(st1, M):
    """Achieved algorithmic HBM rate of the two first-core kernels from the
    single-solve event timing, with the minimum bytes of each launch at the
    final ranks: the projection reads the state Z (M r1 FP32 values), the
    output kernel reads Z and writes Z_out (2 M r1 values)."""
    ms, n = st1["kernel_ms"], st1["kernel_launches"]
    r1 = st1["r1"]
    out = {}
    for cls, words in (("project", 1), ("output", 2)):
        if n[cls] and ms[cls]:
            t = ms[cls] / n[cls] * 1e-3
            out[cls] = {"GB_per_s": words * M * r1 * 4 / t / 1e9, "bytes_per_launch": words * M * r1 * 4,
                        "avg_launch_us": t * 1e6}
    return out


def served_phase(args):
    """The served request mix: 50/50 1D (16 GL mu) / 2D (8 x 8), cells per
    dimension U{64..256}, groups U{16..64}, rank caps U{4..48}, FP32/FP64 split,
    64 steps each.  First all requests arrive at once (capacity = completed
    requests/s); then Poisson arrivals at 0.8 x capacity give p50/p99 latency."""
    import tt_inputs as ti
    from paper_2602_00290_amd.serve import Server, make_requests

    probs = ti.served_requests(args.served, seed=0, steps=64)
    srv = Server(budget_bytes=int(args.served_budget_gb * (1 << 30)), max_active=args.served_slots,
                 n_streams=min(16, args.served_slots), chunk=4)
    cap = srv.run(make_requests(probs))
    rate = 0.8 * cap["throughput_rps"]
    arr = ti.poisson_arrivals(len(probs), rate, seed=0)
    live = srv.run(make_requests(probs, arr))
    keep = ("p50_ms", "p99_ms", "mean_ms", "throughput_rps", "makespan_s", "max_active", "peak_workspace_bytes")
    return {"requests": len(probs), "steps_per_request": 64,
            "mix": "1D (16 GL mu) / 2D (8x8) 50/50, cells/dim U{64..256}, groups U{16..64}, caps U{4..48}, "
                   "FP32 (Gram) / FP64 (QR) 50/50, seed 0",
            "budget_gb": args.served_budget_gb, "slots": args.served_slots,
            "capacity_rps": cap["throughput_rps"], "capacity_run": {k: cap[k] for k in keep},
            "arrival_rate_rps": rate, **{k: live[k] for k in keep}}


def mode_copy(args):
    import torch
    n = args.copy_mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(8):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_per_copy": n * 4, "copies": 8}), flush=True)


def rusanov_scatter_problem(ti):
    """plane2d with the Rusanov flux (S+ = c) and isotropic scattering
    kappa_s = kappa_a (the absorption field of the same seed)."""
    import numpy as np
    prob = ti.plane2d()
    ks = np.outer(prob.kappa0, prob.kappa_scale)
    return prob.copy(flux=ti.FLUX_RUSANOV, rusanov_s=1.0, kappa_s_full=ks)


def mode_probe(args):
    import torch
    import paper_2602_00290_amd as tt
    import tt_inputs as ti
    if args.probe_workload == "clumps3d":
        prob = ti.clumps3d(precision=ti.PREC_BF16X)
    elif args.probe_workload == "plane2d_coupled":
        prob = ti.plane2d()
        prob = prob.copy(heat_capacity=8.0 * ti.radiation_constant(prob.c))
    elif args.probe_workload == "plane2d_rusanov_scatter":
        prob = rusanov_scatter_problem(ti)
    elif args.probe_workload == "plane2d_randomized":
        prob = ti.plane2d().copy(round_method=ti.ROUND_RAND, rand_oversample=4, rand_seed=0)
    else:
        prob = ti.plane2d()
    s = tt.Solver(prob)
    st = s.solve(args.probe_steps)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "probe", "workload": args.probe_workload, "steps": args.probe_steps,
                      "ranks": [st["r1"], st["r2"]]}), flush=True)


def mode_c5_slab(args):
    """The 256^3 spike workload on one GPU's share: a 256 x 256 x 32 z-slab
    (128 groups, 16 x 16 directions, split BF16), at the largest rank cap whose
    projected rank fits the SVD chain (k1 <= 128: cap 18).  Untimed steps until
    the ranks reach the cap, then --steps timed steps with HIP-event kernel
    timing."""
    import tt_inputs as ti
    prob = ti.spikes3d_slab(rank_cap=args.c5_cap)
    return steady_steps(args, prob, "c5-slab",
                        "spikes3d z-slab 256 x 256 x 32 cells (1/8 of the 256^3 cube), 128 groups, "
                        "16 x 16 directions, split BF16 contractions, FP64 rounding, tol 1e-5", args.c5_warmup, 4)


def mode_c3(args):
    """The 64^3 clump workload (64 groups, 8 x 16 directions, cap 64, split
    BF16): untimed steps until the ranks have reached the cap (about 30 steps),
    then --steps timed steps with HIP-event kernel timing (steady state)."""
    import tt_inputs as ti
    prob = ti.clumps3d(precision=ti.PREC_BF16X)
    return steady_steps(args, prob, "c3",
                        "clumps3d 64^3 cells, 64 groups, 8 x 16 directions, split BF16 contractions, "
                        "FP64 rounding, cap 64, tol 1e-5", 48, 32)


def steady_steps(args, prob, mode, workload, max_warm, min_warm):
    import torch
    import paper_2602_00290_amd as tt
    ws = tt.workspace_bytes(prob)
    print(json.dumps({"mode": mode, "phase": "setup", "rows": prob.M, "workspace_gb": ws / 2 ** 30}),
          flush=True)
    s = tt.Solver(prob)
    warm = 0
    while warm < max_warm:
        st = s.solve(1)
        warm += 1
        print(json.dumps({"phase": "warmup", "step": warm, "ranks": [st["r1"], st["r2"]],
                          "ms": st["seconds"] * 1e3}), flush=True)
        if st["r1"] >= prob.rank_cap and warm >= min_warm:
            break
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.solve(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    n = st["kernel_launches"]
    print(json.dumps({
        "mode": mode, "workload": workload, "rows": prob.M, "rank_cap": prob.rank_cap, "warmup_steps": warm,
        "steps": args.steps,
        "ms_per_step": el / args.steps * 1e3, "ranks": [st["r1"], st["r2"]], "max_R": [st["max_R1"], st["max_R2"]],
        "compression": st["compression"], "workspace_gb": ws / 2 ** 30, "timing": "HIP events on",
        "kernel_ms_per_step": {c: st["kernel_ms"][c] / args.steps for c in tt.KERNEL_CLASSES if n[c]},
        "flops_per_step": sum(st["flops"].values()) / args.steps}), flush=True)


def _pmc_rows(path, counter):
    rows = []
    for fn in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
        with open(fn) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    return rows


def mode_pmc_summary(args):
    """profiles/traffic_plane2d.json from four counter runs under --pmc-dir:
    fetch/ and write/ (FETCH_SIZE, WRITE_SIZE of `--mode probe`), copy_fetch/ and
    copy_write/ (the same counters of `--mode copy`).  Counter values are KiB per
    dispatch; each is scaled by copy bytes / counter of the copy kernel."""
    d = args.pmc_dir
    nbytes = args.copy_mb * (1 << 20)

    def copy_factor(sub, counter):
        rows = _pmc_rows(os.path.join(d, sub), counter)
        vals = sorted(v for _, _, v in rows)[-4:]          # the large copies
        return nbytes / (sum(vals) / len(vals) * 1024.0)

    def fused(sub, counter):
        key = FUSED_KERNEL.replace(" ", "")
        rows = [v for _, k, v in _pmc_rows(os.path.join(d, sub), counter) if key in k.replace(" ", "")]
        steady = rows[len(rows) // 2:]                      # second half: ranks at their steady values
        return sum(steady) / len(steady) * 1024.0, len(steady)

    ff, fw = copy_factor("copy_fetch", "FETCH_SIZE"), copy_factor("copy_write", "WRITE_SIZE")
    fetch, nf = fused("fetch", "FETCH_SIZE")
    write, nw = fused("write", "WRITE_SIZE")
    import tt_inputs as ti
    p = ti.plane2d()
    out = {
        "kernel": FUSED_KERNEL,
        "workload": "plane2d steady state (second half of a 64-step probe)",
        "source_hash": kernel_source_hash(),
        "fetch_bytes": fetch * ff,
        "write_bytes": write * fw,
        "raw_fetch_bytes": fetch, "raw_write_bytes": write, "dispatches": [nf, nw],
        "calibration": {"copy_bytes": nbytes, "fetch_factor": ff, "write_factor": fw},
        # Z read once (ld 24 floats) + row table (8 B) + neighbour table (4 ints) + rank-1
        # block (4 floats) per row, + the Gram partials written
        "algorithmic_bytes": p.M * (24 * 4 + 8 + 16 + 16) + 256 * 10 * 256 * 8,
        "commands": [f"rocprofv3 --pmc {c} --output-format csv -d <dir>/{s} -o {s} -- python3 bench.py --mode {m}"
                     for c, s, m in (("FETCH_SIZE", "fetch", "probe"), ("WRITE_SIZE", "write", "probe"),
                                     ("FETCH_SIZE", "copy_fetch", "copy"), ("WRITE_SIZE", "copy_write", "copy"))],
    }
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({"mode": "pmc-summary", **{k: out[k] for k in ("fetch_bytes", "write_bytes")}}), flush=True)


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
    ap.add_argument("--mode", default="bench",
                    choices=["bench", "probe", "copy", "pmc-summary", "served", "c5-slab", "c3"])
    ap.add_argument("--c5-cap", type=int, default=18, help="rank cap of --mode c5-slab")
    ap.add_argument("--c5-warmup", type=int, default=40, help="at most this many untimed steps in --mode c5-slab")
    ap.add_argument("--probe-steps", type=int, default=64)
    ap.add_argument("--probe-workload", default="plane2d",
                    choices=["plane2d", "clumps3d", "plane2d_coupled", "plane2d_rusanov_scatter", "plane2d_randomized"],
                    help="probe workload: plane2d (FP32), clumps3d (64^3 cells, 64 groups, split BF16), "
                         "plane2d_coupled (plane2d with the coupled medium temperature, heat capacity 8 a), "
                         "plane2d_rusanov_scatter (plane2d with the Rusanov flux and scattering kappa_s = kappa_a), "
                         "or plane2d_randomized (plane2d with randomized rounding, sketch ranks = ranks + 4)")
    ap.add_argument("--copy-mb", type=int, default=512)
    ap.add_argument("--pmc-dir", default=os.path.join(ROOT, "gpurun_out", "traffic"))
    ap.add_argument("--plain-fp64", type=int, default=1, help="also time the plain FP64 TT path on seed 0")
    ap.add_argument("--coupled", type=int, default=1,
                    help="also time seed 0 with the coupled medium temperature (heat capacity 8 a)")
    ap.add_argument("--rusanov-scatter", type=int, default=1,
                    help="also time seed 0 with the Rusanov flux and isotropic scattering (kappa_s = kappa_a)")
    ap.add_argument("--randomized", type=int, default=1,
                    help="also time seed 0 with randomized rounding (sketch ranks = ranks + 4) beside Gram rounding")
    ap.add_argument("--c1-batch", type=int, default=256,
                    help="also time this many independent 1D slab solves (FP64, 128 steps) as one batch")
    ap.add_argument("--served", type=int, default=256,
                    help="requests of the served mix (0: skip the serving phase)")
    ap.add_argument("--served-budget-gb", type=float, default=64.0)
    ap.add_argument("--served-slots", type=int, default=32)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.mode == "pmc-summary":
        return mode_pmc_summary(args)
    # one hardware queue per stream: with fewer queues than streams, independent
    # solves wait behind each other's latency-bound small-core kernels.  Must be
    # set before the HIP runtime initialises.
    if args.hw_queues > 0:
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, args.hw_queues))
    if args.mode == "copy":
        return mode_copy(args)
    if args.mode == "probe":
        return mode_probe(args)
    if args.mode == "c5-slab":
        return mode_c5_slab(args)
    if args.mode == "c3":
        return mode_c3(args)
    if args.mode == "served":
        print(json.dumps({"mode": "served", **served_phase(args)}), flush=True)
        return

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
    # internal delta-ranks of the final combined core (discussion of the internal structure of Z)
    internal = {}
    for delta in (1e-3, 1e-6):
        t4 = time.perf_counter()
        ir = single.internal_ranks(delta)
        internal[f"{delta:g}"] = {"r_nux": ir["r_nux"], "r_xnu": ir["r_xnu"], "C_rel_nu": ir["C_rel_nu"],
                                  "C_rel_x": ir["C_rel_x"], "ms": (time.perf_counter() - t4) * 1e3}

    # ---- phase 3: the plain FP64 TT path (FP64 state, Householder TSQR) on seed 0 ----
    plain = None
    if args.plain_fp64:
        sp = tt.Solver(prob.copy(precision=ti.PREC_FP64), device=dev, round_method=tt.TT_ROUND_QR)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        stp = sp.solve(K)
        plain_s = time.perf_counter() - t2
        a, b = single.get_cores(), sp.get_cores()
        plain = {"solves_per_s": 1.0 / plain_s, "ms": plain_s * 1e3, "ranks": [stp["r1"], stp["r2"]],
                 "rel_l2_mixed_vs_fp64": tt_rel_diff(a, b),
                 "speedup_batched_mixed_vs_plain_fp64": value * plain_s}
        sp.destroy()
    # ---- phase 4: seed 0 with the coupled medium temperature (Section 2.1 coupled source stage) ----
    coupled = None
    if args.coupled:
        pc = prob.copy(heat_capacity=8.0 * ti.radiation_constant(prob.c))
        sc = tt.Solver(pc, device=dev, round_method=method)
        sc.set_timing(True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        stc = sc.solve(K)
        coupled_s = time.perf_counter() - t3
        Tc = sc.get_temperature()
        nc = stc["kernel_launches"]["couple"]
        coupled = {"solves_per_s": 1.0 / coupled_s, "ms": coupled_s * 1e3, "timing": "HIP events on",
                   "heat_capacity": "8 a (a = 8 pi^5 / (15 c))", "ranks": [stc["r1"], stc["r2"]],
                   "couple_us_per_launch": stc["kernel_ms"]["couple"] / max(1, nc) * 1e3,
                   "couple_launches": nc, "T_mean": float(Tc.mean()), "T_max": float(Tc.max()),
                   "energy_total": stc["energy"] / pc.c + stc["medium_energy"]}
        sc.destroy()
    # ---- phase 6: the 1D slab (FP64, cap 8, 128 steps), batched: latency-bound solves ----
    c1 = None
    if args.c1_batch > 0:
        p1 = ti.slab1d()
        c1s = [tt.Solver(p1, device=dev) for _ in range(args.c1_batch)]
        c1st = [torch.cuda.Stream(device=dev) for _ in range(min(args.c1_batch, args.streams))]
        for sv in c1s:
            sv.reset()
        tt.solve_batch(c1s, p1.n_steps, c1st)        # warm-up
        torch.cuda.synchronize()
        t6 = time.perf_counter()
        for sv in c1s:
            sv.reset()
        c1stats = tt.solve_batch(c1s, p1.n_steps, c1st)
        torch.cuda.synchronize()
        c1_s = time.perf_counter() - t6
        one = c1s[0]
        one.reset()
        torch.cuda.synchronize()
        t7 = time.perf_counter()
        one.solve(p1.n_steps)
        c1_one = time.perf_counter() - t7
        c1 = {"workload": "slab1d: 64 cells, 8 groups [0.01,10], 16 GL mu, FP64, cap 8, tol 1e-8, 128 steps",
              "batch": args.c1_batch, "streams": len(c1st), "solves_per_s": args.c1_batch / c1_s,
              "single_solve_ms": c1_one * 1e3, "ranks": [c1stats[0]["r1"], c1stats[0]["r2"]]}
        for sv in c1s:
            sv.destroy()
    # ---- phase 5: seed 0 with the Rusanov flux and isotropic scattering ----
    rus = None
    if args.rusanov_scatter:
        pr = rusanov_scatter_problem(ti)
        sr = tt.Solver(pr, device=dev, round_method=method)
        sr.set_timing(True)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        str_ = sr.solve(K)
        rus_s = time.perf_counter() - t5
        nr = str_["kernel_launches"]["couple"]
        rus = {"solves_per_s": 1.0 / rus_s, "ms": rus_s * 1e3, "timing": "HIP events on",
               "flux": "Rusanov, S+ = c", "scattering": "kappa_s = kappa_a", "ranks": [str_["r1"], str_["r2"]],
               "max_R": [str_["max_R1"], str_["max_R2"]],
               "prepass_us_per_launch": str_["kernel_ms"]["couple"] / max(1, nr) * 1e3,
               "kernel_us_per_launch": {c: str_["kernel_ms"][c] / str_["kernel_launches"][c] * 1e3
                                        for c in tt.KERNEL_CLASSES if str_["kernel_launches"][c]}}
        sr.destroy()
    # ---- phase 7: seed 0 with randomized rounding (Section 3.1 footnote), beside Gram rounding ----
    rnd = None
    if args.randomized:
        prr = prob.copy(round_method=ti.ROUND_RAND, rand_oversample=4, rand_seed=0)
        srr = tt.Solver(prr, device=dev)
        srr.solve(2)                                   # warm-up
        srr.reset()
        torch.cuda.synchronize()
        t8 = time.perf_counter()
        strr = srr.solve(K)
        rnd_s = time.perf_counter() - t8
        diff = tt_rel_diff(single.get_cores(), srr.get_cores())
        # the Gram-rounded solve under the same conditions (no events)
        single.reset()
        single.set_timing(False)
        torch.cuda.synchronize()
        t9 = time.perf_counter()
        single.solve(K)
        gram_s = time.perf_counter() - t9
        srr.reset()
        srr.set_timing(True)
        stre = srr.solve(K)
        ns = stre["kernel_launches"]["svd"]
        rnd = {"solves_per_s": 1.0 / rnd_s, "ms": rnd_s * 1e3, "gram_single_solve_ms": gram_s * 1e3,
               "oversample": 4, "ranks": [strr["r1"], strr["r2"]],
               "sketch_ranks_last": [strr["sketch_r1"], strr["sketch_r2"]],
               "rel_l2_vs_gram_solve": diff,
               "svd_class_us_per_round": stre["kernel_ms"]["svd"] / max(1, K) * 1e3,
               "svd_class_launches_per_round": ns / max(1, K),
               "timing": "solve without events; per-class times from a second solve with HIP events"}
        srr.destroy()
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
                               "(sigma 1, l 0.1), FP32 contractions + FP64 Gram/SVD, rank cap 32, tol 1e-6, "
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
        "kernel_us_per_launch": {c: agg_ms[c] / agg_n[c] * 1e3 for c in tt.KERNEL_CLASSES if agg_n[c]},
        "roofline": roofline(st1),
        "hbm_algorithmic": kernel_hbm(st1, prob.M),
        "internal_ranks": internal,
    }
    if plain:
        out["plain_fp64"] = plain
    if coupled is not None:
        out["coupled_temperature"] = coupled
    if rus is not None:
        out["rusanov_scattering"] = rus
    if rnd is not None:
        out["randomized_rounding"] = rnd
    if c1 is not None:
        out["c1_slab1d"] = c1
    if args.served > 0:
        out["served"] = served_phase(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
