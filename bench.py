"""Benchmark: TT multigroup transport solves on one MI355X.

Headline workload (the 3D configuration, the largest that fits one GPU):
64^3 cells on [0,1]^3, 64 groups with log-spaced edges on [0.01, 10], 8
polar x 16 azimuthal product quadrature, seeded lognormal kappa0 (sigma 1,
correlation length 0.1) with two dense spherical clumps (x100), kappa_g =
kappa0 nu_g^-3, medium T = 0.1, Planck T = 1 inflow on x = 0, rank cap 64,
tol 1e-5; a solve is 384 steps (t = L/c at CFL 0.5).  The headline runs it
with an FP64 state, FP64 contractions on FP64 MFMA and FP64 Gram rounding.
One benchmark step is one time step of that solve (the whole apply + round
path over the 16.8M-row first core).  Untimed steps first bring the ranks to
the cap (the solve's steady state, R1 = 450 and k1 = 128), then --warmup
untimed steps, then --steps timed steps; `value` = 1 / (384 x time per step)
= TT solves/s with the state resident in HBM.

Beside it: the same workload in split BF16 and FP32 (with their relative L2
difference from the FP64 state after the same steps) and with Householder QR
rounding in FP64; the 2D configuration (128^2 x 32 groups x 8 x 8 angles) as
16 batched FP32 solves, one FP32 solve and one FP64 solve (Gram and QR
rounding), each compared with the dense FP64 oracle march; the 1D slab as
256 batched solves; the served request mix (p50 / p99 latency, also the
top-level p50_ms / p99_ms); and `cpu_baseline`, the dense FP64 CPU oracle
timed on z-slabs of the same 64^3 cube and scaled to the whole cube.

Prints one JSON line.  `roofline` covers the dominant kernel, the
direction-space stencil of the 3D headline's FP64 projection, from its
HIP-event times; `traffic` its HBM bytes per launch from the committed counter
summary (null when the kernel source has changed since).

Other modes (for profiling runs; they print one line and exit):
  --mode probe        one solve of `--probe-workload` for `--probe-steps` steps (clumps3d_fp64 first
                      brings the ranks to the cap)
  --mode c3           the 64^3 clump workload in split BF16 at steady state, `--steps` timed steps
  --mode c5-slab      one GPU's z-slab of the 256^3 spike workload (cap 18), `--steps` timed steps
  --mode copy         a plain device-to-device copy of `--copy-mb` MiB (counter calibration)
  --mode served       only the served request mix (capacity, then Poisson arrivals)
  --mode pmc-summary  turn rocprofv3 counter CSVs (--pmc-dir) into profiles/traffic_<workload>.json
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
C3_STEPS_PER_SOLVE = 384
# the dominant kernel of the headline: the direction-space stencil of the
# FP64 projection (128 columns); beside it Y = Z W and the gathered projection
HEAD_KERNEL = "k_stencil_f64"
ANGLE_KERNEL = "k_mm_f64<2, 8, false, 1, false>"
GATHER_KERNEL = "k_mm_f64<0, 8, false, 1, false>"
KERNEL_SOURCES = ["paper_2602_00290_amd/csrc/k_f64.hpp", "paper_2602_00290_amd/csrc/k_fused.hpp",
                  "paper_2602_00290_amd/csrc/tt_common.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_clumps3d_fp64.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def host_cores() -> int:
    return len(os.sched_getaffinity(0))


def cpu_baseline_c3(budget_s: float = 15.0, nz: int = 4):
    """Dense FP64 oracle march (C/OpenMP) of z-slabs of the 64^3 clump cube on
    all host cores: steps of one 64 x 64 x nz slab (the cube's field and cell
    spacing) until about budget_s has passed, scaled by 64 / nz to the whole
    cube and by 384 steps to a solve."""
    import tt_inputs as ti
    from oracle import dense
    prob = ti.clumps3d_slab(nz=nz, precision=ti.PREC_FP64)
    cores = host_cores()
    I = dense.initial_dense(prob)
    I = dense.march(prob, I, 1, n_threads=cores)     # warm (page-in, thread pool)
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and steps < 64:
        I = dense.march(prob, I, 2, n_threads=cores)
        steps += 2
    per_slab_step = (time.perf_counter() - t0) / steps
    scale = 64 // nz
    per_step = per_slab_step * scale
    del I
    return {
        "value": 1.0 / (per_step * C3_STEPS_PER_SOLVE),
        "unit": "solves/s",
        "cores": cores,
        "threads": cores,
        "kind": "oracle",
        "sample": f"dense FP64 upwind march (C/OpenMP) of a 64 x 64 x {nz}-cell z-slab of the 64^3 cube "
                  f"(64 groups, 8 x 16 directions, {prob.dense_entries} entries), {steps} steps at "
                  f"{per_slab_step * 1e3:.1f} ms each, scaled x{scale} to the cube ({per_step:.2f} s/step) and "
                  f"x{C3_STEPS_PER_SOLVE} steps to a solve",
        "dof_updates_per_s": prob.dense_entries / per_slab_step,
    }


def stored_traffic(project_blocks=None, kernel=None):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None if it is missing, was taken on different kernel source,
    for another kernel than `kernel` or at a grid other than `project_blocks`
    (when given)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    if kernel is not None and t.get("kernel") != kernel:
        return None
    if project_blocks is not None and t.get("project_blocks") != project_blocks:
        return None
    return t


def tt_diff_norm(x, y):
    """||X - Y||_F and ||Y||_F of two TTs (Z, Theta, Phi) without the full
    tensor: the difference is the TT with Z = [Z_x, Z_y], Theta block-diagonal
    and Phi = [Phi_x; -Phi_y]; its norm is that of R x (Theta, Phi) with R the
    triangular factor of the stacked first core, taken by row chunks (a
    Householder R of the chunk R's), so no cancellation limits it."""
    import numpy as np

    def first_core_r(Zs):
        Rs = []
        M = Zs[0].shape[0]
        for k0 in range(0, M, 1 << 20):
            C = np.hstack([Z[k0:k0 + (1 << 20)] for Z in Zs])
            Rs.append(np.linalg.qr(C, mode="r"))
        return np.linalg.qr(np.vstack(Rs), mode="r")

    def norm_of(R, Th, Ph):
        T = np.einsum("ia,alb->ilb", R, Th)
        return float(np.linalg.norm(np.einsum("ilb,bp->ilp", T, Ph)))

    Zx, Tx, Px = x
    Zy, Ty, Py = y
    r1x, nt, r2x = Tx.shape
    r1y, _, r2y = Ty.shape
    Th = np.zeros((r1x + r1y, nt, r2x + r2y))
    Th[:r1x, :, :r2x] = Tx
    Th[r1x:, :, r2x:] = Ty
    Ph = np.vstack([Px, -Py])
    dn = norm_of(first_core_r([Zx, Zy]), Th, Ph)
    yn = norm_of(first_core_r([Zy]), Ty, Py)
    return dn, yn


def tt_rel_diff(x, y):
    """||X - Y|| / ||Y|| of two TTs (see tt_diff_norm)."""
    dn, yn = tt_diff_norm(x, y)
    return dn / yn if yn > 0 else dn


def roofline_c3(st, M, tuning=None, ndir=128):
    """Roofline of the headline's dominant kernel from its HIP-event times
    over the timed steps.

    In the steady state the first-core pass runs in direction space: Y = Z W
    (FP64 MFMA, K = r1) and the operator's stencil on Y, which is the longest
    kernel of the step and HBM-bound: its algorithmic bytes per launch are one
    read of Y and one write of B, 2 M k1 8 with k1 = N_theta N_phi.  Beside
    it, `projection_stage` counts the whole pass as the method defines it, the
    R factor of the explicit M x R1 sum (2 M R1^2 - 2/3 R1^3 flops per launch,
    R1 = 450 at the cap), over the time of both kernels, and `executed` the
    flops they run.  Without direction-space passes the gathered projection
    is reported by that count as before."""
    ms, n, fl = st["kernel_ms"], st["kernel_launches"], st["flops"]
    R1 = st["max_R1"]
    alg = 2.0 * M * R1 * R1 - 2.0 / 3.0 * R1 ** 3
    peak64 = PEAKS["fp64"]
    if n.get("stencil") and st.get("direction_space_rounds", 0) > 0 and ms["stencil"] > 0:
        t_st = ms["stencil"] / n["stencil"] * 1e-3
        t_ang = ms["angle"] / n["angle"] * 1e-3
        t_pass = t_st + t_ang
        byt = 2.0 * M * ndir * 8
        t = stored_traffic(kernel=HEAD_KERNEL)
        exe = (fl["angle"] + fl["stencil"]) / n["stencil"]
        out = {"bound": "hbm", "kernel": HEAD_KERNEL, "achieved": byt / t_st / 1e9, "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": byt / t_st / 1e9 / HBM_PEAK_GBS,
               "traffic": (t["fetch_bytes"] + t["write_bytes"]) if t else None,
               "avg_launch_ms": t_st * 1e3, "launches": n["stencil"], "algorithmic_bytes_per_launch": byt,
               "projection_stage": {
                   "kernels": [ANGLE_KERNEL, HEAD_KERNEL], "avg_ms": t_pass * 1e3, "angle_ms": t_ang * 1e3,
                   "algorithmic_flops_per_launch": alg, "R1": R1, "achieved": alg / t_pass / 1e12, "peak": peak64,
                   "unit": "TFLOP/s", "frac": alg / t_pass / 1e12 / peak64,
                   "executed": {"flops_per_launch": exe, "TFLOP_per_s": exe / t_pass / 1e12,
                                "frac": exe / t_pass / 1e12 / peak64}}}
        if t:
            out["traffic_detail"] = {k: t[k] for k in ("fetch_bytes", "write_bytes", "algorithmic_bytes")}
        return out
    if not n["project"] or not ms["project"]:
        return None
    t_launch = ms["project"] / n["project"] * 1e-3
    exe = fl["project"] / n["project"]
    t = stored_traffic(tuning["project_blocks"] if tuning else None, kernel=GATHER_KERNEL)
    out = {"bound": "mfma", "kernel": GATHER_KERNEL, "achieved": alg / t_launch / 1e12, "peak": peak64,
           "unit": "TFLOP/s", "frac": alg / t_launch / 1e12 / peak64,
           "traffic": (t["fetch_bytes"] + t["write_bytes"]) if t else None,
           "avg_launch_ms": t_launch * 1e3, "launches": n["project"],
           "algorithmic_flops_per_launch": alg, "R1": R1,
           "executed": {"flops_per_launch": exe, "TFLOP_per_s": exe / t_launch / 1e12,
                        "frac": exe / t_launch / 1e12 / peak64}}
    if t:
        out["traffic_detail"] = {k: t[k] for k in ("fetch_bytes", "write_bytes", "algorithmic_bytes")}
    return out


def c3_run(prob, method, rank_warm, args, label, keep_cores=True, timing_steps=4):
    """The 3D workload from its initial state: rank_warm untimed steps (or,
    when None, until the ranks reach the cap), args.warmup untimed steps,
    args.steps timed steps (no events), then timing_steps more with HIP-event
    timing of every kernel class.  Returns the measurements and the cores."""
    import torch
    import paper_2602_00290_amd as tt
    s = tt.Solver(prob, round_method=method)
    warm = 0
    if rank_warm is None:
        while warm < 48:
            st = s.solve(1)
            warm += 1
            if st["r1"] >= prob.rank_cap and warm >= 24:
                break
    else:
        s.solve(rank_warm)
        warm = rank_warm
    # launch shapes tuned on the state at the cap (untimed set-up)
    tuning = s.tune(args.tune_cache) if args.tune else None
    if args.warmup > 0:
        s.solve(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.solve_async(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s.set_timing(True)
    stt = s.solve(timing_steps)
    s.set_timing(False)
    n = stt["kernel_launches"]
    out = {"label": label, "ms_per_step": el / args.steps * 1e3, "rank_warmup_steps": warm,
           "ranks": [stt["r1"], stt["r2"]], "max_R": [stt["max_R1"], stt["max_R2"]],
           "compression": stt["compression"],
           "kernel_ms_per_step": {c: stt["kernel_ms"][c] / timing_steps for c in tt.KERNEL_CLASSES if n[c]},
           "flops_per_step": sum(stt["flops"].values()) / timing_steps,
           "workspace_gb": s.nbytes / 2 ** 30, "tuning": tuning}
    print(json.dumps({"phase": label, "ms_per_step": out["ms_per_step"], "ranks": out["ranks"]}),
          file=sys.stderr, flush=True)
    cores = s.get_cores() if keep_cores else None
    s.destroy()
    return out, stt, cores


def c3_phase(args):
    """The headline (FP64) and the other precisions and rounding beside it."""
    import tt_inputs as ti
    import paper_2602_00290_amd as tt
    p64 = ti.clumps3d(precision=ti.PREC_FP64)
    head, st64, cores64 = c3_run(p64, tt.TT_ROUND_GRAM, None, args, "clumps3d fp64 gram")
    warm = head["rank_warmup_steps"]
    beside = {}
    if args.c3_beside:
        for name, prob, method in (("bf16x", ti.clumps3d(precision=ti.PREC_BF16X), tt.TT_ROUND_AUTO),
                                   ("fp32", ti.clumps3d(precision=ti.PREC_FP32), tt.TT_ROUND_AUTO),
                                   ("fp64_qr", p64, tt.TT_ROUND_QR)):
            r, _, cores = c3_run(prob, method, warm, args, "clumps3d " + name)
            r["rel_l2_vs_fp64_gram"] = tt_rel_diff(cores, cores64)
            r["solves_per_s"] = 1e3 / (C3_STEPS_PER_SOLVE * r["ms_per_step"])
            beside[name] = r
            del cores
    return head, st64, beside, p64


def served_phase(args):
    """The served request mix: 50/50 1D (16 GL mu) / 2D (8 x 8), cells per
    dimension U{64..256}, groups U{16..64}, rank caps U{4..48}, FP32/FP64 split,
    64 steps each.  First all requests arrive at once (capacity = completed
    requests/s); then Poisson arrivals at 0.8 x capacity give p50/p99 latency."""
    import numpy as np
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

    # latency per request class (dimension, precision) and the slowest
    # requests, to show where the tail comes from
    def cls(p):
        return f"{p.dim}d_" + ("fp64" if p.precision == ti.PREC_FP64 else "fp32")

    lat = live["latency_ms"]
    by = {}
    for i, p in enumerate(probs):
        by.setdefault(cls(p), []).append(lat[i])
    by_class = {c: {"n": len(v), "p50_ms": float(np.percentile(v, 50)), "p99_ms": float(np.percentile(v, 99)),
                    "mean_ms": float(np.mean(v))} for c, v in sorted(by.items())}
    slow = sorted(range(len(probs)), key=lambda i: -lat[i])[:5]
    tail = [{"class": cls(probs[i]), "rows": probs[i].M, "cap": probs[i].rank_cap, "latency_ms": lat[i]} for i in slow]
    return {"requests": len(probs), "steps_per_request": 64,
            "mix": "1D (16 GL mu) / 2D (8x8) 50/50, cells/dim U{64..256}, groups U{16..64}, caps U{4..48}, "
                   "FP32 (Gram) / FP64 (QR) 50/50, seed 0",
            "budget_gb": args.served_budget_gb, "slots": args.served_slots,
            "capacity_rps": cap["throughput_rps"], "capacity_run": {k: cap[k] for k in keep},
            "arrival_rate_rps": rate, **{k: live[k] for k in keep}, "by_class": by_class, "slowest": tail}


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
    if args.probe_workload in ("clumps3d_fp64", "clumps3d_fp32"):
        # the headline (or the same in FP32): ranks brought to the cap, then
        # --probe-steps steps
        fp64 = args.probe_workload == "clumps3d_fp64"
        prob = ti.clumps3d(precision=ti.PREC_FP64 if fp64 else ti.PREC_FP32)
        s = tt.Solver(prob, round_method=tt.TT_ROUND_GRAM)
        warm = 0
        while warm < 48:
            st = s.solve(1)
            warm += 1
            if st["r1"] >= prob.rank_cap and warm >= 24:
                break
        tuning = s.tune(args.tune_cache) if args.tune else None
        st = s.solve(args.probe_steps)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "probe", "workload": args.probe_workload, "rank_warmup_steps": warm,
                          "steps": args.probe_steps, "ranks": [st["r1"], st["r2"]], "tuning": tuning}), flush=True)
        return
    if args.probe_workload == "clumps3d":
        prob = ti.clumps3d(precision=ti.PREC_BF16X)
    elif args.probe_workload == "plane2d_coupled":
        prob = ti.plane2d()
        prob = prob.copy(heat_capacity=8.0 * ti.radiation_constant(prob.c))
    elif args.probe_workload == "plane2d_rusanov_scatter":
        prob = rusanov_scatter_problem(ti)
    elif args.probe_workload == "plane2d_randomized":
        prob = ti.plane2d().copy(round_method=ti.ROUND_RAND, rand_oversample=4, rand_seed=0)
    elif args.probe_workload == "plane2d_fp64_qr":
        prob = ti.plane2d(precision=ti.PREC_FP64)
    else:
        prob = ti.plane2d()
    s = tt.Solver(prob, round_method=tt.TT_ROUND_QR) if args.probe_workload == "plane2d_fp64_qr" else tt.Solver(prob)
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
    """profiles/traffic_clumps3d_fp64.json from four counter runs under
    --pmc-dir: fetch/ and write/ (FETCH_SIZE, WRITE_SIZE of `--mode probe
    --probe-workload clumps3d_fp64`), copy_fetch/ and copy_write/ (the same
    counters of `--mode copy`).  Counter values are KiB per dispatch; each is
    scaled by copy bytes / counter of the copy kernel.  The dominant kernel's
    dispatches of the last --probe-steps steps (ranks at the cap) are averaged."""
    d = args.pmc_dir
    nbytes = args.copy_mb * (1 << 20)

    def copy_factor(sub, counter):
        rows = _pmc_rows(os.path.join(d, sub), counter)
        vals = sorted(v for _, _, v in rows)[-4:]          # the large copies
        return nbytes / (sum(vals) / len(vals) * 1024.0)

    def probe_steps(sub):
        # the steps the probe timed at the cap (its JSON line on stdout); the
        # dispatches before them include passes on which the kernel exits at once
        try:
            for line in open(os.path.join(d, sub + ".log")):
                if line.startswith("{") and '"probe"' in line:
                    return int(json.loads(line)["steps"])
        except (OSError, ValueError, KeyError):
            pass
        return args.probe_steps

    def kernel(sub, counter):
        key = HEAD_KERNEL.replace(" ", "")
        rows = [v for _, k, v in _pmc_rows(os.path.join(d, sub), counter) if key in k.replace(" ", "")]
        steady = rows[-probe_steps(sub):]
        return sum(steady) / len(steady) * 1024.0, len(steady)

    def probe_grid(sub):
        # the projection grid the probe ran at (its JSON line on stdout)
        try:
            for line in open(os.path.join(d, sub + ".log")):
                if line.startswith("{") and '"probe"' in line:
                    tun = json.loads(line).get("tuning")
                    return tun["project_blocks"] if tun else None
        except (OSError, ValueError):
            pass
        return None

    ff, fw = copy_factor("copy_fetch", "FETCH_SIZE"), copy_factor("copy_write", "WRITE_SIZE")
    fetch, nf = kernel("fetch", "FETCH_SIZE")
    write, nw = kernel("write", "WRITE_SIZE")
    grids = {probe_grid("fetch"), probe_grid("write")}
    import tt_inputs as ti
    p = ti.clumps3d(precision=ti.PREC_FP64)
    out = {
        "kernel": HEAD_KERNEL,
        "workload": "clumps3d 64^3 FP64 at the rank cap (R1 = 450, k1 = 128, r1 = 64), direction-space "
                    f"projection, last {nf} steps of a probe",
        "source_hash": kernel_source_hash(),
        "fetch_bytes": fetch * ff,
        "write_bytes": write * fw,
        "raw_fetch_bytes": fetch, "raw_write_bytes": write, "dispatches": [nf, nw],
        # the projection's grid in both counter runs (null if they differ or were not recorded)
        "project_blocks": grids.pop() if len(grids) == 1 else None,
        "calibration": {"copy_bytes": nbytes, "fetch_factor": ff, "write_factor": fw},
        # the stencil's minimum: read Y = Z W once and write B once (M x k1 FP64 each)
        "algorithmic_bytes": 2 * p.M * 128 * 8,
        "commands": [f"rocprofv3 --pmc {c} --output-format csv -d <dir>/{s} -o {s} -- python3 bench.py --mode {m}"
                     + (f" --probe-workload clumps3d_fp64 --probe-steps {args.probe_steps}" if m == "probe" else "")
                     for c, s, m in (("FETCH_SIZE", "fetch", "probe"), ("WRITE_SIZE", "write", "probe"),
                                     ("FETCH_SIZE", "copy_fetch", "copy"), ("WRITE_SIZE", "copy_write", "copy"))],
    }
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({"mode": "pmc-summary", **{k: out[k] for k in ("fetch_bytes", "write_bytes")}}), flush=True)


def plane2d_phase(args, dev):
    """The 2D configuration: B batched FP32 solves (seeds 0..B-1) on B streams;
    seed 0 alone in FP32 (with and without per-kernel HIP events), in FP64 with
    Gram rounding on FP64 MFMA and in FP64 with Householder QR (the plain TT-SVD
    path); each result of seed 0 against the dense FP64 oracle march."""
    import numpy as np
    import torch
    import paper_2602_00290_amd as tt
    import tt_inputs as ti
    from oracle import dense

    prob = ti.plane2d()
    K = prob.n_steps
    B = max(1, args.batch)
    probs = [prob] + [ti.plane2d(seed=b) for b in range(1, B)]
    solvers = [tt.Solver(p, device=dev) for p in probs]
    streams = [torch.cuda.Stream(device=dev) for _ in range(min(B, args.streams))]
    for sv in solvers:
        sv.reset()
    tt.solve_batch(solvers, K, streams)                 # warm-up batch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.c2_batches):
        for sv in solvers:
            sv.reset()
        stats = tt.solve_batch(solvers, K, streams)
    torch.cuda.synchronize()
    batched = B * args.c2_batches / (time.perf_counter() - t0)
    last = stats[0]
    batch_flops = sum(sum(st["flops"].values()) for st in stats)
    for sv in solvers[1:]:
        sv.destroy()
    single = solvers[0]

    def alone(sv, timing):
        sv.reset()
        sv.set_timing(timing)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = sv.solve(K)
        el = time.perf_counter() - t
        sv.set_timing(False)
        return st, el

    st1, single_s = alone(single, False)
    st1t, _ = alone(single, True)
    ms1, n1 = st1t["kernel_ms"], st1t["kernel_launches"]
    cores32 = single.get_cores()
    internal = {}
    for delta in (1e-3, 1e-6):
        t4 = time.perf_counter()
        ir = single.internal_ranks(delta)
        internal[f"{delta:g}"] = {"r_nux": ir["r_nux"], "r_xnu": ir["r_xnu"], "C_rel_nu": ir["C_rel_nu"],
                                  "C_rel_x": ir["C_rel_x"], "ms": (time.perf_counter() - t4) * 1e3}
    p64 = prob.copy(precision=ti.PREC_FP64)
    runs = {}
    for name, method in (("fp64_gram", tt.TT_ROUND_GRAM), ("fp64_qr", tt.TT_ROUND_QR)):
        sv = tt.Solver(p64, device=dev, round_method=method)
        sv.solve(2)
        st, el = alone(sv, False)
        stt, _ = alone(sv, True)
        runs[name] = {"solves_per_s": 1.0 / el, "ms": el * 1e3, "ranks": [st["r1"], st["r2"]],
                      "kernel_us_per_step": {c: stt["kernel_ms"][c] / K * 1e3 for c in tt.KERNEL_CLASSES
                                             if stt["kernel_launches"][c]},
                      "cores": sv.get_cores()}
        sv.destroy()
    # the dense FP64 oracle march of seed 0 (same discretisation, no rounding)
    t5 = time.perf_counter()
    ref = dense.march(prob, dense.initial_dense(prob), K, n_threads=host_cores())
    oracle_s = time.perf_counter() - t5

    def err(c):
        X = np.einsum("ka,alb,bp->klp", *c, optimize=True)
        return float(np.linalg.norm(X - ref) / np.linalg.norm(ref))

    e32 = err(cores32)
    out = {
        "workload": "plane2d: 128x128 cells, 32 groups [0.01,10], 8x8 angles, lognormal kappa0 (sigma 1, l 0.1), "
                    "rank cap 32, tol 1e-6, 512 steps per solve",
        "batched_fp32": {"solves_per_s": batched, "batch": B, "streams": len(streams), "seeds": f"0..{B - 1}",
                         "batches_timed": args.c2_batches,
                         "gflops": batch_flops * args.c2_batches / (B * args.c2_batches / batched) / 1e9,
                         "ranks": [last["r1"], last["r2"]], "max_R": [last["max_R1"], last["max_R2"]],
                         "compression": last["compression"]},
        "single_fp32": {"solves_per_s": 1.0 / single_s, "ms": single_s * 1e3, "rel_l2_vs_dense_oracle": e32,
                        "kernel_us_per_launch": {c: ms1[c] / n1[c] * 1e3 for c in tt.KERNEL_CLASSES if n1[c]}},
        "dense_oracle": {"seconds": oracle_s, "threads": host_cores(), "steps": K},
        "internal_ranks": internal,
    }
    for name, r in runs.items():
        r["rel_l2_vs_dense_oracle"] = err(r.pop("cores"))
        out[name] = r
    # equal accuracy: both meet the same relative L2 bound against the oracle
    bound = max(e32, runs["fp64_qr"]["rel_l2_vs_dense_oracle"]) * 1.01
    out["equal_accuracy_bound"] = bound
    out["speedup_batched_fp32_vs_fp64_qr"] = batched / runs["fp64_qr"]["solves_per_s"]
    out["speedup_batched_fp32_vs_fp64_gram"] = batched / runs["fp64_gram"]["solves_per_s"]
    return out, single


def c1_phase(args, dev):
    """The 1D slab (FP64, cap 8, 128 steps): many independent solves as one batch."""
    import torch
    import paper_2602_00290_amd as tt
    import tt_inputs as ti
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
    ref = one.get_cores()
    # the same batch in the persistent ragged kernel (one workgroup per request)
    for sv in c1s:
        sv.reset()
    tt.solve_small_batch(c1s, p1.n_steps)      # warm-up
    times = []
    for _ in range(3):
        for sv in c1s:
            sv.reset()
        torch.cuda.synchronize()
        t8 = time.perf_counter()
        pst = tt.solve_small_batch(c1s, p1.n_steps)
        times.append(time.perf_counter() - t8)
    diff = tt_rel_diff(c1s[0].get_cores(), ref)
    one.reset()
    torch.cuda.synchronize()
    t9 = time.perf_counter()
    tt.solve_small_batch([one], p1.n_steps)
    p_one = time.perf_counter() - t9
    for sv in c1s:
        sv.destroy()
    return {"workload": "slab1d: 64 cells, 8 groups [0.01,10], 16 GL mu, FP64, cap 8, tol 1e-8, 128 steps",
            "batch": args.c1_batch,
            "persistent_kernel": {"solves_per_s": args.c1_batch / min(times), "batch_ms": min(times) * 1e3,
                                  "single_solve_ms": p_one * 1e3, "ranks": [pst[0]["r1"], pst[0]["r2"]],
                                  "rel_l2_vs_launched_path": diff},
            "launched_kernels": {"streams": len(c1st), "solves_per_s": args.c1_batch / c1_s,
                                 "single_solve_ms": c1_one * 1e3, "ranks": [c1stats[0]["r1"], c1stats[0]["r2"]]}}


def extras_phase(args, dev, single):
    """Seed 0 of the 2D workload with the coupled medium temperature, with the
    Rusanov flux and scattering, and with randomized rounding."""
    import torch
    import paper_2602_00290_amd as tt
    import tt_inputs as ti
    prob = ti.plane2d()
    K = prob.n_steps
    out = {}
    if args.coupled:
        pc = prob.copy(heat_capacity=8.0 * ti.radiation_constant(prob.c))
        sc = tt.Solver(pc, device=dev)
        sc.set_timing(True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        stc = sc.solve(K)
        coupled_s = time.perf_counter() - t3
        Tc = sc.get_temperature()
        nc = stc["kernel_launches"]["couple"]
        out["coupled_temperature"] = {
            "solves_per_s": 1.0 / coupled_s, "ms": coupled_s * 1e3, "timing": "HIP events on",
            "heat_capacity": "8 a (a = 8 pi^5 / (15 c))", "ranks": [stc["r1"], stc["r2"]],
            "couple_us_per_launch": stc["kernel_ms"]["couple"] / max(1, nc) * 1e3, "couple_launches": nc,
            "T_mean": float(Tc.mean()), "T_max": float(Tc.max()),
            "energy_total": stc["energy"] / pc.c + stc["medium_energy"]}
        sc.destroy()
    if args.rusanov_scatter:
        pr = rusanov_scatter_problem(ti)
        sr = tt.Solver(pr, device=dev)
        sr.set_timing(True)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        str_ = sr.solve(K)
        rus_s = time.perf_counter() - t5
        nr = str_["kernel_launches"]["couple"]
        out["rusanov_scattering"] = {
            "solves_per_s": 1.0 / rus_s, "ms": rus_s * 1e3, "timing": "HIP events on",
            "flux": "Rusanov, S+ = c", "scattering": "kappa_s = kappa_a", "ranks": [str_["r1"], str_["r2"]],
            "max_R": [str_["max_R1"], str_["max_R2"]],
            "prepass_us_per_launch": str_["kernel_ms"]["couple"] / max(1, nr) * 1e3,
            "kernel_us_per_launch": {c: str_["kernel_ms"][c] / str_["kernel_launches"][c] * 1e3
                                     for c in tt.KERNEL_CLASSES if str_["kernel_launches"][c]}}
        sr.destroy()
    if args.randomized:
        prr = prob.copy(round_method=ti.ROUND_RAND, rand_oversample=4, rand_seed=0)
        srr = tt.Solver(prr, device=dev)
        srr.solve(2)
        srr.reset()
        torch.cuda.synchronize()
        t8 = time.perf_counter()
        strr = srr.solve(K)
        rnd_s = time.perf_counter() - t8
        single.reset()
        single.solve(K)
        diff = tt_rel_diff(srr.get_cores(), single.get_cores())
        single.reset()
        torch.cuda.synchronize()
        t9 = time.perf_counter()
        single.solve(K)
        gram_s = time.perf_counter() - t9
        out["randomized_rounding"] = {
            "solves_per_s": 1.0 / rnd_s, "ms": rnd_s * 1e3, "gram_single_solve_ms": gram_s * 1e3,
            "oversample": 4, "ranks": [strr["r1"], strr["r2"]],
            "sketch_ranks_last": [strr["sketch_r1"], strr["sketch_r2"]], "rel_l2_vs_gram_solve": diff}
        srr.destroy()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps of the 3D headline")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps after the ranks reach the cap")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=16, help="independent 2D solves advanced together")
    ap.add_argument("--c2-batches", type=int, default=2, help="timed batches of the 2D workload")
    ap.add_argument("--streams", type=int, default=16, help="HIP streams for the batches")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="GPU_MAX_HW_QUEUES for this process (0: keep the environment's)")
    ap.add_argument("--mode", default="bench",
                    choices=["bench", "probe", "copy", "pmc-summary", "served", "c5-slab", "c3"])
    ap.add_argument("--c3-beside", type=int, default=1,
                    help="also run the 3D workload in split BF16, FP32 and FP64 with QR rounding")
    ap.add_argument("--c5-cap", type=int, default=18, help="rank cap of --mode c5-slab")
    ap.add_argument("--c5-warmup", type=int, default=40, help="at most this many untimed steps in --mode c5-slab")
    ap.add_argument("--probe-steps", type=int, default=64)
    ap.add_argument("--probe-workload", default="plane2d",
                    choices=["plane2d", "clumps3d", "clumps3d_fp64", "plane2d_coupled", "plane2d_rusanov_scatter",
                             "plane2d_randomized", "plane2d_fp64_qr", "clumps3d_fp32"],
                    help="probe workload: plane2d (FP32), clumps3d (64^3 cells, 64 groups, split BF16), "
                         "clumps3d_fp64 (the headline: FP64, Gram rounding, ranks at the cap first), "
                         "clumps3d_fp32 (the same in FP32), "
                         "plane2d_coupled (plane2d with the coupled medium temperature, heat capacity 8 a), "
                         "plane2d_rusanov_scatter (plane2d with the Rusanov flux and scattering kappa_s = kappa_a), "
                         "plane2d_randomized (plane2d with randomized rounding, sketch ranks = ranks + 4), "
                         "or plane2d_fp64_qr (plane2d in FP64 with Householder TSQR rounding)")
    ap.add_argument("--tune", type=int, default=1,
                    help="tune the launch shapes of the 3D solves once their ranks reach the cap (untimed)")
    ap.add_argument("--tune-cache", default=None, help="tuning cache file (default: none, always time)")
    ap.add_argument("--copy-mb", type=int, default=512)
    ap.add_argument("--pmc-dir", default=os.path.join(ROOT, "gpurun_out", "traffic"))
    ap.add_argument("--coupled", type=int, default=1,
                    help="also time seed 0 with the coupled medium temperature (heat capacity 8 a)")
    ap.add_argument("--rusanov-scatter", type=int, default=1,
                    help="also time seed 0 with the Rusanov flux and isotropic scattering (kappa_s = kappa_a)")
    ap.add_argument("--randomized", type=int, default=1,
                    help="also time seed 0 with randomized rounding (sketch ranks = ranks + 4) beside Gram rounding")
    ap.add_argument("--c2", type=int, default=1, help="run the 2D workload phase")
    ap.add_argument("--c1-batch", type=int, default=256,
                    help="also time this many independent 1D slab solves (FP64, 128 steps) as one batch")
    ap.add_argument("--served", type=int, default=256,
                    help="requests of the served mix (0: skip the serving phase)")
    ap.add_argument("--served-budget-gb", type=float, default=64.0)
    ap.add_argument("--served-slots", type=int, default=32)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
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

    import torch
    dev = torch.device("cuda:0")

    # ---- the headline: the 3D workload in FP64 at steady state ----
    head, st64, beside, p64 = c3_phase(args)
    ms_step = head["ms_per_step"]
    value = 1e3 / (C3_STEPS_PER_SOLVE * ms_step)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "clumps3d: 64^3 cells on [0,1]^3, 64 groups [0.01,10], 8x16 angles, lognormal "
                               "kappa0 (sigma 1, l 0.1) with two clumps x100, Planck T=1 inflow on x=0, rank cap 64, "
                               "tol 1e-5, 384 steps per solve; FP64 state and contractions (FP64 MFMA), FP64 Gram "
                               "rounding; a step is one time step at the rank cap (R1 = 450, k1 = 128)",
                   "rank_warmup_steps": head["rank_warmup_steps"], "timesteps_per_solve": C3_STEPS_PER_SOLVE,
                   "round_method": "gram"},
        "timesteps_per_s": 1e3 / ms_step,
        "gflops": head["flops_per_step"] / ms_step / 1e6,
        "ranks": head["ranks"], "max_R": head["max_R"], "compression": head["compression"],
        "workspace_gb": head["workspace_gb"],
        "kernel_ms_per_step": head["kernel_ms_per_step"],
        "tuning": head["tuning"],
        "roofline": roofline_c3(st64, p64.M, head["tuning"], p64.n_theta * p64.n_phi),
        "precisions_beside": beside,
    }
    del beside
    # ---- the 2D workload against the dense oracle, the 1D slab, extras ----
    single = None
    if args.c2:
        c2, single = plane2d_phase(args, dev)
        out["plane2d"] = c2
        out.update(extras_phase(args, dev, single))
        single.destroy()
    if args.c1_batch > 0:
        out["c1_slab1d"] = c1_phase(args, dev)
    if args.served > 0:
        sv = served_phase(args)
        out["served"] = sv
        out["p50_ms"] = sv["p50_ms"]
        out["p99_ms"] = sv["p99_ms"]
        out["latency_source"] = ("served request mix (256 requests, Poisson arrivals at 0.8 x capacity): "
                                 "per-request time from arrival to completion")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_c3()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
