#!/usr/bin/env python3
"""Benchmark of the graph-Kuramoto hot path on one MI355X.

A step is one classical RK4 step (four right-hand-side evaluations with localised order
parameters, list and inter-community gathers, the fused stage updates and the compensated phase
update) over the whole graph, with every input resident in HBM before the timed region.

Default workload: heterogeneous stochastic block model, N = 2^20, power-law community sizes in
[256, 16384], intra densities U[0.3, 1], cross-community Erdos-Renyi edges of mean degree 8,
omega ~ Cauchy(0, 0.5), K = 3, dt = 0.005, FP32 (seeded synthetic input).

Prints one JSON line with the throughput, the roofline of the dominant kernel (the row kernel,
timed live with HIP events on its own stream) and the CPU oracle timed on a bounded sample. The
default run also times the other workloads (the 64 x 1024 SBM with its 2000-step adjoint in FP32
and FP64, the N = 512 all-to-all graph in FP64, the 256-instance batch) in child runs and reports
them under "other_configs" (--no-other-configs skips them).

Other workloads (--workload): sbm (64 x 1024 SBM), a2a (N = 512 all-to-all, FP64), pairs (the
paired SBM with dense off-diagonal blocks), paper (M = 4096 in four communities to T = 200, with
the paper's timing as context), homo (a homogeneous N = 2^20 diagnostic), batch (256 independent
instances) and ens (B replicas of one graph on the matrix cores, --dtype f32 or f64).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RK4 steps/s and RHS evals/s at N=2^20 (fraction of HBM roofline); adjoint/fwd ratio"
HBM_PEAK_GBS = 8000.0
# the device code of the row kernel: its source file and the device helpers it includes
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2102_07167_amd", "csrc", f) for f in ("kur_kernels.hip", "kur_device.hpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rows_kernel_traffic.json")
TUNE_CACHE = os.path.join(ROOT, "paper_2102_07167_amd", "tuned_layouts.tsv")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def layout_of(info: dict) -> dict:
    """The layout figures a stored traffic measurement must share with this run."""
    return {k: int(info[k]) for k in ("chunk", "tiles", "list_padded", "dense_blocks")}


def algorithmic_bytes_per_eval(info: dict, elem: int, mask_bytes: int = 0) -> int:
    """Bytes one right-hand-side evaluation must move: the stored index lists (2 B per entry,
    unpadded), the bitmask segments (1 bit per cell, in 128-column units), the inter-block
    columns (4 B), the list and inter row offsets (2 x 8 (N+1)), four per-node vectors (theta, the
    previous stage, omega read; the stage result written) and the block sums. With bitmask
    segments, their per-row sums (one pair per row) are written and read once more."""
    n, nb = info["n"], info["blocks"]
    masks = mask_bytes + (2 * 2 * elem * n if mask_bytes else 0)
    return (2 * info["list_entries"] + masks + 4 * info["inter_entries"] + 16 * (n + 1) + 4 * n * elem
            + 2 * nb * elem * 4)


def make_workload(name: str):
    import gen
    if name == "het":
        return gen.sbm_heterogeneous()
    if name == "sbm":
        return gen.sbm_equal()
    if name == "a2a":
        return gen.all_to_all()
    if name == "pairs":
        return gen.sbm_paired_workload()
    if name == "paper":
        return gen.paper_four_communities()
    if name == "homo":
        # 1024 communities of 1024, inter-community degree about 13
        return gen.sbm_equal(n_comm=1024, comm_size=1024, rho_in=0.97, p_out=13.0 / (1 << 20), seed=1009)
    raise SystemExit("unknown workload %s" % name)


def workload_desc(name: str, w, info) -> dict:
    d = {"n": info["n"], "blocks": info["blocks"], "dense_blocks": info["dense_blocks"],
         "list_entries": info["list_entries"], "inter_entries": info["inter_entries"],
         "K": w.K, "dt": w.dt, "tau": 0.5}
    if name == "het":
        d["workload"] = ("heterogeneous SBM N=2^20: power-law(2) community sizes clipped to [256,16384], "
                         "intra density U[0.3,1], inter ER mean degree 8, omega~Cauchy(0,0.5), K=3, dt=0.005, "
                         "seed 1003")
    elif name == "sbm":
        d["workload"] = "SBM N=65536 = 64x1024, rho_in 0.97, p_out 2e-4, omega~N(0,1), K=4, dt=0.01, seed 1002"
    elif name == "pairs":
        d["workload"] = ("paired SBM N=65536 = 64x1024, rho_in 0.97, communities 2i and 2i+1 joined by a dense "
                         "off-diagonal block of density 0.9, p_out 2e-4, omega~N(0,1), K=4, dt=0.01, seed 1008")
        d["dense_offdiagonal_blocks"] = info.get("pairs")
    elif name == "homo":
        d["workload"] = ("homogeneous SBM N=2^20 = 1024x1024, rho_in 0.97, p_out 13/2^20 (inter degree ~13), "
                         "omega~N(0,1), K=4, dt=0.01, seed 1009: a diagnostic whose ~0.2 GB per evaluation stays "
                         "in the 256 MB Infinity Cache, so its HBM fraction is nominal")
    elif name == "paper":
        d["workload"] = ("paper-shaped: M=4096 in 4 equal communities (rho_in 0.95, p_out 0.05: densities not stated "
                         "in the paper, a stated guess), omega_m the paper's special choice with omega0=2, splay "
                         "theta0, K=3, T=200 with fixed dt=0.01 (20000 classical RK4 steps), seed 1006")
    else:
        d["workload"] = "all-to-all N=512, omega~N(0,1), K=2, dt=0.01, seed 1001"
    return d


def cpu_baseline(w, seconds: float) -> dict:
    """The FP64 oracle (direct summation) on a seeded 1/64 row sample, extrapolated."""
    import numpy as np
    import oracle
    g = w.graph
    rows = np.sort(np.random.default_rng(64).choice(g.n, max(1, g.n // 64), replace=False))
    oracle.rhs_rows(g, w.omega, w.K, w.theta0, rows[:8])  # load and warm
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.rhs_rows(g, w.omega, w.K, w.theta0, rows)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds or reps >= 1000:
            break
    t_eval = el / reps * (g.n / len(rows))  # extrapolated full evaluation
    cores = oracle.threads()  # the OpenMP threads of the oracle's row loop
    return {"value": 1.0 / (4.0 * t_eval), "unit": "RK4 steps/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 direct-summation RHS on a seeded 1/64 row sample (%d rows) x%d repeats in %.1f s, "
                      "extrapolated x%d per RHS and x4 RHS per RK4 step" % (len(rows), reps, el, g.n // len(rows)),
            "rhs_evals_per_s": 1.0 / t_eval}


def bench_batch(args):
    """256 independent instances (N log-uniform in [1024, 65536], all-to-all or SBM, K swept
    over [0, 6]) integrated as one batch, r sampled per instance every 10 steps."""
    import numpy as np
    import torch

    import gen
    from paper_2102_07167_amd import Kuramoto
    t0 = time.perf_counter()
    k = Kuramoto("f32", device=0)
    # chunk width of the per-instance layouts: the batch is bound by per-tile latency, not by
    # bytes, and narrower staging areas let more tiles share a CU (measured: 4096 -> 5.56e9,
    # 2048 -> 5.95e9, 1024 -> 5.83e9 node-steps/s); --option chunk=... overrides
    k.set_option("chunk", 2048)
    for kv in args.option:
        key, v = kv.split("=")
        k.set_option(key, float(v))
    insts = []

    def feed():
        for w in gen.batch_instances_iter():
            insts.append((w.graph.n, w.meta["kind"], w.K))
            yield w.graph, w.K, w.omega, w.theta0
    k.set_batch(feed())
    info = k.graph_info()
    ntot = info["n"]
    log("batch of %d instances, %d nodes, set in %.1f s: %s" % (len(insts), ntot, time.perf_counter() - t0, info))
    tuning = None
    if args.tune_effort >= 0:
        t0 = time.perf_counter()
        tuning = k.tune_tiles(args.tune_effort)
        info = k.graph_info()
        log("tiles tuned in %.1f s: %s" % (time.perf_counter() - t0, tuning))
    dt = 0.01
    k.batch_step(dt, args.warmup, 10)
    k.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r, psi = k.batch_step(dt, args.steps, 10)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert np.isfinite(r).all()
    # row-kernel launch time from HIP events on a separate short run (event timing replaces the
    # graph replay by plain launches of the same kernels)
    k.set_option("timing", 1)
    k.kernel_time()
    k.batch_step(dt, 50, 10)
    k.sync()
    launches, kms = k.kernel_time()
    k.set_option("timing", 0)
    avg_ms = kms / max(1, launches)
    masks = k.graph_masks()
    b_eval = algorithmic_bytes_per_eval(info, 4, masks["mask_bytes"])
    achieved = b_eval / (avg_ms * 1e-3) / 1e9
    out = {"metric": "aggregate node-steps/s of a batched ensemble (RK4)", "value": ntot * args.steps / el,
           "unit": "node-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "256 instances, N log-uniform in [1024,65536], all-to-all or SBM(1024-node "
                                  "communities, rho 0.97, p_out 2e-4) by a coin, K=linspace(0,6,256), dt=0.01, "
                                  "r every 10 steps, seed 1004", "nodes": ntot, "list_entries": info["list_entries"],
                      "inter_entries": info["inter_entries"], "tiles": info["tiles"]},
           "layout": {"tuning": tuning, "chunk": info["chunk"], "masks": masks},
           "r_final_K0": float(r[-1, 0]), "r_final_K6": float(r[-1, -1]),
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "k_mask + k_rows" if masks["mask_segments"] else "k_rows", "avg_launch_ms": avg_ms,
                        "algorithmic_bytes_per_launch": b_eval}}
    print(json.dumps(out), flush=True)
    k.close()


def bench_ensemble(args):
    """B replicas of one graph (the equal-community SBM, 64 x 1024, rho 0.97, p_out 2e-4) with
    K swept over [0, 6], omega ~ N(0, 1) and theta0 ~ U[0, 2 pi) per replica; r of every replica
    every 10 steps. Dense blocks form A_b [sin, cos] on the matrix cores when the tuner says so."""
    import numpy as np
    import torch

    import gen
    from paper_2102_07167_amd import Kuramoto
    B = args.replicas
    w = gen.sbm_paired_workload() if args.ens_graph == "paired" else gen.sbm_equal(seed=1002)
    g = w.graph
    rng = np.random.default_rng(1006)
    K = np.linspace(0.0, 6.0, B)
    om = rng.standard_normal((B, g.n))
    th = rng.uniform(0.0, 2 * np.pi, (B, g.n))
    dtype = args.dtype or "f32"
    k = Kuramoto(dtype, device=0)
    for kv in args.option:
        key, v = kv.split("=")
        k.set_option(key, float(v))
    t0 = time.perf_counter()
    tuning = None
    if args.tune_effort >= 0:
        tuning = k.ens_autotune(g, B, args.tune_effort)
        log("ensemble threshold tuned in %.1f s: %s" % (time.perf_counter() - t0, tuning))
    else:
        k.ens_set_graph(g)
    k.ens_set_params(K, om)
    k.ens_set_phases(th)
    info = k.ens_info()
    log("ensemble layout: %s" % info)
    dt, r_every = 0.01, 10
    k.ens_step(dt, args.warmup, r_every)
    k.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r, _ = k.ens_step(dt, args.steps, r_every)
    k.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert np.isfinite(r).all()
    # per-kernel split from HIP events on a separate short run
    k.set_option("timing", 1)
    k.ens_kernel_time()
    k.ens_step(dt, 50, 0)
    kt = k.ens_kernel_time()
    k.set_option("timing", 0)
    out = {"metric": "aggregate node-steps/s of a shared-graph ensemble (RK4)", "value": g.n * B * args.steps / el,
           "unit": "node-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": dtype, "data": "synthetic",
           "config": {"workload": "%d replicas of the %s N=65536 (64 x 1024, rho 0.97, p_out 2e-4%s), "
                                  "K=linspace(0,6,%d), omega~N(0,1), theta0~U[0,2pi) per replica, dt=0.01, r every 10 "
                                  "steps, seed 1006" % (
                                      B, "paired SBM" if args.ens_graph == "paired" else "equal-community SBM",
                                      ", communities 2i and 2i+1 joined at density 0.9" if args.ens_graph == "paired"
                                      else "", B), "layout": info, "tuning": tuning}}
    if kt["gemm_launches"] > 0:
        # issued matrix-core work per launch: every output tile of a row block (256 x 128 in
        # FP32, 128 x 64 in FP64) runs over its ranges' widths, each padded to 32, with 2 flops
        # per multiply-add; FP32 products issue three bf16 terms, FP64 products one FP64 term
        J = 2 * info["Bp"]
        terms = 3 if dtype == "f32" else 1
        peak = 2500.0 if dtype == "f32" else 78.6
        issued = 2.0 * terms * info["gemm_cells_issued"] * J
        useful = 2.0 * info["gemm_pairs"] * 2 * B
        gms = kt["gemm_ms"] / kt["gemm_launches"]
        out["roofline"] = {"bound": "mfma", "achieved": issued / (gms * 1e-3) / 1e12, "peak": peak, "unit": "TFLOP/s",
                           "frac": issued / (gms * 1e-3) / 1e12 / peak, "traffic": None,
                           "kernel": "k_ens_gemm" if dtype == "f32" else "k_ens_gemm_f64",
                           "avg_launch_ms": gms,
                           ("issued_bf16_flops_per_launch" if dtype == "f32" else "issued_fp64_flops_per_launch"): issued,
                           "useful_%s_flops_per_launch" % ("fp32" if dtype == "f32" else "fp64"): useful,
                           "rows_kernel_avg_ms": kt["rows_ms"] / max(1, kt["rows_launches"])}
    print(json.dumps(out), flush=True)
    k.close()


# The other workloads of the hot path, each timed by a child run of this script before the main
# workload touches the GPU (label, arguments). The 64 x 1024 SBM runs 2000 steps with its adjoint
# over the same 2000 steps (checkpoints every 32) in FP32 and FP64; the all-to-all N = 512 graph
# runs in FP64 with its one-workgroup adjoint; the batch is the 256-instance ensemble.
OTHER_CONFIGS = [
    ("a2a_n512_f64", ["--workload", "a2a", "--steps", "2000", "--warmup", "20", "--adjoint-steps", "2000"]),
    ("sbm_64x1024_f32", ["--workload", "sbm", "--steps", "2000", "--warmup", "20", "--adjoint-steps", "2000"]),
    ("sbm_64x1024_f64", ["--workload", "sbm", "--dtype", "f64", "--steps", "2000", "--warmup", "20",
                         "--adjoint-steps", "2000"]),
    ("batch_256_f32", ["--workload", "batch", "--steps", "200", "--warmup", "20"]),
]


def other_configs(timeout_s: float = 300.0) -> dict:
    """Run every entry of OTHER_CONFIGS as a child process (its progress goes to stderr) and keep
    the figures of its JSON line: throughput, row-kernel launch time and roofline fraction, and
    the adjoint/forward ratios where the run has them."""
    import subprocess
    res = {}
    for label, extra in OTHER_CONFIGS:
        log("other workload %s" % label)
        cmd = [sys.executable, os.path.abspath(__file__), "--no-cpu-baseline", "--no-other-configs"] + extra
        t0 = time.perf_counter()
        try:
            p = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=timeout_s)
        except subprocess.TimeoutExpired:
            res[label] = {"error": "timed out after %.0f s" % timeout_s}
            continue
        lines = [x for x in p.stdout.splitlines() if x.startswith("{")]
        if p.returncode != 0 or not lines:
            res[label] = {"error": "exit status %d" % p.returncode}
            continue
        d = json.loads(lines[-1])
        e = {"metric": d["metric"], "value": d["value"], "unit": d["unit"], "ms_per_step": d["ms_per_step"],
             "steps": d["steps"], "dtype": d["dtype"], "workload": d["config"].get("workload"),
             "row_kernel_avg_launch_ms": d["roofline"]["avg_launch_ms"], "roofline_frac": d["roofline"]["frac"],
             "wall_s": time.perf_counter() - t0}
        a = d.get("adjoint")
        if a:
            e["adjoint"] = {x: a[x] for x in ("steps", "ckpt_every", "ratio", "ratio_with_forward",
                                               "ratio_from_stages", "one_workgroup")}
        res[label] = e
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="het", choices=["het", "sbm", "a2a", "pairs", "paper", "homo", "batch", "ens"])
    ap.add_argument("--replicas", type=int, default=128, help="replicas of the ensemble workload (1..256)")
    ap.add_argument("--ens-graph", choices=["sbm", "paired"], default="sbm",
                    help="graph of the ensemble workload: the equal-community SBM or the paired SBM")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the child runs of the other workloads (default workload only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one 256 MiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--option", action="append", default=[], help="library option key=value")
    ap.add_argument("--dtype", choices=["f32", "f64"], default=None,
                    help="arithmetic type (default: f64 for a2a and paper, else f32)")
    ap.add_argument("--tune-effort", type=int, default=1, choices=[-1, 0, 1, 2],
                    help="layout autotuning effort (-1: defaults and --option values only)")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="tuning cache file (a matching entry skips the timing)")
    ap.add_argument("--adjoint-steps", type=int, default=64,
                    help="steps of the timed adjoint leg (0 skips it); checkpoints every 32 steps")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    others = None
    if args.workload == "het" and not args.no_other_configs:
        others = other_configs()

    import torch

    from paper_2102_07167_amd import Kuramoto

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if args.copy_calibration:
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "ens":
        return bench_ensemble(args)
    t0 = time.perf_counter()
    w = make_workload(args.workload)
    log("workload %s generated in %.1f s (nnz %d)" % (w.name, time.perf_counter() - t0, w.graph.nnz))
    if args.workload == "paper" and "--steps" not in sys.argv:
        args.steps = w.steps  # the whole T = 200 integration
    dtype = args.dtype or ("f64" if args.workload in ("a2a", "paper") else "f32")
    elem = 8 if dtype == "f64" else 4
    k = Kuramoto(dtype, device=0)
    for kv in args.option:
        key, v = kv.split("=")
        k.set_option(key, float(v))
    t0 = time.perf_counter()
    tuning = None
    if args.tune_effort >= 0 and not getattr(w.graph, "complete", False):
        tuning = k.autotune(w.graph, effort=args.tune_effort, cache=args.tune_cache)
        log("layout %s in %.1f s: %s" % ("from the tuning cache" if tuning["cache"] == 1 else "tuned",
                                         time.perf_counter() - t0, tuning))
    else:
        k.set_graph(w.graph)
    k.set_params(w.omega, w.K)
    k.set_phases(w.theta0)
    info = k.graph_info()
    info["pairs"] = k.graph_pairs()
    log("graph set in %.1f s: %s" % (time.perf_counter() - t0, info))

    k.step_rk4(w.dt, args.warmup)
    k.sync()
    torch.cuda.synchronize()
    log("warmup %d steps done" % args.warmup)

    # At N = 2^20 a launch is long, so the row kernel is timed with HIP events inside the timed
    # region. The smaller workloads are timed as they run (graph replay, or the one-workgroup
    # run of small complete graphs), which event timing would replace by plain launches: their
    # launch time comes from a separate run of the same steps.
    in_region = args.workload == "het"
    if in_region:
        k.set_option("timing", 1)
    torch.cuda.synchronize()
    k.sync()
    t0 = time.perf_counter()
    k.step_rk4(w.dt, args.steps)
    k.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if not in_region:
        k.set_phases(w.theta0)
        k.set_option("timing", 1)
        k.kernel_time()
        k.step_rk4(w.dt, min(args.steps, 500))
        k.sync()
    launches, kms = k.kernel_time()
    k.set_option("timing", 0)
    log("timed %d steps in %.3f s; row kernel %d launches, %.3f ms total" % (args.steps, el, launches, kms))
    r, psi = k.order_parameter()
    theta = k.get_phases(wrapped=True)
    assert all(math.isfinite(x) for x in (r, psi)) and bool((abs(theta) <= math.pi + 1e-6).all())

    steps_per_s = args.steps / el
    avg_ms = kms / max(1, launches)
    masks = k.graph_masks()
    b_eval = algorithmic_bytes_per_eval(info, elem, masks["mask_bytes"])
    achieved = b_eval / (avg_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        # counters taken on the same kernel source, workload and layout only
        try:
            tr = json.load(open(TRAFFIC_FILE))
            e = tr.get("workloads", {}).get(args.workload, {})
            if tr.get("kernel_sha") == kernel_hash() and e.get("layout") == layout_of(info):
                traffic = e.get("bytes_per_launch")
        except Exception:
            traffic = None
    out = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "RK4 steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": workload_desc(args.workload, w, info),
        "rhs_evals_per_s": 4 * steps_per_s,
        "layout": {"tuning": tuning, "chunk": info["chunk"], "tiles": info["tiles"], "masks": masks,
                   "dense_blocks": info["dense_blocks"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_mask + k_rows" if masks["mask_segments"] else "k_rows", "avg_launch_ms": avg_ms,
                     "algorithmic_bytes_per_launch": b_eval,
                     "launch_timing": "HIP events around every launch in the timed region" if in_region else
                                      "HIP events on a separate run of plain launches of the same steps"},
    }
    if args.workload == "homo":
        out["roofline"]["note"] = ("cache-resident working set (lists, offsets, per-node vectors fit the 256 MB "
                                   "Infinity Cache): the fraction of the HBM peak is nominal and can exceed 1")
    stream_gbs = k.read_bandwidth(4 << 30, 5)
    out["roofline"]["stream_read_gbs"] = stream_gbs
    out["roofline"]["frac_of_stream_read"] = achieved / stream_gbs
    log("plain streaming read on this GPU: %.0f GB/s" % stream_gbs)
    if args.adjoint_steps > 0:
        import numpy as np
        na, ck = args.adjoint_steps, 32
        seed = np.random.default_rng(7).standard_normal(w.graph.n) / w.graph.n
        k.adjoint_rk4(w.dt, min(na, 4), seed, theta0=w.theta0, ckpt_every=ck)  # warm-up

        def timed(fn):
            k.sync()
            t0 = time.perf_counter()
            res = fn()
            k.sync()
            return time.perf_counter() - t0, res
        # the plain forward twice (the first may capture its step graph); the faster is the
        # denominator of every ratio
        t_fwd = math.inf
        for _ in range(2):
            k.set_phases(w.theta0)
            t_fwd = min(t_fwd, timed(lambda: k.step_rk4(w.dt, na))[0])
        k.set_phases(w.theta0)
        k.set_option("checkpoint_every", ck)
        t_fwd_ck, _ = timed(lambda: k.step_rk4(w.dt, na))
        k.set_option("checkpoint_every", 0)
        t_bwd, (gt, gw, gk) = timed(lambda: k.adjoint_recorded(seed))
        t_full, (gt2, gw2, gk2) = timed(lambda: k.adjoint_rk4(w.dt, na, seed, theta0=w.theta0, ckpt_every=ck))
        assert np.isfinite(gt).all() and np.isfinite(gw).all() and math.isfinite(gk)
        assert np.array_equal(gt, gt2) and np.array_equal(gw, gw2) and gk == gk2
        # the same run recording every stage state (16 N reals per step): no recompute
        k.set_phases(w.theta0)
        k.set_option("checkpoint_every", ck)
        k.set_option("record_stages", 1)
        t_fwd_st, _ = timed(lambda: k.step_rk4(w.dt, na))
        k.set_option("checkpoint_every", 0)
        k.set_option("record_stages", 0)
        t_bwd_st, (gt3, gw3, gk3) = timed(lambda: k.adjoint_recorded(seed))
        # a small complete graph runs the adjoint (and its checkpointed forward) in one workgroup;
        # the stage record comes from the row kernel, whose sums run in another order
        one_wg = getattr(w.graph, "complete", False) and w.graph.n <= 1024
        if one_wg:
            tol = 1e-9 * max(np.abs(gt).max(), np.abs(gw).max())
            assert np.abs(gt - gt3).max() <= tol and np.abs(gw - gw3).max() <= tol
        else:
            assert np.array_equal(gt, gt3) and np.array_equal(gw, gw3) and gk == gk3
        out["adjoint"] = {"steps": na, "ckpt_every": ck, "fwd_ms": 1e3 * t_fwd, "fwd_checkpointed_ms": 1e3 * t_fwd_ck,
                          "backward_ms": 1e3 * t_bwd, "ratio": t_bwd / t_fwd,
                          "adjoint_with_forward_ms": 1e3 * t_full, "ratio_with_forward": t_full / t_fwd,
                          "fwd_recording_stages_ms": 1e3 * t_fwd_st, "backward_from_stages_ms": 1e3 * t_bwd_st,
                          "ratio_from_stages": t_bwd_st / t_fwd,
                          "stage_record_gb": 16 * elem * w.graph.n * na / 1e9,
                          "one_workgroup": bool(one_wg),
                          "note": "ratio = backward (recompute per segment + 4 VJP stages per step, using the "
                                  "forward run's checkpoints) / plain forward; ratio_with_forward also repeats the "
                                  "forward; ratio_from_stages = backward from a forward run that kept every stage "
                                  "state (option record_stages, no recompute) / plain forward; the first two give "
                                  "the same gradients bit for bit, and so does the third unless one_workgroup (a "
                                  "small complete graph, whose adjoint runs in one workgroup per launch)"}
        log("adjoint %d steps: backward %.1f ms, with forward %.1f ms, from recorded stages %.1f ms, forward %.1f ms "
            "(ratios %.2f / %.2f / %.2f)" % (na, 1e3 * t_bwd, 1e3 * t_full, 1e3 * t_bwd_st, 1e3 * t_fwd,
                                             t_bwd / t_fwd, t_full / t_fwd, t_bwd_st / t_fwd))
    if args.workload == "paper":
        # the paper's own wall times for this experiment (MATLAB, hardware and precision not
        # stated, variable-step integrator): context beside the same integration here, not a target
        out["paper_context"] = {"seconds_for_T200": el * w.steps / args.steps,
                                "paper_seconds_localised": 54.0, "paper_seconds_straightforward": 890.0,
                                "paper_hardware": "not stated (MATLAB)",
                                "note": "Sec. 3 numerical comparison, M = 4096, four communities; the paper's "
                                        "integrator and step are not stated for this run, here fixed-step classical "
                                        "RK4 with dt = 0.01"}
    if others is not None:
        out["other_configs"] = others
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, %.0f s budget)" % args.cpu_seconds)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    k.close()


if __name__ == "__main__":
    main()
