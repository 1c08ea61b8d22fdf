#!/usr/bin/env python3
"""Throughput of the fractional LB time step on one MI355X.

Workload: 2D, 1024 x 1024 nodes (walls included), D2Q5, MRT, FP32, 2000 steps;
alpha = (1.3, 1.7), p = (0.3, 0.8), anisotropic D (eigenvalues 0.05 and 0.2
rotated by 30 degrees), u = (0.05, 0.02); seeded sum of 8 Gaussian pulses,
homogeneous Dirichlet walls.  One "step" is one full time step: the
fractional-term GEMM along both axes and the fused collide-stream-boundary-
moment kernel.  Inputs are resident in HBM before the timed region.

Prints ONE JSON line.  Metric: MLUPS = nodes * steps / seconds / 1e6, with
the relative L2 error of the final concentration against the FP64 oracle,
for the FP32 GEMM (headline value) and the 3-term split-BF16 GEMM.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
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

METRIC = "MLUPS (incl. fractional-flux GEMM) FP32 vs split-BF16 at stated L2 error; adjoint/fwd"
WORKLOAD = "c2_1024sq"
PEAK = {"hbm_GBps": 8000.0, "fp32_mfma_TFLOPs": 157.3, "bf16_mfma_TFLOPs": 2500.0}


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gemm_flops_per_step(cfg: dict) -> float:
    """Algorithmic flops of the fractional term per step: an n x n Toeplitz-plus-
    boundary matrix times every line, 2 n flops per node per axis (n + 1 when
    the operator is one-sided, p in {0, 1}: a triangle)."""
    d = cfg["dim"]
    nodes = float(np.prod(cfg["n"][:d]))
    total = 0.0
    for mu in range(d):
        n = cfg["n"][mu]
        one_sided = cfg["p"][mu] in (0.0, 1.0)
        total += (n + 1 if one_sided else 2 * n) * nodes
    return total


def gemm_bytes_per_step(cfg: dict) -> float:
    """Algorithmic HBM bytes of the FP32 GEMM launch: C read once per axis, the
    d fractional terms written (FP32)."""
    d = cfg["dim"]
    return 2.0 * d * 4.0 * float(np.prod(cfg["n"][:d]))


def collide_bytes_per_step(cfg: dict) -> float:
    """Algorithmic HBM bytes of the fused collide-stream kernel: Q populations
    read and written, d fractional terms read, C written (FP32)."""
    d = cfg["dim"]
    Q = 2 * d + 1
    return (2 * Q + d + 1) * 4.0 * float(np.prod(cfg["n"][:d]))


def rel_l2_vs_reference(C: np.ndarray, name: str, steps: int):
    path = os.path.join(ROOT, "tests", "golden", f"ref_{name}_{steps}steps_every4.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path)
    sl = (slice(None, None, int(ref["stride"])),) * C.ndim
    got = C[sl].astype(np.float64)
    r = ref["C"]
    return float(np.linalg.norm((got - r).ravel()) / np.linalg.norm(r.ravel()))


def time_steps(torch, solver, steps: int) -> float:
    """Seconds for `steps` time steps on the current stream, by HIP events."""
    stream = torch.cuda.current_stream()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    solver.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / 1e3


def time_gemm(torch, solver, reps: int) -> float:
    """Average seconds of the fractional-term launch of one step (one kernel,
    all axes, on the solver's current C exactly as inside a step), timed by
    HIP events on the stream it is launched on."""
    out = torch.empty((solver.dim,) + solver.shape, dtype=torch.float32, device="cuda")
    for _ in range(3):
        solver.apply_phi(None, out=out)
    stream = torch.cuda.current_stream()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(reps):
        solver.apply_phi(None, out=out)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / 1e3 / reps


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_fp32__2d_1024sq_pmc.txt")
GEMM_SOURCES = [os.path.join(ROOT, "paper_1706_09161_amd", "csrc", f) for f in ("fractional_gemm.hip", "lbm_internal.h")]


def gemm_source_hash() -> str:
    """Hash of the FP32 GEMM kernel's sources: fractional_gemm.hip and the part
    of lbm_internal.h that declares the operator structures it reads (up to
    the collide-stream constants)."""
    import hashlib

    h = hashlib.sha256()
    for f in GEMM_SOURCES:
        with open(f, "rb") as fh:
            data = fh.read()
        if f.endswith("lbm_internal.h"):
            cut = data.find(b"// Constants of the fused collide-stream kernel")
            data = data if cut < 0 else data[:cut]
        h.update(data)
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the FP32 GEMM from the committed rocprofv3 PMC
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's
    reading for a plain copy of known size); None when the summary is missing
    or was taken from other GEMM sources than the ones built now."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if "=" in line and not line.startswith((" ", "#", "|")):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != gemm_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def profile_run(torch, LbmFade, synth, workload: str = WORKLOAD, reps: int = 20):
    """Launch sequence for rocprofv3 (trace or counters): a plain 256 MiB copy
    (the calibration of FETCH_SIZE / WRITE_SIZE), then, per precision, `reps`
    launches of the fractional-term GEMM on the solver's own C and `reps`
    steps of the workload (the benchmark's by default; with its source, if it
    has one)."""
    a = torch.ones(64 * 1024 * 1024, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    cfg = synth.config(workload)
    C0 = torch.from_numpy(synth.initial_C(cfg).astype(np.float32)).cuda()
    S = synth.source(cfg)
    for precision in ("fp32", "bf16x3"):
        with LbmFade.from_config(cfg, precision=precision) as s:
            s.set_C(C0)
            if S is not None:
                s.set_source(S.astype(np.float32))
            out = torch.empty((cfg["dim"],) + tuple(C0.shape), device="cuda")
            for _ in range(reps):
                s.apply_phi(None, out=out)
            s.step(reps)
            torch.cuda.synchronize()
    log("profile run done")


def profile_adjoint(torch, LbmFade, synth):
    """Launch sequence for a rocprofv3 kernel trace of the adjoint: on the
    512^2 adjoint workload, 500 forward steps and then lbm_fade_adjoint(500
    steps, checkpoint every 50), each twice (the first pass allocates the
    checkpoints and captures the step graph)."""
    cfg = synth.config("c5_512sq_eval")
    steps, K = cfg["steps"], cfg["ckpt_every"]
    C0 = torch.from_numpy(synth.initial_C(cfg).astype(np.float32)).cuda()
    gC = torch.from_numpy(np.random.default_rng(5).standard_normal(synth.shape(cfg)).astype(np.float32)).cuda()
    with LbmFade.from_config(cfg, precision="fp32") as s:
        for _ in range(2):
            s.set_C(C0)
            s.step(steps)
            s.set_C(C0)
            s.adjoint(steps, K, gC)
        torch.cuda.synchronize()
    log("adjoint profile run done")


def adjoint_ratio(torch, LbmFade, synth):
    """Wall time of lbm_fade_adjoint(500 steps, checkpoint every 50) over that of
    500 forward steps on the 512^2 adjoint workload (misfit gradient point)."""
    cfg = synth.config("c5_512sq_eval")
    steps, K = cfg["steps"], cfg["ckpt_every"]
    C0 = torch.from_numpy(synth.initial_C(cfg).astype(np.float32)).cuda()
    gC = torch.from_numpy(np.random.default_rng(5).standard_normal(synth.shape(cfg)).astype(np.float32)).cuda()
    with LbmFade.from_config(cfg, precision="fp32") as s:
        s.set_C(C0)
        s.adjoint(steps, K, gC)  # warm-up (allocates checkpoints)
        s.set_C(C0)
        s.step(steps)  # warm-up (captures the step graph)
        s.set_C(C0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        fwd = time.perf_counter() - t
        s.set_C(C0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        s.adjoint(steps, K, gC)
        adj = time.perf_counter() - t
    return {"value": round(adj / fwd, 3), "adjoint_ms": adj * 1e3, "forward_ms": fwd * 1e3,
            "workload": "2D 512x512 D2Q5 MRT, 500 steps, checkpoint every 50, FP32"}


def cpu_baseline(cfg: dict, budget_s: float = 15.0):
    """The FP64 oracle as it stands, on the host's cores, for a bounded number of
    steps of the same workload (starting from its initial state)."""
    import oracle
    import synth

    C0 = synth.initial_C(cfg).astype(np.float32).astype(np.float64)
    f = oracle.init(cfg, C0)
    t = time.perf_counter()
    f = oracle.step(cfg, f, 1)
    one = time.perf_counter() - t
    steps = int(max(1, min(200, budget_s / max(one, 1e-3))))
    t = time.perf_counter()
    oracle.step(cfg, f, steps)
    dt = time.perf_counter() - t
    nodes = float(np.prod(cfg["n"][: cfg["dim"]]))
    return {"value": nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{steps} steps of the same {cfg['n'][0]}x{cfg['n'][1]} workload (FP64, OpenMP over lines), "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed steps (default: the workload's 2000)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the full-length accuracy runs")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint / forward timing")
    ap.add_argument("--profile-run", action="store_true",
                    help="only the launch sequence profiled by rocprofv3 (copy calibration, GEMM, steps); no JSON")
    ap.add_argument("--profile-workload", default=WORKLOAD,
                    help="workload of --profile-run (a synth configuration name, e.g. c3_256cube)")
    ap.add_argument("--profile-adjoint", action="store_true",
                    help="only the adjoint launch sequence (512^2: 500 steps forward, then the adjoint), twice; no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1706_09161_amd import LbmFade

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.profile_run:
        profile_run(torch, LbmFade, synth, args.profile_workload)
        return
    if args.profile_adjoint:
        profile_adjoint(torch, LbmFade, synth)
        return
    cfg = synth.config(WORKLOAD)
    d = cfg["dim"]
    nodes = int(np.prod(cfg["n"][:d]))
    C0 = torch.from_numpy(synth.initial_C(cfg).astype(np.float32)).cuda()

    results = {}
    for precision in ("fp32", "bf16x3"):
        log(f"{precision}: create")
        try:
            s = LbmFade.from_config(cfg, precision=precision)
        except Exception as e:  # the BF16 kernel may be absent from an older build
            log(f"{precision}: unavailable ({e})")
            continue
        with s:
            s.set_C(C0)
            s.step(args.warmup)
            secs = time_steps(torch, s, args.steps)
            log(f"{precision}: {args.steps} steps in {secs * 1e3:.2f} ms")
            gemm_s = time_gemm(torch, s, reps=max(20, min(500, args.steps)))
            err = None
            if not args.no_accuracy:
                s.set_C(C0)
                s.step(cfg["steps"])
                err = rel_l2_vs_reference(s.get_C(device=False), WORKLOAD, cfg["steps"])
                log(f"{precision}: rel L2 vs FP64 oracle after {cfg['steps']} steps = {err}")
        results[precision] = {"secs": secs, "gemm_s": gemm_s, "err": err}

    r = results["fp32"]
    mlups = nodes * args.steps / r["secs"] / 1e6
    flops = gemm_flops_per_step(cfg)
    achieved = flops / r["gemm_s"] / 1e12
    collide_s = max(r["secs"] / args.steps - r["gemm_s"], 1e-12)
    line = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["secs"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D 1024x1024 D2Q5 MRT, alpha=(1.3,1.7), p=(0.3,0.8), rotated anisotropic D, "
                               "u=(0.05,0.02), 8 seeded Gaussian pulses, Dirichlet 0, FP32 GEMM",
                   "nodes": nodes, "workload_steps": cfg["steps"]},
        "rel_l2_vs_fp64_oracle": r["err"],
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["fp32_mfma_TFLOPs"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK["fp32_mfma_TFLOPs"], 4),
                     "traffic": measured_traffic(),
                     "kernel": "fractional-term GEMM, FP32 (one launch: x and y axes of a step)",
                     "flops_per_launch": flops, "avg_us_per_launch": r["gemm_s"] * 1e6,
                     "algorithmic_bytes_per_launch": gemm_bytes_per_step(cfg)},
        "collide_stream": {"bound": "hbm", "est_us_per_step": collide_s * 1e6,
                           "algorithmic_bytes_per_step": collide_bytes_per_step(cfg),
                           "achieved_GBps": collide_bytes_per_step(cfg) / collide_s / 1e9,
                           "peak_GBps": PEAK["hbm_GBps"]},
    }
    if "bf16x3" in results:
        b = results["bf16x3"]
        bach = 3 * flops / b["gemm_s"] / 1e12
        line["split_bf16"] = {"value": round(nodes * args.steps / b["secs"] / 1e6, 2), "unit": "MLUPS",
                              "ms_per_step": b["secs"] / args.steps * 1e3, "rel_l2_vs_fp64_oracle": b["err"],
                              "gemm_us_per_step": b["gemm_s"] * 1e6,
                              "gemm_mfma_TFLOPs_3terms": round(bach, 3),
                              "gemm_frac_of_bf16_peak": round(bach / PEAK["bf16_mfma_TFLOPs"], 4)}
    if not args.no_adjoint:
        try:
            log("adjoint / forward")
            line["adjoint_over_fwd"] = adjoint_ratio(torch, LbmFade, synth)
        except Exception as e:  # reported, never fatal for the throughput line
            line["adjoint_over_fwd"] = {"value": None, "error": str(e)}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
