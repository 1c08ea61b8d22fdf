#!/usr/bin/env python3
"""Throughput of the fractional LB time step on one MI355X.

Headline workload: 2D, 4096 x 4096 nodes (walls included), D2Q5, MRT, 1000
steps; alpha = (1.2, 1.9), one-sided p = (1, 0), D = 0.1 Id, u = (0.02, 0.02);
seeded sum of 8 Gaussian pulses, homogeneous Dirichlet walls; the
fractional-term GEMM in FP32 (headline value) and in 3-term split BF16 on the
matrix cores.  One "step" is one full time step: the fractional-term GEMM
along both axes and the fused collide-stream-boundary-moment kernel.  Inputs
are resident in HBM before the timed region.  Secondary blocks: the 1024^2
(two-sided operators, rotated anisotropic D) and 256^3 (D3Q7, point source)
workloads, and adjoint / forward on the 512^2 adjoint workload.

Timing: the library replays a captured graph of 10 steps for runs of 10 or
more steps; the graph is captured by an untimed 10-step run before the
warm-up (then the state is reset), so no capture falls in a timed region.
Each figure is the median of 5 timed runs of --steps steps (HIP events on
the stream the kernels run on).  Accuracy: the relative L2 error of C after
the workload's full step count against the stored FP64 oracle result, and
of the fractional term of each axis (one alpha each) of the initial C.

Prints ONE JSON line.  MLUPS = nodes * steps / seconds / 1e6.

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
WORKLOAD = "c4_4096sq"          # headline
SECONDARY = ("c2_1024sq", "c3_256cube")
GRAPH_STEPS = 10                # steps per captured step graph in the library
REPEATS = 5
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


def reference_file(name: str, steps: int):
    """Stored FP64 oracle result of a workload (tests/golden/make_reference.py), or None."""
    import glob

    hits = sorted(glob.glob(os.path.join(ROOT, "tests", "golden", f"ref_{name}_{steps}steps_every*.npz")))
    return np.load(hits[0]) if hits else None


def rel_l2(got: np.ndarray, ref: np.ndarray) -> float:
    got = np.asarray(got, np.float64)
    return float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel()))


def phi_reference(name: str):
    """Stored FP64 oracle fractional terms of a workload's initial C
    (tests/golden/make_phi_reference.py), or None."""
    import glob

    hits = sorted(glob.glob(os.path.join(ROOT, "tests", "golden", f"phi_{name}_C0_every*.npz")))
    return np.load(hits[0]) if hits else None


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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_fp32__2d_4096sq_pmc.txt")
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


def profile_run(torch, LbmFade, synth, workload: str = WORKLOAD, reps: int = 100):
    """Launch sequence for rocprofv3 (trace or counters): a plain 256 MiB copy
    (the calibration of FETCH_SIZE / WRITE_SIZE), then, per precision, `reps`
    launches of the fractional-term GEMM on the solver's own C and `reps`
    steps of the workload (the benchmark's by default; with its source, if it
    has one).  The first GEMM launch of the process runs while the shader
    clock is still ramping up (about 2.5x its later duration at 4096^2); with
    100 launches it moves the trace's average by under 2 %."""
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
            # zero-filled, so the first GEMM launch does not pay the first touch of fresh memory
            out = torch.zeros((cfg["dim"],) + tuple(C0.shape), device="cuda")
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


def copy_ceiling(torch, nbytes: float, repeats: int = 5) -> dict:
    """Reference for the HBM-bound kernels: a plain device-to-device copy
    (torch's copy kernel) that reads and writes nbytes / 2 each, the traffic
    of one collide-stream launch; median of `repeats` timed copies after one
    untimed one."""
    n = int(nbytes / 2 / 4)
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ts = []
    stream = torch.cuda.current_stream()
    for _ in range(repeats):
        st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        st.record(stream)
        b.copy_(a)
        en.record(stream)
        torch.cuda.synchronize()
        ts.append(st.elapsed_time(en) / 1e3)
    sec = float(np.median(ts))
    del a, b
    return {"bytes_moved": 2 * 4 * n, "us": sec * 1e6, "GBps": 2 * 4 * n / sec / 1e9,
            "what": "torch device copy of the same traffic (half read, half written)"}


def adjoint_ratio(torch, LbmFade, synth, repeats: int = 3):
    """Wall time of lbm_fade_adjoint(500 steps, checkpoint every 50) over that of
    500 forward steps on the 512^2 adjoint workload (misfit gradient point);
    median of `repeats` timings of each, after an untimed run of each (it
    allocates the checkpoints and captures the step graph)."""
    cfg = synth.config("c5_512sq_eval")
    steps, K = cfg["steps"], cfg["ckpt_every"]
    C0 = torch.from_numpy(synth.initial_C(cfg).astype(np.float32)).cuda()
    gC = torch.from_numpy(np.random.default_rng(5).standard_normal(synth.shape(cfg)).astype(np.float32)).cuda()
    fwd, adj = [], []
    with LbmFade.from_config(cfg, precision="fp32") as s:
        s.set_C(C0)
        s.adjoint(steps, K, gC)
        s.set_C(C0)
        s.step(steps)
        for _ in range(repeats):
            s.set_C(C0)
            torch.cuda.synchronize()
            t = time.perf_counter()
            s.step(steps)
            torch.cuda.synchronize()
            fwd.append(time.perf_counter() - t)
            s.set_C(C0)
            torch.cuda.synchronize()
            t = time.perf_counter()
            s.adjoint(steps, K, gC)  # synchronises (scalar gradients to the host)
            adj.append(time.perf_counter() - t)
    f, a = float(np.median(fwd)), float(np.median(adj))
    return {"value": round(a / f, 3), "adjoint_ms": a * 1e3, "forward_ms": f * 1e3, "repeats": repeats,
            "workload": "2D 512x512 D2Q5 MRT, 500 steps, checkpoint every 50, FP32"}


def cpu_baseline(cfg: dict, min_s: float = 10.0):
    """The FP64 oracle as it stands, on the host's cores, on a bounded sample of
    the same workload: whole steps from its initial state, at least one and
    at least `min_s` seconds (the set-up of the initial populations is not
    timed)."""
    import oracle
    import synth

    C0 = synth.initial_C(cfg).astype(np.float32).astype(np.float64)
    f = oracle.init(cfg, C0)
    S = synth.source(cfg)
    steps, dt = 0, 0.0
    while steps == 0 or dt < min_s:
        k = 1 if steps == 0 else max(1, int(np.ceil((min_s - dt) / (dt / steps))))
        t = time.perf_counter()
        f = oracle.step(cfg, f, k, S)
        dt += time.perf_counter() - t
        steps += k
    nodes = float(np.prod(cfg["n"][: cfg["dim"]]))
    shape = "x".join(str(v) for v in cfg["n"][: cfg["dim"]])
    return {"value": nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{steps} step(s) of the same {shape} workload from its initial state (FP64, OpenMP over "
                      f"lines), {dt:.1f} s"}


def describe(cfg: dict) -> str:
    d = cfg["dim"]
    shape = "x".join(str(v) for v in cfg["n"][:d])
    lat = "D2Q5" if d == 2 else "D3Q7"
    D = np.asarray(cfg["D"], dtype=np.float64)
    Ds = (f"D={D[0, 0]:g} Id" if np.allclose(D, D[0, 0] * np.eye(d)) else
          "D=" + str(np.round(D, 6).tolist()))
    src = ", point source" if cfg.get("source") else ""
    fmt = lambda v: "(" + ",".join(f"{x:g}" for x in v) + ")"  # noqa: E731
    return (f"{d}D {shape} {lat} {cfg.get('collision', 'MRT')}, alpha={fmt(cfg['alpha'])}, p={fmt(cfg['p'])}, "
            f"{Ds}, u={fmt(cfg['u'])}, {cfg['steps']} steps{src}, Dirichlet 0")


def measure(torch, LbmFade, synth, name: str, steps: int, warmup: int, repeats: int, accuracy: bool):
    """FP32 and split-BF16 figures of one workload: median step time of
    `repeats` timed runs, median GEMM launch time, accuracy vs the oracle."""
    cfg = synth.config(name)
    d = cfg["dim"]
    nodes = int(np.prod(cfg["n"][:d]))
    C0 = torch.from_numpy(synth.initial_C(cfg).astype(np.float32)).cuda()
    S = synth.source(cfg)
    S = None if S is None else torch.from_numpy(S.astype(np.float32)).cuda()
    ref = reference_file(name, cfg["steps"]) if accuracy else None
    phi_ref = phi_reference(name) if accuracy else None
    out = {}
    for precision in ("fp32", "bf16x3"):
        log(f"{name} {precision}: create")
        with LbmFade.from_config(cfg, precision=precision) as s:
            s.set_C(C0)
            s.set_source(S)
            s.step(GRAPH_STEPS)  # captures the step graph; not timed, not a warm-up step
            s.set_C(C0)
            s.step(warmup)
            secs = sorted(time_steps(torch, s, steps) for _ in range(repeats))
            gemm = sorted(time_gemm(torch, s, reps=max(10, min(200, steps))) for _ in range(repeats))
            r = {"secs": float(np.median(secs)), "secs_all": secs, "gemm_s": float(np.median(gemm))}
            log(f"{name} {precision}: {steps} steps in {r['secs'] * 1e3:.3f} ms (median of {repeats}); "
                f"GEMM {r['gemm_s'] * 1e6:.1f} us")
            if accuracy:
                if phi_ref is not None:
                    phi = s.apply_phi(C0).cpu().numpy()
                    st = int(phi_ref["stride"])
                    sl = (slice(None),) + (slice(None, None, st),) * d
                    r["phi_err_per_axis"] = [rel_l2(phi[sl][mu], phi_ref["Phi"][mu]) for mu in range(d)]
                s.set_C(C0)
                s.step(cfg["steps"])
                C = s.get_C(device=False)
                if ref is not None:
                    st = int(ref["stride"])
                    r["err"] = rel_l2(C[(slice(None, None, st),) * d], ref["C"])
                log(f"{name} {precision}: rel L2 vs FP64 oracle after {cfg['steps']} steps = {r.get('err')}, "
                    f"Phi per axis {r.get('phi_err_per_axis')}")
        out[precision] = r
    flops = gemm_flops_per_step(cfg)
    blk = {"workload": describe(cfg), "nodes": nodes}
    for precision, key in (("fp32", "fp32"), ("bf16x3", "split_bf16")):
        r = out[precision]
        terms = 1 if precision == "fp32" else 3
        peak = PEAK["fp32_mfma_TFLOPs"] if precision == "fp32" else PEAK["bf16_mfma_TFLOPs"]
        gemm_tf = terms * flops / r["gemm_s"] / 1e12
        collide_s = max(r["secs"] / steps - r["gemm_s"], 1e-12)
        blk[key] = {"MLUPS": round(nodes * steps / r["secs"] / 1e6, 2), "us_per_step": r["secs"] / steps * 1e6,
                    "rel_l2_vs_fp64_oracle": r.get("err"), "phi_rel_l2_per_axis": r.get("phi_err_per_axis"),
                    "gemm_us": r["gemm_s"] * 1e6, "gemm_TFLOPs": round(gemm_tf, 2),
                    "gemm_frac_of_peak": round(gemm_tf / peak, 4),
                    "collide_us_step_minus_gemm": collide_s * 1e6,
                    "collide_GBps_step_minus_gemm": collide_bytes_per_step(cfg) / collide_s / 1e9}
    return cfg, out, blk


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed steps per run (median of 5 runs)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the full-length accuracy runs")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint / forward timing")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 1024^2 and 256^3 blocks")
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

    cfg, res, head = measure(torch, LbmFade, synth, WORKLOAD, args.steps, args.warmup, REPEATS,
                             not args.no_accuracy)
    d = cfg["dim"]
    nodes = int(np.prod(cfg["n"][:d]))
    r = res["fp32"]
    flops = gemm_flops_per_step(cfg)
    achieved = flops / r["gemm_s"] / 1e12
    line = {
        "metric": METRIC,
        "value": head["fp32"]["MLUPS"],
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
        "config": {"workload": head["workload"] + "; fractional-flux GEMM FP32 (value) vs 3-term split BF16",
                   "nodes": nodes, "workload_steps": cfg["steps"], "timed_runs": REPEATS,
                   "statistic": "median"},
        "rel_l2_vs_fp64_oracle": head["fp32"]["rel_l2_vs_fp64_oracle"],
        "phi_rel_l2_per_axis": head["fp32"]["phi_rel_l2_per_axis"],
        "alpha_per_axis": cfg["alpha"],
        "split_bf16": head["split_bf16"],
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["fp32_mfma_TFLOPs"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK["fp32_mfma_TFLOPs"], 4),
                     "traffic": measured_traffic(),
                     "kernel": "fractional-term GEMM, FP32 (one launch: x and y axes of a step)",
                     "flops_per_launch": flops, "avg_us_per_launch": r["gemm_s"] * 1e6,
                     "algorithmic_bytes_per_launch": gemm_bytes_per_step(cfg)},
        "fp32_detail": head["fp32"],
        "collide_stream": {"bound": "hbm", "algorithmic_bytes_per_step": collide_bytes_per_step(cfg),
                           "us_fp32_step_minus_gemm": head["fp32"]["collide_us_step_minus_gemm"],
                           "GBps": head["fp32"]["collide_GBps_step_minus_gemm"], "peak_GBps": PEAK["hbm_GBps"],
                           "copy_reference": copy_ceiling(torch, collide_bytes_per_step(cfg))},
    }
    if not args.no_secondary:
        line["secondary"] = {}
        for name in SECONDARY:
            try:
                _, _, blk = measure(torch, LbmFade, synth, name, args.steps, args.warmup, REPEATS,
                                    not args.no_accuracy)
                line["secondary"][name] = blk
            except Exception as e:  # reported, never fatal for the headline line
                line["secondary"][name] = {"error": str(e)}
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
