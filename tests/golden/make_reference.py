"""Write oracle reference results used by the GPU tests and the benchmark.

Calls only ``oracle`` and ``synth``: every stored value is the FP64 oracle's.
The final concentration is stored on the sub-grid of every ``stride``-th node
per axis (default 4 in 2D, 8 in 3D), in FP64, together with the workload
name, step count and the L2 norm of the full field.  ``--marks`` also stores
the sub-sampled C after each listed step count (keys ``C_at_<m>``), so a
shorter run can be checked against the same reference.

Long runs can be split: ``--checkpoint DIR`` saves the FP64 populations every
``--every`` steps and resumes from the newest saved state (the step loop is
the oracle's, so a resumed run equals an uninterrupted one bit for bit).
``--flush-subnormals`` reads and writes FP64 values below 2.2e-308 as zero:
the 4096^2 run's fractional tails fill many nodes with such values, which the
x86 FPU handles slowly enough to stall it; the change per value is below
1e-300.

    python tests/golden/make_reference.py c2_1024sq
    python tests/golden/make_reference.py c4_4096sq --stride 8 --marks 10,100 \\
        --checkpoint /some/scratch/dir --every 50 --flush-subnormals
"""
import argparse
import glob
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def stride_of(dim: int) -> int:
    return 4 if dim == 2 else 8


def reference_path(name: str, steps: int, stride: int | None = None) -> str:
    cfg = synth.config(name)
    stride = stride_of(cfg["dim"]) if stride is None else stride
    return os.path.join(HERE, f"ref_{name}_{steps}steps_every{stride}.npz")


def _latest_checkpoint(ckdir: str, name: str):
    best = None
    for p in glob.glob(os.path.join(ckdir, f"{name}_f_step*.npy")):
        m = int(os.path.basename(p).split("_step")[1].split(".")[0])
        if best is None or m > best[0]:
            best = (m, p)
    return best


def make(name: str, steps: int | None = None, stride: int | None = None, marks=(), checkpoint: str | None = None,
         every: int = 50, flush_subnormals: bool = False) -> str:
    cfg = synth.config(name)
    steps = cfg["steps"] if steps is None else steps
    stride = stride_of(cfg["dim"]) if stride is None else stride
    C0 = synth.initial_C(cfg).astype(np.float32).astype(np.float64)  # the GPU starts from FP32 C0
    S = synth.source(cfg)
    if S is not None:
        S = S.astype(np.float32).astype(np.float64)
    sl = (slice(None, None, stride),) * cfg["dim"]
    marks = sorted(m for m in set(marks) if 0 < m < steps)
    snap = {}
    t = time.time()
    done, f = 0, None
    if checkpoint:
        os.makedirs(checkpoint, exist_ok=True)
        last = _latest_checkpoint(checkpoint, name)
        if last is not None:
            done, path = last
            f = np.load(path)
            for m in marks:
                p = os.path.join(checkpoint, f"{name}_C_at_{m}.npy")
                if m <= done and os.path.exists(p):
                    snap[m] = np.load(p)
            print(f"{name}: resuming at step {done} from {path}", flush=True)
    if f is None:
        f = oracle.init(cfg, C0)
    flushed_from = -1  # first step computed with subnormals flushed (-1: none)
    if flush_subnormals:
        oracle.flush_subnormals(True)
        flushed_from = done
    while done < steps:
        # advance to the next mark, checkpoint or the end, whichever comes first
        nxt = min([steps] + [m for m in marks if m > done] + ([done + every - done % every] if checkpoint else []))
        f = oracle.step(cfg, f, nxt - done, S)
        done = nxt
        if done in marks:
            snap[done] = oracle.moment(cfg, f)[sl].copy()
            if checkpoint:
                np.save(os.path.join(checkpoint, f"{name}_C_at_{done}.npy"), snap[done])
        if checkpoint and done % every == 0 and done < steps:
            tmp = os.path.join(checkpoint, f"{name}_f_step{done}.tmp.npy")
            np.save(tmp, f)
            os.replace(tmp, os.path.join(checkpoint, f"{name}_f_step{done}.npy"))
            old = os.path.join(checkpoint, f"{name}_f_step{done - every}.npy")
            if os.path.exists(old):
                os.remove(old)
        print(f"{name}: step {done}/{steps}, {time.time() - t:.0f} s", flush=True)
    C = oracle.moment(cfg, f)
    dt = time.time() - t
    path = reference_path(name, steps, stride)
    extra = {f"C_at_{m}": snap[m] for m in marks if m in snap}
    np.savez(path, C=C[sl], name=name, steps=steps, stride=stride, full_l2=np.linalg.norm(C.ravel()),
             seconds=dt, threads=oracle.threads(), marks=np.array(sorted(extra and [int(k[5:]) for k in extra]),
                                                                  dtype=np.int64),
             subnormals_flushed_from_step=flushed_from, **extra)
    print(f"{name}: {steps} steps in {dt:.1f} s on {oracle.threads()} threads -> {path}")
    return path


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("steps", nargs="?", type=int, default=None)
    ap.add_argument("--stride", type=int, default=None)
    ap.add_argument("--marks", default="", help="comma-separated step counts whose C is also stored")
    ap.add_argument("--checkpoint", default=None, help="directory for resumable FP64 population checkpoints")
    ap.add_argument("--every", type=int, default=50)
    ap.add_argument("--flush-subnormals", action="store_true",
                    help="treat FP64 values below 2.2e-308 as zero (speed of very long runs)")
    a = ap.parse_args()
    make(a.name, a.steps, a.stride, [int(m) for m in a.marks.split(",") if m], a.checkpoint, a.every,
         a.flush_subnormals)
