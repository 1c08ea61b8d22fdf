"""Write oracle reference results used by the GPU tests and the benchmark.

Calls only ``oracle`` and ``synth``: every stored value is the FP64 oracle's.
The final concentration is stored on the sub-grid of every 4th node per
axis in 2D (every 8th in 3D), in FP64, together with the workload name,
step count and the L2 norm of the full field.

    python tests/golden/make_reference.py c2_1024sq
"""
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


def reference_path(name: str, steps: int) -> str:
    cfg = synth.config(name)
    return os.path.join(HERE, f"ref_{name}_{steps}steps_every{stride_of(cfg['dim'])}.npz")


def make(name: str, steps: int | None = None) -> str:
    cfg = synth.config(name)
    steps = cfg["steps"] if steps is None else steps
    C0 = synth.initial_C(cfg).astype(np.float32).astype(np.float64)  # the GPU starts from FP32 C0
    S = synth.source(cfg)
    if S is not None:
        S = S.astype(np.float32).astype(np.float64)
    t = time.time()
    C = oracle.run(cfg, C0, steps, S=S)
    dt = time.time() - t
    stride = stride_of(cfg["dim"])
    sl = (slice(None, None, stride),) * cfg["dim"]
    path = reference_path(name, steps)
    np.savez(path, C=C[sl], name=name, steps=steps, stride=stride, full_l2=np.linalg.norm(C.ravel()),
             seconds=dt, threads=oracle.threads())
    print(f"{name}: {steps} steps in {dt:.1f} s on {oracle.threads()} threads -> {path}")
    return path


if __name__ == "__main__":
    name = sys.argv[1]
    steps = int(sys.argv[2]) if len(sys.argv) > 2 else None
    make(name, steps)
