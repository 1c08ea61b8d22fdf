"""Write the FP64 oracle's fractional term of a workload's initial
concentration, for the benchmark's per-axis (per-alpha) error report and the
GPU tests.

Calls only ``oracle`` and ``synth``: Phi_mu = p I+(g C) + (1 - p) I-(g C) of
every axis (Sec. 2.4, eq. (XXminus_discret)) for the FP32-rounded initial C
the GPU receives, stored in FP64 on the sub-grid of every ``stride``-th node
per axis (key ``Phi``, shape (d, *sub-grid)).

    python tests/golden/make_phi_reference.py c4_4096sq --stride 16
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def phi_reference_path(name: str, stride: int) -> str:
    return os.path.join(HERE, f"phi_{name}_C0_every{stride}.npz")


def make(name: str, stride: int) -> str:
    cfg = synth.config(name)
    d = cfg["dim"]
    C0 = synth.initial_C(cfg).astype(np.float32).astype(np.float64)
    t = time.time()
    Phi = oracle.phi(cfg, C0)
    dt = time.time() - t
    sl = (slice(None),) + (slice(None, None, stride),) * d
    path = phi_reference_path(name, stride)
    np.savez(path, Phi=np.ascontiguousarray(Phi[sl]), name=name, stride=stride, alpha=np.array(cfg["alpha"]),
             seconds=dt, threads=oracle.threads())
    print(f"{name}: Phi of C0 in {dt:.1f} s on {oracle.threads()} threads -> {path}")
    return path


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--stride", type=int, default=8)
    a = ap.parse_args()
    make(a.name, a.stride)
