"""Write the oracle's run of the exact-solution check of the Caputo-type flux
variant (Sec. 3.5) at the paper's setting: 2D, alpha = (1.7, 1.2),
a = (0.3, 1.2), p = 1, D = Id, g = 1, u = 0, dx = 0.02 on [0, 1]^2 (51 nodes
per axis), dt = 2.5e-5, MRT, source (SourceTerm_PS) at t_m and wall values
C(t_{m+1}) set before every step m, in the FP32 values an FP32 run gets
(synth.CaputoPowerLawProblem.schedule32).  Stores C at t = 0.025 and 0.425
(steps 1000 and 17000) in FP64.  Calls only ``oracle`` and ``synth``.

    python tests/golden/make_caputo_reference.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

PATH = os.path.join(HERE, "ref_caputo_2d_51sq_dt2.5e-5.npz")
DT = 2.5e-5
MARKS = (1000, 17000)


def make() -> str:
    P = synth.CaputoPowerLawProblem(2, 51, DT)
    base = P.base.astype(np.float32).astype(np.float64)
    f = oracle.init(P.cfg, base, Cw=base)
    out = {}
    t = time.time()
    for m in range(MARKS[-1]):
        S, Cw = P.schedule32(m)
        f = oracle.step(P.cfg, f, 1, S=S.astype(np.float64), Cw=Cw.astype(np.float64))
        if m + 1 in MARKS:
            out[f"C{m + 1}"] = oracle.moment(P.cfg, f)
    np.savez_compressed(PATH, steps=np.array(MARKS), dt=DT, seconds=time.time() - t, **out)
    print(f"{MARKS[-1]} steps in {time.time() - t:.1f} s -> {PATH}")
    return PATH


if __name__ == "__main__":
    make()
