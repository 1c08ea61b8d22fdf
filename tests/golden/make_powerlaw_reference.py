"""Write the oracle's run of the exact-solution workload of Sec. 3.4 at the
paper's setting (2D, alpha = (1.5, 1.7), a = (0.4, 0.7), dx = 0.01 on [0, 1]^2,
dt = 5e-5, MRT), with the source S(t_m) and the wall values C(t_{m+1}) set
before every step m.  The oracle gets exactly the FP32 fields an FP32 run
gets (the initial and wall values, D(x) and the per-step source, rounded to
FP32 as synth.PowerLawProblem.schedule32 forms them), so a GPU comparison
measures the step's arithmetic, not input rounding.  Stores the
concentration at t = 0.05, 0.5 and 1 (steps 1000, 10000, 20000) in FP64.
Calls only ``oracle`` and ``synth``.

    python tests/golden/make_powerlaw_reference.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

PATH = os.path.join(HERE, "ref_powerlaw_2d_101sq_dt5e-5.npz")
DT = 5e-5
MARKS = (1000, 10000, 20000)


def make() -> str:
    P = synth.PowerLawProblem(2, 101, DT)
    f64 = lambda a: np.asarray(a, np.float32).astype(np.float64)  # noqa: E731
    base, D = f64(P.base), f64(P.D)
    f = oracle.init(P.cfg, base, Cw=base)
    out = {}
    t = time.time()
    for m in range(MARKS[-1]):
        S, Cw = P.schedule32(m)
        f = oracle.step(P.cfg, f, 1, S=f64(S), D=D, Cw=f64(Cw))
        if m + 1 in MARKS:
            out[f"C{m + 1}"] = oracle.moment(P.cfg, f)
    np.savez_compressed(PATH, steps=np.array(MARKS), dt=DT, seconds=time.time() - t, **out)
    print(f"{MARKS[-1]} steps in {time.time() - t:.1f} s -> {PATH}")
    return PATH


if __name__ == "__main__":
    make()
