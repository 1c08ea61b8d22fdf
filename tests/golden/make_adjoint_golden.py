"""Oracle gradients of the adjoint workload's misfit loss (FP64), for the GPU
adjoint test.  Calls only ``oracle`` and ``synth``.

Workload: 2D 512 x 512, D2Q5, MRT, 500 steps.  The observed plume C_obs is
the oracle forward run with the hidden parameters (D = [[0.08, 0.03],
[0.03, 0.15]], u = (0.04, -0.01), p = (0.6, 0.4), alpha = (1.6, 1.4)); the
gradient of L = 1/2 |C_500 - C_obs|^2 is taken at D = 0.1 Id, u = 0,
p = (0.5, 0.5), S = 0 with the same alpha and initial plume.

Stored (JSON): central differences (h = 1e-6 relative) for the entries of D
(a symmetric perturbation of the off-diagonal pair), u and p; directional
derivatives of L along two seeded unit-variance directions for C0 (interior
nodes) and for S; and the oracle adjoint's values of the same quantities.

    python tests/golden/make_adjoint_golden.py [steps]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def directions(cfg, seed=55, count=2):
    """Seeded random directions for the field gradients (zero on the walls)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        v = rng.standard_normal(synth.shape(cfg))
        v[0, :] = v[-1, :] = v[:, 0] = v[:, -1] = 0.0
        out.append(v)
    return out


def main(steps=None):
    hid = synth.config("c5_512sq_hidden")
    ev = synth.config("c5_512sq_eval")
    steps = hid["steps"] if steps is None else steps
    C0 = synth.initial_C(ev).astype(np.float32).astype(np.float64)
    t = time.time()
    C_obs = oracle.run(hid, C0, steps)
    S0 = np.zeros(synth.shape(ev))

    def loss(cfg, c0=C0, S=S0):
        C = oracle.run(cfg, c0, steps, S=S)
        return 0.5 * float(np.sum((C - C_obs) ** 2))

    Cn = oracle.run(ev, C0, steps, S=S0)
    gC = Cn - C_obs
    adj = oracle.adjoint(ev, C0, steps, gC, S=S0)
    out = {"steps": steps, "loss": 0.5 * float(np.sum(gC**2)), "fd": {}, "adjoint": {}}
    D0 = np.array(ev["D"])
    for a, b in ((0, 0), (1, 1), (0, 1)):
        h = 1e-6 * max(1.0, abs(D0[a, b]))
        vals = []
        for sgn in (+1, -1):
            D = D0.copy()
            D[a, b] += sgn * h
            if a != b:
                D[b, a] += sgn * h
            vals.append(loss(dict(ev, D=D.tolist())))
        out["fd"][f"D{a}{b}"] = (vals[0] - vals[1]) / (2 * h)
        out["adjoint"][f"D{a}{b}"] = float(adj["D"][a, b] * (1 if a == b else 2))
    for key in ("u", "p"):
        for k in range(2):
            h = 1e-6 * max(1.0, abs(ev[key][k]))
            vals = []
            for sgn in (+1, -1):
                v = list(ev[key])
                v[k] += sgn * h
                vals.append(loss(dict(ev, **{key: v})))
            out["fd"][f"{key}{k}"] = (vals[0] - vals[1]) / (2 * h)
            out["adjoint"][f"{key}{k}"] = float(adj[key][k])
    for j, v in enumerate(directions(ev)):
        h = 1e-3
        out["fd"][f"C0_dir{j}"] = (loss(ev, c0=C0 + h * v) - loss(ev, c0=C0 - h * v)) / (2 * h)
        out["adjoint"][f"C0_dir{j}"] = float(np.sum(adj["dC0"] * v))
        out["fd"][f"S_dir{j}"] = (loss(ev, S=S0 + h * v) - loss(ev, S=S0 - h * v)) / (2 * h)
        out["adjoint"][f"S_dir{j}"] = float(np.sum(adj["dS"] * v))
    out["seconds"] = time.time() - t
    out["threads"] = oracle.threads()
    path = os.path.join(HERE, f"adjoint_c5_512sq_{steps}steps.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1, sort_keys=True))
    print("->", path)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else None)
