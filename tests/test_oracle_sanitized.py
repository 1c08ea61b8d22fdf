"""The oracle's C code built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and driven through every entry point on small 2D and 3D
problems: the step with and without space-dependent fields, the fractional term
(full and at sampled nodes), the one-step sampled update, the adjoint and the
random walk.  Any out-of-bounds access, use after free or undefined behaviour
aborts the child process and fails the test.  CPU only."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = textwrap.dedent("""
    import sys
    import numpy as np
    sys.path.insert(0, sys.argv[2])
    import oracle
    oracle._LIB_PATH = sys.argv[1]
    import synth

    for dim, n in ((2, [23, 17]), (3, [9, 8, 7])):
        for collision in ("MRT", "BGK"):
            cfg = synth.small(dim, n, seed=3, collision=collision, p=[1.0, 0.0, 0.5][:dim])
            C0 = synth.initial_C(cfg)
            S = np.random.default_rng(1).uniform(0, 1e-3, C0.shape)
            f = oracle.init(cfg, C0)
            f = oracle.step(cfg, f, 4, S)
            oracle.phi(cfg, C0)
            nodes = np.array([0, 5, C0.size // 2, C0.size - 1], np.int64)
            oracle.phi_at(cfg, C0, nodes)
            oracle.step_sampled(cfg, f, nodes, S)
            gC = np.random.default_rng(2).standard_normal(C0.shape)
            oracle.adjoint(cfg, C0, 3, gC, S)
        cfg = synth.small(dim, n, seed=4)
        C0 = synth.initial_C(cfg)
        D = np.zeros((dim, dim) + C0.shape)
        for a in range(dim):
            D[a, a] = 0.1 + 0.05 * np.random.default_rng(a).uniform(size=C0.shape)
        Cw = np.full(C0.shape, 0.3)
        f = oracle.init(cfg, C0, Cw)
        oracle.step(cfg, f, 3, None, D, Cw)
    P = oracle.rw_params(2, [0.0, 0.0], [2.0, 2.0], [1.5, 1.9], [0.5, 0.3], (0.5, 0.5), dt=1e-3, seed=3)
    x, al = oracle.rw_init_gaussian(P, [1.0, 1.0], 0.1, 500)
    x, al = oracle.rw_walk(P, x, al, 20)
    oracle.rw_histogram(P, x, al, [21, 21], 0.1)
    print("sanitized oracle ok", flush=True)
""")


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime")
    lib = str(tmp_path / "libfade_oracle_san.so")
    srcs = [os.path.join(ROOT, "oracle", s) for s in ("fade_oracle.c", "random_walk.c")]
    subprocess.run([gcc, "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-o", lib, *srcs, "-lm"], check=True)
    drv = tmp_path / "drive.py"
    drv.write_text(DRIVER)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, str(drv), lib, ROOT], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
