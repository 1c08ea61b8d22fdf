"""bench.py's contract, the parts checkable without a GPU: it refuses more than
one GPU with a message and exit status 2, and the committed HBM-counter
summary of the FP32 fractional-term GEMM belongs to the GEMM sources built
now (otherwise the bench line would report its traffic as null)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_summary_matches_the_gemm_sources():
    b = _bench()
    traffic = b.measured_traffic()
    assert traffic is not None, f"{b.TRAFFIC_FILE} was taken from other GEMM sources"
    # FETCH + WRITE per launch of the 4096^2 headline workload: at least the
    # algorithmic bytes (C read once per axis, Phi written: 2 x 2 x 64 MiB)
    alg = 2 * 2 * 4 * 4096 * 4096
    assert 0.95 * alg <= traffic <= 8 * alg


def test_profile_commands_use_existing_options_and_workloads():
    """Every bench.py command recorded in profiles/ names options bench.py
    accepts and workloads the synthetic-input module defines, so each summary
    can be taken again from the committed files."""
    import re

    import synth

    src = open(os.path.join(ROOT, "bench.py")).read()
    prof = os.path.join(ROOT, "profiles")
    seen = 0
    for name in sorted(os.listdir(prof)):
        text = open(os.path.join(prof, name)).read()
        for m in re.finditer(r"python3? bench\.py((?: --?[\w-]+(?: [\w.]+)?)*)", text):
            args = m.group(1).split()
            seen += 1
            for i, a in enumerate(args):
                if a.startswith("--"):
                    assert f'"{a}"' in src, (name, a)
                    if a == "--profile-workload":
                        synth.config(args[i + 1])
    assert seen >= 5
