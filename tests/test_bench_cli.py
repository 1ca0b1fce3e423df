"""bench.py's command-line contract, on the CPU: the benchmark runs on one GPU
and refuses a request for several with a message and a non-zero status."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""   # no JSON line for an unsupported run


def test_workload_defaults():
    # the default line times 20 H.psi steps of the 512-atom cell after 3
    # warm-up steps (mixed beside float64: its --precision is not read); the
    # 512-atom solve workload times one mixed solve and no warm-up; the
    # 64-atom solves default to float64 with a basis of 3 nb
    import importlib
    sys.path.insert(0, ROOT)
    argv = sys.argv
    try:
        bench = importlib.import_module("bench")
        for extra, want in [([], ("cell512", "fp64", 20, 3)), (["--workload", "solve512"], ("solve512", "mixed", 1, 0)),
                            (["--workload", "cell64"], ("cell64", "fp64", 3, 1))]:
            sys.argv = ["bench.py"] + extra
            a = bench.parse()
            assert (a.workload, a.precision, a.steps, a.warmup) == want
        sys.argv = ["bench.py", "--workload", "cell64"]
        assert bench.parse().ndim == 3
        # the per-class profile of the 512-atom solve is opt-in
        sys.argv = ["bench.py", "--workload", "solve512"]
        assert bench.parse().class_profile is False
        sys.argv = ["bench.py", "--workload", "solve512", "--class-profile"]
        assert bench.parse().class_profile is True
        # the whole sphere unless the Gamma form is asked for
        sys.argv = ["bench.py", "--workload", "solve512"]
        assert bench.parse().gamma is False
        sys.argv = ["bench.py", "--workload", "solve512", "--gamma"]
        assert bench.parse().gamma is True
    finally:
        sys.argv = argv
        sys.path.remove(ROOT)
