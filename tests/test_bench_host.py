"""Host-side checks of bench.py (no GPU): the one-GPU guard, argument
checks, the algorithmic byte model and the committed profile summaries it
reads its measured traffic from."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("args,msg", [(["--gpus", "2"], "exactly one GPU"), (["--steps", "0"], "--steps >= 1"),
                                      (["--repeats", "0"], "--repeats >= 1")])
def test_bench_rejects_before_touching_a_gpu(args, msg):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and msg in r.stderr, (r.returncode, r.stderr)
    assert r.stdout == ""


def test_algorithmic_bytes_per_stage():
    b = _bench()
    # a stage is a third of a DOF-update's bytes; the mixed path reads more
    assert b.alg_bytes_per_stage_point(4, "mixed") == pytest.approx(445.0 / 3)
    assert b.alg_bytes_per_stage_point(4, "fp64") == pytest.approx(345.0 / 3)
    # 3.15 GB per stage on the 331,776-hex N = 4 shell
    assert b.alg_bytes_per_stage_point(4, "mixed") * 331776 * 64 == pytest.approx(3.1497e9, rel=1e-4)


@pytest.mark.parametrize("precision,kernel", [("mixed", "k_flux_mixed"), ("fp64", "k_flux64")])
def test_profile_summaries_name_the_dominant_kernel(precision, kernel):
    """The committed summaries carry the machine-readable lines the bench
    reads: the dominant kernel, the source hash and a per-launch traffic
    between the algorithmic bytes and ten times them."""
    b = _bench()
    path = os.path.join(ROOT, "profiles", "sd_%s_sun_332k_N4.md" % precision)
    vals = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            for key in ("kernel:", "source_sha256:", "traffic_bytes_per_launch:"):
                if line.startswith(key):
                    vals[key[:-1]] = line.split(":", 1)[1].strip()
    assert vals["kernel"] == kernel
    assert len(vals["source_sha256"]) == 64
    alg = b.alg_bytes_per_stage_point(4, precision) * 331776 * 64
    assert alg < float(vals["traffic_bytes_per_launch"]) < 10 * alg
    # an unknown workload has no summary
    assert b.measured_traffic("no_such_workload", precision, kernel) is None
