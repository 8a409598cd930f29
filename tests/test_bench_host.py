"""Host-side logic of bench.py (no GPU): the one-GPU guard, the traffic figure's
source-hash check and the oracle timing leg on a tiny workload."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single MI355X" in r.stderr
    assert r.stdout.strip() == ""          # no JSON line for a refused run


def test_traffic_figure_follows_the_kernel_source(tmp_path, monkeypatch):
    """The committed counter summary carries the hash of the kernel source it was
    taken on; bench.py reports its bytes only while the source still matches."""
    import hashlib
    import re
    text = open(bench.TRAFFIC_FILE).read()
    assert "x-step traffic per launch (bytes):" in text
    recorded = re.search(r"kernels.hip sha256: ([0-9a-f]{64})", text).group(1)
    current = hashlib.sha256(open(bench.KERNELS_SRC, "rb").read()).hexdigest()
    got = bench.measured_traffic()
    plane = bench.measured_traffic("plane")
    if current == recorded:
        assert isinstance(got, int) and 0.99 < got / (6 * 256 * 256 * 129 * 8) < 1.2
        if "plane traffic per launch (bytes):" in text:
            algorithmic = 2 * 256 * 256 * 129 * 8 + 2 * 256 ** 3 * 4
            assert isinstance(plane, int) and 0.99 < plane / algorithmic < 1.3
    else:                                  # summary older than the source: no figure
        assert got is None and plane is None
    other = tmp_path / "kernels.hip"
    other.write_text(open(bench.KERNELS_SRC).read() + "\n// changed\n")
    monkeypatch.setattr(bench, "KERNELS_SRC", str(other))
    assert bench.measured_traffic() is None


@pytest.mark.parametrize("workers", [1, 2])
def test_oracle_step_timing_on_a_tiny_workload(workers):
    mk, spec = bench.workload_spec("tiny8", None)
    ms = bench.oracle_step_ms(mk, spec, workers, reps=2)
    assert ms > 0.0
    base = bench.cpu_baseline(mk, spec, 0.2)
    assert base["kind"] == "oracle" and base["value"] > 0 and base["unit"] == "leapfrog steps/s"
