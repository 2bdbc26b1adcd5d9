"""Host-side checks of the benchmark's command line (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    """A run over several GPUs is not implemented: bench.py must say so and
    exit non-zero before it touches a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "--gpus 2" in r.stderr and "not implemented" in r.stderr
    assert r.stdout == ""


def test_unknown_variant_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--variants", "f32_nonsense"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "unknown variants" in r.stderr
    assert r.stdout == ""
