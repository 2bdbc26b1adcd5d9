"""Host check of the element offsets of the step, in-place and adjoint
kernels (tests/index_check.hip, built for the host with hipcc; no GPU).

The program runs the kernels' own addressing code (PullIndex and the block
shape of the launches) over every block, lane and population of each grid
below -- the grids of the GPU parity and adjoint tests, and of the benchmark
-- and checks that every access is in bounds and that the pull loads (which
the adjoint's pushes mirror), the step's stores and the in-place pull half's
stores are permutations of the state's elements.
"""
import pathlib
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]

# (D, nx, ny, nz, mode)
GRIDS = [
    (3, 9, 7, 6, "full"), (2, 20, 16, 1, "full"),            # adjoint parity
    (3, 5, 1, 1, "full"), (3, 1, 4, 1, "full"), (3, 1, 1, 3, "full"), (3, 1, 3, 2, "full"),
    (3, 65, 1, 1, "full"), (3, 129, 2, 2, "full"), (3, 257, 1, 5, "full"),  # degenerate, ragged
    (3, 300, 16, 12, "full"), (3, 513, 3, 2, "full"), (3, 70, 24, 20, "full"),
    (2, 1, 1, 1, "full"), (3, 1, 1, 1, "full"), (2, 257, 5, 1, "full"),
    (3, 128, 128, 128, "full"), (2, 256, 256, 1, "full"),     # gradient workloads
    (2, 1024, 1024, 1, "full"), (3, 256, 256, 256, "full"),   # benchmark grids
    (3, 1024, 1024, 1024, "edges"),                           # largest in-place grid
]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not pathlib.Path(hipcc).exists():
        pytest.skip("hipcc not available")
    exe = tmp_path_factory.mktemp("index") / "index_check"
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "--cuda-host-only",
                           "-I", str(ROOT / "include"), str(ROOT / "tests" / "index_check.hip"), "-o", str(exe)])
    return exe


@pytest.mark.parametrize("D,nx,ny,nz,mode", GRIDS)
def test_kernel_offsets(checker, D, nx, ny, nz, mode):
    r = subprocess.run([str(checker), str(D), str(nx), str(ny), str(nz), mode],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
