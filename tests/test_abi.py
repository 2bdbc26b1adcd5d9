"""Host-side checks of the C-ABI library (no GPU needed): it loads, it
exports every function include/eselbm.h declares, the Python binding names
the same functions, and the ABI struct layout matches."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eselbm.h")
LIB = os.path.join(ROOT, "paper_2203_12946_amd", "libeselbm.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(eselbm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libeselbm.so is not built (run python -m paper_2203_12946_amd.build)")
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    names = declared()
    assert len(names) == 23
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (eselbm_[a-z_0-9]+)$", out, flags=re.M))
    assert set(names) <= exported


def test_binding_covers_the_abi():
    import paper_2203_12946_amd.eselbm as es
    assert set(es.EXPORTS) == set(declared())


def test_stats_struct_layout():
    import paper_2203_12946_amd.eselbm as es
    assert ctypes.sizeof(es.Stats) == 9 * 8 + 8 * 8  # 9 doubles, 8 long longs


def test_argument_errors_without_device(lib):
    """Argument checks run before any HIP call: they work without a GPU."""
    lib.eselbm_create.restype = ctypes.c_int
    lib.eselbm_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    assert lib.eselbm_create(None, 0, 4, 4, 1, 1) == 1
    assert lib.eselbm_create(ctypes.byref(h), 7, 4, 4, 1, 1) == 1
    assert b"lattice" in lib.eselbm_last_error()
    assert lib.eselbm_create(ctypes.byref(h), 0, 4, 4, 2, 1) == 1  # D2Q9 with nz != 1
    assert lib.eselbm_create(ctypes.byref(h), 1, 0, 4, 4, 1) == 1
    assert lib.eselbm_create(ctypes.byref(h), 1, 4, 4, 4, 9) == 1
    # limits of the kernels' addressing, rejected before any device call
    assert lib.eselbm_create(ctypes.byref(h), 0, (1 << 28) + 1, 1, 1, 0) == 2  # row beyond 32-bit offsets
    assert b"nx" in lib.eselbm_last_error()
    assert lib.eselbm_create(ctypes.byref(h), 1, 4, 65536, 4, 1) == 2  # grid y beyond the launch limit
    assert lib.eselbm_create(ctypes.byref(h), 1, 1 << 17, 1 << 15, 2, 1) == 2  # 2^33 cells
    assert b"2^32" in lib.eselbm_last_error()
    assert lib.eselbm_step(None, None, None, 1, ctypes.c_double(0.1), None) == 1
    assert lib.eselbm_adjoint_step(None, None, None, None, None, ctypes.c_double(0.1), None, None) == 1
    assert lib.eselbm_adjoint_step_diss(None, None, None, None, ctypes.c_double(1.0), None, ctypes.c_double(0.1),
                                        None, None) == 1
    assert b"eselbm_adjoint_step_diss" in lib.eselbm_last_error()
    assert lib.eselbm_destroy(None) == 0
