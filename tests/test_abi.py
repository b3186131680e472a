"""The C-ABI library loads on the CPU host and exports every symbol the header declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sp2qmd.h")
LIB = os.path.join(ROOT, "paper_1203_6836_amd", "libsp2qmd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def libh():
    if not os.path.exists(LIB):
        import paper_1203_6836_amd.build as b
        b.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("sp2_density_matrix", "sp2_mulliken", "sp2_band_energy", "tb_hamiltonian",
                 "tb_forces", "xlbomd_create", "xlbomd_run", "sp2_ctx_create"):
        assert must in names


def test_library_exports_every_declared_symbol(libh):
    missing = [n for n in declared_functions() if not hasattr(libh, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    import paper_1203_6836_amd as p
    assert set(declared_functions()) <= set(p._SIGS)


def test_host_side_argument_checks_without_gpu(libh):
    """Calls that fail argument checks before touching a device."""
    libh.sp2_strerror.restype = ctypes.c_char_p
    assert libh.sp2_strerror(-4) == b"SP2 did not converge within max_iter"
    libh.sp2_density_matrix.restype = ctypes.c_int
    # null context -> EINVAL, no device access
    assert libh.sp2_density_matrix(None, 16, None, 8, None, None, None) == -1
    libh.xlbomd_run.restype = ctypes.c_int
    assert libh.xlbomd_run(None, 1, None) == -1
