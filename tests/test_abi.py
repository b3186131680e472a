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


STRUCTS = {"sp2_options": "Sp2Options", "sp2_stats": "Sp2Stats", "sp2_tune_result": "TuneResult",
           "tb_params": "TBParams", "xlbomd_options": "XLOptions", "xlbomd_record": "XLRecord",
           "sp2_server_options": "ServerOptions"}


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (a C program built with the host compiler prints them)."""
    import shutil
    import subprocess
    import paper_1203_6836_amd as p
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "sp2qmd.h"', 'int main(void) {']
    for cname, pyname in STRUCTS.items():
        cls = getattr(p, pyname)
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, pyname in STRUCTS.items():
        cls = getattr(p, pyname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
