"""The C-ABI library loads on the CPU and exports every entry point include/pm.h
declares; the Python binding declares exactly those (no GPU calls)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pm.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:pm_status|const char\*)\s+(pm_\w+)\s*\(", src,
                                 flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1611_01545_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1611_01545_amd import build
        build.build(verbose=False)
    return _lib.load()


def test_header_declares_the_calls():
    names = header_functions()
    for required in ("pm_encode", "pm_deposit", "pm_force", "pm_kick_drift", "pm_decode",
                     "pm_step", "pm_step_vjp", "pm_pack", "pm_unpack", "pm_sync"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr)


def test_binding_matches_header():
    from paper_1611_01545_amd import _lib
    assert sorted(n for n, _ in _lib.EXPORTS) == header_functions()


def test_status_strings(lib):
    assert lib.pm_status_str(0) == b"ok"
    assert b"capacity" in lib.pm_status_str(5)


def test_struct_layouts_match_c(tmp_path):
    # compile a probe against include/pm.h with the host C compiler and compare the
    # struct sizes and field offsets with the ctypes declarations
    import shutil
    import subprocess
    from paper_1611_01545_amd._lib import PmConfig, PmSpecies
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    fields = [("pm_config", PmConfig, [f for f, _ in PmConfig._fields_]),
              ("pm_species", PmSpecies, [f for f, _ in PmSpecies._fields_])]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pm.h"', "int main(void){"]
    for cname, _, fs in fields:
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f in fs:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append('printf("%zu\\n", sizeof(pm_shdr)); return 0;}')
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    expect = []
    for _, ct, fs in fields:
        expect.append(ctypes.sizeof(ct))
        expect += [getattr(ct, f).offset for f in fs]
    expect.append(32)
    assert out == expect


def test_null_arguments_rejected_without_gpu(lib):
    # argument checks happen on the host before any device work
    assert lib.pm_create(None, None, None) == 1
    assert lib.pm_sync(None) == 1
    assert lib.pm_encode(None, None, None, None) == 1
