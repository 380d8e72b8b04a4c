"""The C-ABI library loads without a GPU and exports every symbol include/efm.h
declares; the ctypes structures match the C layouts (checked by compiling a
small C program against the header)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1804_02867_amd import efm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "efm.h")


def _declared():
    text = open(HEADER).read()
    # declarations: a return type, then the function name and its parameter list
    return sorted(set(re.findall(r"^(?:efm_status|const char \*)\s*(efm_[a-z_]+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(efm.LIB_PATH):
        from paper_1804_02867_amd import build
        build.build()
    return efm.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert set(names) == set(efm.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    assert lib.efm_status_string(0) == b"ok"
    assert lib.efm_status_string(-2).startswith(b"workspace")


def test_null_arguments_are_rejected(lib):
    out = ctypes.c_void_p()
    assert lib.efm_network_create(0, 0, None, None, None, ctypes.byref(out)) == efm.EINVAL
    assert b"null" in lib.efm_last_error() or b"dimension" in lib.efm_last_error()
    assert lib.efm_enumerate(None, 0, None, None) == efm.EINVAL
    assert lib.efm_result_info(None, None, None, None, None) == efm.EINVAL


def test_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "efm.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu\\n", sizeof(efm_enum_opts), '
                   'offsetof(efm_enum_opts, stream), sizeof(efm_level_stats), '
                   'offsetof(efm_level_stats, ms_expand));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert got == [ctypes.sizeof(efm.EnumOpts), efm.EnumOpts.stream.offset,
                   ctypes.sizeof(efm.LevelStats), efm.LevelStats.ms_expand.offset]
