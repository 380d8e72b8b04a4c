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
    checks = [("efm_enum_opts", efm.EnumOpts, "stream"), ("efm_level_stats", efm.LevelStats, "ms_expand"),
              ("efm_level_stats", efm.LevelStats, "rank_rows"),
              ("efm_trace_opts", efm.TraceOpts, "seed"), ("efm_trace_info", efm.TraceInfo, "status"),
              ("efm_train_opts", efm.TrainOpts, "stream"), ("efm_train_stats", efm.TrainStats, "ms"),
              ("efm_batch_config", efm.BatchConfig, "networks_per_cu")]
    body = "".join(f'printf("%zu %zu\\n", sizeof({c}), offsetof({c}, {f}));' for c, _, f in checks)
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "efm.h"\n'
                   'int main(void){' + body + 'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = []
    for _, cls, f in checks:
        want += [ctypes.sizeof(cls), getattr(cls, f).offset]
    assert got == want


def test_header_constants_match_the_binding(tmp_path):
    src = tmp_path / "k.c"
    src.write_text('#include <stdio.h>\n#include "efm.h"\nint main(void){printf("%d %d %u %d %u %u %u %u %u\\n", '
                   'EFM_FEAT_MAX, EFM_TRACE_WORDS, EFM_OPT_LEARNED, EFM_MAX_DEPTH, EFM_OPT_NO_PRUNE, '
                   'EFM_OPT_EXACT_RANK, EFM_OPT_TIME_KERNELS, EFM_OPT_NO_GF2, EFM_OPT_AUTOTUNE);return 0;}\n')
    exe = tmp_path / "k"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert got == [efm.FEAT_MAX, efm.TRACE_WORDS, efm.OPT_LEARNED, efm.MAX_DEPTH, efm.OPT_NO_PRUNE,
                   efm.OPT_EXACT_RANK, efm.OPT_TIME_KERNELS, efm.OPT_NO_GF2, efm.OPT_AUTOTUNE]
