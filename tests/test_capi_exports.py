"""The C-ABI library loads on the CPU and exports every entry point that
include/afn.h declares (no compute calls: this container has no GPU)."""
import ctypes
import re

import pytest

from conftest import ROOT


def declared_functions():
    text = (ROOT / "include" / "afn.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:afn_status|void|const char \*)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("afn_setup", "afn_apply", "kernel_matvec", "afn_pcg_solve", "afn_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2304_05460_amd import afn
    lib = afn.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(afn.EXPORTED) <= set(declared_functions())


def test_status_strings_without_gpu():
    from paper_2304_05460_amd import afn
    lib = afn.lib()
    for code in range(8):
        assert lib.afn_status_string(code).startswith(b"AFN_")
    assert lib.afn_last_error() is not None


def test_param_struct_layout_matches_header():
    from paper_2304_05460_amd import afn
    assert ctypes.sizeof(afn.afn_params) == 48
    assert afn.afn_params.seed.offset == 24
    assert afn.afn_params.nrhs_max.offset == 40


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Every field offset and struct size the binding uses equals what a C
    compiler computes from include/afn.h."""
    import shutil
    import subprocess
    from paper_2304_05460_amd import afn
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"afn_params": afn.afn_params, "afn_setup_info": afn.afn_setup_info,
               "afn_solve_info": afn.afn_solve_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "afn.h"', "int main(void) {"]
    for sname, cls in structs.items():
        lines.append(f'printf("{sname} size %zu\\n", sizeof({sname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{sname} {fname} %zu\\n", offsetof({sname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", str(ROOT / "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        sname, field, value = line.split()
        cls = structs[sname]
        got = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(value), (sname, field, got, value)
        seen += 1
    assert seen == sum(len(c._fields_) + 1 for c in structs.values())
