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
    assert ctypes.sizeof(afn.afn_params) == 32
    assert afn.afn_params.seed.offset == 24
