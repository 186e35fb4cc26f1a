"""The C-ABI library loads on a machine without a GPU and exports every
entry point that include/kfbi.h declares (no compute calls here)."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "kfbi.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kfbi_\w+)\s*\(", text)))


def test_header_declares_the_named_calls():
    names = declared_functions()
    for must in ("kfbi_domain_create", "kfbi_helmholtz_solve", "kfbi_step_heat",
                 "kfbi_step_wave", "kfbi_step_schrodinger"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2404_14864_amd import kfbi
    if not os.path.exists(kfbi.LIB_PATH):
        pytest.skip("libkfbi.so not built")
    L = kfbi.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(kfbi.EXPORTED) == set(declared_functions())


def test_binding_struct_sizes_match_header_layout():
    import ctypes
    from paper_2404_14864_amd import kfbi
    # sizes implied by the header's field order on LP64
    assert ctypes.sizeof(kfbi.DomainDesc) == 8 + 4 * 4 + 8 * 7 + 4 * 2 + 8
    assert ctypes.sizeof(kfbi.SolveOpts) == 8 + 4 * 6 + 8
    assert ctypes.sizeof(kfbi.SolveStats) == 4 * 2 + 8 + 4 * 2 + 8
    assert ctypes.sizeof(kfbi.DomainInfo) == 4 * 2 + 8 * 2 + 4 * 4 + 8 + 8
    assert ctypes.sizeof(kfbi.StepParams) == 8 * 4 + 8 * 2 + 4 * 2
