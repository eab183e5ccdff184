"""The C-ABI library loads and exports every function include/hsma.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsma.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(hsma_\w+)\s*\(", txt)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("hsma_plan_create", "hsma_energy_forces", "hsma_energy_forces_device",
              "hsma_energy_grad_device", "hsma_plan_destroy", "hsma_workspace_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1806_04801_amd import hsma
    lib = hsma.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding's table covers the header exactly
    assert sorted(hsma.EXPORTS) == declared_functions()


def test_status_strings_without_gpu():
    from paper_1806_04801_amd import hsma
    lib = hsma.load()
    assert lib.hsma_status_string(0) == b"ok"
    assert lib.hsma_status_string(-2) == b"system not neutral"
    assert lib.hsma_status_string(-4) == b"two charges at the same position"
    assert lib.hsma_version() == 6


def test_plan_argument_validation_without_gpu():
    """Invalid descriptions are rejected before any device work."""
    from paper_1806_04801_amd import hsma
    lib = hsma.load()
    h = ctypes.c_void_p()
    assert lib.hsma_plan_create(1.0, 0, 8, 1000, 10, 2.7, ctypes.byref(h)) == -1   # K < unknowns
    assert lib.hsma_plan_create(1.0, 0, 8, 1000, 600, 0.5, ctypes.byref(h)) == -1  # R <= R0
    assert lib.hsma_plan_create(-1.0, 0, 8, 1000, 600, 2.7, ctypes.byref(h)) == -1
    assert lib.hsma_plan_create(1.0, 7, 8, 1000, 600, 2.7, ctypes.byref(h)) == -1
    assert b"boundary condition" in lib.hsma_last_error()


def test_product_path_does_not_import_oracle():
    """The library package never reaches the oracle (no CPU fallback)."""
    pkg = os.path.join(ROOT, "paper_1806_04801_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "hsma_oracle" not in txt, f
