"""The C-ABI library loads and exports every entry point that include/fsi.h declares."""
import ctypes
import os
import re

import pytest

from paper_1810_04289_amd import fsi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols(header=None):
    names = [header] if header else sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    out = set()
    for h in names:
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        out |= set(re.findall(r"\b(fsi_[a-z_0-9]+)\s*\(", src))
    return sorted(out)


def test_header_and_binding_agree():
    assert declared_symbols("fsi.h") == sorted(fsi.SYMBOLS)
    assert declared_symbols("fsi_guess.h") == sorted(fsi.GUESS_SYMBOLS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(fsi.LIB_PATH):
        pytest.fail("libfsi.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(fsi.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_null_arguments_are_rejected_without_a_gpu_call():
    L = fsi.load_library()
    assert L.fsi_create(None, None, None, None, None) == 1
    assert L.fsi_destroy(None) == 0
    assert L.fsi_sizes(None, None, None) == 1
    assert L.fsi_residual(None, None, None) == 1
    assert L.fsi_last_error(None) == b"null solver"


def test_product_path_has_no_oracle_dependency():
    for root, _, files in os.walk(os.path.join(ROOT, "paper_1810_04289_amd")):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                txt = open(os.path.join(root, f)).read()
                assert "import oracle" not in txt and "fsio_" not in txt and "from oracle" not in txt, f
