"""The C ABI library loads without a GPU and exports every entry point that
include/mgdd.h declares (no compute calls here)."""
import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1202_2462_amd", "libmgdd.so")


def test_library_exports_declared_symbols():
    if not os.path.exists(LIB):
        pytest.skip("libmgdd.so not built (run __graft_entry__.build())")
    from paper_1202_2462_amd import mgdd
    names = mgdd.declared_symbols()
    assert len(names) >= 9
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert set(names) <= exported


def test_header_is_plain_c():
    """The boundary carries no C++ or torch types."""
    txt = open(os.path.join(ROOT, "include", "mgdd.h")).read()
    for bad in ("torch", "std::", "template", "class ", "at::"):
        assert bad not in txt, bad
    subprocess.run(["gcc", "-fsyntax-only", "-x", "c", os.path.join(ROOT, "include", "mgdd.h")], check=True)
