"""The C-ABI library loads and exports every entry point that
include/rodlcp.h declares (no compute calls; runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rodlcp.h")
LIB = os.path.join(ROOT, "paper_2109_08206_amd", "librodlcp.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rl_[a-z_A-Z0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("rl_build_pairs", "rl_assemble_D", "rl_solve_lcp", "rl_step", "rl_apply_M", "rl_create"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (rl_\w+)", out))
    assert exported == set(declared_symbols())


def test_binding_names_match_header():
    import paper_2109_08206_amd as rl
    assert set(rl.SYMBOLS) == set(declared_symbols())


def test_status_strings_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    import paper_2109_08206_amd as rl
    lib = rl.load()
    assert lib.rl_status_str(0) == b"ok"
    assert b"capacity" in lib.rl_status_str(-2)
    # a NULL handle is rejected before any device work
    assert lib.rl_reserve(None, 10, 10) == rl.ERR_ARG
    assert lib.rl_create(None, None) == rl.ERR_ARG


def test_missing_library_fails_loudly():
    """No CPU fallback: without the built library the binding raises."""
    import sys
    code = ("import paper_2109_08206_amd as rl\n"
            "try:\n"
            "    rl.load('/nonexistent/librodlcp.so')\n"
            "except RuntimeError as e:\n"
            "    print('raised', e)\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT)
    assert out.returncode == 0 and out.stdout.startswith("raised") and "not built" in out.stdout
