"""The HIP library loads and exports every entry point that include/cgks.h declares.

No compute call is made here (this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "cgks.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cgks_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_documented_calls():
    syms = declared_symbols()
    for s in ("cgks_create", "cgks_mesh_setup", "cgks_coloring", "cgks_residual", "cgks_smooth",
              "cgks_vcycle", "cgks_solve", "cgks_restrict", "cgks_prolong"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2509_06347_amd", "libcgks.so"))
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2509_06347_amd import cgks
    assert set(declared_symbols()) <= set(cgks.EXPORTS)
