"""The C-ABI library loads and exports every symbol include/pcx.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "pcx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pcx_[a-z_]+)\s*\(", src)))


def test_header_declares_the_api():
    syms = declared_symbols()
    for s in ["pcx_mlp_create", "pcx_extract", "pcx_complex_copy", "pcx_last_error"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    lib_path = os.path.join(ROOT, "paper_2306_07212_amd", "libpcx.so")
    assert os.path.exists(lib_path), "libpcx.so not built (python -m paper_2306_07212_amd.build)"
    lib = ctypes.CDLL(lib_path)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, f"not exported: {missing}"


def test_binding_names_match_header():
    from paper_2306_07212_amd import pcx
    assert sorted(pcx.SYMBOLS) == declared_symbols()


def test_error_path_without_gpu():
    """A NULL handle is rejected on the host before any device call."""
    from paper_2306_07212_amd import pcx
    rc = pcx._lib.pcx_complex_info(None, None)
    assert rc == pcx.PCX_ERR_INVALID
    assert "NULL" in pcx.last_error()
