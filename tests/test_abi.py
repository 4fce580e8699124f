"""The C-ABI library loads and exports every entry point include/muffin.h
declares (no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "muffin.h")
LIB = os.path.join(ROOT, "paper_1905_08468_amd", "libmuffin.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(muffin_[a-zA-Z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for n in ["muffin_create", "muffin_set_problem", "muffin_run", "muffin_get_sky",
              "muffin_destroy", "muffin_strerror", "muffin_workspace_bytes"]:
        assert n in names


def test_library_exports_all_declared_symbols():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    from paper_1905_08468_amd import muffin as mm
    assert sorted(mm.EXPORTS) == declared()


def test_config_defaults_and_workspace():
    from paper_1905_08468_amd import muffin as mm
    c = mm.default_config(64, 8)
    assert (c.n_bases, c.levels, c.sigma, c.delta_period) == (8, 3, 10.0, 10)
    assert mm.workspace_bytes(c) > 0
    bad = mm.default_config(48, 8)
    assert mm.workspace_bytes(bad) == 0          # invalid shape
    big = mm.default_config(1024, 256, mode=mm.F32, sure=1, eps_fd=1.0, sigma_w=1.0)
    assert 100e9 < mm.workspace_bytes(big) < 200e9


def test_strerror():
    from paper_1905_08468_amd import muffin as mm
    assert mm._lib.muffin_strerror(-4).decode().startswith("non-finite")
