"""The C-ABI library builds for gfx950, loads, and exports every function that
include/mcl.h declares.  No GPU needed (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcl.h")
LIB = os.path.join(ROOT, "paper_2002_10083_amd", "libmcl.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(mcl_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_north_star_entry_points():
    names = declared_functions()
    for n in ("mcl_expand", "mcl_prune", "mcl_inflate", "mcl_iterate", "mcl_merge_partials"):
        assert n in names
    assert len(names) >= 15


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcl.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcl.so not built")
def test_binding_lists_all_exports():
    from paper_2002_10083_amd import mcl
    assert set(declared_functions()) == set(mcl.EXPORTS)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcl.so not built")
def test_default_params_and_host_only_queries():
    from paper_2002_10083_amd import mcl
    p = mcl.default_params()
    assert p.prune_threshold == 1e-4 and p.select_num == 1100 and p.recover_num == 1400
    assert p.recover_pct == 0.9 and p.inflation == 2.0 and p.cohen_keys == 5
    assert mcl.mlp_packed_bytes() >= 5057 * 2
    assert mcl.mlp_state_floats() >= 3 * 5057


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcl.so not built")
def test_library_is_gfx950_code_object():
    data = open(LIB, "rb").read()
    assert b"gfx950" in data
