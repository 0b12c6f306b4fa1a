"""CPU: the C ABI library loads and exports every function include/xminer.h
declares (no compute call: that needs a GPU)."""
import ctypes
import os
import re

from paper_2404_11105_amd import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "..", "include", "xminer.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)  # drop comments
    return sorted(set(re.findall(r"\b(xm_[a-z0-9_]+)\s*\(", text)) - {"xm_count_opts"})


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("xm_load_graph", "xm_plan", "xm_count", "xm_graph_node_order"):
        assert must in names


def test_library_exports_every_declared_function():
    L = _lib.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value, name
    # the binding's own list matches the header
    assert sorted(_lib.EXPORTS) == declared_functions()
