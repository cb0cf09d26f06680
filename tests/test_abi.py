"""The C-ABI library loads and exports every function include/ann.h declares;
the product package never reaches the CPU oracle (no compute calls here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ann.h")
LIB = os.path.join(ROOT, "paper_2409_16576_amd", "libann.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(ann_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("ann_load_index", "ann_search", "ann_free_index", "ann_last_error",
                 "ann_graph_create", "ann_server_start", "ann_adc_backward"):
        assert must in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build libann.so first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_product_code_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_2409_16576_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f), errors="replace").read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", src, flags=re.M), f
                assert "ann_oracle" not in src, f
