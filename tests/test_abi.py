"""The C-ABI library loads and exports every function include/ann.h declares;
the product package never reaches the CPU oracle (no compute calls here)."""
import ctypes
import os
import re
import subprocess

import pytest

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


def _caller_source(names):
    """A caller that includes the header and takes the address of every
    declared entry point (so the link resolves each one)."""
    body = ",\n  ".join(f"(ann_fn){n}" for n in names)
    return ('#include "ann.h"\n'
            "typedef void (*ann_fn)(void);\n"
            f"static ann_fn const table[] = {{\n  {body}\n}};\n"
            "int main(void) { return table[0] == 0; }\n")


@pytest.mark.parametrize("lang", ["c11", "c++17"])
def test_header_compiles_and_links_for_plain_callers(tmp_path, lang):
    """include/ann.h is self-contained for C11 and C++17 callers (-Wall
    -Werror -pedantic, no HIP headers), and every entry point it declares
    resolves against libann.so at link time and at load time."""
    assert os.path.exists(LIB), "build libann.so first (__graft_entry__.build())"
    names = declared()
    src = tmp_path / ("caller.c" if lang == "c11" else "caller.cpp")
    src.write_text(_caller_source(names))
    exe = tmp_path / "caller"
    cc = ["gcc", "-std=c11"] if lang == "c11" else ["g++", "-std=c++17"]
    cmd = [*cc, "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.dirname(HEADER),
           str(src), "-o", str(exe), LIB, "-Wl,-rpath," + os.path.dirname(LIB),
           "-Wl,-rpath-link,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes structures of the binding have the C header's sizes and
    field offsets (a struct that drifts from the header corrupts calls)."""
    from paper_2409_16576_amd import ann
    pairs = {"ann_index_desc": ann.IndexDesc, "ann_tune_result": ann.TuneResult,
             "ann_profile": ann.Profile, "ann_load_cfg": ann.LoadCfg,
             "ann_server_cfg": ann.ServerCfg, "ann_server_stats": ann.ServerStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ann.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    r = subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    got = dict(ln.split() for ln in subprocess.run([str(exe)], capture_output=True,
                                                   text=True).stdout.splitlines())
    for cname, py in pairs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)
    assert ann.IndexDesc().as_dict()["raw_tier"] == 0
