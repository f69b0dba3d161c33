"""Host-side checks of the C ABI: libgbk.so loads and exports every entry
point that include/gbk.h declares (no compute call, no GPU needed)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    hdrs = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
            if f.endswith(".h")]
    names = set()
    for h in hdrs:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(gk_\w+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    from paper_1510_01815_amd import gbk as G
    lib = ctypes.CDLL(G.LIB_PATH)
    names = declared_symbols()
    assert "gk_chi2_batch" in names and "gk_create_model" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"
    assert set(G.SYMBOLS) <= set(names)


# (ctypes structure of the binding, C type of include/gbk.h)
STRUCTS = [("ModelDesc", "gk_model_desc"), ("ProfileStats", "gk_profile_stats"),
           ("LMOpts", "gk_lm_opts"), ("LMResult", "gk_lm_result"), ("NSOpts", "gk_ns_opts"),
           ("NSResult", "gk_ns_result"), ("GridResult", "gk_grid_result"),
           ("SurrogateOpts", "gk_surrogate_opts"), ("LineOpts", "gk_line_opts"),
           ("TuneResult", "gk_tune_result"), ("NSMode", "gk_ns_mode")]


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    that a C compiler gives the header's struct (compiled here with gcc)."""
    import subprocess
    from paper_1510_01815_amd import gbk as G
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gbk.h"', "int main(void) {"]
    for py, c in STRUCTS:
        lines.append(f'printf("{py} size %zu\\n", sizeof({c}));')
        for name, _ in getattr(G, py)._fields_:
            lines.append(f'printf("{py} {name} %zu\\n", offsetof({c}, {name}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        py, field, val = line.split()
        got[(py, field)] = int(val)
    for py, _ in STRUCTS:
        cls = getattr(G, py)
        assert got[(py, "size")] == ctypes.sizeof(cls), py
        for name, _ in cls._fields_:
            assert got[(py, name)] == getattr(cls, name).offset, (py, name)
