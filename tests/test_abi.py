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
