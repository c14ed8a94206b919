"""The C-ABI library loads and exports every function its header declares (no GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(knnj_\w+)\s*\(", txt, flags=re.M))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("knnj_build_index", "knnj_join", "knnj_join_bf", "knnj_index_free", "knnj_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1011_2807_amd import knnj
    lib = ctypes.CDLL(knnj.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_loads():
    import paper_1011_2807_amd as kj
    lib = kj.load_library()
    assert lib.knnj_last_error() == b""
