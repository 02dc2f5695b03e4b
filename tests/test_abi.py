"""CPU-side checks of the C ABI: the library loads and exports every function
the public header declares; the binding wraps each of them.  No GPU call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "raypc.h")
LIB = os.path.join(ROOT, "paper_2207_12011_amd", "libraypc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(raypc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("raypc_load_fields", "raypc_set_brush", "raypc_set_transfer_function", "raypc_render"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_every_symbol():
    from paper_2207_12011_amd import raypc
    assert sorted(raypc.EXPORTED) == sorted(n for n in declared_functions())
    assert raypc.version() == 10000


def test_binding_has_no_cpu_fallback():
    src = open(os.path.join(ROOT, "paper_2207_12011_amd", "raypc.py")).read()
    assert "import oracle" not in src and "from oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_2207_12011_amd")):
        if f.endswith(".py"):
            s = open(os.path.join(ROOT, "paper_2207_12011_amd", f)).read()
            assert not re.search(r"^\s*(import|from)\s+oracle", s, flags=re.M), f
