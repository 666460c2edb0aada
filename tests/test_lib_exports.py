"""The HIP library loads on any host and exports every entry point its header declares."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2211_17263_amd", "libprdpt.so")


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(prdpt_\w+)\s*\(", text, flags=re.M))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("prdpt_scene_create", "prdpt_render_perturbed", "prdpt_smoothed_loss",
                     "prdpt_grad_estimate"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libprdpt.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT\s+(prdpt_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libprdpt.so not built")
def test_library_loads_and_binding_names_match():
    from paper_2211_17263_amd import native
    L = native.load()
    for n in declared_functions():
        assert hasattr(L, n)
    assert set(native.EXPORTS) == set(declared_functions())
    assert L.prdpt_last_error() == b""
