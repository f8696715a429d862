"""The C-ABI library loads and exports every entry point declared in
include/hyperlag.h (no compute call: this runs without a GPU)."""
import os
import re
import subprocess

import pytest

from paper_2104_02139_amd import hyperlag as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hyperlag.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hl_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert _declared() == sorted(H.EXPORTS)


def test_library_loads_and_exports_every_symbol():
    if not os.path.exists(H.LIB_PATH):
        pytest.skip("libhyperlag.so not built")
    H.load()
    out = subprocess.run(["nm", "-D", "--defined-only", H.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (hl_[a-z_]+)\b", out))
    missing = [s for s in _declared() if s not in exported]
    assert not missing, missing


def test_status_strings():
    if not os.path.exists(H.LIB_PATH):
        pytest.skip("libhyperlag.so not built")
    L = H.load()
    assert L.hl_status_str(0) == b"ok"
    assert b"invalid" in L.hl_status_str(-1)


def test_no_silent_fallback_without_gpu():
    """Without a GPU the binding raises instead of computing elsewhere."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    if not os.path.exists(H.LIB_PATH):
        pytest.skip("libhyperlag.so not built")
    with pytest.raises(H.HyperLagError):
        H.Context(0)
