"""The C-ABI library loads without a GPU and exports every declared entry point."""
import ctypes
import os
import re

import pytest

from paper_2307_00391_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(sv_[a-z0-9_]+)\s*\(", text, re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sv_alloc", "sv_init_b", "sv_apply_gate", "sv_apply_ctrl_unitary", "sv_qft", "sv_hhl",
                     "sv_postselect"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libsv.so not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if getattr(lib, n, None) is None]
    assert not missing, f"declared but not exported: {missing}"
    assert set(declared_functions()) <= set(binding._SIGS), "binding lacks a declared entry point"


def test_validation_errors_without_gpu_work():
    """Argument checks run on the host: a bad qubit count is rejected before any device call."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libsv.so not built")
    with pytest.raises(binding.SvError) as e:
        binding.sv_alloc(0)
    assert e.value.status == binding.SV_EINVAL
    assert binding.sv_plan_passes(20, binding.SV_C64, [("u", 3, [[0, 1], [1, 0]])], 12) == 1
