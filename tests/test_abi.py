"""The C-ABI library loads and exports every symbol include/atm3.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "atm3.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(atm3_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    from paper_2510_21230_amd import _lib
    assert set(_declared()) == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2510_21230_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.atm3_version().startswith(b"atm3")


def test_struct_layouts():
    from paper_2510_21230_amd import _lib
    assert ctypes.sizeof(_lib.Params) == 48
    assert ctypes.sizeof(_lib.Result) == 72


def test_no_device_gives_edevice():
    """Host-side argument handling: with no visible GPU, creation fails cleanly."""
    import torch
    from paper_2510_21230_amd import _lib
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.atm3_create(ctypes.byref(h), 0) == _lib.ATM3_EDEVICE
    assert lib.atm3_create(ctypes.byref(h), -1) == _lib.ATM3_EDEVICE


def test_null_context_is_einval():
    from paper_2510_21230_amd import _lib
    lib = _lib.load()
    assert lib.atm3_set_stream(None, None) == _lib.ATM3_EINVAL
    box = (ctypes.c_double * 3)(10.0, 10.0, 10.0)
    nc = (ctypes.c_int32 * 3)()
    assert lib.atm3_bin_cells(None, None, 0, box, 2.5, None, None, None, nc) == _lib.ATM3_EINVAL


def test_null_model_is_einval():
    from paper_2510_21230_amd import _lib
    lib = _lib.load()
    assert lib.atm3_mlp_create(None, 0, None) == _lib.ATM3_EINVAL
    assert lib.atm3_mlp_get_params(None, None, None, 0) == _lib.ATM3_EINVAL
    assert lib.atm3_mlp_train_step(None, None, None, 0, None, 2.5, None, 1.0, 1e-3, None) == _lib.ATM3_EINVAL
    lib.atm3_mlp_destroy(None)
