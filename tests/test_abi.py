"""CPU checks of the C ABI: the library loads and exports every function the header declares;
calls that need a device fail cleanly with an error code and message when there is none."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsdock.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsd_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("rsd_build_rs_tensor", "rsd_score_poses", "rsd_tensor_import", "rsd_tensor_export",
                 "rsd_context_create", "rsd_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2510_26611_amd import _lib
    lib = _lib.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (rsd_\w+)", out))
    for name in _declared():
        assert name in exported, name
        assert getattr(lib, name) is not None
    assert set(_lib.EXPORTED) == set(_declared())


def test_version_and_error_paths_without_device():
    from paper_2510_26611_amd import _lib
    lib = _lib.lib()
    a, b = ctypes.c_int32(), ctypes.c_int32()
    assert lib.rsd_version(ctypes.byref(a), ctypes.byref(b)) == 0 and a.value >= 1
    # null output pointer is an argument error, checked before any device call
    assert lib.rsd_context_create(0, None, 0, None) == _lib.RSD_E_INVALID
    assert b"NULL" in lib.rsd_last_error()
    # null handles are argument errors
    assert lib.rsd_tensor_query(None, None, None, None, None) == _lib.RSD_E_INVALID
    assert lib.rsd_score_poses(None, None, None, None, 1, None, None, 1, 2.5, 0, None, None, None, None,
                               None) == _lib.RSD_E_INVALID
    lib.rsd_tensor_free(None)
    lib.rsd_context_free(None)


def test_context_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2510_26611_amd import _lib
    lib = _lib.lib()
    h = ctypes.c_void_p()
    st = lib.rsd_context_create(0, None, 0, ctypes.byref(h))
    assert st in (_lib.RSD_E_HIP, _lib.RSD_E_INVALID)
    assert len(lib.rsd_last_error()) > 0
