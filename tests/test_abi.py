"""The C ABI library loads, exports every entry point declared in
include/g4d.h, and rejects bad arguments on the host (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2310_08528_amd import g4d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "g4d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(g4d_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("g4d_deform", "g4d_render", "g4d_deform_batched", "g4d_render_workspace_bytes",
                     "g4d_read_status", "g4d_server_submit"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = g4d.load()
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared_functions()) == set(g4d.SIGNATURES)


def test_workspace_size_and_status_strings():
    a = g4d.workspace_bytes(1000, 128, 128, 10_000)
    b = g4d.workspace_bytes(1000, 128, 128, 20_000)
    assert a > 0 and b > a
    assert g4d.workspace_bytes(-1, 128, 128, 10) == 0
    assert g4d.workspace_bytes(10, 0, 128, 10) == 0
    assert g4d.workspace_bytes(10, 128, 128, 1 << 30) == 0
    lib = g4d.load()
    assert lib.g4d_status_string(g4d.ECAPACITY).decode() == "instance capacity exceeded"
    assert "g4d" in g4d.version()


def test_host_validation_rejects_null_arguments_without_touching_the_device():
    lib = g4d.load()
    assert lib.g4d_render(None, None, None, None, None, None, None) == g4d.EINVAL
    assert lib.g4d_deform(None, None, None, ctypes.c_float(0.5), None, None) == g4d.EINVAL
    assert lib.g4d_deform_batched(None, 0, None) == g4d.EINVAL
    ws = g4d.Workspace(None, 0, 10, 16, 16, 100)
    st = g4d.DeviceStatus()
    assert lib.g4d_read_status(ctypes.byref(ws), ctypes.byref(st), None) == g4d.EINVAL
    # a time outside [0, 1] is rejected before any launch
    G = g4d.Gaussians(0, 0, None, None, None, None, None)
    P = g4d.Planes()
    assert lib.g4d_deform_features(ctypes.byref(G), ctypes.byref(P), ctypes.c_float(2.0), None, None) == g4d.EINVAL
