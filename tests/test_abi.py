"""The C-ABI library loads and exports every function include/snn.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2007_14236_amd import snn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "snn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(snn_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["snn_create_net", "snn_create", "snn_connect_fixed_indegree", "snn_poisson", "snn_build",
                 "snn_simulate", "snn_get_spikes", "snn_get_state", "snn_set_state"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(snn.LIB_PATH), reason="libsnn.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(snn.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(snn.LIB_PATH), reason="libsnn.so not built")
def test_binding_signatures_cover_the_header():
    assert set(declared_functions()) == set(snn._SIGS)
    snn.lib()  # loads and applies every signature


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(snn, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(snn, "_lib", None)
    with pytest.raises(ImportError):
        snn.lib()


@pytest.mark.skipif(not os.path.exists(snn.LIB_PATH), reason="libsnn.so not built")
def test_argument_validation_without_device():
    """Calls that fail before touching the device return their status code."""
    L = snn.lib()
    out = ctypes.c_void_p()
    bad = snn.Config(0.0, 1, 15, 0)  # dt must be positive
    assert L.snn_create_net(ctypes.byref(bad), None, ctypes.byref(out)) == -1
    bad = snn.Config(0.1, 1, 64, 0)  # Dmax above 63
    assert L.snn_create_net(ctypes.byref(bad), None, ctypes.byref(out)) == -1
    bad = snn.Config(0.1, 1, 15, snn.F_DELIVERY_DIRECT | snn.F_DELIVERY_BINNED)  # two delivery modes
    assert L.snn_create_net(ctypes.byref(bad), None, ctypes.byref(out)) == -1
    bad = snn.Config(0.1, 1, 15, 1 << 7)  # unknown flag
    assert L.snn_create_net(ctypes.byref(bad), None, ctypes.byref(out)) == -1
    for tile in (128, 768, 8192):  # tile size: power of two in [256, 4096]
        bad = snn.Config(0.1, 1, 15, 0, tile)
        assert L.snn_create_net(ctypes.byref(bad), None, ctypes.byref(out)) == -1
    assert L.snn_build(None) == -1
