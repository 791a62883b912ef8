"""The C-ABI library loads and exports every function include/gf.h declares
(no compute call: runs without a GPU)."""
import ctypes
import os

import pytest

from paper_1212_5221_amd import gf


def test_header_declares_the_abi():
    names = gf.header_functions()
    for must in ("gf_create", "gf_destroy", "gf_last_error", "gf_add_instance", "gf_set_gauge", "gf_set_group",
                 "gf_set_precision", "gf_workspace_size", "gf_bind_workspace", "gf_upload", "gf_download",
                 "gf_set_overrelax", "gf_set_anneal", "gf_sweep", "gf_measure", "gf_measure_timeslices",
                 "gf_unitarity", "gf_reunitarise"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(gf.LIB_PATH):
        from paper_1212_5221_amd import build
        build.build(verbose=False)
    lib = ctypes.CDLL(gf.LIB_PATH)
    missing = [n for n in gf.header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_has_no_fallback(monkeypatch, tmp_path):
    monkeypatch.setattr(gf, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gf, "_lib", None)
    with pytest.raises(ImportError):
        gf.load()


def test_create_error_without_gpu():
    # without a visible device gf_create reports an error status, never crashes
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = gf.load()
    h = ctypes.c_void_p()
    rc = lib.gf_create(ctypes.byref(h), 0, None)
    assert rc < 0
    assert lib.gf_last_error(None)
