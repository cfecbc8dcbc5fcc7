"""C ABI contract checks that need no GPU: the library loads, exports every
symbol the header declares, and fails cleanly without a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scarff.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scff_[a-z_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared_functions()
    for must in ("scff_create", "scff_destroy", "scff_load_molecule", "scff_load_transitions",
                 "scff_load_transitions_device", "scff_set_options", "scff_eval_grid", "scff_eval_points",
                 "scff_query", "scff_export_vtensors", "scff_last_error", "scff_server_create",
                 "scff_server_submit", "scff_server_wait", "scff_server_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2512_18010_amd import binding
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert binding.scff_version().decode().startswith("scarff")


def test_no_device_is_reported_not_crashed():
    from paper_2512_18010_amd import binding
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = binding.scff_create(0, 0, ctypes.byref(h))
    assert rc == binding.SCFF_EDEVICE
    assert b"device" in binding.scff_last_error()
    with pytest.raises(binding.ScffError) as ei:
        binding.Context(0)
    assert ei.value.code == binding.SCFF_EDEVICE
    assert binding.scff_server_create(0, 0, 2, ctypes.byref(h)) == binding.SCFF_EDEVICE


def test_null_arguments():
    from paper_2512_18010_amd import binding
    binding.scff_destroy(None)          # ignored
    assert binding.scff_create(0, 0, None) == binding.SCFF_EINVAL
    assert binding.scff_query(None, None) == binding.SCFF_EINVAL
    assert binding.scff_set_options(None, 0.0, 1.0) == binding.SCFF_EINVAL
    assert binding.scff_eval_grid(None, None, 0, None, None, 0, None) == binding.SCFF_EINVAL
    assert binding.scff_server_create(0, 0, 0, ctypes.byref(ctypes.c_void_p())) == binding.SCFF_EINVAL
    assert b"max_inflight" in binding.scff_last_error()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    """The product path has no fallback: importing the binding without the
    shared library raises."""
    import importlib.util
    src = os.path.join(ROOT, "paper_2512_18010_amd", "binding.py")
    dst = tmp_path / "binding.py"
    dst.write_text(open(src).read())
    spec = importlib.util.spec_from_file_location("binding_copy", str(dst))
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)
