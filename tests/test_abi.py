"""The C-ABI library loads and exports every entry point its header declares.

CPU-only: no call here touches a GPU.
"""
import ctypes
import os
import re

import pytest
import torch  # noqa: F401  (loads the HIP runtime the library must share)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kdeplugin.h")
LIB = os.path.join(ROOT, "paper_1505_02100_amd", "libkdeplugin.so")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(kde_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("kde_psi", "kde_plugin_bandwidth", "kde_plugin_bandwidth_batch",
                     "kde_ctx_create", "kde_ctx_destroy", "kde_psi_ex",
                     "kde_plugin_bandwidth_ex", "kde_psi_range", "kde_last_error",
                     "kde_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libkdeplugin.so not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_entry_points():
    if not os.path.exists(LIB):
        pytest.skip("libkdeplugin.so not built")
    from paper_1505_02100_amd import kdeplugin as kp
    assert "gfx950" in kp.kde_version()
    assert kp.kde_strerror(kp.KDE_EINVAL) == "invalid argument"
    assert kp.kde_strerror(kp.KDE_EDEGENERATE).startswith("degenerate")
    o = kp.kde_options_init()
    assert o.precision == kp.KDE_FP64_PLAIN and o.device == 0
    # argument validation happens before any device call
    assert kp._lib.kde_psi_num_items(None, 10) == -1
    assert kp.kde_last_error() == kp.KDE_EINVAL
    res = kp.kde_result()
    assert kp._lib.kde_plugin_bandwidth_ex(None, None, 5, 0, 0, None, ctypes.byref(res)) == kp.KDE_EINVAL
    assert kp._lib.kde_eval_ex(None, None, 5, 0, 0, None, 3, 0, 0.5, None, None) == kp.KDE_EINVAL
    # negative options are refused before the device is touched
    for field in ("wait_limit_us", "target_items", "pair_budget", "mem_budget"):
        o = kp.kde_options_init()
        setattr(o, field, -1)
        h = kp._P()
        assert kp._lib.kde_ctx_create(ctypes.byref(h), ctypes.byref(o)) == kp.KDE_EINVAL, field
        assert not h.value


def test_binding_names_match_the_header():
    if not os.path.exists(LIB):
        pytest.skip("libkdeplugin.so not built")
    from paper_1505_02100_amd import kdeplugin as kp
    for name in _declared_functions():
        assert hasattr(kp, name), name


def test_binding_constants_match_the_header():
    # every #define KDE_* value the header states is the binding's constant of the same name
    import re
    from paper_1505_02100_amd import kdeplugin as kp
    text = open(HEADER).read()
    found = re.findall(r"^#define (KDE_[A-Z0-9_]+)\s+\(?(-?\d+)\)?", text, flags=re.M)
    assert ("KDE_NUM_STAGES", "4") in found
    for name, value in found:
        if hasattr(kp, name):
            assert getattr(kp, name) == int(value), name
