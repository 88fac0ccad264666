"""CPU-side checks of the C ABI library: it loads, exports every symbol that
include/lt.h declares, its struct layouts match the header, and it fails
cleanly (no crash) when no device is present."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import lt_inputs as li

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lt.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(lt_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2310_02043_amd import native
    if not os.path.exists(native.LIB_PATH):
        pytest.skip("liblt.so not built")
    return native.load()


def test_header_declares_expected_entry_points():
    names = _declared()
    for n in ("lt_create", "lt_scene_upload", "lt_set_lights", "lt_trace_forward", "lt_trace_adjoint",
              "lt_objective", "lt_record_paths", "lt_sync"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2310_02043_amd import native
    out = subprocess.run(["nm", "-D", "--defined-only", native.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lt_\w+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    assert set(native.EXPORTED) == set(_declared())


def test_struct_layouts_match_header(lib):
    from paper_2310_02043_amd import native
    assert C.sizeof(native.TraceCfg) == 32
    assert C.sizeof(native.Tuning) == 32
    assert native.Tuning.tri_share.offset == 20
    assert li.PATCH_DTYPE.itemsize == native.PATCH_ITEMSIZE == 88
    assert li.LIGHT_DTYPE.itemsize == native.LIGHT_ITEMSIZE == 20
    # field offsets of lt_patch as laid out in the header
    off = {n: li.PATCH_DTYPE.fields[n][1] for n in li.PATCH_DTYPE.names}
    assert off["normal"] == 36 and off["inv_len2_u"] == 48 and off["albedo"] == 64
    assert off["res_u"] == 68 and off["texel_base"] == 80


def test_create_fails_cleanly_without_device(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = C.c_void_p()
    rc = lib.lt_create(0, None, C.byref(h))
    assert rc != 0 and not h.value


def test_null_context_is_rejected(lib):
    assert lib.lt_set_stream(None, None) == -1
    assert lib.lt_sync(None, None) == -1
    assert lib.lt_trace_forward(None, None, None, None, None) == -1
    assert lib.lt_last_error(None) == b"null context"


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2310_02043_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "lt_oracle" not in txt, f
