"""The C ABI library builds, loads and exports every symbol include/hgs.h
declares; host-side argument validation returns error codes (no GPU work)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hgs.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hgs_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2512_02932_amd import _hgs
    if not os.path.exists(_hgs.LIB_PATH):
        from paper_2512_02932_amd import build
        build()
    return _hgs.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hgs_create", "hgs_destroy", "hgs_scene_init", "hgs_scene_release",
                     "hgs_render", "hgs_render_backward", "hgs_state_free", "hgs_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2512_02932_amd import _hgs
    out = subprocess.run(["nm", "-D", "--defined-only", _hgs.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (hgs_\w+)", out))
    for name in declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None
    assert set(_hgs.EXPORTS) <= exported


def test_null_arguments_are_rejected(lib):
    from paper_2512_02932_amd import _hgs
    assert lib.hgs_create(0, None) == _hgs.HGS_EINVAL
    assert b"NULL" in lib.hgs_last_error()
    sid = C.c_int32()
    assert lib.hgs_scene_init(None, None, 0, C.byref(sid)) == _hgs.HGS_EINVAL
    assert lib.hgs_render(None, 0, None, 1, None, None, None, None) == _hgs.HGS_EINVAL
    assert lib.hgs_render_backward(None, None, None, None, None) == _hgs.HGS_EINVAL
    assert lib.hgs_state_check(None, None) == _hgs.HGS_EINVAL
    sizes = (C.c_int64 * 5)()
    assert lib.hgs_state_sizes(None, None, sizes) == _hgs.HGS_EINVAL
    assert lib.hgs_type_exchange(None, 0, None, None, None, 2.05, None, None) == _hgs.HGS_EINVAL
    lib.hgs_state_free(None, None)  # no-op
    lib.hgs_destroy(None)           # no-op


def test_product_path_has_no_oracle_dependency():
    """The GPU package never imports the oracle package."""
    pkg = os.path.join(ROOT, "paper_2512_02932_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dp, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "hgs_oracle" not in txt and "liboracle" not in txt, f
