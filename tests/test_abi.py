"""The C ABI library loads and exports every function include/ccm.h declares
(no compute calls: this runs without a GPU)."""
import os
import re

import pytest

from paper_1905_00565_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(ccm\w*)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(capi.LIBRARY):
        from paper_1905_00565_amd import build
        build.build_library()
    return capi.lib()


def test_header_declares_the_binding_exports():
    assert set(declared_functions()) == set(capi.EXPORTS)


@pytest.mark.parametrize("name", declared_functions())
def test_symbol_exported(lib, name):
    assert hasattr(lib, name)


def test_library_is_gfx950_code_object(lib):
    data = open(capi.LIBRARY, "rb").read()
    assert b"gfx950" in data


def test_last_error_of_null_context(lib):
    assert capi.lib().ccm_last_error(None) == b"NULL context"
