"""The C ABI library builds, loads, and exports every entry point its header declares (no GPU calls)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "bddc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bddc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("bddc_setup", "bddc_solve", "bddc_stats", "bddc_destroy", "bddc_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1901_02090_amd import bddc
    if not os.path.exists(bddc.LIB_PATH):
        pytest.skip("libbddc.so not built")
    lib = bddc.load_library()
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(bddc.EXPORTED) == _declared()


def test_binding_has_no_cpu_fallback(tmp_path):
    """A missing library is an error, never a silent fallback."""
    from paper_1901_02090_amd import bddc
    saved = bddc._lib
    bddc._lib = None
    try:
        with pytest.raises(FileNotFoundError):
            bddc.load_library(str(tmp_path / "missing.so"))
    finally:
        bddc._lib = saved


def test_allocator_hooks_are_host_only_and_checked():
    from paper_1901_02090_amd import bddc
    if not os.path.exists(bddc.LIB_PATH):
        pytest.skip("libbddc.so not built")
    lib = bddc.load_library()
    keep = bddc.FREE_FN(lambda p, c: None)
    assert lib.bddc_set_allocator(bddc.ALLOC_FN(), keep, None) == bddc.BDDC_EINVAL
    bddc.set_allocator(lambda n: 0, lambda p: None)
    bddc.set_allocator()                 # back to hipMalloc / hipFree
    with pytest.raises(ValueError):
        bddc.set_allocator(lambda n: 0, None)
