"""The C-ABI library loads and exports every symbol the header declares
(no compute: runs without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cbie.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cbie_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_surface():
    from paper_2408_17116_amd import cbie
    assert set(_declared()) == set(cbie.EXPORTED)


def test_library_exports_every_declared_symbol():
    from paper_2408_17116_amd import cbie
    path = cbie.LIB_PATH
    if not os.path.exists(path):
        pytest.skip("libcbie.so not built")
    lib = cbie.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_missing_library_fails_loudly(tmp_path):
    from paper_2408_17116_amd import cbie
    saved = cbie._lib
    cbie._lib = None
    try:
        with pytest.raises(ImportError):
            cbie.load(str(tmp_path / "missing.so"))
    finally:
        cbie._lib = saved
