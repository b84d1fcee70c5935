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


def test_create_rejects_invalid_objects_before_any_device_work():
    """Argument checks of cbie_create run on the host before any HIP call,
    so they are exercised here without a GPU: each malformed object (or
    argument) gives EINVAL and no context; a null context gives EINVAL from
    the stage entry points."""
    import ctypes as C
    from paper_2408_17116_amd import cbie
    if not os.path.exists(cbie.LIB_PATH):
        pytest.skip("libcbie.so not built")
    lib = cbie.load()

    def obj(form=cbie.MFIE_PEC, k0=1.0, q=4, axes=(1.0, 1.0, 1.0),
            patches=((0, 0, 0, 1),), eps_r=1.0, mu_r=1.0):
        arr = (cbie._Patch * len(patches))(*[cbie._Patch(f, i, j, s) for (f, i, j, s) in patches])
        o = cbie._Object(form=form, k0=k0, q=q, n_patches=len(patches), patches=arr, eps_r=eps_r, mu_r=mu_r)
        o.axes[:] = list(axes)
        o._keep = arr
        return o

    def create(objs, n=None, out=True):
        a = (cbie._Object * len(objs))(*objs)
        h = C.c_void_p(1234)
        st = lib.cbie_create(a, len(objs) if n is None else n, None, C.byref(h) if out else None)
        return st, h.value

    bad = [
        [obj(q=12)], [obj(form=cbie.NMULLER, q=9, eps_r=4.0)], [obj(q=1)], [obj(k0=0.0)], [obj(k0=float("nan"))], [obj(axes=(1.0, -1.0, 1.0))],
        [obj(patches=((6, 0, 0, 1),))], [obj(patches=((0, 2, 0, 2),))], [obj(patches=((0, 0, 0, 0),))],
        [obj(form=7)], [obj(form=cbie.NMULLER, eps_r=-4.0)], [obj(form=cbie.NMULLER, mu_r=0.0)],
        [obj(form=cbie.NMULLER, eps_r=float("inf"))],
        [obj(), obj(form=cbie.NMULLER, eps_r=4.0)],             # one formulation per context
    ]
    for objs in bad:
        st, h = create(objs)
        assert st == cbie.EINVAL and h is None
    assert create([obj()], n=0)[0] == cbie.EINVAL
    assert create([obj()], out=False)[0] == cbie.EINVAL
    assert lib.cbie_build_tree(None, 256, 1.0, 1.0) == cbie.EINVAL
    assert lib.cbie_fill(None, 0, 0) == cbie.EINVAL
    assert lib.cbie_compress(None, 1e-6, 0) == cbie.EINVAL
    assert lib.cbie_factor(None, 0) == cbie.EINVAL


def test_library_leaves_none_of_its_own_symbols_undefined():
    """A shared library links with undefined symbols and fails only when one
    is first called: every function of the library's own namespace must be
    defined in it."""
    import shutil
    import subprocess
    from paper_2408_17116_amd import cbie
    if not os.path.exists(cbie.LIB_PATH) or shutil.which("nm") is None:
        pytest.skip("libcbie.so not built or nm missing")
    out = subprocess.run(["nm", "-C", "-u", cbie.LIB_PATH], capture_output=True, text=True, check=True).stdout
    assert [l for l in out.splitlines() if "cbie::" in l or " cbie_" in l] == []
