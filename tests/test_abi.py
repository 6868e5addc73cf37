"""The C-ABI library loads, exports every symbol include/bsp.h declares, and
rejects invalid geometries before touching a GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

import paper_1708_05303_amd as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "bsp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bsp_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_binding_names():
    assert declared_symbols() == sorted(B.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    for name in declared_symbols():
        assert hasattr(lib, name), name
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr)


def _geom(**kw):
    g = B.Geom()
    d = dict(n=64, n_reduce=0, box=1000.0, window=1, compensate=1, interlace=0, los=0, lmax=0, nbins=10,
             k0=2.0, dk=2.0)
    d.update(kw)
    for k, v in d.items():
        if k == "observer":
            v = (ctypes.c_double * 3)(*v)
        setattr(g, k, v)
    return g


@pytest.mark.parametrize("kw,status", [
    (dict(n=100), 2),                    # no transform kernel for 100
    (dict(lmax=3), 1),                   # lmax must be 0, 2, 4
    (dict(nbins=12), 3),                 # 3 c = 3 * 24 >= 64
    (dict(k0=2.25), 1),                  # 2 k0 must be an integer
    (dict(nbins=0), 1),
    (dict(box=-1.0), 1),
    (dict(n=64, n_reduce=48), 2),        # 48 is not a supported size
    (dict(n=128, n_reduce=32, nbins=6), 3),  # c = 13: 3c >= 32
    (dict(los=2), 1),                    # los must be 0 or 1
    (dict(los=1, observer=(32.0, 32.0, 32.0)), 1),            # observer on a node: x_hat undefined
    (dict(los=1, interlace=1, observer=(31.5, 7.5, 0.5)), 1),  # on a node of the shifted grid
    (dict(los=1, observer=(float("nan"), 0.0, -100.0)), 1),
])
def test_plan_create_rejects_invalid_geometry(kw, status):
    with pytest.raises(B.BspError) as e:
        B.bsp_plan_create(_geom(**kw))
    assert e.value.status == status
    assert B.lib().bsp_last_error(None)


def test_plan_create_accepts_observer_off_the_nodes():
    """The same positions are fine where no node sits: half-integers without
    interlacing, outside the grid, or off the lattice in one coordinate (the
    check runs before any device work, so only its outcome is looked at)."""
    for kw in (dict(los=1, observer=(31.5, 7.5, 0.5)), dict(los=1, observer=(-32.0, 32.0, 32.0)),
               dict(los=1, interlace=1, observer=(32.0, 32.0, 32.25))):
        try:
            B.bsp_plan_destroy(B.bsp_plan_create(_geom(**kw)))
        except B.BspError as e:
            assert "observer" not in str(e), (kw, str(e))
        except Exception:  # no GPU here: plan creation stops at its first device call
            pass


def test_modal_basis_validation():
    import numpy as np
    modes = np.array([[0, 0, 0], [0, 2, 1]], np.int32)  # second is not sorted
    pf = np.ones(2000)
    b = B.ModalBasis()
    b.P, b.nmodes, b.pfid_len = 3, 2, pf.size
    b.modes = modes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    b.pfid = pf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    with pytest.raises(B.BspError) as e:
        B.bsp_plan_create(_geom(), b)
    assert e.value.status == 1


@pytest.mark.parametrize("lang,std", [("c", "-std=c99"), ("c++", "-std=c++17")])
def test_header_compiles_on_its_own(lang, std):
    """include/bsp.h is a plain C header: it compiles alone as C and as C++ with
    every warning an error (a stray comment end or a C++-only construct fails)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    header = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "bsp.h")
    r = subprocess.run([gcc, "-x", lang, std, "-fsyntax-only", "-Wall", "-Wextra", "-Werror", header],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
