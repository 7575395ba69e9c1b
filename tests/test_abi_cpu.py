"""Host-side checks of the C ABI library: it loads without a GPU and exports
every function include/lsqr.h declares. No compute calls."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsqr.h")
LIB = os.path.join(ROOT, "paper_2308_00778_amd", "liblsqr.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(lsqr_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2308_00778_amd import build

        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lsqr_create", "lsqr_destroy", "lsqr_solve", "lsqr_aprod1", "lsqr_aprod2",
                     "lsqr_solve_refined", "lsqr_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_symbol_list_matches_header():
    import paper_2308_00778_amd as pkg

    assert sorted(pkg.SYMBOLS) == declared_functions()


def test_error_paths_without_gpu(lib):
    # argument checks that return before any HIP call
    lib.lsqr_last_error.restype = ctypes.c_char_p
    lib.lsqr_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    out = ctypes.c_void_p()
    assert lib.lsqr_create(None, ctypes.byref(out)) == -1
    assert b"null" in lib.lsqr_last_error()
    assert lib.lsqr_destroy(None) == 0
    lib.lsqr_set_option.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double]
    assert lib.lsqr_set_option(None, 1, 1.0) == -1


def test_descriptor_checks_without_gpu(lib):
    import paper_2308_00778_amd.lsqr as L

    L.load_library()
    d = L._System(n_rows=100, n_stars=1, n_astro=5, n_axes=2, n_par_axis=4, n_instr=6,
                  n_dfa=10, n_instr_cols=10, n_glob=1, value_type=0, precondition=1,
                  values=1, star_of_row=1, att_start=1, instr_idx=1, stream=None)
    h = ctypes.c_void_p()
    # an attitude section other than 3 axes x 4 parameters is not built
    assert L._lib.lsqr_create(ctypes.byref(d), ctypes.byref(h)) == L.LSQR_E_UNSUPPORTED
    d.n_axes = 3
    for field, bad in (("n_instr", 7), ("n_astro", 6), ("n_glob", 6), ("n_astro", -1)):
        good = getattr(d, field)
        setattr(d, field, bad)
        assert L._lib.lsqr_create(ctypes.byref(d), ctypes.byref(h)) == L.LSQR_E_INVALID
        setattr(d, field, good)
    d.n_astro, d.n_axes, d.n_instr, d.n_glob = 0, 0, 0, 0
    assert L._lib.lsqr_create(ctypes.byref(d), ctypes.byref(h)) == L.LSQR_E_INVALID
    d.n_astro, d.n_axes, d.n_instr, d.n_glob = 5, 3, 6, 1
    d.n_rows = 0
    assert L._lib.lsqr_create(ctypes.byref(d), ctypes.byref(h)) == L.LSQR_E_INVALID
    d.n_rows = 100
    d.values = None
    assert L._lib.lsqr_create(ctypes.byref(d), ctypes.byref(h)) == L.LSQR_E_INVALID
    d.values = 1
    d.n_dfa = 3
    assert L._lib.lsqr_create(ctypes.byref(d), ctypes.byref(h)) == L.LSQR_E_INVALID
    d.n_dfa = 10
    d.value_type = 7
    assert L._lib.lsqr_create(ctypes.byref(d), ctypes.byref(h)) == L.LSQR_E_INVALID
