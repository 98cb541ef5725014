"""The C-ABI library builds, loads and exports every entry point that
include/agf2.h declares (no compute: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "agf2.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(agf2_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2106_03508_amd import agf2, build
    if not os.path.exists(agf2.LIB_PATH):
        build.build(verbose=False)
    return ctypes.CDLL(agf2.LIB_PATH)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("agf2_build_moments", "agf2_compress", "agf2_fock_loop", "agf2_energy_gf",
              "agf2_create", "agf2_destroy", "agf2_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_2106_03508_amd import agf2
    assert set(declared_functions()) <= set(agf2.SIGNATURES)


def test_null_handle_is_rejected(lib):
    lib.agf2_last_error.restype = ctypes.c_char_p
    lib.agf2_last_error.argtypes = [ctypes.c_void_p]
    assert b"NULL" in lib.agf2_last_error(None)
    lib.agf2_destroy.argtypes = [ctypes.c_void_p]
    assert lib.agf2_destroy(None) == -1


def test_run_state_size(lib):
    """The checkpoint size of agf2_run is a host-side formula: header plus
    the saved arrays (poles, density, previous moments, DIIS history)."""
    from paper_2106_03508_amd import agf2
    lib = agf2.load_library()
    for n, sp, nb in ((24, 8, 1), (30, 3, 2)):
        nn = n * n
        npmax = n * (1 + 2 * nb)
        ln = 4 * nb * nn
        doubles = npmax + n * npmax + nn + ln + ln + sp * 2 * ln + sp * sp
        o = agf2.run_opts(diis_space=sp, nblock=nb)
        b = lib.agf2_run_state_bytes(n, ctypes.byref(o))
        assert 0 < b - 8 * doubles <= 512
    assert lib.agf2_run_state_bytes(0, None) == -1
    assert lib.agf2_run_state_bytes(10, ctypes.byref(agf2.run_opts(diis_space=65))) == -1
    assert lib.agf2_run_state_bytes(10, ctypes.byref(agf2.run_opts(nblock=0))) == -1
