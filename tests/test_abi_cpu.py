"""Host-side checks of the C ABI (no GPU needed): every symbol declared in
include/wcamg.h is exported by libwcamg.so, and argument validation rejects
bad input before any device call."""
import ctypes
import os
import re

import pytest

from paper_2111_05012_amd import wcamg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'wcamg.h')


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r'/\*.*?\*/', '', txt, flags=re.S)
    return sorted(set(re.findall(r'\b(wcamg_[a-z_A-Z0-9]+)\s*\(', txt)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ('wcamg_create', 'wcamg_load_gauge', 'wcamg_apply_D', 'wcamg_setup', 'wcamg_solve',
                 'wcamg_destroy'):
        assert name in syms


def test_library_exports_every_declared_symbol():
    lib = wcamg.load_library()
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    # the binding declares exactly the header's entry points
    assert sorted(wcamg.SIGNATURES) == declared_symbols()


def _lat(dims=(4, 4, 4, 4), block=(2, 2, 2, 2), bc=(1, 1, 1, -1), kappa=0.12, csw=1.0):
    return wcamg.Lattice(wcamg._c_int4(*dims), wcamg._c_int4(*block), wcamg._c_int4(*bc), kappa, csw)


@pytest.mark.parametrize('kw', [dict(dims=(4, 4, 3, 4)), dict(dims=(4, 4, 0, 4)), dict(block=(3, 2, 2, 2)),
                                dict(block=(0, 2, 2, 2)), dict(bc=(1, 1, 1, 0)), dict(kappa=float('nan')),
                                dict(dims=(64, 64, 64, 64), block=(8, 8, 8, 8))])
def test_create_rejects_invalid_lattice(kw):
    lib = wcamg.load_library()
    h = ctypes.c_void_p()
    lat = _lat(**kw)
    assert lib.wcamg_create(ctypes.byref(h), ctypes.byref(lat), None) == wcamg.EINVAL
    assert not h.value


def test_null_arguments():
    lib = wcamg.load_library()
    h = ctypes.c_void_p()
    assert lib.wcamg_create(ctypes.byref(h), None, None) == wcamg.EINVAL
    assert lib.wcamg_create(None, ctypes.byref(_lat()), None) == wcamg.EINVAL
    assert lib.wcamg_apply_D(None, None, None, 1, 0, 0) == wcamg.EINVAL
    assert lib.wcamg_solve(None, None, None, 1, None, None) == wcamg.EINVAL
    lib.wcamg_destroy(None)
    assert lib.wcamg_last_error(None) == b'null context'


def test_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(FileNotFoundError):
        wcamg._lib_backup = wcamg._lib
        wcamg._lib = None
        try:
            wcamg.load_library(str(tmp_path / 'missing.so'))
        finally:
            wcamg._lib = wcamg._lib_backup
