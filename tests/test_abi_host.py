"""C ABI checks that need no GPU: the library loads, exports every entry
point declared in include/bh.h, its host tables match the oracle, and bad
arguments are rejected with the documented codes."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import basis
from paper_2509_01180_amd import _lib, api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bh.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bh_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 12
    L = _lib.lib()
    for n in names:
        assert hasattr(L, n), n
        assert n in _lib.SIGNATURES, f"{n} not bound in the Python layer"


@pytest.mark.parametrize("L", [0, 1, 4, 8, 16, 24, 32, 42])
def test_index_tables_match_oracle(L):
    idx = basis.IndexSet(L)
    assert api.index_size(L) == idx.size
    l, k, m, lam = api.index_table(L)
    np.testing.assert_array_equal(l, idx.l)
    np.testing.assert_array_equal(k, idx.k)
    np.testing.assert_array_equal(m, idx.m)
    np.testing.assert_allclose(lam, idx.lam, rtol=1e-13)
    rl, rk, rlam, rc = api.radial_table(L)
    assert len(rl) == len(idx.radial)
    np.testing.assert_allclose(rc, [e[3] for e in idx.radial], rtol=1e-12)


@pytest.mark.parametrize("N", [2, 7, 16, 32, 33, 64, 96])
def test_ball_voxels(N):
    _h, _x, ball = basis.grid(N)
    assert api.ball_voxels(N) == int(ball.sum())


def test_error_codes():
    L = _lib.lib()
    assert L.bh_index_size(-1) == _lib.BH_EINVAL
    assert L.bh_index_size(_lib.BH_MAX_L + 1) == _lib.BH_EINVAL
    assert b"bandlimit" in L.bh_last_error()
    assert L.bh_ball_voxels(0) == _lib.BH_EINVAL
    assert L.bh_plan_create(32, 8, 0, None) == _lib.BH_EINVAL
    h = ctypes.c_void_p()
    assert L.bh_plan_create(1, 8, 0, ctypes.byref(h)) == _lib.BH_EINVAL
    assert L.bh_plan_create(32, -1, 0, ctypes.byref(h)) == _lib.BH_EINVAL
    # calls on a NULL plan
    assert L.bh_expand(None, None, 1, None, None) == _lib.BH_EINVAL
    assert L.bh_plan_num_coeffs(None, 0) == _lib.BH_EINVAL
    assert L.bh_expand_ex(None, None, 1, 0, None, None, None) == _lib.BH_EINVAL
    assert L.bh_expand_rows(None, None, 4, None, 1, 0, None, 0, None, None) == _lib.BH_EINVAL
    assert L.bh_correlate_hess(None, None, None, 1, 0, None, 1, None, None, None, None) == _lib.BH_EINVAL
    assert L.bh_degree_energy(None, None, None, 1, 0, None, None) == _lib.BH_EINVAL
    o = _lib.AlignOpts()
    assert L.bh_align_t(None, None, None, 1, None, 1, ctypes.byref(o), None, None, None, None,
                        None, None) == _lib.BH_EINVAL
    L.bh_plan_destroy(None)   # accepted
    with pytest.raises(_lib.BhError):
        api.index_size(-3)
