"""C-ABI contract checks that need no GPU: the library loads, exports every
function its headers declare, and rejects invalid geometries and arguments
on the host before touching the device."""
import ctypes
import glob
import math
import os
import re

import numpy as np

import pytest

from paper_2512_21180_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cb():
    from paper_2512_21180_amd import cbct
    return cbct


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(cbct_\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_function(cb):
    names = declared_functions()
    assert "cbct_forward" in names and "cbct_batch_adjoint" in names
    lib = ctypes.CDLL(cb.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_error_strings(cb):
    lib = cb.lib()
    for code in range(-7, 1):
        s = lib.cbct_error_string(code).decode()
        assert s and s != "unknown status"
    assert lib.cbct_error_string(-99).decode() == "unknown status"


def _create(cb, g):
    desc, keep = cb.make_desc(g)
    h = ctypes.c_void_p()
    st = cb.lib().cbct_geom_create(ctypes.byref(desc), ctypes.byref(h))
    del keep
    return st, h


BAD = {
    "sdd_not_beyond_sid": dict(sdd=900.0),
    "zero_angles": dict(n_angles=0),
    "negative_pitch": dict(du=-0.8),
    "zero_voxel_pitch": dict(vz=0.0),
    "zero_columns": dict(nu=0),
    "nan_offset": dict(off_u=float("nan")),
    "volume_reaches_panel": dict(nx=400, ny=400),          # 802 mm wide at 2 mm > 2*536
    "volume_off_centre": dict(origin=(400.0, 0.0, 0.0)),
    "cone_too_steep": dict(nv=5000, dv=1.0),              # |d_z| > |d_xy| at the panel edge
    "too_many_elements": dict(n_angles=100000),
}


@pytest.mark.parametrize("name", sorted(BAD))
def test_invalid_geometry_rejected_on_host(cb, name):
    g = W.scaled(W.C2, **BAD[name])
    st, h = _create(cb, g)
    assert st == -2, (name, st)
    assert not h.value


def test_non_finite_angle_rejected(cb):
    g = W.scaled(W.cropped(W.C1, n_angles=3), angles=[0.0, float("inf"), 1.0])
    st, _ = _create(cb, g)
    assert st == -2


def test_wide_fan_switching_axis_twice_rejected(cb):
    # a panel wide enough that one angle's columns cross two 45-degree
    # boundaries of the sampling axis
    g = W.geometry(4, 4000, 8, 1.0, 1.0, 16, 16, 16, 2.0, sid=1000.0, sdd=1536.0,
                   angles=[0.0, math.pi / 2, math.pi, 1.5 * math.pi])
    st, _ = _create(cb, g)
    assert st == -2


def test_null_arguments(cb):
    lib = cb.lib()
    h = ctypes.c_void_p()
    assert lib.cbct_geom_create(None, ctypes.byref(h)) == -1
    assert lib.cbct_forward(None, None, 0, None, 0, 1, None) == -1
    assert lib.cbct_adjoint(None, None, 0, None, 0, 1, None) == -1
    assert lib.cbct_sample_count(None, None) == -1
    assert lib.cbct_geom_destroy(None) == 0
    assert lib.cbct_batch_forward(0, None, None, None, 0, 0, None) == -4
    assert lib.cbct_batch_adjoint(1, None, None, None, 0, 0, None) == -1


def test_valid_geometry_passes_host_validation(cb):
    """A valid descriptor gets past validation: with a GPU it is created, on a
    host without one the first HIP call reports CBCT_E_HIP."""
    for g in (W.C1, W.C2, W.C4, *W.c3_geometries()):
        st, h = _create(cb, W.cropped(g, n_angles=4, nv=8))
        assert st in (0, -5), st
        if st == 0:
            assert cb.lib().cbct_geom_destroy(h) == 0


def test_poly_bins_are_the_papers(cb, oracle):
    """cbct_poly_bins (host only): the ten energy-bin centres and the
    detector response at them, as the oracle defines them."""
    c, r = cb.poly_bins()
    assert c.tolist() == oracle.energy_bins().tolist()
    np.testing.assert_allclose(r, oracle.detector_response(c), rtol=0, atol=1e-12)
    n = ctypes.c_int32()
    assert cb.lib().cbct_poly_bins(4, None, None, ctypes.byref(n)) == 0 and n.value == 10
    buf = (ctypes.c_double * 4)()
    assert cb.lib().cbct_poly_bins(4, buf, None, ctypes.byref(n)) == -4
