"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and rejects invalid arguments on the host before any HIP
call (so these run without a GPU)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lc.h")


@pytest.fixture(scope="module")
def lc():
    from paper_2305_11998_amd import lc as mod
    return mod


def declared_entry_points():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lc_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_four_core_calls():
    names = declared_entry_points()
    for n in ("lc_build_rays", "lc_sweep", "lc_moments", "lc_step"):
        assert n in names


def test_library_exports_every_declared_symbol(lc):
    lib = C.CDLL(lc.LIB_PATH)
    for name in declared_entry_points():
        assert hasattr(lib, name), name
    assert set(declared_entry_points()) <= set(lc.EXPORTED)
    assert lc.lc_version() >= 10000


def _quad(n_az=8, n_pol=2):
    import workloads as W
    return W.product_quadrature(n_az, n_pol)


@pytest.mark.parametrize("kw,needle", [
    (dict(nx=0), "nx, ny"),
    (dict(lx=-1.0), "lx, ly"),
    (dict(h_moc=0.0), "h_moc"),
    (dict(h_moc=float("nan")), "h_moc"),
    (dict(mode=7), "ray mode"),
    (dict(n_az=7), "n_az"),
    (dict(mu_bad=True), "mu"),
    (dict(axis=True), "parallel"),
    (dict(unpaired=True), "pi"),
    (dict(n_pol=9), "n_pol"),
])
def test_build_rays_rejects_bad_arguments(lc, kw, needle):
    nx, ny, lx = kw.get("nx", 4), 4, kw.get("lx", 1.0)
    n_az, n_pol = kw.get("n_az", 8), kw.get("n_pol", 2)
    if n_az % 2:
        phi = np.linspace(0.1, 6.0, n_az)
        mu, om = np.array([-0.5, 0.5]), np.ones(n_az * 2)
    else:
        phi, mu, om = _quad(n_az, min(n_pol, 8))
        if n_pol > 8:
            mu = np.linspace(-0.9, 0.9, n_pol)
            om = np.ones(n_az * n_pol)
    if kw.get("mu_bad"):
        mu = mu.copy(); mu[0] = 1.0
    if kw.get("axis"):
        phi = phi.copy(); phi[0] = 0.0; phi[n_az // 2] = math.pi
    if kw.get("unpaired"):
        phi = phi.copy(); phi[n_az // 2] += 0.1
    with pytest.raises(lc.LcError) as e:
        lc.lc_build_rays(nx, ny, lx, 1.0, phi, mu, om, kw.get("h_moc", 0.1), kw.get("mode", 0), stream=0)
    assert e.value.status == lc.LC_ERR_ARG
    assert needle in str(e.value)


def test_invalid_handles_are_rejected(lc):
    lib = C.CDLL(lc.LIB_PATH)
    lib.lc_state_bytes.restype = C.c_size_t
    lib.lc_state_bytes.argtypes = [C.c_void_p]
    assert lib.lc_state_bytes(None) == 0
    bogus = (C.c_uint32 * 64)()
    assert lc._lib.lc_plan_free(C.cast(bogus, C.c_void_p)) == lc.LC_ERR_STATE
    assert lc._lib.lc_rays_free(C.cast(bogus, C.c_void_p)) == lc.LC_ERR_STATE
    assert lc._lib.lc_sweep(None, None, None, 1.0, None, None, None, None, None) == lc.LC_ERR_STATE
    assert lc._lib.lc_step(C.cast(bogus, C.c_void_p), 1, None, None, 0, 1.0, 1.0, None, None, None,
                           None, None, None, None, None, None) == lc.LC_ERR_STATE
    # freeing NULL is a no-op
    assert lc._lib.lc_rays_free(None) == lc.LC_OK
    assert lc._lib.lc_plan_free(None) == lc.LC_OK


def test_out_pointer_required(lc):
    phi, mu, om = _quad()
    g = lc.lc_grid(4, 4, 1.0, 1.0)
    dp = C.POINTER(C.c_double)
    q = lc.lc_quad(len(phi), len(mu), phi.ctypes.data_as(dp), mu.ctypes.data_as(dp), om.ctypes.data_as(dp))
    assert lc._lib.lc_build_rays(C.byref(g), C.byref(q), 0.1, 0, None, None) == lc.LC_ERR_ARG
    assert b"out" in lc._lib.lc_last_error()


def test_grey_closures_dims_rejects_bad_sizes(lc):
    nul = (None,) * 7
    assert lc._lib.lc_grey_closures_dims(0, 4, *nul) == lc.LC_ERR_ARG
    assert b"cells and G" in lc._lib.lc_last_error()
    assert lc._lib.lc_grey_closures_dims(5, 0, *nul) == lc.LC_ERR_ARG
    assert lc._lib.lc_grey_closures_dims(5, 3, *nul) == lc.LC_ERR_ARG
    assert b"NULL" in lc._lib.lc_last_error()
