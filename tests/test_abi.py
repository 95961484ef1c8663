"""The C ABI on the CPU: the library loads, exports every declared function,
and its host-side logic (defaults, validation, geometry, allocation failure)
behaves as documented.  No compute call is made here."""
import ctypes
import os

import pytest


@pytest.fixture(scope="module")
def B():
    from paper_2205_03133_amd import bdis, build
    if not os.path.exists(bdis.LIB_PATH):
        build.build()
    bdis.lib()
    return bdis


def test_exports_every_declared_function(B):
    names = B.header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(B.lib(), n), n


def test_defaults_follow_paper(B):
    p = B.params()
    assert (p.patch, p.stride, p.iters) == (10, 4, 12)
    assert p.sigma_s == 4.0 and p.valid_ratio == 0.75 and p.sigma_r_dynamic == 1
    assert abs(p.var_fit_thresh - 0.1) < 1e-7
    assert list(p.level_weight) == [float(2 ** n) for n in range(8)]
    assert B.check(p) == B.OK


@pytest.mark.parametrize("kw", [dict(patch=2), dict(patch=17), dict(stride=0), dict(stride=11),
                                dict(iters=0), dict(levels=0), dict(levels=9), dict(sigma_s=0.0),
                                dict(sigma_r=-1.0), dict(finest_level=5), dict(finest_level=-1), dict(float_pyramid=2),
                                dict(level_weight=[0.0] * 8), dict(sigma_s=float("nan")), dict(fusion=3),
                                dict(fusion=-1), dict(propagate=2), dict(valid_ratio=0.0),
                                dict(valid_ratio=-0.5), dict(valid_ratio=1.25), dict(valid_ratio=float("inf"))])
def test_bad_params_rejected(B, kw):
    assert B.check(B.params(**kw)) == B.E_ARG


def test_level_dims(B):
    p = B.params(levels=6, patch=12, stride=4)
    dims = [B.level_dims(p, 1920, 1080, n) for n in range(6)]
    assert dims[0] == (1920, 1080, 478, 268)
    assert dims[5][:2] == (60, 34)
    assert sum(d[2] * d[3] for d in dims) == 169913
    with pytest.raises(B.BdisError) as e:
        B.level_dims(B.params(levels=6, patch=12, stride=4), 300, 200, 0)
    assert e.value.code == B.E_SIZE


def test_create_validation_before_any_device_call(B, monkeypatch):
    h = ctypes.c_void_p()
    p = B.params(levels=3, patch=8, stride=4)
    assert B.lib().bdis_create(None, ctypes.byref(p), 64, 64, 1, 0) == B.E_ARG
    assert B.lib().bdis_create(ctypes.byref(h), ctypes.byref(B.params(patch=1)), 64, 64, 1, 0) == B.E_ARG
    assert B.lib().bdis_create(ctypes.byref(h), ctypes.byref(p), 20, 20, 1, 0) == B.E_SIZE
    assert B.lib().bdis_create(ctypes.byref(h), ctypes.byref(p), 64, 64, 0, 0) == B.E_ARG
    monkeypatch.setenv("BDIS_FAULT", "alloc")
    assert B.lib().bdis_create(ctypes.byref(h), ctypes.byref(p), 64, 64, 1, 0) == B.E_NOMEM
    assert b"BDIS_FAULT" in B.lib().bdis_last_error(None)
    assert not h.value


def test_static_entry_validation_before_any_device_call(B):
    L = B.lib()
    p = B.params(levels=6, patch=8, stride=3, iters=16, variance=1)
    fake = 1  # never dereferenced: every case below is refused on the host
    assert L.bdis_compute_static(None, fake, fake, 64, 64, 64, fake, None, None, None) == B.E_ARG
    assert L.bdis_compute_static(ctypes.byref(p), None, fake, 64, 64, 64, fake, None, None, None) == B.E_ARG
    assert L.bdis_compute_static(ctypes.byref(p), fake, fake, 64, 64, 63, fake, None, None, None) == B.E_ARG
    assert L.bdis_compute_static(ctypes.byref(B.params(variance=0)), fake, fake, 640, 480, 640, fake, fake, None,
                                 None) == B.E_ARG
    assert L.bdis_compute_static(ctypes.byref(p), fake, fake, 40, 40, 40, fake, None, None, None) == B.E_SIZE
    assert L.bdis_compute_static(ctypes.byref(p), fake, fake, 3840, 2160, 3840, fake, None, None, None) == \
        B.E_CAPACITY
    assert b"static scratch" in L.bdis_last_error(None)


def test_null_context_calls(B):
    assert B.lib().bdis_compute(None, None, None, 1, 1, 1, None, None, None, None) == B.E_ARG
    assert B.lib().bdis_compute_batch(None, 0, None, None) == B.E_ARG
    assert B.lib().bdis_compute_f32(None, None, None, 1, 1, 1, None, None, None, None) == B.E_ARG
    assert B.lib().bdis_backward(None, None, None, None, None, None, None) == B.E_ARG
    h = ctypes.c_void_p()
    assert B.lib().bdis_create(ctypes.byref(h), ctypes.byref(B.params()), 64, 64, 1, 4) == B.E_ARG
    B.lib().bdis_destroy(None)
    assert B.lib().bdis_version().startswith(b"bdis")


def test_product_path_has_no_fallback():
    """The binding never imports the oracle and refuses to run without the library."""
    import importlib
    import sys
    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "paper_2205_03133_amd", "bdis.py")).read()
    assert "oracle" not in src
    assert "raise RuntimeError" in src


def test_smoke_parameters_are_valid(B):
    """The smoke pass's parameters build on both sides (library and oracle)."""
    import __graft_entry__ as ge
    from oracle import ref
    kw = ge.smoke_params()
    assert B.check(B.params(**kw)) == B.OK
    assert ref.default_params(**kw)["variance"] == 1
