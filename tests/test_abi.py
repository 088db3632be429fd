"""The C ABI library loads, exports every entry point include/wamct.h declares, and
rejects bad geometry on the host (no GPU needed for any of this)."""
import ctypes
import math
import os
import re

import pytest

from paper_1508_04458_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wamct.h")


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:wamct_status|const char\*)\s+(wamct_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1508_04458_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib.lib, name), name
    assert set(names) == set(lib.SYMBOLS)


def test_version(lib):
    assert lib.lib.wamct_version().startswith(b"wamct")


def _valid():
    return synth.fan_geometry(64, 30, 96)


@pytest.mark.parametrize("change,levels,dtype,needle", [
    (dict(n=1), 1, "f32", "image size"),
    (dict(n=10), 2, "f32", "divisible"),
    (dict(pixel=0.0), 1, "f32", "pixel"),
    (dict(n_views=0), 1, "f32", "n_views"),
    (dict(bin_pitch=-1.0), 1, "f32", "pitch"),
    (dict(sod=40.0), 1, "f32", "circumradius"),
    (dict(sdd=500.0), 1, "f32", "sdd"),
    (dict(kind=7), 1, "f32", "kind"),
    (dict(angle0=math.inf), 1, "f32", "finite"),
    ({}, 9, "f32", "levels"),
    ({}, -1, "f32", "levels"),
    ({}, 1, "f16", "dtype"),
    ({}, 1, "f64/f32", "at least"),
])
def test_validation_rejects(lib, change, levels, dtype, needle):
    import dataclasses
    from paper_1508_04458_amd import api
    g = dataclasses.replace(_valid(), **change)
    dtype, _, geometry = dtype.partition("/")
    msg = api.validate(g, levels, dtype, geometry or "f64")
    assert msg is not None and needle in msg, msg


def test_validation_accepts_configs(lib):
    from paper_1508_04458_amd import api
    for name, cfg in synth.CONFIGS.items():
        assert api.validate(cfg["geom"](), cfg["levels"], cfg["dtype"]) is None, name
        assert api.validate(cfg["geom"](), 0, "f64") is None, name
        assert api.validate(cfg["geom"](), 0, "f32", "f32") is None, name


def test_create_rejects_invalid_geometry_before_touching_the_gpu(lib):
    g = lib.Geometry(1, 64, 1.0, 30, 0.0, 6.0, 96, 1.0, 10.0, 20.0)   # sod inside the image
    opt = lib.Options(1, lib.F32, lib.F64)
    h = ctypes.c_void_p()
    st = lib.lib.wamct_create(ctypes.byref(g), ctypes.byref(opt), None, ctypes.byref(h))
    assert st == lib.E_INVALID and not h.value
    assert b"circumradius" in lib.lib.wamct_last_error(None)
    assert lib.lib.wamct_create(ctypes.byref(g), ctypes.byref(opt), None, None) == lib.E_INVALID
    assert lib.lib.wamct_iterate(None, 1, None) == lib.E_INVALID


@pytest.mark.parametrize("change,levels,dtype,batch,needle", [
    (dict(n=1024), 2, "f32", 1, "outside [2, 512]"),
    (dict(nz=0), 2, "f32", 1, "nz"),
    (dict(nz=12), 3, "f32", 1, "divisible"),
    (dict(n_rows=0), 2, "f32", 1, "n_rows"),
    (dict(row_pitch=0.0), 2, "f32", 1, "pitch"),
    (dict(sod=20.0), 2, "f32", 1, "circumradius"),
    (dict(sdd=50.0), 2, "f32", 1, "sdd"),
    ({}, 5, "f32", 1, "levels"),
    ({}, 2, "f32/f32", 1, "FP64 only"),
    ({}, 2, "f32", 2, "one scan"),
])
def test_cone_validation_rejects(lib, change, levels, dtype, batch, needle):
    import dataclasses
    from paper_1508_04458_amd import api
    g = dataclasses.replace(synth.CONE_CONFIGS["cone32"]["geom"](), **change)
    dtype, _, geometry = dtype.partition("/")
    msg = api.validate(g, levels, dtype, geometry or "f64", batch)
    assert msg is not None and needle in msg, msg


def test_cone_validation_accepts_configs(lib):
    from paper_1508_04458_amd import api
    for name, cfg in synth.CONE_CONFIGS.items():
        assert api.validate(cfg["geom"](), cfg["levels"], "f32") is None, name
        assert api.validate(cfg["geom"](), 0, "f64") is None, name


def test_idiv_noalloc_rejects_bad_sizes_on_the_host(lib):
    """Every rejection happens before any HIP call (so it runs without a GPU)."""
    L = lib.lib
    x = ctypes.c_void_p(16)    # never dereferenced: the calls fail validation first
    too_many = (1 << 20) * 256 + 1
    for args in ((lib.F32, too_many, 1, x, x, x), (lib.F32, 0, 1, x, x, x), (lib.F64, 1 << 31, 1, x, x, x),
                 (lib.F32, 4, 0, x, x, x), (lib.F32, 4, 65536, x, x, x), (5, 4, 1, x, x, x),
                 (lib.F32, 4, 1, None, x, x), (lib.F32, 4, 1, x, None, x), (lib.F32, 4, 1, x, x, None),
                 (lib.F32, 256 * 4096, 257, x, x, x)):
        assert L.wamct_idiv_noalloc(*args, None) == lib.E_INVALID, args
    assert b"static buffer" in L.wamct_last_error(None)


def test_d4_validation_on_the_host(lib):
    """Daubechies-4 options: accepted for 2-D scans with n >> levels >= 4; rejected (with the
    reason) for levels 0, wrapping supports, stacks, the cone beam and unknown families."""
    from paper_1508_04458_amd import api
    fan = synth.fan_geometry(96, 75, 131)
    assert api.validate(fan, 3, "f32", wavelet="d4") is None
    assert api.validate(synth.parallel_geometry(64, 90, 96, 1.0), 4, "f64", wavelet="d4") is None
    for args, kw, needle in (((fan, 0, "f32"), {}, "levels >= 1"),
                             ((synth.parallel_geometry(64, 90, 96, 1.0), 5, "f32"), {}, "n >> levels >= 4"),
                             ((fan, 2, "f32", "f64", 2), {}, "one scan per context"),
                             ((synth.CONE_CONFIGS["cone32"]["geom"](), 1, "f32"), {}, "only the Haar basis")):
        msg = api.validate(*args, wavelet="d4", **kw)
        assert msg is not None and needle in msg, msg
    assert "unknown wavelet" in api.validate(fan, 2, "f32", wavelet="coiflet")
