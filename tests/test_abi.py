"""Host-side tests of the C ABI: the library loads, exports every declared symbol,
and rejects bad arguments before any device work (no GPU needed)."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cuth.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cuth_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2606_17850_amd import _lib
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_2606_17850_amd import _lib
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTED)


def test_default_options(lib):
    from paper_2606_17850_amd import _lib
    o = _lib.Options()
    lib.cuth_default_options(ctypes.byref(o))
    assert o.precision == _lib.CUTH_MIXED and o.tol == 0.0
    assert o.cheb_degree == 30 and o.lanczos_steps == 30
    assert o.preconditioner == 0 and o.storage == 0
    # the ctypes mirror has the header's size (no field missing or misplaced)
    assert ctypes.sizeof(_lib.Options) == 48


def _desc(nx=4, ny=3, nz=2, dx=1e-3, dy=1e-3, dz=(1e-3, 1e-3), kl=(1.0, 2.0), kv=(1.0, 2.0),
          cap=None, h_top=10.0, h_bottom=0.0, t_amb=300.0):
    from paper_2606_17850_amd import _lib
    keep = []

    def arr(x):
        a = np.ascontiguousarray(x, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data_as(_lib.c_double_p)

    d = _lib.GridDesc()
    d.nx, d.ny, d.nz = nx, ny, nz
    d.dx, d.dy = dx, dy
    d.dz = arr(dz) if dz is not None else None
    d.k_lat = arr(kl) if kl is not None else None
    d.k_vert = arr(kv) if kv is not None else None
    d.k_lat_mult = None
    d.heat_cap = arr(cap) if cap is not None else None
    d.h_top, d.h_bottom, d.t_amb = h_top, h_bottom, t_amb
    return d, keep


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-1), dict(nz=65, dz=[1e-3] * 65, kl=[1.0] * 65, kv=[1.0] * 65),
    dict(dx=0.0), dict(dy=math.nan), dict(dz=(1e-3, -1e-3)), dict(kl=(1.0, 0.0)),
    dict(kv=(math.inf, 1.0)), dict(h_top=-1.0), dict(h_bottom=math.nan),
    dict(t_amb=math.inf), dict(cap=(1e6, -1.0)), dict(dz=None),
])
def test_create_rejects_bad_descriptor(lib, bad):
    from paper_2606_17850_amd import _lib
    d, keep = _desc(**bad)
    h = ctypes.c_void_p()
    st = lib.cuth_grid_create(ctypes.byref(d), None, ctypes.byref(h))
    assert st == _lib.CUTH_E_INVALID
    assert h.value is None
    assert len(lib.cuth_last_error()) > 0


def test_null_handles_are_rejected(lib):
    from paper_2606_17850_amd import _lib
    st = _lib.Stats()
    assert lib.cuth_solve(None, None, None, None, ctypes.byref(st)) == _lib.CUTH_E_INVALID
    assert lib.cuth_transient_step(None, 1.0, None, None, None, None, None) == _lib.CUTH_E_INVALID
    assert lib.cuth_adjoint(None, None, None, None, None, None, None) == _lib.CUTH_E_INVALID
    assert lib.cuth_apply(None, 0.0, 0, None, None) == _lib.CUTH_E_INVALID
    assert lib.cuth_solve_batch(0, None, 1, None, None, None, None) == _lib.CUTH_OK
    assert lib.cuth_solve_batch(-1, None, 1, None, None, None, None) == _lib.CUTH_E_INVALID
    lib.cuth_grid_destroy(None)
    assert lib.cuth_grid_create(None, None, None) == _lib.CUTH_E_INVALID


def test_package_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2606_17850_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


def test_precision_names_match_header(lib):
    """The binding's precision table equals the header's enum, and an unknown
    name is refused instead of falling back to another precision."""
    import re

    import paper_2606_17850_amd as cuth
    from paper_2606_17850_amd import _lib
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "cuth.h")).read()
    enum = dict((k, int(v)) for k, v in
                re.findall(r"(CUTH_FP64|CUTH_FP32|CUTH_MIXED16|CUTH_MIXED|CUTH_ADAPTIVE)\s*=\s*(\d+)", hdr))
    assert enum == {"CUTH_FP64": _lib.CUTH_FP64, "CUTH_MIXED": _lib.CUTH_MIXED,
                    "CUTH_MIXED16": _lib.CUTH_MIXED16, "CUTH_ADAPTIVE": _lib.CUTH_ADAPTIVE,
                    "CUTH_FP32": _lib.CUTH_FP32}
    assert cuth.options("fp32").precision == enum["CUTH_FP32"]
    auto = re.search(r"#define\s+CUTH_DEGREE_AUTO\s+\((-?\d+)\)", hdr)
    assert auto and int(auto.group(1)) == _lib.CUTH_DEGREE_AUTO
    assert cuth.options(cheb_degree="auto").cheb_degree == _lib.CUTH_DEGREE_AUTO
    assert cuth.options("mixed16").precision == enum["CUTH_MIXED16"]
    assert cuth.options("fp64").precision == enum["CUTH_FP64"]
    with pytest.raises(ValueError):
        cuth.options("fp16")


def _struct_fields(name):
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", text).group(1)
    return [f for decl in body.split(";") if decl.strip()
            for f in re.findall(r"\*?\s*([a-z_0-9]+)\s*(?:,|$)", decl.strip().split(None, 1)[1])]


def test_ctypes_mirrors_match_header_structs():
    """Field names and order of the ctypes mirrors equal the header's structs
    (a field added on one side only would shift every later field)."""
    from paper_2606_17850_amd import _lib
    for cls, name in ((_lib.Stats, "cuth_stats"), (_lib.Options, "cuth_options"),
                      (_lib.GridDesc, "cuth_grid_desc")):
        assert [f for f, _ in cls._fields_] == _struct_fields(name), name
    assert ctypes.sizeof(_lib.Stats) == 88
