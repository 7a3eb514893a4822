"""The C-ABI library loads and exports every symbol include/oecdg.h declares;
host-only argument checks (no GPU needed: nothing here launches a kernel)."""
import ctypes as C
import math
import os
import re

import pytest

from paper_2503_12473_amd import _lib
from paper_2503_12473_amd.api import make_desc
from paper_2503_12473_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "oecdg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(oecdg_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_documented_entry_points():
    assert set(_declared()) == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_state_size_host_only():
    L = _lib.lib()
    prob = inputs.Problem1D(k=2, nc=3, flux=inputs.FLUX_EULER, bc=inputs.BC_OUTFLOW, n=100, xlo=0.0, xhi=1.0)
    d = make_desc(prob, 0.15)
    npr, ndu = C.c_int64(), C.c_int64()
    assert L.oecdg_state_size(C.byref(d), C.byref(npr), C.byref(ndu)) == 0
    assert (npr.value, ndu.value) == (3 * 3 * 100, 3 * 3 * 101)
    p2 = inputs.Problem2D(k=2, nc=4, flux=inputs.FLUX_EULER, nx=8, ny=6, xlo=0, xhi=1, ylo=0, yhi=1)
    d2 = make_desc(p2, 0.3)
    assert L.oecdg_state_size(C.byref(d2), C.byref(npr), C.byref(ndu)) == 0
    assert npr.value == ndu.value == 4 * 9 * 48


@pytest.mark.parametrize("field,value,code", [
    ("k", 4, _lib.EINVAL), ("nx", 1, _lib.EINVAL), ("cfl", 0.0, _lib.EINVAL), ("flux", 7, _lib.EINVAL),
    ("rk", 5, _lib.EINVAL), ("rk", -1, _lib.EINVAL), ("dim", 3, _lib.EINVAL), ("space", 2, _lib.EINVAL),
    ("flags", 2, _lib.EINVAL), ("bc", 4, _lib.EINVAL),
])
def test_invalid_descriptors_are_rejected_before_any_gpu_work(field, value, code):
    L = _lib.lib()
    prob = inputs.Problem1D(k=2, nc=1, flux=inputs.FLUX_ADVECTION, bc=inputs.BC_PERIODIC, n=64, xlo=0.0, xhi=1.0)
    d = make_desc(prob, 0.2)
    setattr(d, field, value)
    h = C.c_void_p()
    assert L.oecdg_init(C.byref(d), 1, None, C.byref(h)) == code
    assert not h.value
    npr, ndu = C.c_int64(), C.c_int64()
    assert L.oecdg_state_size(C.byref(d), C.byref(npr), C.byref(ndu)) == code


def test_2d_degrees():
    """2D handles take k = 1, 2, 3 (the paper's P^k and the tensor Q^k); k = 0 has
    no damping and no 2D kernel."""
    L = _lib.lib()
    npr, ndu = C.c_int64(), C.c_int64()
    for k, code in ((0, _lib.EUNSUPPORTED), (1, 0), (2, 0), (3, 0)):
        p2 = inputs.Problem2D(k=k, nc=1, flux=inputs.FLUX_ADVECTION, nx=8, ny=8, xlo=0, xhi=1, ylo=0, yhi=1)
        d2 = make_desc(p2, 0.3)
        assert L.oecdg_state_size(C.byref(d2), C.byref(npr), C.byref(ndu)) == code, k
        if code == 0:
            assert npr.value == ndu.value == (k + 1) ** 2 * 64


def test_descriptor_layout_matches_the_header():
    assert C.sizeof(_lib.Desc) == 104
    assert _lib.Desc.rk.offset == 92 and _lib.Desc.space.offset == 96


def test_2d_rk_methods():
    """2D handles take every RK method of eq:RKCDG that 1D takes; rk 5 is refused."""
    L = _lib.lib()
    p2 = inputs.Problem2D(k=2, nc=1, flux=inputs.FLUX_ADVECTION, nx=8, ny=8, xlo=0, xhi=1, ylo=0, yhi=1)
    npr, ndu = C.c_int64(), C.c_int64()
    for rk, code in ((0, 0), (1, 0), (2, 0), (3, 0), (4, 0), (5, _lib.EINVAL)):
        d2 = make_desc(p2, 0.3, rk=rk)
        assert L.oecdg_state_size(C.byref(d2), C.byref(npr), C.byref(ndu)) == code, rk


def test_batch_with_two_rk_methods_is_refused_before_any_gpu_work():
    L = _lib.lib()
    prob = inputs.Problem1D(k=2, nc=1, flux=inputs.FLUX_ADVECTION, bc=inputs.BC_PERIODIC, n=64, xlo=0.0, xhi=1.0)
    arr = (_lib.Desc * 2)(make_desc(prob, 0.2, rk=3), make_desc(prob, 0.2, rk=4))
    h = C.c_void_p()
    assert L.oecdg_init(arr, 2, None, C.byref(h)) == _lib.EUNSUPPORTED
    assert not h.value


def test_strerror_covers_every_code():
    L = _lib.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.oecdg_strerror(code).decode() != "unknown error"


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built library a solver handle cannot be made: the binding
    raises instead of computing anything another way."""
    from paper_2503_12473_amd import api, inputs
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(os.path.dirname(_lib.LIB_PATH), "missing", "liboecdg.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError, match="missing"):
        _lib.lib()
    prob, _, _ = inputs.advection_sine(16, 2)
    with pytest.raises(ImportError):
        api.OECDG(prob, 0.2)


def test_noalloc_host_checks():
    """oecdg_run_noalloc refuses bad arguments and oversized problems before it
    touches the device (the pointers below are never dereferenced)."""
    L = _lib.lib()
    prob = inputs.Problem1D(k=2, nc=3, flux=inputs.FLUX_EULER, bc=inputs.BC_OUTFLOW, n=100, xlo=0.0, xhi=1.0)
    d = make_desc(prob, 0.15)
    fake = C.c_void_p(16)
    assert L.oecdg_run_noalloc(None, None, fake, fake, 1.0, 1, 0.0, None, None) == _lib.EINVAL
    assert L.oecdg_run_noalloc(C.byref(d), None, None, fake, 1.0, 1, 0.0, None, None) == _lib.EINVAL
    assert L.oecdg_run_noalloc(C.byref(d), None, fake, fake, math.inf, -1, 0.0, None, None) == _lib.EINVAL
    bad = make_desc(prob, 0.15)
    bad.k = 5
    assert L.oecdg_run_noalloc(C.byref(bad), None, fake, fake, 1.0, 1, 0.0, None, None) == _lib.EINVAL
    p2 = inputs.Problem2D(k=2, nc=4, flux=inputs.FLUX_EULER, nx=8, ny=8, xlo=0, xhi=1, ylo=0, yhi=1)
    assert L.oecdg_run_noalloc(C.byref(make_desc(p2, 0.3)), None, fake, fake, 1.0, 1, 0.0, None, None) == \
        _lib.EUNSUPPORTED
    big = make_desc(prob, 0.15)
    big.nx = 200000
    assert L.oecdg_run_noalloc(C.byref(big), None, fake, fake, 1.0, 1, 0.0, None, None) == _lib.ETOOBIG
    assert "scratch" in L.oecdg_strerror(_lib.ETOOBIG).decode()
