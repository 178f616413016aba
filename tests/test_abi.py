"""The C-ABI library loads, exports every symbol the header declares, and
rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1510_01831_amd import hz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    txt = open(os.path.join(ROOT, "include", "hz.h")).read()
    return sorted(set(re.findall(r"\b(hz_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_header_symbols():
    if not os.path.exists(hz.LIB_PATH):
        pytest.skip("libhz.so not built")
    L = hz.lib()
    syms = _header_symbols()
    assert "hz_setup" in syms and "hz_solve" in syms
    for name in syms:
        assert hasattr(L, name), name
    assert set(hz.EXPORTED) == set(syms)


def test_status_strings():
    if not os.path.exists(hz.LIB_PATH):
        pytest.skip("libhz.so not built")
    L = hz.lib()
    for code in (hz.HZ_OK, hz.HZ_EINVAL, hz.HZ_ENOMEM, hz.HZ_ESTATE, hz.HZ_ENOCONV,
                 hz.HZ_ESINGULAR, hz.HZ_EDEVICE):
        assert L.hz_strerror(code)


@pytest.mark.parametrize("change", [
    dict(n_z=100), dict(h=0.5), dict(omega=0.0), dict(omega=float("nan")), dict(n_pml=-1),
    dict(layers=0), dict(layers=64), dict(cells=0), dict(cells=64), dict(precision=7),
    dict(model_kind=5), dict(inner=5), dict(inner=1, precision=1), dict(inner=1, krylov=1),
    dict(inner=1, n_pml=0), dict(inner=1, inner_tol=2.0), dict(n_pml=0),
    dict(n_pml=0, layers=1, cells=2)])
def test_setup_rejects_bad_parameters_before_device_work(change):
    if not os.path.exists(hz.LIB_PATH):
        pytest.skip("libhz.so not built")
    L = hz.lib()
    n = 63
    base = dict(n_x=n, n_z=n, h=1.0 / (n + 1), omega=30.0, n_pml=8, pml_beta=2.0, layers=4,
                cells=2, precision=0, model_kind=0, max_batch=1)
    base.update(change)
    prm = hz.Params(**base)
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(16)          # never dereferenced: validation fails first
    st = L.hz_setup(fake, ctypes.byref(prm), ctypes.byref(ctx))
    assert st == hz.HZ_EINVAL
    assert ctx.value is None
    assert L.hz_last_error()


def test_null_arguments():
    if not os.path.exists(hz.LIB_PATH):
        pytest.skip("libhz.so not built")
    L = hz.lib()
    assert L.hz_setup(None, None, None) == hz.HZ_EINVAL
    assert L.hz_factor(None) == hz.HZ_EINVAL
    assert L.hz_solve(None, None, 1, None, 1e-10, 10, None, None) == hz.HZ_EINVAL
