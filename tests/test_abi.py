"""The C ABI library loads and exports every function include/adiwave.h declares;
argument validation that happens before any device work, checked on the CPU."""
import ctypes

import pytest

from paper_2006_10142_amd import _lib


def test_header_declares_the_boundary():
    names = _lib.header_functions()
    for required in ("adi_wave_create", "adi_wave_step", "adi_wave_start", "adi_wave_destroy",
                     "tridiag_solve_batched", "adi_last_error"):
        assert required in names


def test_library_exports_every_header_symbol():
    lib = _lib.load()
    missing = [n for n in _lib.header_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_lib.header_functions()) == set(_lib._SIGNATURES)


@pytest.mark.parametrize("nx,ny,h,dt,speed,code", [
    (0, 4, 0.1, 0.1, 1.0, _lib.ADI_EINVAL),
    (4, 0, 0.1, 0.1, 1.0, _lib.ADI_EINVAL),
    (4, 4, 0.0, 0.1, 1.0, _lib.ADI_EINVAL),
    (4, 4, 0.1, -1.0, 1.0, _lib.ADI_EINVAL),
    (4, 4, 0.1, float("nan"), 1.0, _lib.ADI_EINVAL),
    (4, 4, 0.1, 0.1, 0.0, _lib.ADI_EINVAL),
    (4, 4, 0.1, 0.1, -2.0, _lib.ADI_EINVAL),
    (20000, 4, 0.1, 0.1, 1.0, _lib.ADI_EUNSUPPORTED),
    (46341, 46341, 0.1, 0.1, 1.0, _lib.ADI_EUNSUPPORTED),
    (64, 16385, 0.1, 0.1, 1.0, _lib.ADI_EUNSUPPORTED),
])
def test_create_rejects_bad_arguments_before_device_work(nx, ny, h, dt, speed, code):
    lib = _lib.load()
    hnd = ctypes.c_void_p(123)
    rc = lib.adi_wave_create(ctypes.byref(hnd), nx, ny, h, dt, None, speed, _lib.ADI_F32, None)
    assert rc == code
    assert hnd.value is None
    assert lib.adi_last_error()


def test_f64_row_limit():
    lib = _lib.load()
    hnd = ctypes.c_void_p()
    rc = lib.adi_wave_create(ctypes.byref(hnd), 8193, 4, 0.1, 0.1, None, 1.0, _lib.ADI_F64, None)
    assert rc == _lib.ADI_EUNSUPPORTED


def test_null_handle_and_pointers_rejected():
    lib = _lib.load()
    assert lib.adi_wave_step(None, None, None, None, None, 1) == _lib.ADI_EINVAL
    assert lib.adi_wave_start(None, None, None, None, 0, None) == _lib.ADI_EINVAL
    assert lib.adi_wave_set_kappa(None, None, 1.0) == _lib.ADI_EINVAL
    assert lib.adi_wave_destroy(None) == _lib.ADI_OK
    info = _lib.AdiWaveInfo()
    assert lib.adi_wave_get_info(None, ctypes.byref(info)) == _lib.ADI_EINVAL


def test_tridiag_argument_checks():
    lib = _lib.load()
    # empty problems are a no-op
    assert lib.tridiag_solve_batched(0, 0, 5, None, None, None, None, 1, 1, None) == _lib.ADI_OK
    assert lib.tridiag_solve_batched(0, 5, 0, None, None, None, None, 1, 1, None) == _lib.ADI_OK
    # null arrays, bad dtype, bad strides, aliasing
    assert lib.tridiag_solve_batched(0, 5, 1, None, None, None, None, 5, 1, None) == _lib.ADI_EINVAL
    assert lib.tridiag_solve_batched(7, 5, 1, 16, 32, 48, 64, 5, 1, None) == _lib.ADI_EINVAL
    assert lib.tridiag_solve_batched(0, 5, 2, 16, 32, 48, 64, 0, 1, None) == _lib.ADI_EINVAL
    assert lib.tridiag_solve_batched(0, 5, 2, 16, 32, 48, 64, 5, 0, None) == _lib.ADI_EINVAL
    assert lib.tridiag_solve_batched(0, 5, 1, 16, 32, 48, 16, 5, 1, None) == _lib.ADI_EINVAL
    assert lib.tridiag_solve_batched(0, -1, 1, 16, 32, 48, 64, 5, 1, None) == _lib.ADI_EINVAL


def test_stream_copy_argument_checks():
    lib = _lib.load()
    assert lib.adi_stream_copy(None, 16, 16, None) == _lib.ADI_EINVAL
    assert lib.adi_stream_copy(16, 32, 15, None) == _lib.ADI_EINVAL
    assert lib.adi_stream_copy(8, 32, 16, None) == _lib.ADI_EINVAL
