"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, and its host-only validation layer rejects bad input before any GPU
work.  No compute call is made here."""
import ctypes
import os
import re

import pytest

import paper_1903_02581_amd as P
from paper_1903_02581_amd.hom4d import EXPORTS, make_cfg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hom4d.h")


def _lib():
    if not os.path.exists(P.hom4d.LIB_PATH):
        pytest.fail("libhom4d.so is not built; run __graft_entry__.build()")
    return P.load_library()


def test_header_symbols_exported():
    lib = _lib()
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(hom4d_[a-z_0-9]+)\s*\(", text))
    assert declared, "no declarations parsed"
    assert declared == set(EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_status_strings():
    lib = _lib()
    for code in range(0, -10, -1):
        s = lib.hom4d_strerror(code)
        assert s and s != b"unknown status"
    assert lib.hom4d_strerror(-99) == b"unknown status"


@pytest.mark.parametrize("n", [4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256])
def test_supported_sizes_validate(n):
    lib = _lib()
    cfg = make_cfg(n, n, 100.0, 100.0, dt_fs=1.0, b_tesla=5.0)
    assert lib.hom4d_validate_cfg(ctypes.byref(cfg)) == 0
    assert lib.hom4d_state_bytes(ctypes.byref(cfg)) == (n * n) ** 2 * 16
    cfg = make_cfg(n, n, 100.0, 100.0, dt_fs=1.0, b_tesla=5.0, precision="mixed")
    assert lib.hom4d_state_bytes(ctypes.byref(cfg)) == (n * n) ** 2 * 8


@pytest.mark.parametrize("kw", [
    dict(nx=10), dict(ny=5), dict(nx=512), dict(lx=0.0), dict(ly=-1.0), dict(dt_fs=0.0),
    dict(mstar_rel=0.0), dict(eps_r=-2.0), dict(soft_nm=0.0), dict(b_tesla=float("nan")),
    dict(screen_nm=-1.0),
])
def test_invalid_cfg_rejected(kw):
    lib = _lib()
    base = dict(nx=16, ny=16, lx=100.0, ly=100.0, dt_fs=1.0, b_tesla=5.0, soft_nm=2.0)
    base.update(kw)
    nx, ny, lx, ly = base.pop("nx"), base.pop("ny"), base.pop("lx"), base.pop("ly")
    cfg = make_cfg(nx, ny, lx, ly, **base)
    assert lib.hom4d_validate_cfg(ctypes.byref(cfg)) == -1
    assert lib.hom4d_state_bytes(ctypes.byref(cfg)) == 0
    assert len(lib.hom4d_last_error()) > 0
    h = ctypes.c_void_p()
    assert lib.hom4d_create(ctypes.byref(cfg), None, ctypes.byref(h)) == -1
    assert not h.value


def test_bad_precision_and_null_args():
    lib = _lib()
    cfg = make_cfg(16, 16, 100.0, 100.0, dt_fs=1.0, b_tesla=5.0)
    cfg.precision = 7
    assert lib.hom4d_validate_cfg(ctypes.byref(cfg)) == -1
    assert lib.hom4d_validate_cfg(None) == -1
    assert lib.hom4d_create(None, None, None) == -1
    assert lib.hom4d_destroy(None) == -1
    assert lib.hom4d_step(None, 1) == -1
    assert lib.hom4d_observables(None, None, None) == -1
    assert lib.hom4d_grad_backward(None, None, None, None, None, None, None) == -1


def test_soft_zero_allowed_without_coulomb():
    lib = _lib()
    cfg = make_cfg(16, 16, 100.0, 100.0, dt_fs=1.0, b_tesla=5.0, soft_nm=0.0, coulomb_c=0.0)
    assert lib.hom4d_validate_cfg(ctypes.byref(cfg)) == 0


def test_checkpoint_calls_reject_null_handle():
    lib = _lib()
    assert lib.hom4d_checkpoint_bytes(None) == 0
    buf = ctypes.create_string_buffer(128)
    assert lib.hom4d_save_checkpoint(None, buf, 128) == -1
    assert lib.hom4d_load_checkpoint(None, buf, 128) == -1
