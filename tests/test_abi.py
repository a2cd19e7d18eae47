"""The C ABI: the library loads, exports every function include/amqft.h
declares, and rejects invalid arguments with the documented status codes
before making any HIP call (so these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1404_1810_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amqft.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(amqft_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1404_1810_amd.build import build
        build(verbose=False)
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_status_strings(lib):
    for s in range(6):
        assert lib.amqft_status_string(s)
    assert b"gfx950" in lib.amqft_version()


def _create(lib, n, batch=1, variant=4, dtype=1, flags=0, null_out=False):
    h = ctypes.c_void_p(12345)
    rc = lib.amqft_plan_create(None if null_out else ctypes.byref(h), n, batch, variant, dtype, flags)
    return rc, h


@pytest.mark.parametrize("n", [0, -4, 3, 6, 12, 1000, 4097])
def test_not_pow2(lib, n):
    rc, h = _create(lib, n)
    assert rc == _lib.ERR_NOT_POW2
    assert not h.value


@pytest.mark.parametrize("kw", [dict(variant=0), dict(variant=9), dict(dtype=7), dict(dtype=-1),
                                dict(batch=-1), dict(flags=64), dict(null_out=True)])
def test_invalid_args(lib, kw):
    rc, _ = _create(lib, 64, **kw)
    assert rc == _lib.ERR_INVALID_ARG


def test_too_large(lib):
    rc, _ = _create(lib, 1 << 30)
    assert rc == _lib.ERR_UNSUPPORTED


def test_null_plan_calls(lib):
    assert lib.amqft_exec(None, None, None, None) == _lib.ERR_INVALID_ARG
    assert lib.amqft_exec_adjoint(None, None, None, None) == _lib.ERR_INVALID_ARG
    assert lib.amqft_power_loss_grad(None, None, None, None, None, None) == _lib.ERR_INVALID_ARG
    assert lib.amqft_exec_graph(None, None, None, 0, None) == _lib.ERR_INVALID_ARG
    assert lib.amqft_plan_destroy(None) == _lib.OK
    sz = ctypes.c_size_t(7)
    assert lib.amqft_plan_workspace_size(None, ctypes.byref(sz)) == _lib.ERR_INVALID_ARG
    assert lib.amqft_plan_constants(None, 64, None, 0) == _lib.ERR_INVALID_ARG


def test_create_many_validation(lib):
    import numpy as np
    h = ctypes.c_void_p()
    L = np.array([16, 32, 48], dtype=np.int64)
    O = np.array([0, 16, 48, 96], dtype=np.int64)
    rc = lib.amqft_plan_create_many(ctypes.byref(h), 3, L.ctypes.data, O.ctypes.data, 4, 1, 0)
    assert rc == _lib.ERR_NOT_POW2
    L = np.array([16, 32, 64], dtype=np.int64)
    O = np.array([0, 16, 40, 104], dtype=np.int64)  # second signal overlaps the third
    rc = lib.amqft_plan_create_many(ctypes.byref(h), 3, L.ctypes.data, O.ctypes.data, 4, 1, 0)
    assert rc == _lib.ERR_INVALID_ARG
    O = np.array([0, 16, 48, 112], dtype=np.int64)
    rc = lib.amqft_plan_create_many(ctypes.byref(h), 3, L.ctypes.data, O.ctypes.data, 0, 1, 0)
    assert rc == _lib.ERR_INVALID_ARG
    rc = lib.amqft_plan_create_many(ctypes.byref(h), -1, L.ctypes.data, O.ctypes.data, 4, 1, 0)
    assert rc == _lib.ERR_INVALID_ARG
    rc = lib.amqft_plan_create_many(ctypes.byref(h), 3, None, O.ctypes.data, 4, 1, 0)
    assert rc == _lib.ERR_INVALID_ARG


@pytest.mark.parametrize("kw", [dict(n=1024, flags=8), dict(n=4096, variant=3, flags=8),
                                dict(n=4096, variant=1, flags=8), dict(n=4096, dtype=2, flags=8),
                                dict(n=1 << 17, dtype=0, flags=8), dict(n=4096, flags=12)])
def test_force_large_validation(lib, kw):
    """The large-N paths can be forced only where they exist (variants 4, 8
    and their transposed programs 2, 6; N >= 2^11, FP64 / FP32 storage below
    2^15) and not with the multi-pass force flag; the refusal happens before
    any HIP call."""
    n = kw.pop("n")
    rc, h = _create(lib, n, **kw)
    assert rc == _lib.ERR_UNSUPPORTED
    assert not h.value


def test_noalloc_validation(lib):
    """amqft_exec_noalloc rejects bad arguments, and lengths whose single
    signal does not fit its fixed scratch array, before any HIP call."""
    f = lib.amqft_exec_noalloc
    assert f(1 << 22, 1, 4, 1, 0, None, None, None) == _lib.ERR_UNSUPPORTED  # FP32: 3 x 32 MiB workspace
    assert f(1 << 21, 1, 2, 0, 0, None, None, None) == _lib.ERR_UNSUPPORTED  # FP64: 3 x 32 MiB
    assert f(1 << 25, 1, 4, 1, 0, None, None, None) == _lib.ERR_UNSUPPORTED
    assert f(3, 1, 4, 1, 0, None, None, None) == _lib.ERR_NOT_POW2
    assert f(64, 1, 9, 1, 0, None, None, None) == _lib.ERR_INVALID_ARG
    assert f(64, -1, 4, 1, 0, None, None, None) == _lib.ERR_INVALID_ARG
    assert f(64, 1, 4, 4, 0, None, None, None) == _lib.ERR_INVALID_ARG
    assert f(64, 0, 4, 1, 0, None, None, None) == _lib.OK  # empty batch: nothing to do
    assert f(64, 2, 4, 1, 0, None, None, None) == _lib.ERR_INVALID_ARG  # null buffers


@pytest.mark.parametrize("args,status", [((2, 1, 0, 4, 1, 0), _lib.ERR_UNSUPPORTED),        # n below 4
                                         ((1 << 15, 1, 0, 4, 1, 0), _lib.ERR_UNSUPPORTED),  # above LDS (FP32)
                                         ((1 << 14, 1, 1, 4, 0, 0), _lib.ERR_UNSUPPORTED),  # above LDS (FP64)
                                         ((64, 1, 0, 4, 2, 0), _lib.ERR_UNSUPPORTED),       # FP16 storage
                                         ((64, 1, 0, 4, 1, 4), _lib.ERR_UNSUPPORTED),       # force flag
                                         ((64, 1, 3, 4, 1, 0), _lib.ERR_INVALID_ARG),       # kind
                                         ((64, 1, 0, 0, 1, 0), _lib.ERR_INVALID_ARG),       # variant
                                         ((64, -1, 0, 4, 1, 0), _lib.ERR_INVALID_ARG),      # batch
                                         ((48, 1, 0, 4, 1, 0), _lib.ERR_NOT_POW2)])
def test_create_real_validation(lib, args, status):
    h = ctypes.c_void_p(5)
    assert lib.amqft_plan_create_real(ctypes.byref(h), *args) == status
    assert not h.value


@pytest.mark.parametrize("n,variant,dtype", [(64, 4, 1), (1 << 15, 4, 1), (1 << 14, 2, 0), (128, 6, 0)])
def test_transposed_adjoint_validation(lib, n, variant, dtype):
    """The transposed-flow-graph adjoint exists where both compile-time kernels
    do (2^8 .. 2^14, FP64 to 2^13); elsewhere plan creation refuses it before
    any HIP call."""
    rc, h = _create(lib, n, variant=variant, dtype=dtype, flags=16)
    assert rc == _lib.ERR_UNSUPPORTED
    assert not h.value


def test_transposed_adjoint_not_for_many_or_real(lib):
    import numpy as np
    h = ctypes.c_void_p(3)
    L = np.array([256, 256], dtype=np.int64)
    O = np.array([0, 256, 512], dtype=np.int64)
    assert lib.amqft_plan_create_many(ctypes.byref(h), 2, L.ctypes.data, O.ctypes.data, 4, 1, 16) == _lib.ERR_UNSUPPORTED
    assert lib.amqft_plan_create_real(ctypes.byref(h), 256, 1, 0, 4, 1, 16) == _lib.ERR_UNSUPPORTED


@pytest.mark.parametrize("n,variant,flags", [(1024, 2, 0), (1024, 4, 0), (1024, 6, 0), (1024, 8, 0),  # 1/(2cos) family
                                             (128, 1, 0), (1 << 15, 1, 0), (1 << 15, 3, 0),  # outside 2^8..2^14
                                             (1024, 1, 4), (1024, 3, 8)])  # force flags
def test_fixed_point_validation(lib, n, variant, flags):
    """Fixed point (AMQFT_C32I) exists for the variants with 2cos / 2sin
    constants on the compile-time kernels (2^8 .. 2^14); elsewhere plan
    creation refuses it before any HIP call."""
    rc, h = _create(lib, n, variant=variant, dtype=_lib.C32I, flags=flags)
    assert rc == _lib.ERR_UNSUPPORTED
    assert not h.value


def test_fixed_point_not_for_many_or_real(lib):
    import numpy as np
    h = ctypes.c_void_p(3)
    L = np.array([256, 256], dtype=np.int64)
    O = np.array([0, 256, 512], dtype=np.int64)
    assert lib.amqft_plan_create_many(ctypes.byref(h), 2, L.ctypes.data, O.ctypes.data, 1, _lib.C32I, 0) \
        == _lib.ERR_UNSUPPORTED
    assert lib.amqft_plan_create_real(ctypes.byref(h), 256, 1, 0, 1, _lib.C32I, 0) == _lib.ERR_UNSUPPORTED
    assert lib.amqft_exec_noalloc(256, 1, 1, _lib.C32I, 0, None, None, None) == _lib.ERR_INVALID_ARG


@pytest.mark.parametrize("n,variant,dtype,flags", [(1 << 15, 1, 1, 32), (1 << 15, 2, 1, 32), (1 << 18, 4, 1, 32),
                                                   (1 << 15, 4, 2, 32), (1 << 17, 8, 0, 32), (1 << 10, 4, 0, 32 | 8),
                                                   (1 << 12, 4, 1, 32 | 4), (1 << 10, 4, 1, 32 | 8),
                                                   (1 << 15, 5, 1, 32), (1 << 16, 3, 0, 32)])
def test_in_place_validation(lib, n, variant, dtype, flags):
    """Above one workgroup's LDS the in-place flag exists for variants 4 and 8
    with FP32 storage at 2^15 .. 2^17 (FP64 2^14 .. 2^16, forced from 2^11)
    and not with the multi-pass force flag; elsewhere plan creation refuses
    it before any HIP call."""
    rc, h = _create(lib, n, variant=variant, dtype=dtype, flags=flags)
    assert rc == _lib.ERR_UNSUPPORTED
    assert not h.value


def test_in_place_not_for_many_or_real(lib):
    import numpy as np
    h = ctypes.c_void_p(3)
    L = np.array([256, 256], dtype=np.int64)
    O = np.array([0, 256, 512], dtype=np.int64)
    assert lib.amqft_plan_create_many(ctypes.byref(h), 2, L.ctypes.data, O.ctypes.data, 4, 1, 32) == _lib.ERR_UNSUPPORTED
    assert lib.amqft_plan_create_real(ctypes.byref(h), 256, 1, 0, 4, 1, 32) == _lib.ERR_UNSUPPORTED
