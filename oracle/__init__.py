"""AM-QFT oracle -- TEST INFRASTRUCTURE ONLY.

Python loader for the plain C oracle in ``amqft_oracle.c`` (a slow, recursive
CPU implementation of the eight AM-QFT variants of Pasquini, arXiv:1404.1810,
plus the direct O(N^2) DFT / DCT-0 / DST-0 definitions).  Only ``tests/``, the
smoke check and the CPU-baseline leg of ``bench.py`` may import this package;
the GPU library never does.

Three builds of the same C source exist: ``f64`` (REAL = double, the truth),
``f32`` (REAL = float, the same-precision emulation used to state per-variant
bounds) and ``q29`` (32-bit fixed point with Q2.29 constants, variants 1, 3,
5, 7; Sec. 7.2 / 7.4).  All are compiled with ``-O2 -ffp-contract=off`` and no
fast-math so that every rounding happens where the source says it does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "amqft_oracle.c")
_LIBS = {"f64": ("double", "liboracle_f64.so"), "f32": ("float", "liboracle_f32.so"),
         "q29": (None, "liboracle_q29.so")}
_lock = threading.Lock()
_loaded: dict = {}

# kinds understood by oracle_sub (same order as the C enum)
KINDS = ("dct", "dst", "dct_ot", "dst_ot", "dct_to", "dst_to", "dct_oo", "dst_oo")


class Counts(ctypes.Structure):
    _fields_ = [("adds", ctypes.c_longlong), ("mults", ctypes.c_longlong),
                ("halves", ctypes.c_longlong), ("base_const_uses", ctypes.c_longlong)]

    def as_dict(self):
        return {"adds": self.adds, "mults": self.mults, "halves": self.halves,
                "base_const_uses": self.base_const_uses}


def build(force: bool = False) -> None:
    """Compile both oracle builds with gcc (plain C99, no contraction)."""
    for prec, (ctype, name) in _LIBS.items():
        out = os.path.join(_HERE, name)
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
            continue
        tmp = out + ".tmp%d" % os.getpid()
        mode = "-DORACLE_FIXED" if ctype is None else "-DORACLE_REAL=%s" % ctype
        cmd = ["gcc", "-std=gnu99", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", mode, _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, out)


def _lib(prec: str = "f64"):
    with _lock:
        if prec in _loaded:
            return _loaded[prec]
        name = _LIBS[prec][1]
        path = os.path.join(_HERE, name)
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L = ctypes.c_long
        lib.oracle_cdft.argtypes = [L, L, ctypes.c_int, P, P, P, P, P, P]
        lib.oracle_rdft.argtypes = [L, ctypes.c_int, P, P, P, P, P]
        lib.oracle_sub.argtypes = [ctypes.c_int, L, L, ctypes.c_int, P, P, P, P]
        want = 8 if prec == "f64" else 4
        if lib.oracle_real_size() != want or lib.oracle_is_fixed() != (prec == "q29"):
            raise RuntimeError("oracle build %s is not the %s build" % (name, prec))
        if prec == "q29":
            I = ctypes.c_int
            lib.oracle_fixed_wraps.restype = ctypes.c_longlong
            lib.oracle_fixed_mul.argtypes = [I, I]
            lib.oracle_fixed_half.argtypes = [I]
            lib.oracle_fixed_konst.argtypes = [I, L, L]
        else:
            lib.oracle_dft_direct.argtypes = [L, L, ctypes.c_int, P, P, P, P]
            lib.oracle_dcst_direct.argtypes = [ctypes.c_int, L, P, P, P, P]
        _loaded[prec] = lib
        return lib


def _dt(prec):
    return {"f64": np.float64, "f32": np.float32, "q29": np.int32}[prec]


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def cdft(x, variant: int = 4, prec: str = "f64", counts: bool = False, touched: bool = False):
    """AM-QFT CDFT of the last axis of complex array ``x`` (any leading shape).

    Returns the complex spectrum (complex128 for f64, complex64 for f32); with
    ``counts``/``touched`` also the op counts (summed over the batch) and the
    0/1 array of constant indexes p (theta_N * p) that were used.
    """
    x = np.asarray(x)
    n = x.shape[-1]
    batch = int(np.prod(x.shape[:-1], dtype=np.int64)) if x.ndim > 1 else 1
    dt = _dt(prec)
    xr = np.ascontiguousarray(x.real, dtype=dt).reshape(batch, n)
    xi = np.ascontiguousarray(np.imag(x), dtype=dt).reshape(batch, n)
    Xr = np.empty_like(xr)
    Xi = np.empty_like(xi)
    cnt = Counts()
    tch = np.zeros(max(n // 4, 1), dtype=np.uint8)
    rc = _lib(prec).oracle_cdft(n, batch, int(variant), _ptr(xr), _ptr(xi), _ptr(Xr), _ptr(Xi),
                                ctypes.byref(cnt), _ptr(tch))
    if rc != 0:
        raise ValueError("oracle_cdft rejected n=%d variant=%d" % (n, variant))
    ct = np.complex128 if prec == "f64" else np.complex64
    X = (Xr + 1j * Xi).astype(ct).reshape(x.shape)
    out = [X]
    if counts:
        out.append(cnt.as_dict())
    if touched:
        out.append(tch[: n // 4].copy())
    return out[0] if len(out) == 1 else tuple(out)


def cdft_fixed(xr, xi, variant: int = 1, counts: bool = False):
    """Fixed-point AM-QFT CDFT (the ``q29`` build) of the last axis of the
    int32 arrays ``xr``, ``xi`` (real and imaginary parts, in units of the
    input's last bit).  Variants 1, 3, 5, 7 only.  Returns int32 arrays (Xr, Xi)
    and the number of results that wrapped around the int32 range."""
    xr = np.asarray(xr)
    xi = np.asarray(xi)
    assert xr.shape == xi.shape
    n = xr.shape[-1]
    batch = int(np.prod(xr.shape[:-1], dtype=np.int64)) if xr.ndim > 1 else 1
    for a in (xr, xi):
        if np.any(a != a.astype(np.int32)):
            raise ValueError("fixed-point input must be int32 values")
    ar = np.ascontiguousarray(xr, dtype=np.int32).reshape(batch, n)
    ai = np.ascontiguousarray(xi, dtype=np.int32).reshape(batch, n)
    Xr = np.empty_like(ar)
    Xi = np.empty_like(ai)
    lib = _lib("q29")
    cnt = Counts()
    with _lock:
        lib.oracle_fixed_wraps()
        rc = lib.oracle_cdft(n, batch, int(variant), _ptr(ar), _ptr(ai), _ptr(Xr), _ptr(Xi),
                             ctypes.byref(cnt), None)
        wraps = int(lib.oracle_fixed_wraps())
    if rc != 0:
        raise ValueError("fixed-point oracle rejected n=%d variant=%d" % (n, variant))
    out = (Xr.reshape(xr.shape), Xi.reshape(xr.shape), wraps)
    return out + (cnt.as_dict(),) if counts else out


def fixed_scalar(op: str, *args) -> int:
    """The fixed-point build's scalar rules: ``mul`` (a, k), ``half`` (a),
    ``konst`` (family 0 = 2cos / 1 = 2sin, j, L), ``base_const`` ()."""
    lib = _lib("q29")
    return int({"mul": lib.oracle_fixed_mul, "half": lib.oracle_fixed_half,
                "konst": lib.oracle_fixed_konst, "base_const": lib.oracle_fixed_base_const}[op](*args))


def cdft_adjoint(g, variant: int = 4, prec: str = "f64"):
    """F^H g = conj(F conj(g)): the DFT matrix of eq. qft_0A is symmetric."""
    return np.conj(cdft(np.conj(np.asarray(g)), variant, prec))


def rdft(r, variant: int = 4, prec: str = "f64", counts: bool = False):
    """AM-QFT RDFT of a real 1-D signal: returns R(k), k = 0..n/2 (complex)."""
    r = np.ascontiguousarray(r, dtype=_dt(prec))
    n = r.shape[0]
    Rr = np.zeros(n // 2 + 1, dtype=r.dtype)
    Ri = np.zeros(n // 2 + 1, dtype=r.dtype)
    cnt = Counts()
    rc = _lib(prec).oracle_rdft(n, int(variant), _ptr(r), _ptr(Rr), _ptr(Ri), ctypes.byref(cnt), None)
    if rc != 0:
        raise ValueError("oracle_rdft rejected n=%d" % n)
    R = Rr + 1j * Ri
    return (R, cnt.as_dict()) if counts else R


def sub(kind: str, L: int, s, variant: int = 4, ntop: int | None = None, prec: str = "f64",
        counts: bool = False, touched: bool = False):
    """Run one recursive function (dct, dst, dct_ot, ...) on a full-index array
    ``s`` of length L/2+1; returns the full-index output array of length L/2+1
    (entries outside sto_k are zero)."""
    dt = _dt(prec)
    s = np.ascontiguousarray(s, dtype=dt)
    assert s.shape == (L // 2 + 1,)
    S = np.zeros(L // 2 + 1, dtype=dt)
    ntop = L if ntop is None else ntop
    cnt = Counts()
    tch = np.zeros(max(ntop // 4, 1), dtype=np.uint8)
    rc = _lib(prec).oracle_sub(KINDS.index(kind), L, ntop, int(variant), _ptr(s), _ptr(S),
                               ctypes.byref(cnt), _ptr(tch))
    if rc != 0:
        raise ValueError("oracle_sub rejected kind=%s L=%d" % (kind, L))
    out = [S]
    if counts:
        out.append(cnt.as_dict())
    if touched:
        out.append(tch[: ntop // 4].copy())
    return out[0] if len(out) == 1 else tuple(out)


def dft_direct(x, sign: int = -1, prec: str = "f64"):
    """Direct O(N^2) DFT (eq. qft_0A for sign = -1), long-double accumulation."""
    x = np.asarray(x)
    n = x.shape[-1]
    batch = int(np.prod(x.shape[:-1], dtype=np.int64)) if x.ndim > 1 else 1
    dt = _dt(prec)
    xr = np.ascontiguousarray(x.real, dtype=dt).reshape(batch, n)
    xi = np.ascontiguousarray(np.imag(x), dtype=dt).reshape(batch, n)
    Xr = np.empty_like(xr)
    Xi = np.empty_like(xi)
    rc = _lib(prec).oracle_dft_direct(n, batch, int(sign), _ptr(xr), _ptr(xi), _ptr(Xr), _ptr(Xi))
    if rc != 0:
        raise ValueError("oracle_dft_direct rejected n=%d" % n)
    return (Xr + 1j * Xi).reshape(x.shape)


def dcst_direct(is_sine: bool, L: int, s, mask_n, mask_k, prec: str = "f64"):
    """Direct DCT-0 (eq. qft_0B) or DST-0 (eq. qft_0C) of a pruned signal."""
    dt = _dt(prec)
    s = np.ascontiguousarray(s, dtype=dt)
    mn = np.ascontiguousarray(mask_n, dtype=np.uint8)
    mk = np.ascontiguousarray(mask_k, dtype=np.uint8)
    S = np.zeros(L // 2 + 1, dtype=dt)
    rc = _lib(prec).oracle_dcst_direct(1 if is_sine else 0, L, _ptr(s), _ptr(mn), _ptr(mk), _ptr(S))
    if rc != 0:
        raise ValueError("oracle_dcst_direct rejected L=%d" % L)
    return S


# sto_n / sto_k of every signal type (Table tab:notation), as index sets of a
# full-index array of length L/2+1.
def sto(kind: str, L: int):
    q = L // 4
    h = L // 2
    odd_lt = lambda m: list(range(1, m, 2))
    table = {
        "dct": (list(range(0, h + 1)), list(range(0, h + 1))),
        "dst": (list(range(1, h)), list(range(1, h))),
        "dct_ot": (odd_lt(h), list(range(0, q))),
        "dst_ot": (odd_lt(h), list(range(1, q + 1))),
        "dct_to": (list(range(0, q)), odd_lt(h)),
        "dst_to": (list(range(1, q + 1)), odd_lt(h)),
        "dct_oo": (odd_lt(q), odd_lt(q)),
        "dst_oo": (odd_lt(q), odd_lt(q)),
    }
    return table[kind]
