"""RDFT, DCT-0 and DST-0 entry points (amqft_plan_create_real) against the
oracle's functions of the same name: the RDFT of eqs. qft_22-25 and the dct /
dst functions (eqs. qft_0B, qft_0C) of the recursion, every variant, FP64 and
FP32, sizes from the smallest periodization to one workgroup's LDS, odd and
even batches (two real signals share one complex lane; an odd batch leaves
the last lane's imaginary part empty).  Pins as for the CDFT: variants 1-4 at
1e-12 / 1e-5, variants 5-8 at 20x their own same-precision oracle error where
that stays within 1e-3, reported and xfail beyond."""
import sys

import numpy as np
import pytest

import oracle
from gpu_common import PIN_CAP, rel, xfail_unpinned
from paper_1404_1810_amd import inputs

torch = pytest.importorskip("torch")

VARIANTS = list(range(1, 9))


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _oracle(kind, n, s, variant, prec):
    """The oracle's transform of each row of s (real, FP64 or FP32 build)."""
    out = []
    for row in s:
        if kind == "rdft":
            out.append(oracle.rdft(row, variant, prec=prec))
        elif kind == "dct0":
            out.append(oracle.sub("dct", n, row, variant, prec=prec))
        else:
            full = np.zeros(n // 2 + 1)
            full[1:n // 2] = row
            out.append(oracle.sub("dst", n, full, variant, prec=prec)[1:n // 2])
    return np.array(out)


def _check(kind, n, batch, variant, f64, seed):
    from paper_1404_1810_amd import _lib, api
    in_len = {"rdft": n, "dct0": n // 2 + 1, "dst0": n // 2 - 1}[kind]
    s = inputs.real_normal(seed, batch, in_len)
    if not f64:
        s = s.astype(np.float32)
    _say(kind, "variant", variant, "n", n, "batch", batch, "f64" if f64 else "f32")
    plan = api.RealPlan(n, batch, kind, variant, _lib.C128 if f64 else _lib.C64)
    x = torch.from_numpy(np.ascontiguousarray(s)).cuda()
    y = plan.exec(x).cpu().numpy()
    if kind != "rdft":
        ya = plan.exec(x, adjoint=True).cpu().numpy()  # symmetric: the same transform
        assert np.array_equal(ya, y)
    plan.close()
    ref = _oracle(kind, n, s.astype(np.float64), 4, "f64")
    e = rel(y, ref)
    base = 1e-12 if f64 else 1e-5
    if variant <= 4:
        assert e <= base, (kind, n, variant, e)
        return None
    emu = rel(_oracle(kind, n, s, variant, "f64" if f64 else "f32"), ref)
    b = max(base, 20 * emu) if np.isfinite(emu) else None
    if b is None or b > PIN_CAP:
        return "%s n=%d: no pin (variant %d's own emulation error %.1e); GPU rel err %.3e" % (kind, n, variant, emu, e)
    assert e <= b, (kind, n, variant, e, b)
    return None


SIZES_F32 = [4, 8, 16, 64, 256, 1024, 4096, 16384]
SIZES_F64 = [4, 16, 128, 512, 2048, 8192]


@pytest.mark.gpu
@pytest.mark.parametrize("kind", ["rdft", "dct0", "dst0"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_real_fp32(kind, variant):
    reports = [_check(kind, n, 5 if n >= 4096 else 37, variant, False, 70 + n) for n in SIZES_F32]
    xfail_unpinned(reports)


@pytest.mark.gpu
@pytest.mark.parametrize("kind", ["rdft", "dct0", "dst0"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_real_fp64(kind, variant):
    reports = [_check(kind, n, 4 if n >= 4096 else 18, variant, True, 80 + n) for n in SIZES_F64]
    xfail_unpinned(reports)


@pytest.mark.gpu
def test_rdft_matches_cdft_of_real_input():
    """The RDFT of real signals equals the first n/2+1 values of the CDFT
    entry point on the same signals as complex input (same recursion)."""
    from paper_1404_1810_amd import api
    n, batch = 1024, 9
    s = inputs.real_normal(5, batch, n)
    x = torch.from_numpy(s).cuda()
    _say("rdft vs cdft")
    r = api.rdft(x, 4)
    c = api.fft(x.to(torch.complex128), 4)[:, : n // 2 + 1]
    torch.cuda.synchronize()
    assert rel(r.cpu().numpy(), c.cpu().numpy()) < 1e-14
    assert rel(r.cpu().numpy(), np.fft.rfft(s, axis=-1)) < 1e-13
