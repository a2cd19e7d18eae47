"""FP16 / BF16 storage with FP32 arithmetic.

Reference: the FP64 oracle run on the same stored (quantised) input.  The
error then comes from FP32 arithmetic plus the rounding of the output to the
storage type; bounds 5e-4 (FP16) and 4e-3 (BF16, 8x the unit roundoff of FP16)
for variants 1-4.  Variants 5-8 keep those bounds only where FP32 keeps them
accurate (N <= 64 here); beyond that their error and their count of
non-finite outputs are reported and the case is marked xfail.
"""
import sys

import numpy as np
import pytest

from gpu_common import rel, truth, xfail_unpinned
from paper_1404_1810_amd import inputs

torch = pytest.importorskip("torch")

BOUND = {"fp16": 5e-4, "bf16": 4e-3}


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _half_pairs(z):
    out = np.empty(z.shape + (2,), dtype=np.float16)
    out[..., 0] = z.real
    out[..., 1] = z.imag
    return out


def _to_device(kind, z):
    """(device tensor, FP64 complex of the stored values) for storage kind."""
    if kind == "fp16":
        h = _half_pairs(z)
        return torch.from_numpy(h).cuda(), h[..., 0].astype(np.float64) + 1j * h[..., 1].astype(np.float64)
    bits = inputs.to_bf16_bits(np.stack([z.real, z.imag], axis=-1))
    q = inputs.from_bf16_bits(bits).astype(np.float64)
    return torch.from_numpy(bits.view(np.int16)).cuda().view(torch.bfloat16), q[..., 0] + 1j * q[..., 1]


def _from_device(kind, y):
    if kind == "fp16":
        yn = y.cpu().numpy().astype(np.float64)
    else:
        yn = inputs.from_bf16_bits(y.view(torch.int16).cpu().numpy().view(np.uint16)).astype(np.float64)
    return yn[..., 0] + 1j * yn[..., 1]


def _judge(kind, variant, n, yc, ref, label):
    """Assert the storage bound where the variant has one at this size; report
    and return a message otherwise."""
    finite = np.isfinite(yc)
    e = rel(yc, ref) if finite.all() else np.inf
    _say("  %s rel err %.3e, non-finite %d" % (label, e, int((~finite).sum())))
    if variant <= 4 or n <= 64:
        assert e < BOUND[kind], (kind, variant, n, e)
        return None
    return "%s variant %d n=%d: no pin in FP32 arithmetic; rel err %s, %d non-finite values" % (
        kind, variant, n, "%.3e" % e if np.isfinite(e) else "inf", int((~finite).sum()))


@pytest.mark.gpu
@pytest.mark.parametrize("n", [64, 1024, 16384])
@pytest.mark.parametrize("kind", ["fp16", "bf16"])
@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7, 8])
def test_reduced_storage(variant, kind, n):
    from paper_1404_1810_amd import api
    batch = 3
    _say(kind, "variant", variant, "n", n)
    xt, xq = _to_device(kind, inputs.complex_uniform(40 + n + (7 if kind == "bf16" else 0), batch, n))
    yc = _from_device(kind, api.fft(xt, variant))
    xfail_unpinned([_judge(kind, variant, n, yc, truth(xq), "")])


@pytest.mark.gpu
@pytest.mark.parametrize("kind", ["fp16", "bf16"])
@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7, 8])
def test_n2p20_sampled(variant, kind):
    """The precision workload's shape: N = 2^20, FP16 (and BF16) storage,
    U[-1,1) entries, on-the-fly constants; two sampled signals of the seeded
    stream against the FP64 oracle on the quantised input.  Variants 5-8
    overflow or lose all accuracy at this size (Sec. 7.3): reported only."""
    from paper_1404_1810_amd import api
    n = 1 << 20
    _say(kind, "n=2^20 variant", variant)
    h = inputs.cfg_fp16_rows(2, n)
    z = h[..., 0].astype(np.float64) + 1j * h[..., 1].astype(np.float64)
    xt, xq = _to_device(kind, z)
    yc = _from_device(kind, api.fft(xt, variant, flags=1))
    xfail_unpinned([_judge(kind, variant, n, yc, truth(xq), "")])


@pytest.mark.gpu
@pytest.mark.parametrize("variant", [4, 8, 2, 6])
def test_reduced_storage_large_path(variant, monkeypatch):
    """FP16 and BF16 storage on the four-kernel path (N above one workgroup's
    LDS), workspaces cut to 1 MiB so that the batch runs in chunks."""
    from paper_1404_1810_amd import _lib, api
    monkeypatch.setenv("AMQFT_LARGE_WS_MB", "1")
    reports = []
    for kind, n, batch in (("fp16", 1 << 15, 5), ("bf16", 1 << 17, 2)):
        _say(kind, "large path variant", variant, "n", n, "batch", batch)
        xt, xq = _to_device(kind, inputs.complex_uniform(60 + n, batch, n))
        plan = api.Plan(n, batch, variant, _lib.C32H if kind == "fp16" else _lib.C32B, 0)
        assert "amqft_kL" in plan.describe(), plan.describe()
        y = plan.exec(xt)
        torch.cuda.synchronize()
        yc = _from_device(kind, y)
        plan.close()
        reports.append(_judge(kind, variant, n, yc, truth(xq), "large path"))
    xfail_unpinned(reports)
