"""Fixed-point AM-QFT on the GPU (AMQFT_C32I: int32 values, Q2.29 constants;
Sec. 7.2 binary translations, Sec. 7.4 fixed-point implementations).

Sums are exact, so the kernels -- whatever order they form the sums in, with
the recurrences as lane scans and skeleton B as the transposed program -- must
round exactly the values the recursion rounds: every output is compared with
the fixed-point oracle bit for bit (integer work, no tolerance).
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_common import rel

torch = pytest.importorskip("torch")

FLAG_ONTHEFLY, FLAG_TRANSPOSED_ADJOINT = 1, 16


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _scale_bits(variant, logn):
    """Input scale that keeps every value inside int32 (measured with the
    oracle; variants 5 / 7 wrap at larger sizes whatever the scale -- the
    comparison stays bit-exact, wrapping included)."""
    if variant == 3:
        return 15 if logn <= 11 else {12: 12, 13: 10, 14: 8}[logn]
    return 15


def _inputs(seed, batch, n, bits):
    from paper_1404_1810_amd import inputs
    return inputs.int_pairs(seed, batch, n, bits)


def _oracle(x, variant, adjoint=False):
    sgn = -1 if adjoint else 1
    Xr, Xi, wraps = oracle.cdft_fixed(x[..., 0], sgn * x[..., 1], variant)
    return np.stack([Xr, sgn * Xi], axis=-1), wraps


@pytest.mark.gpu
@pytest.mark.parametrize("logn", [8, 9, 10, 11, 12, 13, 14])
@pytest.mark.parametrize("variant", [1, 3, 5, 7])
def test_fixed_bit_exact(variant, logn):
    from paper_1404_1810_amd import api
    n = 1 << logn
    batch = 5 if logn <= 11 else 2  # ragged against the signals a workgroup holds
    x = _inputs(1000 * variant + logn, batch, n, _scale_bits(variant, logn))
    _say("fixed variant", variant, "n", n, "batch", batch)
    y = api.fft(torch.from_numpy(x).cuda(), variant).cpu().numpy()
    ref, wraps = _oracle(x, variant)
    bad = int(np.sum(y != ref))
    assert bad == 0, (bad, wraps)
    if variant in (1, 3):
        assert wraps == 0


@pytest.mark.gpu
@pytest.mark.parametrize("variant,logn", [(1, 12), (3, 10), (5, 9), (7, 14)])
def test_fixed_adjoint_bit_exact(variant, logn):
    """F^H x = conj(F conj x): conjugation is an exact negation."""
    from paper_1404_1810_amd import api
    n = 1 << logn
    x = _inputs(77 + logn, 3, n, _scale_bits(variant, logn))
    _say("fixed adjoint variant", variant, "n", n)
    y = api.adjoint(torch.from_numpy(x).cuda(), variant).cpu().numpy()
    ref, _ = _oracle(x, variant, adjoint=True)
    assert np.array_equal(y, ref)


@pytest.mark.gpu
@pytest.mark.parametrize("variant,logn", [(1, 12), (3, 11), (5, 8), (7, 13)])
def test_fixed_transposed_adjoint_is_the_dual_variant(variant, logn):
    """The transposed-flow-graph adjoint runs the dual variant's program (1 <->
    3, 5 <-> 7) conjugated: bit-exact against the oracle's dual variant."""
    from paper_1404_1810_amd import _lib, api
    n = 1 << logn
    dual = {1: 3, 3: 1, 5: 7, 7: 5}[variant]
    x = _inputs(5 + logn, 2, n, min(_scale_bits(variant, logn), _scale_bits(dual, logn)))
    _say("fixed transposed adjoint variant", variant, "n", n)
    plan = api.Plan(n, 2, variant, _lib.C32I, FLAG_TRANSPOSED_ADJOINT)
    y = plan.exec(torch.from_numpy(x).cuda(), adjoint=True)
    torch.cuda.synchronize()
    plan.close()
    ref, _ = _oracle(x, dual, adjoint=True)
    assert np.array_equal(y.cpu().numpy(), ref)


@pytest.mark.gpu
@pytest.mark.parametrize("variant,logn", [(1, 12), (3, 9), (5, 14), (7, 10)])
def test_fixed_onthefly_constants(variant, logn):
    """Constants generated on the device in FP64 and rounded once to Q2.29 are
    the host's long-double ones here, so the output stays bit-exact."""
    from paper_1404_1810_amd import _lib, api
    n = 1 << logn
    plan = api.Plan(n, 3, variant, _lib.C32I, FLAG_ONTHEFLY)
    dev_table = plan.constants()
    ref_plan = api.Plan(n, 3, variant, _lib.C32I, 0)
    host_table = ref_plan.constants()
    ref_plan.close()
    diff = np.nonzero(dev_table != host_table)[0]
    assert diff.size == 0, ("device constants differ from the host's at", diff[:8])
    x = _inputs(321 + logn, 3, n, _scale_bits(variant, logn))
    _say("fixed on-the-fly variant", variant, "n", n)
    y = plan.exec(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    plan.close()
    ref, _ = _oracle(x, variant)
    assert np.array_equal(y.cpu().numpy(), ref)


@pytest.mark.gpu
def test_fixed_full_batch_sampled():
    """The benchmark shape (16384 signals of 4096 points) in one launch:
    sampled signals against the oracle, bit for bit; the fixed-point spectrum
    of variant 1 is also within 3e-4 of the FP64 one."""
    from paper_1404_1810_amd import api
    n, batch = 4096, 16384
    x = _inputs(2024, batch, n, 15)
    _say("fixed full batch", batch, "x", n)
    y = api.fft(torch.from_numpy(x).cuda(), 1)
    torch.cuda.synchronize()
    rows = [0, 1, 255, 256, 8191, batch - 1]
    ys = y[rows].cpu().numpy()
    ref, wraps = _oracle(x[rows], 1)
    assert wraps == 0
    assert np.array_equal(ys, ref)
    truth = oracle.cdft(x[rows, :, 0] + 1j * x[rows, :, 1], 1)
    assert rel(ys[..., 0] + 1j * ys[..., 1], truth) < 3e-4
