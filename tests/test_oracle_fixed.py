"""Pins of the oracle's fixed-point build (32-bit values, Q2.29 constants;
Sec. 7.2 binary translations, Sec. 7.4 fixed-point implementations).

The recursion itself is the one the FP64 pins fix; what is new here are the
scalar rules (the rounded product with a constant, the rounded halving), the
Q2.29 constants and the integer data path.  Each is pinned against exact
arithmetic (Python integers and fractions, high-precision decimals), closed
forms of the DFT, and the FP64 oracle's spectrum -- never against itself.
"""
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import oracle

FIXED_VARIANTS = (1, 3, 5, 7)


def _round_away(fr: Fraction) -> int:
    """Round a fraction to the nearest integer, ties away from zero."""
    q, r = divmod(abs(fr.numerator), fr.denominator)
    if 2 * r >= fr.denominator:
        q += 1
    return q if fr >= 0 else -q


def test_product_rule_is_rounded_exact_product():
    rng = np.random.default_rng(1)
    cases = [(3, 1 << 28), (-3, 1 << 28), (1, 1 << 28), (-1, 1 << 28), (5, -(1 << 28)),
             (2 ** 31 - 1, 2 ** 30 - 1), (-2 ** 31, 2 ** 30 - 1), (12345, 379625062), (0, 7)]
    cases += [(int(a), int(k)) for a, k in zip(rng.integers(-2 ** 31, 2 ** 31, 400),
                                               rng.integers(-2 ** 30, 2 ** 30, 400))]
    for a, k in cases:
        want = _round_away(Fraction(a * k, 1 << 29))
        want = (want + 2 ** 31) % 2 ** 32 - 2 ** 31  # int32 wrap
        assert oracle.fixed_scalar("mul", a, k) == want, (a, k)


def test_halving_is_rounded_binary_translation():
    for a in list(range(-9, 10)) + [2 ** 31 - 1, -2 ** 31, 2 ** 31 - 2, -2 ** 31 + 1]:
        assert oracle.fixed_scalar("half", a) == _round_away(Fraction(a, 2)), a
    # odd symmetry: a sign flip of the data changes no rounding
    for a in range(-50, 51):
        assert oracle.fixed_scalar("half", -a) == -oracle.fixed_scalar("half", a)
        assert oracle.fixed_scalar("mul", -a, 123456789) == -oracle.fixed_scalar("mul", a, 123456789)


def test_constants_are_q229_of_closed_forms():
    getcontext().prec = 60
    two = Decimal(2)
    s2 = two.sqrt()
    q = Decimal(1 << 29)
    # 2 cos(2 pi / 8) = sqrt 2; 2 cos(2 pi / 16) = sqrt(2 + sqrt 2); 2 sin(2 pi 3 / 16) = sqrt(2 + sqrt 2)
    closed = [((0, 1, 8), s2), ((0, 1, 16), (two + s2).sqrt()), ((1, 3, 16), (two + s2).sqrt()),
              ((0, 3, 16), (two - s2).sqrt()), ((1, 1, 16), (two - s2).sqrt()), ((1, 2, 8), two)]
    for (fam, j, L), v in closed:
        exact = v * q
        want = int(exact.to_integral_value(rounding="ROUND_HALF_UP"))
        assert oracle.fixed_scalar("konst", fam, j, L) == want, (fam, j, L)
    assert oracle.fixed_scalar("base_const") == int((q / s2).to_integral_value(rounding="ROUND_HALF_UP"))


@pytest.mark.parametrize("variant", FIXED_VARIANTS)
@pytest.mark.parametrize("n", [1, 2, 4])
def test_small_sizes_are_the_exact_integer_dft(variant, n):
    """N <= 4 has no product and no halving: the integer DFT exactly."""
    rng = np.random.default_rng(n)
    xr = rng.integers(-2 ** 20, 2 ** 20, (5, n))
    xi = rng.integers(-2 ** 20, 2 ** 20, (5, n))
    Xr, Xi, wraps = oracle.cdft_fixed(xr, xi, variant)
    # exact: W^{nk} is 1, -i, -1, i for n = 4
    k = np.arange(n)
    W = np.exp(-2j * np.pi * np.outer(k, k) / n).round().astype(np.complex128)
    T = (xr + 1j * xi) @ W.T
    assert wraps == 0
    assert np.array_equal(Xr, T.real.astype(np.int64)) and np.array_equal(Xi, T.imag.astype(np.int64))


@pytest.mark.parametrize("variant", FIXED_VARIANTS)
@pytest.mark.parametrize("n", [8, 64, 1024])
def test_impulse_gives_constant_spectrum_exactly(variant, n):
    """x = A delta(0): every product and halving sees zero, so X(k) = A."""
    xr = np.zeros((2, n), np.int64)
    xi = np.zeros((2, n), np.int64)
    xr[0, 0], xi[1, 0] = 12345, -777
    Xr, Xi, wraps = oracle.cdft_fixed(xr, xi, variant)
    assert wraps == 0
    assert np.all(Xr[0] == 12345) and np.all(Xi[0] == 0)
    assert np.all(Xr[1] == 0) and np.all(Xi[1] == -777)


@pytest.mark.parametrize("variant", FIXED_VARIANTS)
def test_same_operation_counts_as_floating_point(variant):
    rng = np.random.default_rng(3)
    x = rng.integers(-100, 100, (1, 256))
    _, _, _, cq = oracle.cdft_fixed(x, x, variant, counts=True)
    _, cf = oracle.cdft(x + 1j * x, variant, counts=True)
    assert cq == cf


@pytest.mark.parametrize("variant,n,bound", [(1, 256, 1e-4), (1, 4096, 3e-4), (3, 256, 2e-4), (3, 4096, 1e-3),
                                             (5, 256, 3e-3), (7, 256, 3e-4)])
def test_close_to_fp64_spectrum(variant, n, bound):
    """Inputs of 16-bit scale: the rounding of products and halvings (half a
    unit each) leaves a small relative error against the FP64 spectrum; a
    wrong sign, index, scale or constant would leave an error of order 1."""
    rng = np.random.default_rng(n + variant)
    xr = rng.integers(-2 ** 15, 2 ** 15, (4, n))
    xi = rng.integers(-2 ** 15, 2 ** 15, (4, n))
    Xr, Xi, wraps = oracle.cdft_fixed(xr, xi, variant)
    T = oracle.cdft(xr + 1j * xi, variant)
    err = np.linalg.norm(Xr + 1j * Xi - T) / np.linalg.norm(T)
    assert wraps == 0
    assert err < bound, err


@pytest.mark.parametrize("variant", (1, 3))
def test_rounding_error_scales_with_the_input(variant):
    """The error is rounding, not structure: the absolute error stays of the
    order of a unit while the input grows 256-fold, so the relative error
    falls about 256-fold."""
    n = 1024
    rng = np.random.default_rng(7)
    xr = rng.integers(-2 ** 7, 2 ** 7, (4, n))
    xi = rng.integers(-2 ** 7, 2 ** 7, (4, n))
    errs = []
    for s in (0, 8):
        ar, ai = xr << s, xi << s
        Xr, Xi, wraps = oracle.cdft_fixed(ar, ai, variant)
        T = oracle.cdft(ar + 1j * ai, variant)
        errs.append(np.linalg.norm(Xr + 1j * Xi - T) / np.linalg.norm(T))
        assert wraps == 0
    assert 64 < errs[0] / errs[1] < 1024, errs


def test_unbounded_constant_families_are_rejected():
    x = np.zeros((1, 64), np.int64)
    for v in (2, 4, 6, 8):
        with pytest.raises(ValueError):
            oracle.cdft_fixed(x, x, v)
