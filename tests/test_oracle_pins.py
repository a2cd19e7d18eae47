"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every expected value is a
brute-force sum, a closed form, a library FFT, an invariant of the DFT, or a
number printed in the paper (tests/golden/, each with its citation).
"""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
VARIANTS = range(1, 9)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return d / n if n > 0 else d


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------------------
# the direct DFT itself (eq. qft_0A) against a library FFT and a plain numpy sum
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 12, 64, 256])
def test_direct_dft_matches_numpy(n):
    rng = np.random.default_rng(n)
    x = rand_c(rng, 3, n)
    X = oracle.dft_direct(x)
    assert rel(X, np.fft.fft(x, axis=-1)) < 1e-14
    # plain matrix-vector definition, independent of the C code
    k = np.arange(n)
    Fm = np.exp(-2j * np.pi * np.outer(k, k) / n)
    assert rel(X, x @ Fm.T) < 1e-12
    # sign = +1 is the unnormalised inverse
    assert rel(oracle.dft_direct(X, sign=+1) / n, x) < 1e-13


# ---------------------------------------------------------------------------
# P1 brute force: every variant equals the O(N^2) DFT
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("variant", VARIANTS)
def test_brute_force_small(variant):
    rng = np.random.default_rng(100 + variant)
    for m in range(0, 7):
        n = 1 << m
        x = rand_c(rng, 4, n)
        X = oracle.cdft(x, variant)
        assert rel(X, oracle.dft_direct(x)) < 1e-13, (variant, n)


@pytest.mark.parametrize("variant", VARIANTS)
def test_library_cross_check_medium(variant):
    """P7: numpy.fft in FP64 up to N=4096; variants 5-8 lose accuracy as the
    paper says (Sec. 7.3), so their bound grows with N."""
    rng = np.random.default_rng(200 + variant)
    for m in range(7, 13):
        n = 1 << m
        x = rand_c(rng, 2, n)
        e = rel(oracle.cdft(x, variant), np.fft.fft(x, axis=-1))
        bound = 2e-14 if variant <= 4 else 1e-5
        assert e < bound, (variant, n, e)


# ---------------------------------------------------------------------------
# P2 closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("n", [4, 16, 64, 256])
def test_closed_forms(variant, n):
    k = np.arange(n)
    tol = 1e-12 if variant <= 4 else 1e-9
    for m in (0, 1, n // 2 - 1, n - 1):
        x = np.zeros(n, complex)
        x[m] = 1.0
        assert np.max(np.abs(oracle.cdft(x, variant) - np.exp(-2j * np.pi * m * k / n))) < tol
    X = oracle.cdft(np.ones(n, complex), variant)
    ref = np.zeros(n, complex)
    ref[0] = n
    assert np.max(np.abs(X - ref)) < tol * n
    for f in (1, 3, n // 4):
        x = np.cos(2 * np.pi * f * k / n) + 0j
        ref = np.zeros(n, complex)
        ref[f] += n / 2
        ref[(-f) % n] += n / 2
        assert np.max(np.abs(oracle.cdft(x, variant) - ref)) < tol * n
        x = np.exp(2j * np.pi * f * k / n)
        ref = np.zeros(n, complex)
        ref[f] = n
        assert np.max(np.abs(oracle.cdft(x, variant) - ref)) < tol * n


# ---------------------------------------------------------------------------
# P3 invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("variant", VARIANTS)
def test_invariants(variant):
    rng = np.random.default_rng(300 + variant)
    n = 128
    tol = 1e-13 if variant <= 4 else 1e-11
    x, y = rand_c(rng, n), rand_c(rng, n)
    X, Y = oracle.cdft(x, variant), oracle.cdft(y, variant)
    # Parseval
    assert abs(np.sum(abs(X) ** 2) - n * np.sum(abs(x) ** 2)) < tol * n * np.sum(abs(x) ** 2)
    # linearity
    a, b = 0.7 - 0.2j, -1.3 + 0.5j
    assert rel(oracle.cdft(a * x + b * y, variant), a * X + b * Y) < tol
    # shift theorem: x(n - s) -> X(k) exp(-2 pi i k s / N)
    s = 5
    k = np.arange(n)
    assert rel(oracle.cdft(np.roll(x, s), variant), X * np.exp(-2j * np.pi * k * s / n)) < tol
    # real input: X(N-k) = conj X(k)
    r = rng.standard_normal(n) + 0j
    R = oracle.cdft(r, variant)
    assert rel(R[(-k) % n], np.conj(R)) < tol
    # adjoint: <F x, y> = <x, F^H y>, and F^H F = N I
    g = rand_c(rng, n)
    lhs = np.vdot(g, X)
    rhs = np.vdot(oracle.cdft_adjoint(g, variant), x)
    assert abs(lhs - rhs) < tol * np.linalg.norm(X) * np.linalg.norm(g)
    assert rel(oracle.cdft_adjoint(X, variant), n * x) < tol


# ---------------------------------------------------------------------------
# P4 operation counts equal the paper's tables (exact integers)
# ---------------------------------------------------------------------------
def _golden_counts():
    rows = []
    with open(os.path.join(GOLDEN, "cdft_op_counts_var_qft.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return rows


def _golden_formulas():
    forms = {}
    with open(os.path.join(GOLDEN, "cost_formulas.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                t, qty, a, b, c, d = line.split()
                forms[(t, qty)] = tuple(float(v) for v in (a, b, c, d))
    return forms


@pytest.mark.parametrize("variant", VARIANTS)
def test_counts_equal_tables(variant):
    for n, adds, mults, fa, fb in _golden_counts():
        _, c = oracle.cdft(np.ones(n, complex), variant, counts=True)
        halves = c["halves"]
        assert c["adds"] == adds, (variant, n)
        assert c["mults"] == mults, (variant, n)
        assert c["adds"] + c["mults"] == fa, (variant, n)
        if variant in (1, 3, 5, 7):
            assert c["adds"] + c["mults"] + halves == fb, (variant, n)
        else:
            assert halves == 0


@pytest.mark.parametrize("variant", VARIANTS)
def test_counts_equal_formulas(variant):
    forms = _golden_formulas()
    rng = np.random.default_rng(7)
    for m in range(3, 13):
        n = 1 << m

        def f(t, q):
            a, b, c, d = forms[(t, q)]
            return a * n * m + b * n + c * m + d

        has_half = variant in (1, 3, 5, 7)
        _, c = oracle.cdft(rand_c(rng, n), variant, counts=True)
        _, r = oracle.rdft(rng.standard_normal(n), variant, counts=True)
        _, dc = oracle.sub("dct", n, rng.standard_normal(n // 2 + 1), variant, counts=True)
        _, ds = oracle.sub("dst", n, rng.standard_normal(n // 2 + 1), variant, counts=True)
        for t, got in (("CDFT", c), ("RDFT", r), ("DCT", dc), ("DST", ds)):
            assert got["mults"] == f(t, "mults"), (t, n)
            assert got["adds"] == f(t, "adds"), (t, n)
            assert got["halves"] == (f(t, "halves") if has_half else 0), (t, n)
            assert got["adds"] + got["mults"] == f(t, "flopsA"), (t, n)
            if has_half:
                assert got["adds"] + got["mults"] + got["halves"] == f(t, "flopsB"), (t, n)


# ---------------------------------------------------------------------------
# P5 constants touched: p = 1..N/4-1 except N/8 (the N=8 base uses cos(pi/4))
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("variant", VARIANTS)
def test_constants_touched(variant):
    for m in range(3, 12):
        n = 1 << m
        _, t = oracle.cdft(np.ones(n, complex), variant, touched=True)
        want = np.zeros(n // 4, dtype=np.uint8)
        want[1:] = 1
        want[n // 8] = 0
        assert np.array_equal(t, want), (variant, n)


# ---------------------------------------------------------------------------
# P6 all variants are bitwise identical for N <= 8 (no M step below L = 16)
# ---------------------------------------------------------------------------
def test_small_n_bitwise_equal():
    rng = np.random.default_rng(11)
    for n in (1, 2, 4, 8):
        x = rand_c(rng, 5, n)
        ref = oracle.cdft(x, 1)
        for v in range(2, 9):
            assert np.array_equal(oracle.cdft(x, v), ref)


# ---------------------------------------------------------------------------
# every recursive function against its direct DCT-0 / DST-0 definition on its
# own sto_n / sto_k (Table tab:notation), at several periodizations
# ---------------------------------------------------------------------------
MIN_L = {"dct": 2, "dst": 4, "dct_ot": 4, "dst_ot": 4, "dct_to": 4, "dst_to": 4,
         "dct_oo": 8, "dst_oo": 8}
SKEL_A = {1, 4, 5, 8}


@pytest.mark.parametrize("kind", oracle.KINDS)
@pytest.mark.parametrize("variant", VARIANTS)
def test_subfunctions_against_definition(kind, variant):
    if kind.endswith("_ot") and variant not in SKEL_A:
        pytest.skip("dct_ot/dst_ot belong to skeleton A (variants 1, 4, 5, 8)")
    if kind.endswith("_to") and variant in SKEL_A:
        pytest.skip("dct_to/dst_to belong to skeleton B (variants 2, 3, 6, 7)")
    rng = np.random.default_rng(17 * variant + len(kind))
    for m in range(1, 11):
        L = 1 << m
        if L < MIN_L[kind]:
            continue
        sn, sk = oracle.sto(kind, L)
        if not sn or not sk:
            continue
        mn = np.zeros(L // 2 + 1, np.uint8)
        mk = np.zeros(L // 2 + 1, np.uint8)
        mn[sn] = 1
        mk[sk] = 1
        s = np.zeros(L // 2 + 1)
        s[sn] = rng.standard_normal(len(sn))
        S = oracle.sub(kind, L, s, variant)
        ref = oracle.dcst_direct(kind.startswith("dst"), L, s, mn, mk)
        tol = 1e-13 if variant <= 4 else 1e-9
        assert rel(S[sk], ref[sk]) < tol, (kind, variant, L)
        # nothing outside sto_k is produced
        assert np.all(S[mk == 0] == 0)


# ---------------------------------------------------------------------------
# accuracy ordering claim (Sec. 7.3): sine variants are far less accurate
# ---------------------------------------------------------------------------
def test_sine_variants_less_accurate():
    rng = np.random.default_rng(5)
    n = 2048
    x = rand_c(rng, 2, n)
    ref = np.fft.fft(x, axis=-1)
    cos_err = max(rel(oracle.cdft(x, v), ref) for v in (1, 2, 3, 4))
    sin_err = min(rel(oracle.cdft(x, v), ref) for v in (5, 6, 7, 8))
    assert sin_err > 100 * cos_err


# ---------------------------------------------------------------------------
# the float build emulates the same algorithm in float32
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("variant", (2, 4))
def test_float_build(variant):
    rng = np.random.default_rng(9)
    x = rand_c(rng, 4, 1024).astype(np.complex64)
    X32 = oracle.cdft(x, variant, prec="f32")
    assert X32.dtype == np.complex64
    e = rel(X32, np.fft.fft(x.astype(np.complex128), axis=-1))
    assert 1e-8 < e < 2e-6


# ---------------------------------------------------------------------------
# P9 gradient of loss = sum |W * F x|^2: closed form 2 F^H(|W|^2 F x) against
# central finite differences (PyTorch convention grad = dL/dRe + i dL/dIm)
# ---------------------------------------------------------------------------
def test_power_loss_gradient_fd():
    rng = np.random.default_rng(21)
    n = 64
    x, w = rand_c(rng, n), rand_c(rng, n)

    def loss(z):
        return float(np.sum(np.abs(w * oracle.cdft(z, 4)) ** 2))

    g = 2 * oracle.cdft_adjoint(np.abs(w) ** 2 * oracle.cdft(x, 4), 4)
    h = 1e-6
    fd = np.zeros(n, complex)
    for i in range(n):
        e = np.zeros(n, complex)
        e[i] = h
        fd[i] = (loss(x + e) - loss(x - e)) / (2 * h)
        e[i] = 1j * h
        fd[i] += 1j * (loss(x + e) - loss(x - e)) / (2 * h)
    assert rel(fd, g) < 1e-7
