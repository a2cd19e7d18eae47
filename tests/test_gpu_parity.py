"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every case prints its identity before it touches the GPU.
"""
import sys

import numpy as np
import pytest

from gpu_common import assess, bound, rel, truth, xfail_unpinned
from paper_1404_1810_amd import inputs

torch = pytest.importorskip("torch")

VARIANTS = list(range(1, 9))


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _api():
    from paper_1404_1810_amd import api
    return api


def _run(x_np, variant, dtype, flags=0, adjoint=False):
    api = _api()
    if dtype == "c128":
        x = torch.from_numpy(np.ascontiguousarray(x_np, dtype=np.complex128)).cuda()
    else:
        x = torch.from_numpy(np.ascontiguousarray(x_np, dtype=np.complex64)).cuda()
    f = api.adjoint if adjoint else api.fft
    y = f(x, variant, flags=flags)
    torch.cuda.synchronize()
    return y.cpu().numpy()


SIZES_F32 = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384]
SIZES_F64 = [1, 2, 4, 8, 16, 64, 256, 512, 1024, 2048, 4096, 8192]


@pytest.mark.gpu
@pytest.mark.parametrize("n", SIZES_F32)
@pytest.mark.parametrize("variant", VARIANTS)
def test_parity_fp32(variant, n):
    batch = 3 if n >= 4096 else 37  # ragged: not a multiple of signals-per-workgroup
    _say("fp32 parity variant", variant, "n", n, "batch", batch)
    x = inputs.complex_normal(1000 + n, batch, n).astype(np.complex64)
    ref = truth(x, 2 if variant in (2, 3, 6, 7) else 4)
    y = _run(x, variant, "c64")
    assert y.dtype == np.complex64
    xfail_unpinned([assess(y, ref, variant, False, x, "fp32 n=%d" % n)])


@pytest.mark.gpu
@pytest.mark.parametrize("n", SIZES_F64)
@pytest.mark.parametrize("variant", VARIANTS)
def test_parity_fp64(variant, n):
    batch = 2 if n >= 4096 else 19
    _say("fp64 parity variant", variant, "n", n, "batch", batch)
    x = inputs.complex_uniform(2000 + n, batch, n)
    ref = truth(x, 4)
    y = _run(x, variant, "c128")
    xfail_unpinned([assess(y, ref, variant, True, x, "fp64 n=%d" % n)])


@pytest.mark.gpu
@pytest.mark.parametrize("variant", VARIANTS)
def test_adjoint_parity(variant):
    n, batch = 512, 9
    _say("adjoint variant", variant)
    g = inputs.complex_normal(77, batch, n)
    ref = np.conj(truth(np.conj(g), 4))  # F^H g
    y = _run(g, variant, "c128", adjoint=True)
    b = bound(variant, True, np.conj(g), np.conj(ref))
    assert b is not None and rel(y, ref) <= b


@pytest.mark.gpu
def test_onthefly_constants_match_table():
    n, batch = 1024, 5
    x = inputs.complex_normal(5, batch, n).astype(np.complex64)
    for v in VARIANTS:
        _say("on-the-fly constants variant", v)
        a = _run(x, v, "c64", flags=0)
        b = _run(x, v, "c64", flags=1)
        # the FP64 device constants round to the same FP32 table entries
        # except for rare double-rounding ties, so the results agree closely
        assert rel(b, a) < 1e-6, v


@pytest.mark.gpu
def test_in_place_and_empty():
    api = _api()
    n = 256
    x_np = inputs.complex_normal(9, 7, n).astype(np.complex64)
    x = torch.from_numpy(x_np).cuda()
    _say("in-place n", n)
    y = api.fft(x.clone(), 4)
    z = x.clone()
    api.fft(z, 4, out=z)
    torch.cuda.synchronize()
    assert torch.equal(y, z)
    _say("empty batch")
    e = torch.empty((0, n), dtype=torch.complex64, device="cuda")
    assert api.fft(e, 4).shape == (0, n)


@pytest.mark.gpu
def test_deterministic():
    api = _api()
    x = torch.from_numpy(inputs.complex_normal(3, 64, 4096).astype(np.complex64)).cuda()
    for v in (1, 2, 4, 6, 7):
        _say("determinism variant", v)
        a = api.fft(x, v)
        b = api.fft(x, v)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


@pytest.mark.gpu
@pytest.mark.parametrize("n", [2048, 8192, 1 << 15])
def test_fp64_repeated_launches_identical(n):
    """FP64 results of 40 launches on the same input agree bit for bit and
    with the oracle.  Guards the 16-byte output stores: a store whose data
    registers were overwritten by the next instruction wrote the low word of
    a real part wrong in a few launches out of ten (lanes 12..15 of 16-lane
    rows), an error of 1e-7 relative that a single launch rarely shows."""
    from paper_1404_1810_amd import _lib
    api = _api()
    batch = 64 if n <= 8192 else 4
    _say("fp64 repeated launches n", n, "batch", batch)
    xn = inputs.complex_uniform(2000 + n, batch, n)
    ref = truth(xn, 4)
    x = torch.from_numpy(xn).cuda()
    plan = api.Plan(n, batch, 4, _lib.C128, 0)
    first = torch.empty_like(x)
    plan.exec(x, out=first)
    y = torch.empty_like(x)
    for it in range(40):
        y.fill_(0)
        plan.exec(x, out=y)
        torch.cuda.synchronize()
        assert torch.equal(y, first), (n, it)
    e = rel(first.cpu().numpy(), ref)
    assert e <= 1e-12, (n, e)


@pytest.mark.gpu
@pytest.mark.parametrize("variant", VARIANTS)
def test_transposed_graph_adjoint(variant):
    """F^H by the transposed flow graph (AMQFT_FLAG_TRANSPOSED_ADJOINT): the
    real transpose of variant v's program, which is the program of its dual
    variant (M4^T = M2, M8^T = M6, M1^T = M3, M5^T = M7) with the sign of i
    flipped.  Against the oracle's F^H (pinned by the dual variant's own
    error, since that is the arithmetic performed); bit for bit against the
    conjugation-fused adjoint of the dual variant (the same program); its
    rounding compared with the conjugation-fused adjoint of variant v; the
    forward transform of the plan unchanged."""
    api = _api()
    from paper_1404_1810_amd import _lib
    dual = {1: 3, 2: 4, 3: 1, 4: 2, 5: 7, 6: 8, 7: 5, 8: 6}[variant]
    reports = []
    for dtype, n, batch in (("c128", 256, 5), ("c128", 4096, 2), ("c64", 4096, 3), ("c64", 16384, 2)):
        f64 = dtype == "c128"
        code = _lib.C128 if f64 else _lib.C64
        g_np = inputs.complex_normal(88 + n, batch, n)
        if not f64:
            g_np = g_np.astype(np.complex64)
        _say("transposed-graph adjoint variant", variant, dtype, "n", n)
        ref = np.conj(truth(np.conj(g_np), 4))
        g = torch.from_numpy(g_np).cuda()
        pt = api.Plan(n, batch, variant, code, _lib.FLAG_TRANSPOSED_ADJOINT)
        pc = api.Plan(n, batch, variant, code, 0)
        pd = api.Plan(n, batch, dual, code, 0)
        yt = pt.exec(g, adjoint=True)
        yc = pc.exec(g, adjoint=True)
        yd = pd.exec(g, adjoint=True)
        ft, fc = pt.exec(g), pc.exec(g)
        torch.cuda.synchronize()
        assert "amqft_k" in pt.describe()
        assert torch.equal(ft, fc)
        assert torch.equal(yt, yd)
        yt_np = yt.cpu().numpy()
        _say("  rel to oracle %.3e, to the conjugation-fused adjoint %.3e" % (rel(yt_np, ref), rel(yt_np, yc.cpu().numpy())))
        reports.append(assess(np.conj(yt_np), np.conj(ref), dual, f64, np.conj(g_np), "%s n=%d" % (dtype, n)))
        for p in (pt, pc, pd):
            p.close()
    xfail_unpinned(reports)


MP_FORCED = (("c64", 32), ("c64", 128), ("c64", 1024), ("c64", 4096), ("c128", 256), ("c128", 1024), ("c128", 2048))


@pytest.mark.gpu
@pytest.mark.parametrize("dtype,n", MP_FORCED)
@pytest.mark.parametrize("variant", VARIANTS)
def test_multipass_forced_small(variant, dtype, n):
    """The multi-pass path (global levels + LDS sub-blocks + tail) forced at
    small N, where it uses 4..64-point sub-blocks and several global levels.
    Its FP64 cases up to 2^11 pin every kernel of the engine for all eight
    variants (the same kernels serve N = 2^15 .. 2^24)."""
    batch = 3
    _say("forced multipass", dtype, "variant", variant, "n", n)
    x = inputs.complex_normal(3000 + n, batch, n)
    if dtype == "c64":
        x = x.astype(np.complex64)
    ref = truth(x, 4)
    y = _run(x, variant, dtype, flags=4)
    xfail_unpinned([assess(y, ref, variant, dtype == "c128", x, "forced multipass %s n=%d" % (dtype, n))])


@pytest.mark.gpu
@pytest.mark.parametrize("dtype,n", (("c64", 1 << 15), ("c64", 1 << 16), ("c128", 1 << 14)))
@pytest.mark.parametrize("variant", VARIANTS)
def test_multipass_large(variant, dtype, n):
    """Signals above the LDS capacity: 2^15 and 2^16 (FP32), 2^14 (FP64)."""
    batch = 2
    _say("multipass", dtype, "variant", variant, "n", n)
    x = inputs.complex_normal(4000 + n, batch, n)
    if dtype == "c64":
        x = x.astype(np.complex64)
    ref = truth(x, 4)
    y = _run(x, variant, dtype)
    xfail_unpinned([assess(y, ref, variant, dtype == "c128", x, "%s n=%d" % (dtype, n))])


def _large_case(api, _lib, variant, dtype, n, batch, flags_extra, want_chunk=None, adjoint=True):
    x_np = inputs.complex_normal(5000 + n, batch, n)
    if dtype == "c64":
        x_np = x_np.astype(np.complex64)
    f64 = dtype == "c128"
    ref = truth(x_np, 4)
    aref = np.conj(truth(np.conj(x_np), 4))
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    reports = []
    for flags in (0, _lib.FLAG_ONTHEFLY_CONSTANTS):
        plan = api.Plan(n, batch, variant, _lib.C128 if f64 else _lib.C64, flags | flags_extra)
        d = plan.describe()
        assert "amqft_kL" in d, d
        if want_chunk is not None:
            assert ("chunk=%d" % want_chunk) in d, d
        y = plan.exec(x)
        torch.cuda.synchronize()
        reports.append(assess(y.cpu().numpy(), ref, variant, f64, x_np, "%s n=%d flags=%d" % (dtype, n, flags)))
        if flags == 0 and adjoint:
            g = x.clone()
            plan.exec(g, out=g, adjoint=True)  # in place
            torch.cuda.synchronize()
            reports.append(assess(np.conj(g.cpu().numpy()), np.conj(aref), variant, f64, np.conj(x_np),
                                  "%s n=%d adjoint in place" % (dtype, n)))
        plan.close()
    return reports


@pytest.mark.gpu
@pytest.mark.parametrize("dtype,n,batch,chunk", (("c64", 1 << 15, 5, 3), ("c64", 1 << 17, 3, 1),
                                                 ("c128", 1 << 14, 5, 3), ("c128", 1 << 15, 3, 2),
                                                 ("c128", 1 << 16, 2, 1)))
@pytest.mark.parametrize("variant", [4, 8, 2, 6])
def test_large_path(variant, dtype, n, batch, chunk, monkeypatch):
    """The four-kernel path for N above one workgroup's LDS (variants 4 and 8:
    2^15 .. 2^17 FP32, 2^14 .. 2^16 FP64) and its transposed program (the
    five kernels of variants 2 and 6), workspaces cut to 1 MiB so that
    every batch runs in several chunks with a ragged last one; forward with the
    table and with on-the-fly constants, adjoint, in place.  Variants 6 and 8
    have no pin at these sizes (their own FP64 error is above 1e-3 from 2^13);
    their kernels are pinned by test_large_path_forced."""
    api = _api()
    from paper_1404_1810_amd import _lib
    monkeypatch.setenv("AMQFT_LARGE_WS_MB", "1")
    _say("large path", dtype, "variant", variant, "n", n, "batch", batch)
    xfail_unpinned(_large_case(api, _lib, variant, dtype, n, batch, 0, want_chunk=chunk))


LARGE_FORCED = (("c128", 1 << 11, 5), ("c128", 1 << 12, 3), ("c128", 1 << 13, 2), ("c64", 1 << 11, 5),
                ("c64", 1 << 12, 3), ("c64", 1 << 13, 2), ("c64", 1 << 14, 2))


@pytest.mark.gpu
@pytest.mark.parametrize("dtype,n,batch", LARGE_FORCED)
@pytest.mark.parametrize("variant", [4, 8, 2, 6])
def test_large_path_forced(variant, dtype, n, batch, monkeypatch):
    """The same kernels (top, rows, back, bchain; for 2 and 6 c0, fold, b0,
    rows, top) forced at N = 2^11 .. 2^14, where the rows are 2^8 .. 2^11-point
    transforms that share a workgroup.  At FP64 2^11 and 2^12 every kernel of
    variants 8 and 6 is pinned at 20x its own FP64 error (<= 5e-5); forward with
    table and on-the-fly constants, adjoint in place, chunks of 1 MiB of
    workspace."""
    api = _api()
    from paper_1404_1810_amd import _lib
    monkeypatch.setenv("AMQFT_LARGE_WS_MB", "1")
    _say("forced large path", dtype, "variant", variant, "n", n, "batch", batch)
    xfail_unpinned(_large_case(api, _lib, variant, dtype, n, batch, _lib.FLAG_FORCE_LARGE))


@pytest.mark.gpu
@pytest.mark.parametrize("n", [1 << 18, 1 << 20])
@pytest.mark.parametrize("variant", [4, 8, 2, 6])
def test_large_path_deep(variant, n):
    """N = 2^18 and 2^20 (FP32) on the six-kernel path (variants 4, 8) and its
    transpose (2, 6): depth-3 rows split once more into depth-6 rows; table
    and device-generated constants, adjoint.  The depth-6 kernels (rtop,
    rback and their transposes) exist only from 2^18, where variants 6 and 8
    have no pin: their cases are reported, not asserted."""
    api = _api()
    from paper_1404_1810_amd import _lib
    batch = 2 if n == 1 << 18 else 1
    _say("deep large path c64 variant", variant, "n", n, "batch", batch)
    x_np = inputs.complex_normal(6000 + n, batch, n).astype(np.complex64)
    ref = truth(x_np, 4)
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    reports = []
    for flags in (0, _lib.FLAG_ONTHEFLY_CONSTANTS):
        plan = api.Plan(n, batch, variant, _lib.C64, flags)
        assert "rtop" in plan.describe(), plan.describe()
        y = plan.exec(x)
        torch.cuda.synchronize()
        reports.append(assess(y.cpu().numpy(), ref, variant, False, x_np, "n=%d flags=%d" % (n, flags)))
        if flags == 0 and n == 1 << 18:
            g = plan.exec(x, adjoint=True)
            torch.cuda.synchronize()
            reports.append(assess(np.conj(g.cpu().numpy()), np.conj(np.conj(truth(np.conj(x_np), 4))), variant,
                                  False, np.conj(x_np), "n=%d adjoint" % n))
        plan.close()
    xfail_unpinned(reports)


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("variant", VARIANTS)
def test_plan_constants_device_table(variant, dtype):
    """amqft_plan_constants returns what the kernels read: the host table
    (long double, rounded once) without the on-the-fly flag, the device FP64
    table with it.  The two agree bit for bit in FP32 except where the FP64
    value lies within 2^-40 (relative) of a halfway point between two floats
    (double rounding); in FP64 within 4 ulp (the device's cospi / sinpi and the
    reciprocal round separately)."""
    api = _api()
    from paper_1404_1810_amd import _lib
    for n in (1 << 10, 1 << 16):
        _say("constants variant", variant, "dtype", dtype, "n", n)
        host = api.Plan(n, 1, variant, dtype, 0)
        dev = api.Plan(n, 1, variant, dtype, _lib.FLAG_ONTHEFLY_CONSTANTS)
        a, b = host.constants(), dev.constants()
        host.close()
        dev.close()
        assert a.shape == b.shape == (n // 4,)
        assert a[0] == 0 and b[0] == 0
        fam = {1: 0, 2: 1, 3: 0, 4: 1, 5: 2, 6: 3, 7: 2, 8: 3}[variant]
        p = np.arange(1, n // 4, dtype=np.longdouble)
        ang = 2 * np.pi * p / np.longdouble(n)  # numpy's pi: exact to double, enough for the tie test
        exact = {0: 2 * np.cos(ang), 1: 1 / (2 * np.cos(ang)), 2: 2 * np.sin(ang), 3: 1 / (2 * np.sin(ang))}[fam]
        if dtype == 1:
            diff = np.nonzero(a[1:] != b[1:])[0]
            for i in diff:
                lo, hi = sorted((np.float32(a[1 + i]), np.float32(b[1 + i])))
                assert np.nextafter(lo, np.float32(np.inf)) == hi, (variant, n, i)
                mid = (np.longdouble(lo) + np.longdouble(hi)) / 2
                assert abs(exact[i] - mid) <= abs(mid) * 2.0 ** -40, (variant, n, i, a[1 + i], b[1 + i])
            assert len(diff) <= max(2, n // 4 // 1000), (variant, n, len(diff))
        else:
            ulp = np.spacing(np.abs(a[1:]))
            assert np.all(np.abs(a[1:] - b[1:]) <= 4 * ulp), (variant, n)


@pytest.mark.gpu
def test_alloc_failure_status(monkeypatch):
    """A plan whose workspace cannot be allocated returns AMQFT_ERR_ALLOC (and
    no plan); nothing is launched.  2^21 signals of 2^15 points with one chunk
    spanning all of them: 512 GiB per workspace buffer."""
    from paper_1404_1810_amd import _lib
    import ctypes
    lib = _lib.load()
    monkeypatch.setenv("AMQFT_LARGE_WS_MB", str(1 << 20))
    h = ctypes.c_void_p(1)
    _say("allocation failure")
    st = lib.amqft_plan_create(ctypes.byref(h), 1 << 15, 1 << 21, 4, _lib.C64, 0)
    assert st == _lib.ERR_ALLOC, st
    assert not h.value
    torch.cuda.synchronize()
    x = torch.ones(4, 64, dtype=torch.complex64, device="cuda")  # the device still works
    assert torch.allclose(_api().fft(x, 4)[:, 0], torch.full((4,), 64, dtype=torch.complex64, device="cuda"))


def _closed_form_inputs(n):
    """delta(0), delta(N/2), ones, i delta(0): spectra ones, (-1)^k, N delta(k),
    i -- exact in the FP32 oracle of every variant at these sizes, because the
    ill-conditioned constants of variants 5-8 multiply only zeros."""
    k = np.arange(n)
    x = np.zeros((4, n), np.complex128)
    x[0, 0] = 1
    x[1, n // 2] = 1
    x[2, :] = 1
    x[3, 0] = 1j
    want = np.stack([np.ones(n), (-1.0) ** k, n * (k == 0), 1j * np.ones(n)]).astype(np.complex128)
    return x, want


@pytest.mark.gpu
@pytest.mark.parametrize("dtype,n,flags", (("c64", 1 << 15, 0), ("c64", 1 << 17, 0), ("c128", 1 << 15, 0),
                                           ("c64", 1 << 20, 0), ("c64", 1 << 16, 32), ("c128", 1 << 12, 4)))
@pytest.mark.parametrize("variant", [5, 6, 7, 8])
def test_closed_forms_where_random_inputs_have_no_pin(variant, dtype, n, flags):
    """Variants 5-8 above one workgroup's LDS have no pin for random inputs
    (their own error in the oracle is of order one or not finite).  Four
    inputs with closed-form spectra pin every path they take there -- the
    large-N path (8), its transposed program (6), the multi-pass engine (5,
    7; also forced), in place where it exists -- to the exact result: a
    kernel that drops, misplaces or mis-signs any output fails."""
    api = _api()
    from paper_1404_1810_amd import _lib
    if flags == 32 and variant != 8:
        pytest.skip("in place above LDS: variants 4 and 8")
    x_np, want = _closed_form_inputs(n)
    code = _lib.C128 if dtype == "c128" else _lib.C64
    _say("closed forms variant", variant, dtype, "n", n, "flags", flags)
    x = torch.from_numpy(x_np.astype(np.complex128 if dtype == "c128" else np.complex64)).cuda()
    plan = api.Plan(n, 4, variant, code, flags)
    if flags == 32:
        plan.exec(x, out=x)
        y = x
    else:
        y = plan.exec(x)
    torch.cuda.synchronize()
    plan.close()
    got = y.cpu().numpy().astype(np.complex128)
    assert np.all(np.isfinite(got))
    for row in range(4):
        e = np.linalg.norm(got[row] - want[row]) / np.linalg.norm(want[row])
        assert e <= 1e-6, (row, e)
