"""CPU emulation of the HIP kernel sources (no GPU): the compile-time kernels
of both skeletons, the large-N path and the generic engines, compiled for the
host with the shim of tests/emu under AddressSanitizer and UBSan, every
workgroup's LDS filled with NaN bytes, LDS accesses checked for races between
barriers and buffer accesses for their bounds, and the results compared with
the oracle under the pins of the GPU tests.  This is how a kernel is run
before its first GPU launch; here it guards the sources on every CPU run."""
import os
import subprocess
import sys

import numpy as np
import pytest

from gpu_common import bound, rel, truth
from paper_1404_1810_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "emu"))


@pytest.fixture(scope="module")
def emu_exe():
    import build_emu
    try:
        return build_emu.build()
    except FileNotFoundError:  # pragma: no cover
        pytest.skip("host clang++ not available")


CASES = [
    # (path, variant, dtype 0 = FP64 / 1 = FP32, log2 N, batch, conjugated in and out)
    ("lds", 4, 1, 12, 2, 0),     # amqft_kA_kernel, headline geometry
    ("lds", 4, 0, 13, 1, 0),
    ("lds", 1, 1, 14, 1, 0),     # recurrences across several waves
    ("lds", 5, 0, 9, 3, 1),      # two signals per workgroup, adjoint
    ("lds", 8, 0, 11, 2, 0),
    ("lds", 4, 1, 10, 40, 1),    # one-wave workgroups, many of them
    ("lds", 5, 0, 9, 23, 0),     # two signals a workgroup, ragged last one
    ("tkernel", 2, 0, 8, 5, 0),  # amqft_kB_kernel: four signals per workgroup
    ("tkernel", 2, 0, 11, 2, 1),
    ("tkernel", 2, 1, 12, 2, 0),
    ("tkernel", 6, 0, 10, 2, 0),
    ("tkernel", 6, 1, 8, 3, 1),
    ("tkernel", 2, 1, 14, 1, 1),
    ("tkernel", 2, 1, 13, 1, 0),  # both fold walks with four values a lane in the second
    ("tkernel", 3, 0, 8, 5, 0),  # transposed recurrences, four signals per workgroup
    ("tkernel", 3, 1, 14, 1, 0),  # ... across several waves
    ("tkernel", 7, 0, 12, 1, 1),
    ("large", 4, 0, 11, 2, 0),   # top / rows / back / bchain, rows sharing workgroups
    ("large", 8, 0, 12, 1, 1),
    ("large", 4, 0, 11, 16, 1),  # 16 chain workgroups: the XCD remap of bchain permutes them
    ("large", 2, 0, 11, 3, 0),   # transposed large path (c0 / fold / b0 / rows / top), rows sharing workgroups
    ("large", 6, 0, 12, 2, 1),
    ("large", 2, 1, 12, 2, 0),
    ("large", 2, 0, 13, 1, 1),   # two-walk fold, 4096-point rows
    ("generic", 3, 0, 10, 3, 0),  # level engine
    ("multipass", 1, 0, 10, 3, 0),  # multi-pass engine: global recurrence scans (skeleton A), LDS sub-blocks
    ("multipass", 3, 0, 11, 2, 1),  # ... skeleton B, adjoint, two chunks
    ("multipass", 5, 0, 9, 3, 0),
    ("multipass", 7, 0, 10, 2, 0),
    ("multipass", 4, 1, 11, 2, 0),  # gather levels only
    ("lds", 7, 0, 12, 1, 0),     # amqft_fast_kernel
]


@pytest.mark.parametrize("path,variant,dtype,logn,batch,conj", CASES)
def test_kernel_source_on_cpu(emu_exe, tmp_path, path, variant, dtype, logn, batch, conj):
    n = 1 << logn
    x = inputs.complex_normal(7 + logn, batch, n).astype(np.complex128 if dtype == 0 else np.complex64)
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    x.tofile(fin)
    r = subprocess.run([emu_exe, path, str(variant), str(dtype), str(logn), str(batch), str(conj), fin, fout],
                       capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1"))
    assert r.returncode == 0, r.stderr[-4000:]
    y = np.fromfile(fout, dtype=x.dtype).reshape(batch, n)
    src = np.conj(x) if conj else x
    ref = truth(src)
    if conj:
        ref = np.conj(ref)
    b = bound(variant, dtype == 0, src, ref if not conj else np.conj(ref))
    assert b is not None, "every emulated case is chosen where its variant has a pin"
    assert rel(y, ref) <= b, (rel(y, ref), b)


# In-place large path: (variant, dtype, log2 N, batch, conjugated).  2^13,
# 2^14 and 2^15 have two, four and eight chain workgroups a signal (2^15: a
# size the path runs at unforced); 16 signals in chunks of 15 with the XCD
# remap of the chain kernel.
IP_CASES = [(4, 0, 13, 2, 0), (8, 0, 12, 1, 1), (4, 1, 12, 3, 0), (8, 0, 11, 16, 1), (4, 0, 14, 1, 0),
            (4, 1, 15, 2, 0)]


def _run_emu(exe, tmp_path, path, variant, dtype, logn, batch, conj, x, track=True):
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / ("out_%s.bin" % path))
    x.tofile(fin)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    if track:
        env["EMU_TRACK_GLOBAL"] = "1"
    r = subprocess.run([exe, path, str(variant), str(dtype), str(logn), str(batch), str(conj), fin, fout],
                       capture_output=True, text=True, timeout=600, env=env)
    y = np.fromfile(fout, dtype=x.dtype).reshape(x.shape) if r.returncode == 0 else None
    return r, y


@pytest.mark.parametrize("variant,dtype,logn,batch,conj", IP_CASES)
def test_in_place_large_path(emu_exe, tmp_path, variant, dtype, logn, batch, conj):
    """The in-place form of the large-N path keeps the rows in the signal's own
    buffer: no workgroup may read or write a word that another workgroup of
    the same launch writes (checked on every access to the signal), and the
    result is the out-of-place path's, bit for bit (same operations, same
    order), within the variant's pin of the exact DFT."""
    n = 1 << logn
    x = inputs.complex_normal(7 + logn, batch, n).astype(np.complex128 if dtype == 0 else np.complex64)
    r_ip, y_ip = _run_emu(emu_exe, tmp_path, "large_ip", variant, dtype, logn, batch, conj, x)
    assert r_ip.returncode == 0, r_ip.stderr[-4000:]
    r, y = _run_emu(emu_exe, tmp_path, "large", variant, dtype, logn, batch, conj, x)
    assert r.returncode == 0, r.stderr[-4000:]
    assert np.array_equal(y_ip, y)
    src = np.conj(x) if conj else x
    ref = truth(src)
    b = bound(variant, dtype == 0, src, ref)
    if conj:
        ref = np.conj(ref)
    assert rel(y_ip, ref) <= b, (rel(y_ip, ref), b)


def test_in_place_checker_rejects_a_layout_that_ignores_the_readers(emu_exe, tmp_path):
    """The cross-workgroup checker's own test: with every slot left in its own
    orbit (no ownership, nothing shared) chain workgroups overwrite rows that
    other chain workgroups still read."""
    x = inputs.complex_normal(20, 2, 1 << 13)
    r, _ = _run_emu(emu_exe, tmp_path, "large_ip_naive", 4, 0, 13, 2, 0, x)
    assert r.returncode == 5 and "cross-workgroup hazards" in r.stderr, (r.returncode, r.stderr[-2000:])


# The depth-6 split of the transposed large path (N >= 2^18) takes about
# three minutes here; AMQFT_EMU_DEEP=1 adds it.
DUAL_CASES = [("tkernel", 2, 12), ("tkernel", 6, 9), ("tkernel", 2, 8), ("tkernel", 6, 8),
              ("large", 2, 12), ("large", 6, 11)] + ([("large", 2, 18)] if os.environ.get("AMQFT_EMU_DEEP") else [])


@pytest.mark.parametrize("path,vb,logn", DUAL_CASES)
def test_transposed_program_is_the_dual_variant(emu_exe, tmp_path, path, vb, logn):
    """The duality of the paper's M steps (M4^T = M2, M8^T = M6; skeleton A
    <-> B): the transposed program of the skeleton-A kernel of variant 4 (8),
    and of its large-N path, run without FMA contraction, reproduces the
    oracle's FP32 build of
    variant 2 (6) bit for bit -- including variant 6's ill-conditioned
    rounding, which differs from variant 8's by more than the error itself."""
    import oracle
    n, batch = 1 << logn, 3
    x = inputs.complex_normal(31 + logn, batch, n).astype(np.complex64)
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    x.tofile(fin)
    r = subprocess.run([emu_exe, path, str(vb), "1", str(logn), str(batch), "0", fin, fout],
                       capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1"))
    assert r.returncode == 0, r.stderr[-4000:]
    y = np.fromfile(fout, dtype=np.complex64).reshape(batch, n)
    emu = oracle.cdft(x, vb, prec="f32")
    assert np.array_equal(y, emu), rel(y, emu)
    if vb == 6:  # the skeleton-A twin rounds differently
        assert not np.array_equal(y, oracle.cdft(x, 8, prec="f32"))


FIXED_CASES = [
    # (path, variant, log2 N, batch, conjugated in and out): int32 fixed point
    ("lds", 1, 12, 2, 0),      # amqft_kA_kernel, M1 recurrences as lane scans
    ("lds", 5, 9, 3, 1),       # two signals per workgroup, adjoint
    ("lds", 1, 14, 1, 0),
    ("tkernel", 3, 12, 1, 0),  # amqft_kB_kernel: the transposed recurrences
    ("tkernel", 7, 8, 5, 1),
    ("tkernel", 3, 13, 1, 1),
]


@pytest.mark.parametrize("path,variant,logn,batch,conj", FIXED_CASES)
def test_fixed_point_kernel_source_is_bit_exact(emu_exe, tmp_path, path, variant, logn, batch, conj):
    """Fixed point: sums are exact, so the kernels (scans, transposed levels,
    any order of the sums) must round exactly the values the recursion
    rounds -- the output equals the fixed-point oracle's bit for bit."""
    import oracle
    n = 1 << logn
    rng = np.random.default_rng(100 + logn + variant)
    x = rng.integers(-2 ** 15, 2 ** 15, size=(batch, n, 2), dtype=np.int32)
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    x.tofile(fin)
    r = subprocess.run([emu_exe, path, str(variant), "4", str(logn), str(batch), str(conj), fin, fout],
                       capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1"))
    assert r.returncode == 0, r.stderr[-4000:]
    y = np.fromfile(fout, dtype=np.int32).reshape(batch, n, 2)
    sgn = -1 if conj else 1  # adjoint: conj(F conj(x)); negation is exact
    Xr, Xi, wraps = oracle.cdft_fixed(x[..., 0], sgn * x[..., 1], variant)
    assert np.array_equal(y[..., 0], Xr) and np.array_equal(y[..., 1], sgn * Xi), \
        (int(np.sum(y[..., 0] != Xr)), int(np.sum(y[..., 1] != sgn * Xi)), wraps)
