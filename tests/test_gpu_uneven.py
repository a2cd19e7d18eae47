"""Uneven batches: one plan over signals of many power-of-two lengths in a
packed buffer (persistent launch + long-length classes), its autotuning,
its HIP graph, against the oracle and against plain per-length plans."""
import sys

import numpy as np
import pytest

from gpu_common import assess, rel, truth, xfail_unpinned
from paper_1404_1810_amd import inputs

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _layout(ks, gap=0):
    lengths = np.array([1 << int(k) for k in ks], dtype=np.int64)
    offsets = np.zeros(len(ks) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lengths + gap)
    return lengths, offsets


@pytest.mark.gpu
@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7, 8])
def test_uneven_against_oracle(variant):
    from paper_1404_1810_amd import api
    rng = np.random.default_rng(variant)
    ks = list(range(0, 17)) + list(rng.integers(0, 17, size=40))
    lengths, offsets = _layout(ks, gap=3)  # gaps between signals stay untouched
    _say("uneven variant", variant, "signals", len(ks), "points", int(offsets[-1]))
    buf = (rng.standard_normal(int(offsets[-1])) + 1j * rng.standard_normal(int(offsets[-1]))).astype(np.complex64)
    plan = api.ManyPlan(lengths, offsets, variant, 1)
    x = torch.from_numpy(buf).cuda()
    y = torch.full_like(x, complex(7.0, 7.0))
    plan.exec(x, out=y)
    got = y.cpu().numpy()
    reports = []
    for i, (n, o) in enumerate(zip(lengths, offsets[:-1])):
        seg = buf[o:o + n]
        ref = truth(seg[None, :], 4)[0]
        assert np.all(got[o + n:offsets[i + 1]] == np.complex64(7 + 7j))  # gaps untouched
        reports.append(assess(got[o:o + n][None, :], ref[None, :], variant, False, seg[None, :],
                              "signal %d n=%d" % (i, n)))
    xfail_unpinned(reports)


@pytest.mark.gpu
@pytest.mark.parametrize("variant", [2, 4])
def test_uneven_matches_plain_per_length(variant):
    from paper_1404_1810_amd import api
    lengths, offsets = inputs.uneven_lengths(count=300, seed=7)
    total = int(offsets[-1])
    _say("uneven vs plain variant", variant, "points", total)
    buf = inputs.uneven_entries(lengths, offsets, seed=8)
    x = torch.from_numpy(buf).cuda()
    plan = api.ManyPlan(lengths, offsets, variant, 1)
    y = plan.exec(x)
    # plain path: gather each length, batched plan, scatter
    ref = torch.empty_like(x)
    for k in np.unique(lengths):
        idx = np.nonzero(lengths == k)[0]
        rows = torch.stack([x[offsets[i]:offsets[i] + k] for i in idx])
        out = api.fft(rows.contiguous(), variant)
        for r, i in enumerate(idx):
            ref[offsets[i]:offsets[i] + k] = out[r]
    torch.cuda.synchronize()
    # the persistent kernel and the per-length kernels schedule the same
    # relations differently (different rounding order): compare per length
    yn, rn = y.cpu().numpy(), ref.cpu().numpy()
    for k in np.unique(lengths):
        idx = np.nonzero(lengths == k)[0]
        a = np.concatenate([yn[offsets[i]:offsets[i] + k] for i in idx])
        b = np.concatenate([rn[offsets[i]:offsets[i] + k] for i in idx])
        assert rel(a, b) < 1e-5, (k, rel(a, b))


@pytest.mark.gpu
def test_uneven_graph_replay_and_adjoint():
    from paper_1404_1810_amd import api
    lengths, offsets = inputs.uneven_lengths(count=200, seed=9)
    buf = inputs.uneven_entries(lengths, offsets, seed=10)
    x = torch.from_numpy(buf).cuda()
    plan = api.ManyPlan(lengths, offsets, 4, 1)
    eager = plan.exec(x)
    eager_adj = plan.exec(x, adjoint=True)
    y = torch.zeros_like(x)
    for rep in range(4):
        _say("graph replay", rep)
        y.zero_()
        plan.exec(x, out=y, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(y, eager), rep
        z = x * 2  # eager work between replays
        torch.cuda.synchronize()
        del z
    ya = torch.zeros_like(x)
    plan.exec(x, out=ya, adjoint=True, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(ya, eager_adj)
    # adjoint against the oracle on a few signals
    ga = eager_adj.cpu().numpy()
    for i in (0, 1, len(lengths) - 1):
        n, o = lengths[i], offsets[i]
        ref = np.conj(truth(np.conj(buf[o:o + n])[None, :], 4))[0]
        assert rel(ga[o:o + n], ref) < 1e-5


@pytest.mark.gpu
def test_single_plan_graph_replay():
    from paper_1404_1810_amd import api
    x = torch.from_numpy(inputs.complex_normal(12, 33, 1024).astype(np.complex64)).cuda()
    plan = api.get_plan(1024, 33, 4, 1)
    eager = plan.exec(x)
    y = torch.zeros_like(x)
    for rep in range(3):
        _say("single graph replay", rep)
        y.zero_()
        api.exec_graph(plan, x, y)
        torch.cuda.synchronize()
        assert torch.equal(y, eager)


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_uneven_long_classes_only(dtype):
    """Only lengths above one workgroup's LDS (no persistent launch, no side
    stream): 2^15 and 2^16 signals interleaved, FP32 and FP64, forward and
    adjoint against the oracle."""
    from paper_1404_1810_amd import api, _lib
    ks = [15, 16, 15, 16, 15]
    lengths, offsets = _layout(ks, gap=5)
    _say("uneven long classes", dtype, "points", int(offsets[-1]))
    rng = np.random.default_rng(21)
    buf = rng.standard_normal(int(offsets[-1])) + 1j * rng.standard_normal(int(offsets[-1]))
    f64 = dtype == "c128"
    buf = buf.astype(np.complex128 if f64 else np.complex64)
    plan = api.ManyPlan(lengths, offsets, 4, _lib.C128 if f64 else _lib.C64)
    x = torch.from_numpy(buf).cuda()
    for adjoint in (False, True):
        y = torch.full_like(x, complex(7.0, 7.0))
        plan.exec(x, out=y, adjoint=adjoint)
        got = y.cpu().numpy()
        for i, (n, o) in enumerate(zip(lengths, offsets[:-1])):
            seg = buf[o:o + n]
            src = np.conj(seg) if adjoint else seg
            ref = truth(src[None, :], 4)[0]
            if adjoint:
                ref = np.conj(ref)
            assert assess(got[o:o + n][None, :], ref[None, :], 4, f64, src[None, :],
                          "signal %d n=%d adjoint=%s" % (i, n, adjoint)) is None
            assert np.all(got[o + n:offsets[i + 1]] == 7 + 7j)
