"""In-place execution (AMQFT_FLAG_IN_PLACE; Sec. 7.1 states that every
variant can run in place and leaves an efficient in-place form open).

Above one workgroup's LDS the in-place large-N path keeps the recursion's
depth-3 rows in the signal's own buffer and needs about a quarter of a signal
of workspace.  It performs the out-of-place path's operations in the same
order: without FMA contraction (the CPU emulation of the kernel sources) the
two agree bit for bit; here the compiler contracts the two instantiations
differently, so they must agree to within a few times the out-of-place
path's own rounding error, and (where the variant has a pin) the in-place
result must meet the oracle's pin.

Every case prints its identity before it touches the GPU.
"""
import ctypes
import sys

import numpy as np
import pytest

from gpu_common import assess, rel, truth, xfail_unpinned
from paper_1404_1810_amd import inputs

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _agree(y_ip, y_op, x_np, adjoint):
    """The two paths differ by rounding only: their distance is within four
    times the out-of-place result's own distance from the exact DFT (and at
    most a few units of the working precision where that is tiny)."""
    ref = np.conj(truth(np.conj(x_np), 4)) if adjoint else truth(x_np, 4)
    own = rel(y_op, ref)
    eps = np.finfo(y_op.dtype).eps
    d = rel(y_ip, y_op)
    assert d <= max(4 * own, 8 * eps), (d, own)


def _both(api, _lib, variant, dtype, n, batch, flags_extra, adjoint):
    """(in-place result, out-of-place result, input) for one batch."""
    f64 = dtype == "c128"
    x_np = inputs.complex_normal(7000 + n + variant, batch, n)
    if not f64:
        x_np = x_np.astype(np.complex64)
    code = _lib.C128 if f64 else _lib.C64
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    pi = api.Plan(n, batch, variant, code, _lib.FLAG_IN_PLACE | flags_extra)
    d = pi.describe()
    large = bool(flags_extra & _lib.FLAG_FORCE_LARGE) or n > (1 << (13 if f64 else 14))
    assert ("in place" in d) == bool(large), d
    y_ip = x.clone()
    pi.exec(y_ip, out=y_ip, adjoint=adjoint)
    po = api.Plan(n, batch, variant, code, flags_extra)
    y_op = po.exec(x, adjoint=adjoint)
    torch.cuda.synchronize()
    pi.close()
    po.close()
    return y_ip.cpu().numpy(), y_op.cpu().numpy(), x_np


IP_LARGE = (("c64", 1 << 15, 5), ("c64", 1 << 16, 3), ("c64", 1 << 17, 2), ("c128", 1 << 14, 3),
            ("c128", 1 << 16, 2))


@pytest.mark.gpu
@pytest.mark.parametrize("dtype,n,batch", IP_LARGE)
@pytest.mark.parametrize("variant", [4, 8])
@pytest.mark.parametrize("adjoint", [False, True])
def test_in_place_large_equals_out_of_place(variant, dtype, n, batch, adjoint, monkeypatch):
    """Forward and adjoint, workspaces cut to 1 MiB so that batches run in
    several chunks with a ragged last one."""
    api = __import__("paper_1404_1810_amd.api", fromlist=["api"])
    from paper_1404_1810_amd import _lib
    monkeypatch.setenv("AMQFT_LARGE_WS_MB", "1")
    _say("in-place large path", dtype, "variant", variant, "n", n, "batch", batch, "adjoint", adjoint)
    y_ip, y_op, x_np = _both(api, _lib, variant, dtype, n, batch, 0, adjoint)
    _agree(y_ip, y_op, x_np, adjoint)
    if not adjoint:
        xfail_unpinned([assess(y_ip, truth(x_np, 4), variant, dtype == "c128", x_np, "%s n=%d" % (dtype, n))])


@pytest.mark.gpu
@pytest.mark.parametrize("dtype,n,batch", (("c128", 1 << 11, 5), ("c128", 1 << 12, 3), ("c128", 1 << 13, 2),
                                           ("c64", 1 << 12, 3), ("c64", 1 << 14, 2)))
@pytest.mark.parametrize("variant", [4, 8])
def test_in_place_large_forced(variant, dtype, n, batch, monkeypatch):
    """The in-place kernels forced at N = 2^11 .. 2^14: at FP64 2^11 and 2^12
    variant 8 is pinned at 20x its own FP64 error, so every in-place kernel of
    both variants meets a pin; the output agrees with the forced out-of-place
    path's to rounding."""
    api = __import__("paper_1404_1810_amd.api", fromlist=["api"])
    from paper_1404_1810_amd import _lib
    monkeypatch.setenv("AMQFT_LARGE_WS_MB", "1")
    _say("forced in-place large path", dtype, "variant", variant, "n", n, "batch", batch)
    y_ip, y_op, x_np = _both(api, _lib, variant, dtype, n, batch, _lib.FLAG_FORCE_LARGE, False)
    _agree(y_ip, y_op, x_np, False)
    xfail_unpinned([assess(y_ip, truth(x_np, 4), variant, dtype == "c128", x_np, "forced %s n=%d" % (dtype, n))])


@pytest.mark.gpu
@pytest.mark.parametrize("variant,dtype,n", ((4, "c64", 4096), (2, "c64", 1 << 14), (1, "c128", 1024),
                                             (7, "c64", 256), (5, "c128", 64), (3, "c64", 16)))
def test_in_place_within_lds(variant, dtype, n):
    """Up to one workgroup's LDS every variant runs in place with no
    workspace (each workgroup loads its signals before it stores them): the
    same kernel as out of place, so the same bits."""
    api = __import__("paper_1404_1810_amd.api", fromlist=["api"])
    from paper_1404_1810_amd import _lib
    _say("in place within LDS variant", variant, dtype, "n", n)
    y_ip, y_op, _ = _both(api, _lib, variant, dtype, n, 7, 0, False)
    assert np.array_equal(y_ip, y_op)
    p = api.Plan(n, 7, variant, _lib.C128 if dtype == "c128" else _lib.C64, _lib.FLAG_IN_PLACE)
    ws = ctypes.c_size_t(1)
    _lib.check(_lib.load().amqft_plan_workspace_size(p.handle, ctypes.byref(ws)), "workspace")
    p.close()
    assert ws.value == 0


@pytest.mark.gpu
@pytest.mark.parametrize("dtype,n", (("c64", 1 << 16), ("c128", 1 << 15)))
def test_in_place_workspace_and_rejection(dtype, n):
    """The in-place plan's workspace is below 0.25 N values a signal (the
    out-of-place path: 2 N + 16), and executing it out of place is refused."""
    api = __import__("paper_1404_1810_amd.api", fromlist=["api"])
    from paper_1404_1810_amd import _lib
    esz = 16 if dtype == "c128" else 8
    batch = 4
    _say("in-place workspace", dtype, "n", n)
    code = _lib.C128 if dtype == "c128" else _lib.C64
    sizes = {}
    for flags in (0, _lib.FLAG_IN_PLACE):
        p = api.Plan(n, batch, 4, code, flags)
        ws = ctypes.c_size_t(0)
        _lib.check(_lib.load().amqft_plan_workspace_size(p.handle, ctypes.byref(ws)), "workspace")
        sizes[flags] = ws.value
        if flags:
            x = torch.zeros(batch, n, dtype=torch.complex128 if dtype == "c128" else torch.complex64, device="cuda")
            with pytest.raises(_lib.AmqftError):
                p.exec(x)  # a fresh output buffer: not in place
            torch.cuda.synchronize()
        p.close()
    assert sizes[_lib.FLAG_IN_PLACE] <= 0.25 * n * esz * batch, sizes
    assert sizes[0] >= 2 * n * esz * batch, sizes


@pytest.mark.gpu
def test_in_place_large_full_chunk_sampled():
    """A 2^17-point batch of 64 signals in place with the default workspace
    (one chunk): sampled signals against the oracle (variant 4, FP32)."""
    api = __import__("paper_1404_1810_amd.api", fromlist=["api"])
    from paper_1404_1810_amd import _lib
    n, batch = 1 << 17, 64
    _say("in-place 2^17 x 64 sampled")
    x_np = inputs.complex_normal(4242, batch, n).astype(np.complex64)
    x = torch.from_numpy(x_np).cuda()
    p = api.Plan(n, batch, 4, _lib.C64, _lib.FLAG_IN_PLACE)
    p.exec(x, out=x)
    torch.cuda.synchronize()
    p.close()
    rows = [0, 31, 63]
    y = x[rows].cpu().numpy()
    xfail_unpinned([assess(y, truth(x_np[rows], 4), 4, False, x_np[rows], "in-place 2^17 sampled")])


@pytest.mark.gpu
@pytest.mark.parametrize("variant,dtype,n", ((4, "c64", 1 << 15), (8, "c128", 1 << 14)))
def test_in_place_large_onthefly_constants(variant, dtype, n):
    """With AMQFT_FLAG_ONTHEFLY_CONSTANTS the in-place path reads the table
    the device generated; it agrees with the out-of-place path on the same
    flag to rounding, and (variant 4) with the oracle within the pin."""
    api = __import__("paper_1404_1810_amd.api", fromlist=["api"])
    from paper_1404_1810_amd import _lib
    _say("in-place on-the-fly constants variant", variant, dtype, "n", n)
    y_ip, y_op, x_np = _both(api, _lib, variant, dtype, n, 3, _lib.FLAG_ONTHEFLY_CONSTANTS, False)
    _agree(y_ip, y_op, x_np, False)
    xfail_unpinned([assess(y_ip, truth(x_np, 4), variant, dtype == "c128", x_np, "on-the-fly %s n=%d" % (dtype, n))])


@pytest.mark.gpu
@pytest.mark.parametrize("variant,n,batch", ((4, 1 << 16, 3), (2, 4096, 5), (8, 1 << 15, 2)))
def test_binding_in_place_forward_and_adjoint(variant, n, batch):
    """api.fft_ / api.adjoint_ overwrite their argument with the result the
    out-of-place calls return (to rounding above LDS; the same kernel below)."""
    from paper_1404_1810_amd import api
    _say("binding in place variant", variant, "n", n)
    x_np = inputs.complex_normal(99 + n, batch, n).astype(np.complex64)
    x = torch.from_numpy(x_np).cuda()
    want = api.fft(x, variant).cpu().numpy()
    y = x.clone()
    r = api.fft_(y, variant)
    assert r.data_ptr() == y.data_ptr()
    _agree(y.cpu().numpy(), want, x_np, False)
    g = x.clone()
    api.adjoint_(g, variant)
    _agree(g.cpu().numpy(), api.adjoint(x, variant).cpu().numpy(), x_np, True)
    with pytest.raises(ValueError):
        api.fft_(x[:, ::2], variant)


@pytest.mark.gpu
def test_in_place_empty_batch_and_small_chunks(monkeypatch):
    """An empty batch does nothing; a 1 MiB workspace runs 9 signals of 2^17
    points in place in two chunks (N/8 + 16 values of 8 B a signal: 7 fit,
    so 5 + 4)."""
    from paper_1404_1810_amd import _lib, api
    n = 1 << 17
    _say("in-place empty batch and small chunks")
    p0 = api.Plan(n, 0, 4, _lib.C64, _lib.FLAG_IN_PLACE)
    e = torch.empty(0, n, dtype=torch.complex64, device="cuda")
    p0.exec(e, out=e)
    p0.close()
    monkeypatch.setenv("AMQFT_LARGE_WS_MB", "1")
    p = api.Plan(n, 9, 4, _lib.C64, _lib.FLAG_IN_PLACE)
    assert "chunk=5" in p.describe(), p.describe()
    p.close()
    y_ip, y_op, x_np = _both(api, _lib, 4, "c64", n, 9, 0, False)
    _agree(y_ip, y_op, x_np, False)


@pytest.mark.gpu
def test_in_place_graph_replays():
    """The in-place large path captured in a HIP graph (amqft_exec_graph with
    in == out): every replay, with eager work and synchronisation between,
    equals the eager in-place result on a fresh copy of the input; a graph
    execution with distinct buffers is refused before any capture."""
    from paper_1404_1810_amd import _lib, api
    n, batch = 1 << 15, 3
    _say("in-place graph replays")
    x_np = inputs.complex_normal(31337, batch, n).astype(np.complex64)
    x0 = torch.from_numpy(x_np).cuda()
    p = api.Plan(n, batch, 4, _lib.C64, _lib.FLAG_IN_PLACE)
    ref = x0.clone()
    p.exec(ref, out=ref)
    torch.cuda.synchronize()
    buf = torch.empty_like(x0)
    for rep in range(3):
        buf.copy_(x0)
        torch.cuda.synchronize()
        api.exec_graph(p, buf, buf)
        torch.cuda.synchronize()
        assert torch.equal(buf, ref), rep
        _ = (x0 * 2).sum().item()  # eager work between the replays
    other = torch.empty_like(x0)
    with pytest.raises(_lib.AmqftError):
        api.exec_graph(p, x0, other)
    torch.cuda.synchronize()
    p.close()
