"""amqft_exec_noalloc (no plan, no allocation; workspace in a fixed device
array per GPU) against amqft_exec on a plan with device-generated constants:
the same kernels and constants, so the outputs must agree bit for bit.  Each
case runs two calls in a row on the shared scratch array, the second with a
smaller input, and checks a few signals of the pinned variant against the
oracle as well."""
import sys

import numpy as np
import pytest

from gpu_common import rel, truth
from paper_1404_1810_amd import inputs

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _tensor(dtype, n, batch, seed):
    z = inputs.complex_normal(seed, batch, n)
    if dtype == "c128":
        return torch.from_numpy(z).cuda()
    if dtype == "c64":
        return torch.from_numpy(z.astype(np.complex64)).cuda()
    h = np.empty((batch, n, 2), dtype=np.float16)
    h[..., 0] = z.real / 4
    h[..., 1] = z.imag / 4
    return torch.from_numpy(h).cuda()


def _check(api, _lib, variant, dtype, n, batch, adjoint, seed):
    code = {"c128": _lib.C128, "c64": _lib.C64, "f16": _lib.C32H}[dtype]
    _say("noalloc", dtype, "variant", variant, "n", n, "batch", batch, "adjoint", adjoint)
    x = _tensor(dtype, n, batch, seed)
    y = torch.full_like(x, 3.0) if dtype == "f16" else torch.full_like(x, complex(3.0, 3.0))
    api.exec_noalloc(x, variant, adjoint=adjoint, out=y)
    plan = api.Plan(n, batch, variant, code, _lib.FLAG_ONTHEFLY_CONSTANTS)
    ref = plan.exec(x, adjoint=adjoint)
    torch.cuda.synchronize()
    plan.close()
    assert torch.equal(y, ref), (variant, dtype, n, batch)
    if variant in (2, 4) and dtype != "f16":
        xs = x[:2].cpu().numpy()
        want = np.conj(truth(np.conj(xs), 4)) if adjoint else truth(xs, 4)
        assert rel(y[:2].cpu().numpy(), want) <= (1e-12 if dtype == "c128" else 1e-5)


CASES = [
    # (variant, dtype, (n, batch) of the first call, (n, batch) of the second, smaller call)
    (4, "c64", (1 << 16, 130), (1 << 15, 5)),    # large-N path, 3 chunks then 1
    (2, "c64", (1 << 16, 50), (1 << 15, 3)),     # multi-pass path, 2 chunks then 1
    (4, "c64", (4096, 33), (1024, 5)),           # LDS kernel (no scratch)
    (4, "c128", (1 << 15, 9), (1 << 14, 2)),     # FP64 large-N path
    (4, "f16", (1 << 20, 4), (1 << 18, 2)),      # FP16 storage, six-kernel path
]


@pytest.mark.gpu
@pytest.mark.parametrize("variant,dtype,first,second", CASES)
def test_noalloc_matches_plan(variant, dtype, first, second):
    from paper_1404_1810_amd import _lib, api
    for k, (n, batch) in enumerate((first, second)):
        _check(api, _lib, variant, dtype, n, batch, adjoint=False, seed=900 + k)
    _check(api, _lib, variant, dtype, second[0], second[1], adjoint=True, seed=950)


@pytest.mark.gpu
def test_noalloc_in_place_and_empty():
    from paper_1404_1810_amd import _lib, api
    n, batch = 1 << 16, 7
    x = _tensor("c64", n, batch, 990)
    _say("noalloc in place n", n)
    ref = api.Plan(n, batch, 4, _lib.C64, _lib.FLAG_ONTHEFLY_CONSTANTS).exec(x)
    z = x.clone()
    api.exec_noalloc(z, 4, out=z)
    torch.cuda.synchronize()
    assert torch.equal(z, ref)
    e = torch.empty((0, n), dtype=torch.complex64, device="cuda")
    assert api.exec_noalloc(e, 4).shape == (0, n)
