"""Seeded synthetic workloads (inputs only -- no transform arithmetic here).

The paper publishes no data set; its accuracy study uses unstated inputs.  The
workloads below are the five benchmark configurations of this project, each
generated from fixed seeds.  Every signal ``b`` of a batch is drawn from its
own generator ``numpy.random.default_rng([seed, b])`` so that any single
signal of a full-size batch can be regenerated on its own (sampled parity
checks at full size need this).

Both the GPU tests/benchmark and the CPU oracle consume these arrays; nothing
in this module depends on either side.
"""
from __future__ import annotations

import numpy as np

#: seeds of the five configurations
SEEDS = {"fp64_n256": 0, "fp32_n4096": 0, "uneven_lengths": 2, "uneven_entries": 3,
         "grad_x": 0, "grad_w": 1, "fp16_n2p20": 0, "fixed_n4096": 5}


def _rows(seed: int, batch: int, n: int, kind: str, start: int = 0, out: np.ndarray | None = None) -> np.ndarray:
    """complex128 array (batch, n); rows start..start+batch-1 of the stream
    (written into ``out`` when given, which avoids fresh page faults)."""
    if out is None:
        out = np.empty((batch, n), dtype=np.complex128)
    parts = out.view(np.float64).reshape(batch, n, 2)  # (re, im) interleaved
    for b in range(batch):
        g = np.random.default_rng([seed, start + b])
        if kind == "normal":
            re = g.standard_normal(n)
            im = g.standard_normal(n)
        elif kind == "uniform":  # U[-1, 1)
            re = g.random(n) * 2.0 - 1.0
            im = g.random(n) * 2.0 - 1.0
        else:
            raise ValueError(kind)
        parts[b, :, 0] = re
        parts[b, :, 1] = im
    return out


def complex_normal(seed: int, batch: int, n: int, start: int = 0, out: np.ndarray | None = None) -> np.ndarray:
    """Re and Im i.i.d. N(0,1), generated in float64 (cast by the caller)."""
    return _rows(seed, batch, n, "normal", start, out)


def complex_uniform(seed: int, batch: int, n: int, start: int = 0) -> np.ndarray:
    """Re and Im i.i.d. uniform on [-1, 1), generated in float64."""
    return _rows(seed, batch, n, "uniform", start)


def real_normal(seed: int, batch: int, n: int) -> np.ndarray:
    """Real signals, i.i.d. N(0,1), float64 (batch, n); signal b from
    default_rng([seed, b]) like the complex rows."""
    out = np.empty((batch, n), dtype=np.float64)
    for b in range(batch):
        out[b] = np.random.default_rng([seed, b]).standard_normal(n)
    return out


def cfg_fp64_n256(batch: int = 64, n: int = 256) -> np.ndarray:
    """Configuration 1: complex128, 64 x N=256, U[-1,1), seed 0."""
    return complex_uniform(SEEDS["fp64_n256"], batch, n)


def chunks(kind: str, seed: int, batch: int, n: int, chunk: int = 512):
    """Yield (start, rows) of a large batch, chunk rows at a time, reusing one
    complex128 buffer (the caller copies each chunk out before the next)."""
    buf = np.empty((min(chunk, max(batch, 1)), n), dtype=np.complex128)
    for s0 in range(0, batch, chunk):
        m = min(chunk, batch - s0)
        yield s0, _rows(seed, m, n, kind, s0, buf[:m])


def cfg_fp32_n4096(batch: int = 16384, n: int = 4096, start: int = 0) -> np.ndarray:
    """Configuration 2: complex64, 16384 x N=4096, N(0,1), seed 0."""
    return complex_normal(SEEDS["fp32_n4096"], batch, n, start).astype(np.complex64)


def uneven_lengths(count: int = 20000, kmin: int = 4, kmax: int = 16, seed: int | None = None):
    """Configuration 3 layout: lengths 2^k with k i.i.d. uniform on {kmin..kmax}
    (seed 2), packed in generation order; offsets = exclusive prefix sum in
    complex elements, int64, length count+1."""
    g = np.random.default_rng(SEEDS["uneven_lengths"] if seed is None else seed)
    k = g.integers(kmin, kmax + 1, size=count)
    lengths = (np.int64(1) << k.astype(np.int64)).astype(np.int64)
    offsets = np.zeros(count + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    return lengths, offsets


def uneven_entries(lengths: np.ndarray, offsets: np.ndarray, seed: int | None = None,
                   dtype=np.complex64) -> np.ndarray:
    """Entries of configuration 3: signal i gets N(0,1) Re/Im from its own
    generator default_rng([3, i])."""
    s = SEEDS["uneven_entries"] if seed is None else seed
    out = np.empty(int(offsets[-1]), dtype=dtype)
    for i, (n, o) in enumerate(zip(lengths, offsets[:-1])):
        g = np.random.default_rng([s, i])
        re = g.standard_normal(int(n))
        im = g.standard_normal(int(n))
        out[o:o + n] = (re + 1j * im).astype(dtype)
    return out


def cfg_grad(batch: int = 4096, n: int = 1024):
    """Configuration 4: x ~ complex N(0,1) (seed 0), W ~ complex N(0,1) fixed
    (seed 1, one weight vector per batch row), both complex64."""
    x = complex_normal(SEEDS["grad_x"], batch, n).astype(np.complex64)
    w = complex_normal(SEEDS["grad_w"], batch, n).astype(np.complex64)
    return x, w


def cfg_fp16_rows(batch: int, n: int = 1 << 20, start: int = 0) -> np.ndarray:
    """Configuration 5 rows: U[-1,1) Re/Im (seed 0), returned as float16 pairs,
    shape (batch, n, 2) -- the interleaved half2 storage layout."""
    z = complex_uniform(SEEDS["fp16_n2p20"], batch, n, start)
    out = np.empty((batch, n, 2), dtype=np.float16)
    out[..., 0] = z.real.astype(np.float16)
    out[..., 1] = z.imag.astype(np.float16)
    return out


def to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round float32/float64 values to bfloat16 (round to nearest even) and
    return the raw 16-bit patterns as uint16."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    r = ((u + rounding) >> 16).astype(np.uint16)
    nan = np.isnan(f)
    if nan.any():
        r[nan] = 0x7FC0
    return r


def from_bf16_bits(b: np.ndarray) -> np.ndarray:
    """Widen raw bfloat16 patterns (uint16) to float32."""
    return (np.ascontiguousarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def int_pairs(seed: int, batch: int, n: int, bits: int) -> np.ndarray:
    """int32 array (batch, n, 2) of (re, im) pairs uniform on [-2^bits, 2^bits)
    (fixed-point storage)."""
    return np.random.default_rng(seed).integers(-2 ** bits, 2 ** bits, size=(batch, n, 2), dtype=np.int32)
