"""The oracle's pins catch plausible mistakes.

Each case below plants one mistake (a flipped sign, a dropped term, a wrong
trigonometric function, a wrong index, the paper's own sign typo in eq.
qft_19A) into a temporary copy of the oracle source, builds it, and checks
that the brute-force pin against the direct DFT fails for at least one
variant.  Nothing is planted in the GPU code.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "amqft_oracle.c")

# (description, text in the source, replacement, variants that must notice)
MUTATIONS = [
    ("dct_ot D_k sum -> difference", "e[n] = add(c, s[n], s[L / 2 - n]);\n        o[n] = sub(c, s[n], s[L / 2 - n]);\n    }\n    /* H_k: s_dc_oe",
     "e[n] = sub(c, s[n], s[L / 2 - n]);\n        o[n] = sub(c, s[n], s[L / 2 - n]);\n    }\n    /* H_k: s_dc_oe", (4,)),
    ("skeleton-A dct reflection sign", "S[L / 2 - k] = sub(c, E[k], O[k]);\n        }\n        S[q] = E[q];",
     "S[L / 2 - k] = add(c, E[k], O[k]);\n        }\n        S[q] = E[q];", (4,)),
    ("M4 dropped neighbour", "S[k] = add(c, E[k - 1], E[k + 1]);\n        S[q - 1] = E[q - 2];",
     "S[k] = E[k - 1];\n        S[q - 1] = E[q - 2];", (4,)),
    ("cos constant replaced by sin", "case COS2: v = 2.0 * cos(a); break;",
     "case COS2: v = 2.0 * sin(a); break;", (1, 3)),
    ("eq. qft_19A sign as printed", "Xi[k]     = add(c, R1i[k], R2r[k]);",
     "Xi[k]     = sub(c, R1i[k], R2r[k]);", (1, 2, 3, 4)),
    ("M2 neighbour sum -> difference", "for (long n = 2; n <= q - 2; n += 2) e[n] = add(c, s[n - 1], s[n + 1]);",
     "for (long n = 2; n <= q - 2; n += 2) e[n] = sub(c, s[n - 1], s[n + 1]);", (2,)),
    ("M7 dropped halving", "e[q] = half(c, add(c, s[q - 1], e[q - 2]));",
     "e[q] = add(c, s[q - 1], e[q - 2]);", (7,)),
    ("base constant wrong", "return (REAL)cos(M_PI / 4.0);", "return (REAL)cos(M_PI / 8.0);",
     (1, 2, 3, 4)),
    ("dst_to reflection operands transposed", "S[L / 2 - k] = sub(c, O[k], E[k]);\n    }\n    free(t); free(E); free(o); free(O);\n}\n\n/* ------------------------------------------------------------------ */\n/* dct_oo",
     "S[L / 2 - k] = sub(c, E[k], O[k]);\n    }\n    free(t); free(E); free(o); free(O);\n}\n\n/* ------------------------------------------------------------------ */\n/* dct_oo", (2,)),
    ("rdft imaginary part sign", "Ri[k] = -D[k];", "Ri[k] = D[k];", (1, 4)),
    ("M5 recurrence index", "S[k - 1] = add(c, E[k], S[k + 1]);", "S[k - 1] = add(c, E[k - 2], S[k + 1]);",
     (5,)),
    ("M8 (DST context) operands transposed", "for (long k = 1; k <= q - 3; k += 2) S[k] = sub(c, E[k - 1], E[k + 1]);",
     "for (long k = 1; k <= q - 3; k += 2) S[k] = sub(c, E[k + 1], E[k - 1]);", (8,)),
]


def _build(tmp_path, text, idx):
    src = tmp_path / ("mut%d.c" % idx)
    src.write_text(text)
    so = tmp_path / ("libmut%d.so" % idx)
    subprocess.check_call(["gcc", "-std=gnu99", "-O1", "-ffp-contract=off", "-fPIC", "-shared",
                           "-DORACLE_REAL=double", str(src), "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    P, L = ctypes.c_void_p, ctypes.c_long
    lib.oracle_cdft.argtypes = [L, L, ctypes.c_int, P, P, P, P, P, P]
    return lib


def _cdft(lib, x, v):
    n = x.shape[-1]
    xr = np.ascontiguousarray(x.real)
    xi = np.ascontiguousarray(x.imag)
    Xr = np.empty_like(xr)
    Xi = np.empty_like(xi)
    assert lib.oracle_cdft(n, 1, v, xr.ctypes.data, xi.ctypes.data, Xr.ctypes.data, Xi.ctypes.data,
                           None, None) == 0
    return Xr + 1j * Xi


@pytest.mark.parametrize("idx", range(len(MUTATIONS)))
def test_planted_mistake_is_caught(tmp_path, idx):
    desc, old, new, variants = MUTATIONS[idx]
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation site must be unique: " + desc
    lib = _build(tmp_path, text.replace(old, new), idx)
    rng = np.random.default_rng(idx)
    x = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    ref = np.fft.fft(x)
    for v in variants:
        err = np.linalg.norm(_cdft(lib, x, v) - ref) / np.linalg.norm(ref)
        assert err > 1e-6, "pin did not notice: %s (variant %d)" % (desc, v)
