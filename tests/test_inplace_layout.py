"""The slot layout of the in-place large-N path (host code,
amqft_iplayout.h), checked on the CPU through a small C++ driver: a bijection
of the rows' output slots onto the orbits 1 .. N/16 - 1, every slot that only
one chain workgroup reads placed in that workgroup's orbits, and every slot
that two workgroups read listed for the copy to the shared workspace."""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1404_1810_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "amqft_iplayout.h"
int main(int argc, char** argv) {
    std::vector<int> tab;
    const int nsh = amqft::ip_layout_build(std::atoi(argv[1]), tab);
    std::printf("%d\n", nsh);
    for (int v : tab) std::printf("%d\n", v);
    return 0;
}
"""


@pytest.fixture(scope="module")
def layout_exe(tmp_path_factory):
    d = tmp_path_factory.mktemp("iplayout")
    src, exe = str(d / "drv.cpp"), str(d / "drv")
    with open(src, "w") as f:
        f.write(DRIVER)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", CSRC, src, "-o", exe])
    return exe


def _readers(logn):
    """Chain workgroups that read each depth-3 output slot (restated from
    the chain kernel's B0 windows: seven windows of 34 groups of eight
    harmonics a workgroup of 256 chain threads, each group reading its slot
    and its neighbours inside its block)."""
    N = 1 << logn
    W3, N8, Q = N // 16, N // 8, N // 4
    readers = [set() for _ in range(W3)]
    for w in range((W3 + 255) // 256):
        K = 256 * w
        starts = [K // 8 - 1, (N8 - K) // 8 - 33, (N8 + K) // 8 - 1, (Q - K) // 8 - 33,
                  K // 8 - 1, (N8 - K) // 8 - 33, K // 8 - 1]
        for r, g0 in enumerate(starts):
            a = 0 if r < 4 else 1 if r < 6 else 2
            sp = W3 >> (a + 1)
            for g in range(g0, g0 + 34):
                if 0 <= g < sp:
                    p = W3 - (W3 >> a) + g
                    readers[p].add(w)
                    if g >= 1:
                        readers[p - 1].add(w)
                    if g + 1 < sp:
                        readers[p + 1].add(w)
    return readers


@pytest.mark.parametrize("logn", [11, 12, 13, 14, 15, 16, 17])
def test_in_place_slot_layout(layout_exe, logn):
    out = subprocess.run([layout_exe, str(logn)], capture_output=True, text=True, check=True).stdout.split()
    vals = np.array([int(v) for v in out])
    nsh, tab = int(vals[0]), vals[1:]
    W3 = (1 << logn) // 16
    orb, shx, shl = tab[:W3], tab[W3:2 * W3], tab[2 * W3:]
    assert len(shl) == nsh
    # a bijection of the output slots 0 .. W3-2 onto the orbits 1 .. W3-1
    assert orb[W3 - 1] == -1
    assert sorted(orb[:W3 - 1].tolist()) == list(range(1, W3))
    readers = _readers(logn)
    for s in range(W3 - 1):
        if len(readers[s]) == 1:
            w = next(iter(readers[s]))
            assert 256 * w <= orb[s] < 256 * (w + 1), (s, w, orb[s])
            assert shx[s] == -1
        elif len(readers[s]) > 1:
            assert shx[s] >= 0 and shl[shx[s]] == s, s
        else:
            assert shx[s] == -1
    assert sum(1 for r in readers if len(r) > 1) == nsh
    # the shared workspace stays small: at most 11 % of the slots
    assert nsh <= 0.11 * W3
