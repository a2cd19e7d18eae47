// Slot layout of the in-place large-N path (host code).
//
// The path keeps the depth-3 rows of an N-point signal (Sec. 4: the sixteen
// dct_ot / dst_ot problems of length N/16 the recursion reaches after three
// levels) inside the signal's own buffer.  Position sets:
//
//   orbit o (1 <= o < N/16): the 16 positions o + j N/8 and (j+1) N/8 - o,
//   j = 0..7, which the first kernel reads for its thread o and the last
//   kernel writes for its chain thread o.  Row r keeps one value in every
//   orbit: member(r, o) = r N/8 + o for r < 8, (r - 7) N/8 - o for r >= 8.
//
// The rows enter the row kernel with slot s at member(r, s) (so the first
// kernel writes what it read) and leave it in block layout (block a at
// N/16 - N/16 / 2^a) with slot s at member(r, orb[s]).  The chain kernel's
// workgroup K (threads k0 = K .. K+255) writes orbits K .. K+255 and reads,
// for the backward levels 2..0 of the blocks 0..2, the slots of seven windows
// of groups (see amqft_kL_bchain); orb places every slot that only workgroup
// K reads in one of the orbits K .. K+255, so that no workgroup reads a
// position another one writes.  Slots read by two workgroups ("shared": the
// ends of neighbouring windows) are copied to a small workspace beforehand.
//
// tab layout (ints): [0, W) orb, [W, 2W) index into the shared list or -1,
// [2W, 2W + nsh) the shared list; W = N/16.  Slot W - 1 is unused (-1).
#pragma once

#include <algorithm>
#include <cstdint>
#include <set>
#include <vector>

namespace amqft {

// the chain kernel's workgroup size and B0 window geometry
constexpr int kIpChainThreads = 256, kIpWindows = 7, kIpGroups = 34;

// fills tab for N = 2^logn (logn >= 11); returns the number of shared slots,
// or -1 if some workgroup owns more slots than it has orbits (not the case
// for any supported N)
inline int ip_layout_build(int logn, std::vector<int>& tab) {
    const int N = 1 << logn, W3 = N / 16, N8 = N / 8, Q = N / 4;
    const int nwg = (W3 + kIpChainThreads - 1) / kIpChainThreads;
    // reader workgroup of each slot: -1 none, -2 several
    std::vector<int> reader(W3, -1);
    auto touch = [&](int s, int w) { reader[s] = reader[s] == -1 || reader[s] == w ? w : -2; };
    for (int w = 0; w < nwg; ++w) {
        const int K = w * kIpChainThreads;
        for (int r = 0; r < kIpWindows; ++r) {
            const int a = r < 4 ? 0 : r < 6 ? 1 : 2;
            const int g0 = (r == 0 || r == 4 || r == 6) ? K / 8 - 1
                           : (r == 1 || r == 5)         ? (N8 - K) / 8 - 33
                           : r == 2                     ? (N8 + K) / 8 - 1
                                                        : (Q - K) / 8 - 33;
            const int sp = W3 >> (a + 1);
            for (int t = 0; t < kIpGroups; ++t) {
                const int g = g0 + t;
                if (g < 0 || g >= sp) continue;
                const int p = W3 - (W3 >> a) + g;
                touch(p, w);
                if (g >= 1) touch(p - 1, w);
                if (g + 1 < sp) touch(p + 1, w);
            }
        }
    }
    tab.assign(2 * W3, -1);
    std::vector<int> owned_count(nwg, 0);
    std::vector<char> used(W3, 0);
    used[0] = 1;  // orbit 0 carries the chain thread's values, no row slots
    // owned slots, in increasing order, to the first orbits of their workgroup
    for (int s = 0; s < W3 - 1; ++s) {
        const int w = reader[s];
        if (w < 0) continue;
        const int o = w * kIpChainThreads + (w == 0 ? 1 : 0) + owned_count[w]++;
        if (o >= std::min(W3, (w + 1) * kIpChainThreads)) return -1;
        tab[s] = o;
        used[o] = 1;
    }
    // the rest (shared, and the blocks >= 3 that only the back kernel reads)
    int nsh = 0, next = 1;
    for (int s = 0; s < W3 - 1; ++s) {
        if (reader[s] == -2) {
            tab[W3 + s] = nsh++;
            tab.push_back(s);
        }
        if (reader[s] >= 0) continue;
        while (used[next]) ++next;
        tab[s] = next;
        used[next] = 1;
    }
    return nsh;
}

}  // namespace amqft
