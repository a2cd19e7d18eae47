// Register-resident leaves of the AM-QFT recursion: one thread computes a
// whole dct_ot/dst_ot (skeleton A) or dct_to/dst_to (skeleton B) of a small
// size entirely in registers, forward and backward phase, following the same
// relations as the level functions (Tables tab:elabora_relations_B,
// tab:DCT_odd_transformations, tab:DST_odd_transformations; base cases of
// Sec. 4).  The recurrences of M1/M3/M5/M7 run sequentially, in the order the
// paper states them.
//
// v[]: the sub-block's values in its growing-order array (time values in,
// spectrum out).  SG: arithmetic context, 0 = DCT, 1 = DST.  Constants are
// read from the table kt (entry p = f(2 pi p / N), N = 2^(D+2)) at the index
// (2i+1) << (D - 1 - log2(h)) of the butterfly's odd sample 2i+1 inside a
// sub-block of 2h points.
#pragma once
#include "amqft_device.h"

namespace amqft {
namespace leaf {

template <int X> struct ilog2 { static constexpr int v = 1 + ilog2<X / 2>::v; };
template <> struct ilog2<1> { static constexpr int v = 0; };

// ---------------------------------------------------------------------------
// skeleton A: dct_ot (SG = 0) / dst_ot (SG = 1) of SZ points
// ---------------------------------------------------------------------------
template <int V, int SZ, int SG, typename R>
__device__ __forceinline__ void ot(cx<R>* v, const R* kt, int D) {
    if constexpr (SZ == 1) {
        return;  // dct_ot[4] / dst_ot[4]: S = s(1)
    } else if constexpr (SZ == 2) {
        // D_k then the L = 8 base of dct_oo / dst_oo: o * cos(pi/4)
        const cx<R> x = v[0], y = v[1];
        const cx<R> lo = SG == 0 ? x + y : x - y;
        const cx<R> hi = (SG == 0 ? x - y : x + y) * cos_pi_4<R>();
        if (SG == 0) { v[0] = lo; v[1] = hi; }
        else { v[0] = hi; v[1] = lo; }
    } else {
        constexpr int h = SZ / 2;
        constexpr int hb = ilog2<h>::v;
        constexpr bool SW = variant_traits<V>::switches;
        constexpr int SC = SW ? 1 - SG : SG;  // context of the hi child
        cx<R> lo[h], hi[h];
#pragma unroll
        for (int i = 0; i < h; ++i) {
            const cx<R> x = v[i], y = v[SZ - 1 - i];
            lo[i] = SG == 0 ? x + y : x - y;
            hi[i] = (SG == 0 ? x - y : x + y) * kt[(2 * i + 1) << (D - 1 - hb)];  // M^T
        }
        ot<V, h, SG, R>(lo, kt, D);
        ot<V, h, SC, R>(hi, kt, D);
        // M^F on the hi child's spectrum F = hi[]
        cx<R> odd[h];
        if constexpr (V == 4) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                if (SG == 0) odd[j] = (j + 1 < h) ? hi[j] + hi[j + 1] : hi[j];
                else odd[j] = (j >= 1) ? hi[j - 1] + hi[j] : hi[j];
            }
        } else if constexpr (V == 8) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                if (SG == 0) odd[j] = (j >= 1) ? hi[j] - hi[j - 1] : hi[j];
                else odd[j] = (j + 1 < h) ? hi[j] - hi[j + 1] : hi[j];
            }
        } else {  // M1 (c = -1) and M5 (c = +1): recurrences, first term halved
            constexpr R c = R(variant_traits<V>::sign);
            constexpr bool asc = (V == 1) ? (SG == 0) : (SG != 0);
            if (asc) {
                odd[0] = hi[0] * R(0.5);
#pragma unroll
                for (int j = 1; j < h; ++j) odd[j] = hi[j] + odd[j - 1] * c;
            } else {
                odd[h - 1] = hi[h - 1] * R(0.5);
#pragma unroll
                for (int j = h - 2; j >= 0; --j) odd[j] = hi[j] + odd[j + 1] * c;
            }
        }
#pragma unroll
        for (int j = 0; j < h; ++j) {
            if (SG == 0) { v[2 * j] = lo[j]; v[2 * j + 1] = odd[j]; }
            else { v[2 * j] = odd[j]; v[2 * j + 1] = lo[j]; }
        }
    }
}

// ---------------------------------------------------------------------------
// skeleton B: dct_to (SG = 0) / dst_to (SG = 1) of SZ points
// ---------------------------------------------------------------------------
template <int V, int SZ, int SG, typename R>
__device__ __forceinline__ void to(cx<R>* v, const R* kt, int D) {
    if constexpr (SZ == 1) {
        return;  // dct_to[4]: S(1) = s(0); dst_to[4]: S(1) = s(1)
    } else {
        constexpr int h = SZ / 2;
        constexpr int hb = ilog2<h>::v;
        constexpr bool SW = variant_traits<V>::switches;
        constexpr int SC = SW ? 1 - SG : SG;
        cx<R> lo[h], o[h], t[h];
        // D_n: even n -> lo child (through H_n), odd n -> dct_oo / dst_oo
#pragma unroll
        for (int i = 0; i < h; ++i) {
            lo[i] = SG == 0 ? v[2 * i] : v[2 * i + 1];
            o[i] = SG == 0 ? v[2 * i + 1] : v[2 * i];
        }
        if constexpr (SZ == 2) {
            t[0] = o[0] * cos_pi_4<R>();  // L = 8 base of dct_oo / dst_oo
        } else {
            // M^T of M2, M6 (neighbour sums / differences) or M3, M7 (recurrences)
            if constexpr (V == 2) {
#pragma unroll
                for (int j = 0; j < h; ++j) {
                    if (SG == 0) t[j] = (j >= 1) ? o[j - 1] + o[j] : o[j];
                    else t[j] = (j + 1 < h) ? o[j] + o[j + 1] : o[j];
                }
            } else if constexpr (V == 6) {
#pragma unroll
                for (int j = 0; j < h; ++j) {
                    if (SG == 0) t[j] = (j + 1 < h) ? o[j] - o[j + 1] : o[j];
                    else t[j] = (j >= 1) ? o[j] - o[j - 1] : o[j];
                }
            } else {  // M3 (c = -1), M7 (c = +1): the last term halved
                constexpr R c = R(variant_traits<V>::sign);
                constexpr bool asc = (V == 3) ? (SG != 0) : (SG == 0);
                if (asc) {
                    t[0] = o[0];
#pragma unroll
                    for (int j = 1; j < h; ++j) t[j] = o[j] + t[j - 1] * c;
                    t[h - 1] = t[h - 1] * R(0.5);
                } else {
                    t[h - 1] = o[h - 1];
#pragma unroll
                    for (int j = h - 2; j >= 0; --j) t[j] = o[j] + t[j + 1] * c;
                    t[0] = t[0] * R(0.5);
                }
            }
            to<V, h, SC, R>(t, kt, D);
#pragma unroll
            for (int i = 0; i < h; ++i) t[i] = t[i] * kt[(2 * i + 1) << (D - 1 - hb)];  // M^F
        }
        to<V, h, SG, R>(lo, kt, D);
        // D_n^F
#pragma unroll
        for (int i = 0; i < h; ++i) {
            if (SG == 0) { v[i] = lo[i] + t[i]; v[SZ - 1 - i] = lo[i] - t[i]; }
            else { v[i] = t[i] + lo[i]; v[SZ - 1 - i] = t[i] - lo[i]; }
        }
    }
}

}  // namespace leaf
}  // namespace amqft
