// Level functions of the AM-QFT recursion, shared by the LDS-resident
// engine (amqft_lds.hip) and the multi-pass engine (amqft_multipass.hip).
//
// Data layout in LDS (per signal of length N = 2^m, H = N/2, D = m-2):
//   w[0, H)   DCT side, w[H, 2H) DST side.  On each side the chain of the
//             paper's dct[] (dst[]) recursion -- dct[N] = dct[N/2] + dct_ot[N]
//             (skeleton A) or dct[N/2] + dct_to[N] (skeleton B) -- is laid
//             out as blocks: block j (the ot/to function of periodization
//             N/2^j, 2^(D-j) values) occupies [2^(D-j), 2^(D-j+1)).
//   w[0]      DCT chain base (dct[2] input/output, first value)
//   w[H]      "extra" slot: c(N/2) and the top harmonic of the DCT chain
//   Within a block, the sub-blocks that the ot/to recursion creates at depth
//   l are contiguous ([lo child | hi child] under their parent) and hold the
//   paper's growing-order arrays (Table tab:implementation, 0-based).
//
// A "level" pass has every thread handle up to 8 items (one butterfly, one
// interleave pair, ...); items are decoded from a flat index with shifts and
// masks: item t on one side, t in [2^l, 2^D), belongs to block
// j = D-1-floor(log2 t), sub-block P and index i.  Reads go to registers,
// then a barrier, then the writes (in-place permutations are therefore
// safe), then a barrier.
#pragma once
#include "amqft_device.h"

namespace amqft {
namespace lv {

constexpr int KMAX = 8;  // items per thread per level

// LDS address of signal position p: identity, or one pad slot per 16 points
// (keeps the 16-point leaves of the fast kernel free of bank conflicts)
struct ad_identity {
    static __device__ __forceinline__ int at(int p) { return p; }
};
struct ad_pad16 {
    static __device__ __forceinline__ int at(int p) { return p + (p >> 4); }
};

struct item {
    int side;   // 0 = DCT side, 1 = DST side
    int hb;     // log2 of h
    int h;      // half the sub-block size
    int P;      // sub-block path (first choice = most significant bit)
    int i;      // index inside the half
    int base;   // offset of the sub-block in the signal's LDS array
    int sigma;  // arithmetic context of the sub-block: 0 = DCT, 1 = DST
    bool active;
};

__device__ __forceinline__ item decode(int t, int D, int l, int H, bool switches, int min_hb = 0) {
    item it;
    it.side = t >> D;
    const int tt = t & ((1 << D) - 1);
    const int b = 31 - __clz(tt | 1);
    it.active = tt >= (1 << l) && (b - l) >= min_hb;
    const int u = tt - (1 << b);
    it.hb = b - l;
    it.h = 1 << (it.hb < 0 ? 0 : it.hb);
    it.P = it.hb < 0 ? 0 : (u >> it.hb);
    it.i = u & (it.h - 1);
    it.base = it.side * H + (2 << b) + it.P * 2 * it.h;
    it.sigma = it.side ^ (switches ? (__popc(it.P) & 1) : 0);
    return it;
}

// table index p of theta_N * p for odd index 2i+1 inside a sub-block of
// size 2h at depth l: p = (2i+1) * N / (8h)  (Sec. 7.1)
__device__ __forceinline__ int kidx(int i, int hb, int D) { return (2 * i + 1) << (D - 1 - hb); }

// ---------------------------------------------------------------------------
// load x (N points) with the decomposition D_c + D_r on complex data:
//   c(m) = x(m) + x(N-m), d(m) = x(m) - x(N-m), m = 1..N/2-1 (eqs. qft_22-23)
// Skeleton A places c(m), m = 2^j (2i+1), at block j slot i (the odd-n part
// that the D_n chain hands to dct_ot[N/2^j]); skeleton B keeps natural order.
// ---------------------------------------------------------------------------
template <bool SKEL_A, typename S, typename R, typename AD = ad_identity>
__device__ void load_signal(cx<R>* w, const S* x, int ltid, int T, int D, int H, bool conj, bool valid) {
    if (!valid) return;
    for (int m = ltid; m < H; m += T) {
        cx<R> a = storage<S>::ld(x + (m == 0 ? 0 : m));
        cx<R> b = storage<S>::ld(x + (m == 0 ? H : 2 * H - m));
        if (conj) { a = cconj(a); b = cconj(b); }
        if (m == 0) {
            w[AD::at(0)] = a;  // c(0)
            w[AD::at(H)] = b;  // c(N/2)
        } else {
            int pos = m;
            if (SKEL_A) {
                const int j = __ffs(m) - 1;
                pos = (1 << (D - j)) + (m >> (j + 1));
            }
            w[AD::at(pos)] = a + b;
            w[AD::at(H + pos)] = a - b;
        }
    }
}

// ---------------------------------------------------------------------------
// D_c^F and store: X(k) = C(k) - i D(k), X(N-k) = C(k) + i D(k) (eqs.
// qft_17-21 with the sign of qft_19A corrected), X(0) = C(0), X(N/2) = C(N/2)
// ---------------------------------------------------------------------------
template <typename S, typename R, typename AD = ad_identity>
__device__ void store_signal(const cx<R>* w, S* y, int ltid, int T, int H, bool conj, bool valid) {
    if (!valid) return;
    for (int k = ltid; k < H; k += T) {
        if (k == 0) {
            cx<R> a = w[AD::at(0)], b = w[AD::at(H)];
            if (conj) { a = cconj(a); b = cconj(b); }
            storage<S>::st(y, a);
            storage<S>::st(y + H, b);
        } else {
            const cx<R> C = w[AD::at(k)], Dd = w[AD::at(H + k)];
            cx<R> xk = {C.re + Dd.im, C.im - Dd.re};
            cx<R> xnk = {C.re - Dd.im, C.im + Dd.re};
            if (conj) { xk = cconj(xk); xnk = cconj(xnk); }
            storage<S>::st(y + k, xk);
            storage<S>::st(y + 2 * H - k, xnk);
        }
    }
}

// ---------------------------------------------------------------------------
// Skeleton A, forward phase of dct_ot / dst_ot at depth l:
//   D_k^T: e = s(n) +- s(L/2-n), o = s(n) -+ s(L/2-n)  (Table tab:elabora_relations_B)
//   M^T (M1, M4, M5, M8): o times 2cos, 1/(2cos), 2sin, 1/(2sin) of theta*n
//   (Tables tab:DCT/DST_odd_transformations); L = 8 base: o * cos(pi/4).
// ---------------------------------------------------------------------------
template <int V, typename R, typename AD = ad_identity>
__device__ void a_fwd_level(cx<R>* w, const R* kt, int ltid, int T, int D, int H, int l, int min_hb = 0) {
    constexpr bool SW = variant_traits<V>::switches;
    const int n2 = 2 << D;
    cx<R> xa[KMAX], xb[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int t = ltid + k * T;
        if (t < n2) {
            const item it = decode(t, D, l, H, SW, min_hb);
            if (it.active) {
                xa[k] = w[AD::at(it.base + it.i)];
                xb[k] = w[AD::at(it.base + 2 * it.h - 1 - it.i)];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int t = ltid + k * T;
        if (t < n2) {
            const item it = decode(t, D, l, H, SW, min_hb);
            if (it.active) {
                cx<R> lo, hi;
                if (it.sigma == 0) { lo = xa[k] + xb[k]; hi = xa[k] - xb[k]; }
                else { lo = xa[k] - xb[k]; hi = xa[k] + xb[k]; }
                const R kk = (it.h == 1) ? cos_pi_4<R>() : kt[kidx(it.i, it.hb, D)];
                w[AD::at(it.base + it.i)] = lo;
                w[AD::at(it.base + it.h + it.i)] = hi * kk;
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Skeleton A, backward phase at depth l for M4 and M8 (no recurrence):
//   D_k^F interleave: even k from the lo child, odd k from M^F of the hi child
//   (DCT context; the DST context has the roles of even/odd array slots
//   swapped because its harmonics start at k = 1).
// ---------------------------------------------------------------------------
template <int V, typename R, typename AD = ad_identity>
__device__ void a_bwd_level(cx<R>* w, int ltid, int T, int D, int H, int l, int min_hb = 0) {
    constexpr bool SW = variant_traits<V>::switches;
    const int n2 = 2 << D;
    cx<R> lo[KMAX], f[KMAX], fn[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int t = ltid + k * T;
        if (t < n2) {
            const item it = decode(t, D, l, H, SW, min_hb);
            if (it.active) {
                const int j = it.i, h = it.h;
                lo[k] = w[AD::at(it.base + j)];
                f[k] = w[AD::at(it.base + h + j)];
                // neighbour of the hi child's output used by M^F
                bool up;  // true: f[j+1], false: f[j-1]
                if (V == 4) up = (it.sigma == 0);
                else up = (it.sigma != 0);  // V == 8
                const int jn = up ? j + 1 : j - 1;
                fn[k] = (jn >= 0 && jn < h) ? w[AD::at(it.base + h + jn)] : cx<R>{R(0), R(0)};
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int t = ltid + k * T;
        if (t < n2) {
            const item it = decode(t, D, l, H, SW, min_hb);
            if (it.active) {
                const int j = it.i;
                cx<R> odd;  // value of the hi child's slot after M^F
                if (it.h == 1) odd = f[k];  // L = 8 base: already final
                else if (V == 4) odd = f[k] + fn[k];   // S(k) = E(k-1) + E(k+1)
                else odd = (it.sigma == 0) ? f[k] - fn[k] : f[k] - fn[k];  // M8
                if (it.sigma == 0) {
                    w[AD::at(it.base + 2 * j)] = lo[k];
                    w[AD::at(it.base + 2 * j + 1)] = odd;
                } else {
                    w[AD::at(it.base + 2 * j)] = odd;
                    w[AD::at(it.base + 2 * j + 1)] = lo[k];
                }
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// segmented carry for the recurrences of M1, M3, M5, M7.
// Each thread owns KMAX consecutive items; a segment (one hi child, h items)
// longer than KMAX spans h/KMAX consecutive threads.  Because KMAX is even
// and the recurrence coefficient is +-1, the carry out of a chunk is its
// local result plus the carry in, so the carries are plain sums of the chunk
// totals of the preceding (forward) or following (backward) threads.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ cx<R> shfl_up_cx(cx<R> v, int d) {
    return cx<R>{__shfl_up(v.re, d), __shfl_up(v.im, d)};
}
template <typename R>
__device__ __forceinline__ cx<R> shfl_down_cx(cx<R> v, int d) {
    return cx<R>{__shfl_down(v.re, d), __shfl_down(v.im, d)};
}

// max_tps: the largest threads_per_seg of any thread of the workgroup (the
// same value in every thread).  Segments of at most 64 threads are aligned
// groups of lanes inside one wave, and their exclusive scan runs on lane
// shuffles; longer segments go through LDS.  Both forms contain a barrier,
// which callers use to order their LDS reads before their writes.
template <typename R>
__device__ cx<R> chunk_carry(cx<R>* scr, int ltid, cx<R> total, bool participates, bool fwd, int threads_per_seg,
                             int max_tps = 1 << 30) {
    const cx<R> z = {R(0), R(0)};
    if (max_tps <= 64) {
        const int tps = participates ? threads_per_seg : 1;
        const int pos = ltid & (tps - 1);
        const cx<R> own = participates ? total : z;
        // w_p = t_{p-1} (forward) or t_{p+1} (backward) inside the segment,
        // then an inclusive Hillis-Steele scan of w over the segment
        const cx<R> up1 = shfl_up_cx(own, 1), dn1 = shfl_down_cx(own, 1);
        cx<R> w = fwd ? (pos >= 1 ? up1 : z) : (pos + 1 < tps ? dn1 : z);
        for (int d = 1; d < max_tps; d <<= 1) {
            const cx<R> u = fwd ? shfl_up_cx(w, d) : shfl_down_cx(w, d);
            if (fwd ? pos >= d : pos + d < tps) w = w + u;
        }
        __syncthreads();
        return participates && threads_per_seg > 1 ? w : z;
    }
    scr[ltid] = participates ? total : z;
    __syncthreads();
    cx<R> c = z;
    if (participates && threads_per_seg > 1) {
        const int first = ltid & ~(threads_per_seg - 1);
        const int last = first + threads_per_seg - 1;
        if (fwd) {
            for (int u = first; u < ltid; ++u) c = c + scr[u];
        } else {
            for (int u = ltid + 1; u <= last; ++u) c = c + scr[u];
        }
    }
    __syncthreads();
    return c;
}

// ---------------------------------------------------------------------------
// Skeleton A, backward phase at depth l for M1 and M5 (frequency-side
// recurrence with the first term halved):
//   M1 DCT: S(1) = E(0)/2, S(k+1) = E(k) - S(k-1) (ascending)
//   M1 DST: S(q-1) = E(q)/2, S(k-1) = E(k) - S(k+1) (descending)
//   M5 DCT: S(q-1) = E(q)/2, S(k-1) = E(k) + S(k+1) (descending)
//   M5 DST: S(1) = E(0)/2, S(k+1) = E(k) + S(k-1) (ascending)
// ---------------------------------------------------------------------------
template <int V, typename R, typename AD = ad_identity, int KM = KMAX, bool TOP = false>
__device__ void a_bwd_scan_level(cx<R>* w, cx<R>* scr, int ltid, int T, int D, int H, int l, int min_hb = 0) {
    constexpr bool SW = variant_traits<V>::switches;
    constexpr R c = R(variant_traits<V>::sign);
    // TOP: only the top block of each side (items 2^(D-1) .. 2^D - 1 of the
    // side), packed onto the threads KM items each
    const int n2 = TOP ? (1 << D) : (2 << D);
    auto tmap = [&](int u) {
        if constexpr (TOP) {
            const int half = 1 << (D - 1);
            return ((u >> (D - 1)) << D) + half + (u & (half - 1));
        } else {
            return u;
        }
    };
    cx<R> lo[KM], a[KM], y[KM];
    bool fwdk[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int t = ltid * KM + k;
        fwdk[k] = true;
        if (t < n2) {
            const item it = decode(tmap(t), D, l, H, SW, min_hb);
            if (it.active) {
                lo[k] = w[AD::at(it.base + it.i)];
                a[k] = w[AD::at(it.base + it.h + it.i)];
                fwdk[k] = (V == 1) ? (it.sigma == 0) : (it.sigma != 0);
            }
        }
    }
    // local recurrences, ascending segments then descending ones
    {
        cx<R> Y = {R(0), R(0)};
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const int t = ltid * KM + k;
            if (t < n2) {
                const item it = decode(tmap(t), D, l, H, SW, min_hb);
                if (it.active && it.h > 1 && fwdk[k]) {
                    cx<R> v = a[k];
                    if (it.i == 0) { Y = {R(0), R(0)}; v = v * R(0.5); }
                    Y = v + Y * c;
                    y[k] = Y;
                }
            }
        }
        Y = {R(0), R(0)};
#pragma unroll
        for (int k = KM - 1; k >= 0; --k) {
            const int t = ltid * KM + k;
            if (t < n2) {
                const item it = decode(tmap(t), D, l, H, SW, min_hb);
                if (it.active && it.h > 1 && !fwdk[k]) {
                    cx<R> v = a[k];
                    if (it.i == it.h - 1) { Y = {R(0), R(0)}; v = v * R(0.5); }
                    Y = v + Y * c;
                    y[k] = Y;
                }
            }
        }
    }
    // carries across threads (only segments longer than KM)
    int hseg = 0;
    bool act0 = false;
    {
        const int t = ltid * KM;
        if (t < n2) {
            const item it = decode(tmap(t), D, l, H, SW, min_hb);
            act0 = it.active;
            hseg = it.h;
        }
    }
    const bool long_seg = act0 && hseg > KM;
    const bool fwd0 = fwdk[0];
    const cx<R> total = fwd0 ? y[KM - 1] : y[0];
    const int max_tps = ((1 << (D - 1 - l)) / KM) > 1 ? (1 << (D - 1 - l)) / KM : 1;
    const cx<R> Yin = chunk_carry(scr, ltid, total, long_seg, fwd0, long_seg ? hseg / KM : 1, max_tps);
    if (long_seg) {
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const int dist = fwd0 ? k + 1 : KM - k;
            const R sg = (c < R(0) && (dist & 1)) ? R(-1) : R(1);
            y[k] = y[k] + Yin * sg;
        }
    }
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int t = ltid * KM + k;
        if (t < n2) {
            const item it = decode(tmap(t), D, l, H, SW, min_hb);
            if (it.active) {
                const int j = it.i;
                const cx<R> odd = (it.h == 1) ? a[k] : y[k];
                if (it.sigma == 0) {
                    w[AD::at(it.base + 2 * j)] = lo[k];
                    w[AD::at(it.base + 2 * j + 1)] = odd;
                } else {
                    w[AD::at(it.base + 2 * j)] = odd;
                    w[AD::at(it.base + 2 * j + 1)] = lo[k];
                }
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Skeleton A, backward phase of the dct / dst chain (D_n^F, Table
// tab:elabora_relations_B):
//   dct[L]: S(k) = E(k) + O(k), S(L/2-k) = E(k) - O(k), S(q) = E(q)
//   dst[L]: S(k) = O(k) + E(k), S(L/2-k) = O(k) - E(k), S(q) = O(q)
// The DCT chain's top harmonic (k = L/2) lives in the extra slot w[AD::at(H)].
// ---------------------------------------------------------------------------
template <typename R, typename AD = ad_identity>
__device__ void a_chain(cx<R>* w, int ltid, int T, int D, int H, int jmax = 1 << 30, bool base = true) {
    // base dct[2]: (s0 + s1, s0 - s1) with s1 in the extra slot
    if (base && ltid == 0) {
        const cx<R> s0 = w[AD::at(0)], s1 = w[AD::at(H)];
        w[AD::at(0)] = s0 + s1;
        w[AD::at(H)] = s0 - s1;
    }
    __syncthreads();
    for (int j = (jmax < D ? jmax : D); j >= 0; --j) {
        const int q = 1 << (D - j);
        cx<R> ra[KMAX], rb[KMAX], rx[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int t = ltid + k * T;
            if (t < 2 * q) {
                const int side = t >= q, kk = t - side * q;
                if (side == 0) {
                    ra[k] = w[AD::at(kk)];       // E(k)
                    rb[k] = w[AD::at(q + kk)];   // O(k)
                    if (kk == 0) rx[k] = w[AD::at(H)];  // E(q)
                } else if (kk > 0) {
                    ra[k] = w[AD::at(H + kk)];           // E(k)
                    rb[k] = w[AD::at(H + q + kk - 1)];   // O(k)
                } else {
                    rb[k] = w[AD::at(H + 2 * q - 1)];    // O(q)
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int t = ltid + k * T;
            if (t < 2 * q) {
                const int side = t >= q, kk = t - side * q;
                if (side == 0) {
                    w[AD::at(kk)] = ra[k] + rb[k];
                    if (kk > 0) {
                        w[AD::at(2 * q - kk)] = ra[k] - rb[k];
                    } else {
                        w[AD::at(H)] = ra[k] - rb[k];  // S(L/2)
                        w[AD::at(q)] = rx[k];          // S(q) = E(q)
                    }
                } else if (kk > 0) {
                    w[AD::at(H + kk)] = rb[k] + ra[k];
                    w[AD::at(H + 2 * q - kk)] = rb[k] - ra[k];
                } else {
                    w[AD::at(H + q)] = rb[k];
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Skeleton B, forward phase of the dct / dst chain (D_k^T):
//   dct[L]: e(n) = s(n) + s(L/2-n), e(q) = s(q), o(n) = s(n) - s(L/2-n)
//   dst[L]: e(n) = s(n) - s(L/2-n), o(n) = s(n) + s(L/2-n), o(q) = s(q)
// e stays in place as the next chain signal, o goes to block j.
// ---------------------------------------------------------------------------
template <typename R, typename AD = ad_identity>
__device__ void b_chain_fwd(cx<R>* w, int ltid, int T, int D, int H, int jmax = 1 << 30) {
    for (int j = 0; j <= (jmax < D ? jmax : D); ++j) {
        const int q = 1 << (D - j);
        cx<R> ra[KMAX], rb[KMAX], rm[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int t = ltid + k * T;
            if (t < 2 * q) {
                const int side = t >= q, n = t - side * q;
                if (side == 0) {
                    ra[k] = w[AD::at(n)];
                    rb[k] = (n == 0) ? w[AD::at(H)] : w[AD::at(2 * q - n)];
                    if (n == 0) rm[k] = w[AD::at(q)];
                } else if (n > 0) {
                    ra[k] = w[AD::at(H + n)];
                    rb[k] = w[AD::at(H + 2 * q - n)];
                } else {
                    rm[k] = w[AD::at(H + q)];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int t = ltid + k * T;
            if (t < 2 * q) {
                const int side = t >= q, n = t - side * q;
                if (side == 0) {
                    w[AD::at(n)] = ra[k] + rb[k];
                    w[AD::at(q + n)] = ra[k] - rb[k];
                    if (n == 0) w[AD::at(H)] = rm[k];
                } else if (n > 0) {
                    w[AD::at(H + n)] = ra[k] - rb[k];
                    w[AD::at(H + q + n - 1)] = ra[k] + rb[k];
                } else {
                    w[AD::at(H + 2 * q - 1)] = rm[k];
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Skeleton B, backward phase of the chain: the harmonics are re-interleaved
// (even k from dct[L/2], odd k from dct_to[L]); the dct[2] base first.
// ---------------------------------------------------------------------------
template <typename R, typename AD = ad_identity>
__device__ void b_chain_bwd(cx<R>* w, int ltid, int T, int D, int H, int jmax = 1 << 30, bool base = true) {
    if (base && ltid == 0) {
        const cx<R> s0 = w[AD::at(0)], s1 = w[AD::at(H)];
        w[AD::at(0)] = s0 + s1;
        w[AD::at(H)] = s0 - s1;
    }
    __syncthreads();
    for (int j = (jmax < D ? jmax : D); j >= 0; --j) {
        const int q = 1 << (D - j);
        cx<R> re[KMAX], ro[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int t = ltid + k * T;
            if (t < 2 * q) {
                const int side = t >= q, i = t - side * q;
                const int off = side * H;
                if (side == 0 || i > 0) re[k] = w[AD::at(off + i)];
                ro[k] = w[AD::at(off + q + i)];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int t = ltid + k * T;
            if (t < 2 * q) {
                const int side = t >= q, i = t - side * q;
                const int off = side * H;
                if (side == 0 || i > 0) w[AD::at(off + 2 * i)] = re[k];
                w[AD::at(off + 2 * i + 1)] = ro[k];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Skeleton B, forward phase of dct_to / dst_to at depth l for M2 and M6:
//   D_n^T split (even n -> lo child through H_n, odd n -> dct_oo/dst_oo),
//   then M^T on the odd part: neighbour sums (M2) or differences (M6);
//   L = 8 base: o * cos(pi/4).
// ---------------------------------------------------------------------------
template <int V, typename R, typename AD = ad_identity>
__device__ void b_fwd_level(cx<R>* w, int ltid, int T, int D, int H, int l, int min_hb = 0) {
    constexpr bool SW = variant_traits<V>::switches;
    const int n2 = 2 << D;
    cx<R> lo[KMAX], xo[KMAX], xn[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int t = ltid + k * T;
        if (t < n2) {
            const item it = decode(t, D, l, H, SW, min_hb);
            if (it.active) {
                const int i = it.i, h = it.h;
                const bool dctc = (it.sigma == 0);
                // DCT context: n = 2i even -> slot 2i, odd -> slot 2i+1;
                // DST context (n starts at 1): even n -> slot 2i+1, odd -> 2i
                lo[k] = w[AD::at(it.base + (dctc ? 2 * i : 2 * i + 1))];
                xo[k] = w[AD::at(it.base + (dctc ? 2 * i + 1 : 2 * i))];
                bool up;  // neighbour o[i+1] (true) or o[i-1]
                if (V == 2) up = !dctc;
                else up = dctc;  // V == 6
                const int in = up ? i + 1 : i - 1;
                xn[k] = (in >= 0 && in < h) ? w[AD::at(it.base + (dctc ? 2 * in + 1 : 2 * in))] : cx<R>{R(0), R(0)};
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int t = ltid + k * T;
        if (t < n2) {
            const item it = decode(t, D, l, H, SW, min_hb);
            if (it.active) {
                cx<R> hi;
                if (it.h == 1) hi = xo[k] * cos_pi_4<R>();
                else if (V == 2) hi = xo[k] + xn[k];   // o(n-1) + o(n+1)
                else hi = xo[k] - xn[k];               // M6: differences
                w[AD::at(it.base + it.i)] = lo[k];
                w[AD::at(it.base + it.h + it.i)] = hi;
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Skeleton B, forward phase for M3 and M7 (time-side recurrence, the last
// term halved):
//   M3 DCT: e(q-2) = s(q-1), e(n) = s(n+1) - e(n+2) desc., e(0) = [s(1) - e(2)]/2
//   M3 DST: e(2) = s(1), e(n) = s(n-1) - e(n-2) asc., e(q) = [s(q-1) - e(q-2)]/2
//   M7 DCT: e(2) = s(1), e(n) = s(n-1) + e(n-2) asc., e(q) = [s(q-1) + e(q-2)]/2
//   M7 DST: e(q-2) = s(q-1), e(n) = s(n+1) + e(n+2) desc., e(0) = [s(1) + e(2)]/2
// ---------------------------------------------------------------------------
template <int V, typename R, typename AD = ad_identity, int KM = KMAX, bool TOP = false>
__device__ void b_fwd_scan_level(cx<R>* w, cx<R>* scr, int ltid, int T, int D, int H, int l, int min_hb = 0) {
    constexpr bool SW = variant_traits<V>::switches;
    constexpr R c = R(variant_traits<V>::sign);
    // TOP: only the top block of each side (items 2^(D-1) .. 2^D - 1 of the
    // side), packed onto the threads KM items each
    const int n2 = TOP ? (1 << D) : (2 << D);
    auto tmap = [&](int u) {
        if constexpr (TOP) {
            const int half = 1 << (D - 1);
            return ((u >> (D - 1)) << D) + half + (u & (half - 1));
        } else {
            return u;
        }
    };
    cx<R> lo[KM], a[KM], y[KM];
    bool fwdk[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int t = ltid * KM + k;
        fwdk[k] = true;
        if (t < n2) {
            const item it = decode(tmap(t), D, l, H, SW, min_hb);
            if (it.active) {
                const bool dctc = (it.sigma == 0);
                lo[k] = w[AD::at(it.base + (dctc ? 2 * it.i : 2 * it.i + 1))];
                a[k] = w[AD::at(it.base + (dctc ? 2 * it.i + 1 : 2 * it.i))];
                fwdk[k] = (V == 3) ? !dctc : dctc;
            }
        }
    }
    {
        cx<R> Y = {R(0), R(0)};
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const int t = ltid * KM + k;
            if (t < n2) {
                const item it = decode(tmap(t), D, l, H, SW, min_hb);
                if (it.active && it.h > 1 && fwdk[k]) {
                    if (it.i == 0) Y = {R(0), R(0)};
                    Y = a[k] + Y * c;
                    y[k] = Y;
                }
            }
        }
        Y = {R(0), R(0)};
#pragma unroll
        for (int k = KM - 1; k >= 0; --k) {
            const int t = ltid * KM + k;
            if (t < n2) {
                const item it = decode(tmap(t), D, l, H, SW, min_hb);
                if (it.active && it.h > 1 && !fwdk[k]) {
                    if (it.i == it.h - 1) Y = {R(0), R(0)};
                    Y = a[k] + Y * c;
                    y[k] = Y;
                }
            }
        }
    }
    int hseg = 0;
    bool act0 = false;
    {
        const int t = ltid * KM;
        if (t < n2) {
            const item it = decode(tmap(t), D, l, H, SW, min_hb);
            act0 = it.active;
            hseg = it.h;
        }
    }
    const bool long_seg = act0 && hseg > KM;
    const bool fwd0 = fwdk[0];
    const cx<R> total = fwd0 ? y[KM - 1] : y[0];
    const int max_tps = ((1 << (D - 1 - l)) / KM) > 1 ? (1 << (D - 1 - l)) / KM : 1;
    const cx<R> Yin = chunk_carry(scr, ltid, total, long_seg, fwd0, long_seg ? hseg / KM : 1, max_tps);
    if (long_seg) {
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const int dist = fwd0 ? k + 1 : KM - k;
            const R sg = (c < R(0) && (dist & 1)) ? R(-1) : R(1);
            y[k] = y[k] + Yin * sg;
        }
    }
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int t = ltid * KM + k;
        if (t < n2) {
            const item it = decode(tmap(t), D, l, H, SW, min_hb);
            if (it.active) {
                cx<R> hi;
                if (it.h == 1) {
                    hi = a[k] * cos_pi_4<R>();
                } else {
                    hi = y[k];
                    const bool last = fwdk[k] ? (it.i == it.h - 1) : (it.i == 0);
                    if (last) hi = hi * R(0.5);
                }
                w[AD::at(it.base + it.i)] = lo[k];
                w[AD::at(it.base + it.h + it.i)] = hi;
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Skeleton B, backward phase of dct_to / dst_to at depth l:
//   M^F (M2, M3, M6, M7): O = F times 1/(2cos), 2cos, 1/(2sin), 2sin of theta*k
//   D_n^F: DCT S(k) = E + O, S(L/2-k) = E - O; DST S(k) = O + E, S(L/2-k) = O - E
// ---------------------------------------------------------------------------
template <int V, typename R, typename AD = ad_identity>
__device__ void b_bwd_level(cx<R>* w, const R* kt, int ltid, int T, int D, int H, int l, int min_hb = 0) {
    constexpr bool SW = variant_traits<V>::switches;
    const int n2 = 2 << D;
    cx<R> e[KMAX], f[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int t = ltid + k * T;
        if (t < n2) {
            const item it = decode(t, D, l, H, SW, min_hb);
            if (it.active) {
                e[k] = w[AD::at(it.base + it.i)];
                f[k] = w[AD::at(it.base + it.h + it.i)];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int t = ltid + k * T;
        if (t < n2) {
            const item it = decode(t, D, l, H, SW, min_hb);
            if (it.active) {
                const cx<R> O = (it.h == 1) ? f[k] : f[k] * kt[kidx(it.i, it.hb, D)];
                const int s1 = 2 * it.h - 1 - it.i;
                if (it.sigma == 0) {
                    w[AD::at(it.base + it.i)] = e[k] + O;
                    w[AD::at(it.base + s1)] = e[k] - O;
                } else {
                    w[AD::at(it.base + it.i)] = O + e[k];
                    w[AD::at(it.base + s1)] = O - e[k];
                }
            }
        }
    }
    __syncthreads();
}

// constants of the variant's family for length N = 2^logn, entries p < N/4
template <int V, typename R>
__device__ void load_constants(R* kt, const R* ktab, int Q, int kshift, bool onthefly, int logn) {
    for (int p = threadIdx.x; p < Q; p += blockDim.x) {
        if (!onthefly) {
            kt[p] = ktab[(long)p << kshift];
        } else {
            // FP64 on the device, rounded once: x = 2p/N, angle = pi*x
            const double x = (double)p * 2.0 / (double)(1 << logn);
            constexpr int fam = const_family(V);
            double v;
            if (fam == 0) v = 2.0 * cospi(x);
            else if (fam == 1) v = 1.0 / (2.0 * cospi(x));
            else if (fam == 2) v = 2.0 * sinpi(x);
            else v = 1.0 / (2.0 * sinpi(x));
            kt[p] = (p == 0) ? R(0) : R(v);
        }
    }
}

// the recursion of both sides between the D_r split and the D_c combine
template <int V, typename R, typename AD = ad_identity>
__device__ void core(cx<R>* w, const R* kt, cx<R>* scr, int ltid, int T, int D, int H) {
    using VT = variant_traits<V>;
    if constexpr (VT::skel_a) {
        for (int l = 0; l < D; ++l) a_fwd_level<V, R, AD>(w, kt, ltid, T, D, H, l);
        for (int l = D - 1; l >= 0; --l) {
            if constexpr (VT::recurrence) a_bwd_scan_level<V, R, AD>(w, scr, ltid, T, D, H, l);
            else a_bwd_level<V, R, AD>(w, ltid, T, D, H, l);
        }
        a_chain<R, AD>(w, ltid, T, D, H);
    } else {
        b_chain_fwd<R, AD>(w, ltid, T, D, H);
        for (int l = 0; l < D; ++l) {
            if constexpr (VT::recurrence) b_fwd_scan_level<V, R, AD>(w, scr, ltid, T, D, H, l);
            else b_fwd_level<V, R, AD>(w, ltid, T, D, H, l);
        }
        for (int l = D - 1; l >= 0; --l) b_bwd_level<V, R, AD>(w, kt, ltid, T, D, H, l);
        b_chain_bwd<R, AD>(w, ltid, T, D, H);
    }
}

}  // namespace lv
}  // namespace amqft
