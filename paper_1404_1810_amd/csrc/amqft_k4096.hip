// Skeleton-A AM-QFT for N = 4096 (variants 4 and 8), six passes over LDS,
// one workgroup of 256 threads per signal.
//
// View of one side (DCT or DST, 2048 positions) used by the forward passes:
// after the forward levels 0..l-1 of the dct_ot / dst_ot recursion the data
// form 2^l "rows" of W_l = 2048 / 2^l slots.  Slot m of a row holds the
// element of chain block a = v2(m) (the ot function of periodization
// N / 2^a) with odd index m / 2^a, at sub-block path "row".  A forward level
// pairs slot m with W_l - m (m < W_l / 2) inside a row and sends the
// sum/difference to rows 2P / 2P+1 at the same slot (the D_k split, Table
// tab:elabora_relations_B), the hi half scaled by the M4 / M8 constant of
// index p = m * 2^l (Sec. 7.1; the L = 8 base case is p = N/8, whose table
// entry is set to cos(pi/4)).
//
// Storage: the two LDS halves hold rows by arithmetic context, not by side:
// row (side, path) lives in half side ^ parity(path) for the switching
// variant M8 and in half side for M4.  Every row of a half therefore has the
// same context, so a wave that works on one half runs code whose DCT/DST
// context is a compile-time constant.  Positions inside a half carry one pad
// slot per 16 (p + p / 16), which keeps rows of 16 bank-conflict free.
//
// Passes (each reads everything it needs, waits at a barrier, then writes):
//   F1  load + D_c/D_r + levels 0..2 on the orbits {+-m0 + 512 j}; thread 0
//       does blocks 8..10 and the chain up to dct[16] / dst[16].  The
//       loads are issued before the constant tables are filled.  Output:
//       depth-3 rows, slot layout.
//   F2  levels 3..6 on the orbits {+-m0 + 32 j} of each depth-3 row (lanes
//       0..14 of a 16-lane group); lane 15 finishes the row's slots that are
//       multiples of 16 (blocks 4..7, whole sub-blocks of 8, 4, 2, 1 points).
//       Output: depth-7 rows (16 slots), slot layout.
//   P3  every depth-7 row (blocks 0..3 of 8, 4, 2, 1 points): whole
//       sub-blocks forward and backward in registers.  Output: the row's
//       spectra block-contiguous [8 | 4 | 2 | 1] in slots 1..15.
//   B2  backward levels 6..3 of blocks 0..3: a thread combines one child
//       index j of 16 descendant rows into 16 consecutive parent harmonics,
//       with the +-1 neighbours that M4 / M8 read from the same rows.
//       Output: depth-3 rows, blocks 0..3 block-contiguous from slot 16.
//   B1  backward levels 2..0 of blocks 0..7, thread = position in the
//       depth-3 layout.  Output: depth 0, block a at 2048 - 2048 / 2^a.
//   C0  chain (D_n^F of dct/dst): levels 3..7 evaluated along each output's
//       reflection path, levels 0..2 on the orbit of 8 harmonics, then D_c
//       and the store.
// Blocks 4..7 of the depth-3 rows and the chain values live in the pad
// slots (one per 16 positions), which no layout uses otherwise.  LDS
// accesses of a 16-lane group hit distinct banks (stride 1 or 17).
#include <type_traits>

#include "amqft_device.h"
#include "amqft_internal.h"
#include "amqft_leaf.h"

namespace amqft {

namespace {

constexpr int N4 = 4096, H4 = 2048, D4 = 10, Q4 = 1024;
constexpr int THREADS4 = 256;
constexpr int HS = H4 + H4 / 16;  // padded positions of one half
constexpr int WLEN = 2 * HS + 2;  // both halves and two guard slots
// constants of levels 3..6 in the order F2 reads them: [t][r][w] for level
// 3 + t, orbit slot r < 8 >> t, lane w = m0 - 1 (stride-1 reads)
constexpr int KF2 = 225;
constexpr int KF2_ALLOC = 232;
constexpr int kf2_off(int t) { return t == 0 ? 0 : t == 1 ? 120 : t == 2 ? 180 : 210; }

constexpr int par(int x) { return x ? ((x & 1) ^ par(x >> 1)) : 0; }

__device__ __forceinline__ int pad(int p) { return p + (p >> 4); }

// Pad slot k (0..127) of half hh: index 17 k + 16, never a padded position.
// Blocks 4..7 of depth-3 row P (half h) finish into pad slots 16 P + i,
// i = 0..14; the chain values E_8(0..8), D_8(1..7) (c = 0..15) use slot
// 16 (c & 7) + 15 of half c >> 3.
__device__ __forceinline__ int pslot(int hh, int k) { return hh * HS + 17 * k + 16; }
__device__ __forceinline__ int chslot(int c) { return (c >> 3) * HS + 272 * (c & 7) + 271; }

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

template <typename R>
__device__ __forceinline__ cx<R> zero() { return cx<R>{R(0), R(0)}; }

// forward butterfly in context SG (0 = DCT, 1 = DST), hi scaled by k
template <int SG, typename R>
__device__ __forceinline__ void bfly(cx<R> x, cx<R> y, R k, cx<R>& lo, cx<R>& hi) {
    if constexpr (SG == 0) {
        lo = x + y;
        hi = (x - y) * k;
    } else {
        lo = x - y;
        hi = (x + y) * k;
    }
}

// M^F of one child index in parent context SG: hm = F[i-1], h0 = F[i],
// hp = F[i+1] of the hi child (zero outside its sub-block)
template <int V, int SG, typename R>
__device__ __forceinline__ cx<R> mf(cx<R> hm, cx<R> h0, cx<R> hp) {
    if constexpr (V == 4) return SG == 0 ? h0 + hp : hm + h0;  // neighbour sums
    else return SG == 0 ? h0 - hm : h0 - hp;                    // M8: neighbour differences
}

// one backward level on extended runs: n = run length of the children;
// L, Hh: children arrays of n + 2 (index 0 = left halo, n + 1 = right halo),
// P: parent array of 2n + 2.  A halo that the run cannot reach comes out as
// zero; the relations of M4 / M8 only consume a hi child's halo on the side
// that is filled from its own lo child, so those values are never read.
template <int V, int SG, int n, typename R>
__device__ __forceinline__ void combine(const cx<R>* L, const cx<R>* Hh, cx<R>* P) {
#pragma unroll
    for (int rho = -1; rho <= 2 * n; ++rho) {
        const bool even = ((rho + 2) & 1) == 0;
        const int i = even ? rho / 2 : (rho - 1) / 2;  // child index feeding parent index rho
        if ((SG == 0) == even) {
            P[rho + 1] = L[i + 1];  // the lo child fills the even slots in DCT context, the odd in DST
        } else {
            const cx<R> hm = i >= 0 ? Hh[i] : zero<R>();
            const cx<R> hp = i + 1 <= n ? Hh[i + 2] : zero<R>();
            P[rho + 1] = mf<V, SG, R>(hm, Hh[i + 1], hp);
        }
    }
}

// backward levels t .. r-1: cur[q] holds the extended runs of the 2^(r-t)
// rows at this level (length 2^t + 2); (2q, 2q+1) are the lo / hi children
// of parent q, whose context is SGB ^ parity(q) for switching variants
template <int V, int SGB, int r, int t, typename R>
__device__ __forceinline__ void bwd_levels(cx<R> (&cur)[1 << r][(1 << r) + 2]) {
    if constexpr (t < r) {
        constexpr bool SW = variant_traits<V>::switches;
        constexpr int nrow = 1 << (r - t - 1);
        constexpr int n = 1 << t;
        sfor<0, nrow>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int sg = SGB ^ (SW ? par(q) : 0);
            cx<R> tmp[2 * n + 2];
            combine<V, sg, n, R>(cur[2 * q], cur[2 * q + 1], tmp);
#pragma unroll
            for (int e = 0; e < 2 * n + 2; ++e) cur[q][e] = tmp[e];
        });
        bwd_levels<V, SGB, r, t + 1, R>(cur);
    }
}

// r backward levels from 2^r rows (local paths q below a parent of context
// SGB) for one child index j: ext[q] = {F[j-1], F[j], F[j+1]} (zero outside
// the sub-block); out = parent values 2^r j .. 2^r j + 2^r - 1
template <int V, int SGB, int r, typename R>
__device__ __forceinline__ void bwd_run(const cx<R> (&ext)[1 << r][3], cx<R>* out) {
    cx<R> cur[1 << r][(1 << r) + 2];
#pragma unroll
    for (int q = 0; q < (1 << r); ++q) {
        cur[q][0] = ext[q][0];
        cur[q][1] = ext[q][1];
        cur[q][2] = ext[q][2];
    }
    bwd_levels<V, SGB, r, 0, R>(cur);
#pragma unroll
    for (int e = 0; e < (1 << r); ++e) out[e] = cur[0][e + 1];
}

// whole sub-blocks of one 16-slot row in context SG: s[e-1] = slot e
// (e = 1..15; blocks of 8, 4, 2, 1 points at the odd slots, slots 2 mod 4,
// slots 4 and 12, slot 8); o[0..14] = their spectra, block-contiguous
template <int V, int SG, typename R>
__device__ __forceinline__ void row16(const cx<R>* s, cx<R>* o, const R* kt) {
    cx<R> b0[8], b1[4], b2[2];
#pragma unroll
    for (int i = 0; i < 8; ++i) b0[i] = s[2 * i];
#pragma unroll
    for (int i = 0; i < 4; ++i) b1[i] = s[4 * i + 1];
    b2[0] = s[3];
    b2[1] = s[11];
    leaf::ot<V, 8, SG, R>(b0, kt, D4);
    leaf::ot<V, 4, SG, R>(b1, kt, D4);
    leaf::ot<V, 2, SG, R>(b2, kt, D4);
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = b0[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) o[8 + i] = b1[i];
    o[12] = b2[0];
    o[13] = b2[1];
    o[14] = s[7];
}

// ---------------------------------------------------------------------- F1
// global loads of a thread: orbit of m0 = tid (x(m0 + 512 j), x(512 (j+1) - m0))
// or, for thread 0, the multiples of 256
template <typename S, typename R>
__device__ __forceinline__ void f1_load(const S* x, int tid, cx<R> (&raw)[16]) {
    if (tid > 0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            raw[j] = storage<S>::ld(x + tid + 512 * j);
            raw[8 + j] = storage<S>::ld(x + 512 * (j + 1) - tid);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) raw[k] = storage<S>::ld(x + 256 * k);
    }
}

// orbit of m0 in [1, 255]: slots m0 + 512 i, 512 (i+1) - m0 of both sides
template <int V, typename R>
__device__ __forceinline__ void f1_orbit(cx<R>* w, const R* kt, const cx<R> (&raw)[16], int m0, bool conj_in) {
    constexpr bool SW = variant_traits<V>::switches;
    cx<R> xa[8], xb[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        xa[j] = conj_in ? cconj(raw[j]) : raw[j];
        xb[j] = conj_in ? cconj(raw[8 + j]) : raw[8 + j];
    }
    // D_c / D_r on the orbit slots m_{2i} = m0 + 512 i, m_{2i+1} = 512 (i+1) - m0
    cx<R> cd[2][8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        cd[0][2 * i] = xa[i] + xb[7 - i];
        cd[1][2 * i] = xa[i] - xb[7 - i];
        cd[0][2 * i + 1] = xb[i] + xa[7 - i];
        cd[1][2 * i + 1] = xb[i] - xa[7 - i];
    }
    const R k0[4] = {kt[m0], kt[512 - m0], kt[512 + m0], kt[1024 - m0]};
    const R k1[2] = {kt[2 * m0], kt[1024 - 2 * m0]};
    const R k2 = kt[4 * m0];
    const int pm = pad(m0);
    sfor<0, 2>([&](auto sc) {
        constexpr int side = decltype(sc)::value;
        const cx<R>* v = cd[side];
        cx<R> l1[2][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) bfly<side, R>(v[r], v[7 - r], k0[r], l1[0][r], l1[1][r]);
        cx<R> l2[4][2];
        sfor<0, 2>([&](auto pc) {
            constexpr int P = decltype(pc)::value;
            constexpr int sg = side ^ (SW ? par(P) : 0);
#pragma unroll
            for (int r = 0; r < 2; ++r) bfly<sg, R>(l1[P][r], l1[P][3 - r], k1[r], l2[2 * P][r], l2[2 * P + 1][r]);
        });
        sfor<0, 4>([&](auto pc) {
            constexpr int P = decltype(pc)::value;
            constexpr int sg = side ^ (SW ? par(P) : 0);
            constexpr int h0 = side ^ (SW ? par(2 * P) : 0);
            constexpr int h1 = side ^ (SW ? par(2 * P + 1) : 0);
            cx<R> lo, hi;
            bfly<sg, R>(l2[P][0], l2[P][1], k2, lo, hi);
            stc(w + h0 * HS + 272 * (2 * P) + pm, lo);  // depth-3 row 2P, slot m0
            stc(w + h1 * HS + 272 * (2 * P + 1) + pm, hi);
        });
    });
}

// multiples of 256: blocks of 4, 2, 1 points and the chain to dct[16] / dst[16]
template <int V, typename R>
__device__ __forceinline__ void f1_chain(cx<R>* w, const R* kt, const cx<R> (&raw)[16], bool conj_in) {
    cx<R> xs[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) xs[k] = conj_in ? cconj(raw[k]) : raw[k];
    cx<R> c[8], d[8];
    c[0] = xs[0];
    d[0] = zero<R>();
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        c[k] = xs[k] + xs[16 - k];
        d[k] = xs[k] - xs[16 - k];
    }
    const cx<R> cN2 = xs[8];
    {
        // DCT side: block 8 = c(256 {1,3,5,7}), block 9 = c(512 {1,3}), block 10 = c(1024)
        cx<R> b8[4] = {c[1], c[3], c[5], c[7]}, b9[2] = {c[2], c[6]};
        leaf::ot<V, 4, 0, R>(b8, kt, D4);
        leaf::ot<V, 2, 0, R>(b9, kt, D4);
        const cx<R> e0 = c[0] + cN2, e1 = c[0] - cN2;  // dct[2]
        const cx<R> O10 = c[4];
        const cx<R> E10[3] = {e0 + O10, e1, e0 - O10};  // dct[4], k = 0..2
        const cx<R> E9[5] = {E10[0] + b9[0], E10[1] + b9[1], E10[2], E10[1] - b9[1], E10[0] - b9[0]};
        cx<R> E8[9];  // dct[16], k = 0..8
#pragma unroll
        for (int k = 0; k < 4; ++k) E8[k] = E9[k] + b8[k];
        E8[4] = E9[4];
#pragma unroll
        for (int k = 1; k < 4; ++k) E8[8 - k] = E9[k] - b8[k];
        E8[8] = E9[0] - b8[0];
#pragma unroll
        for (int k = 0; k < 9; ++k) stc(w + chslot(k), E8[k]);
    }
    {
        // DST side: dst[4] = d(1024), dst[8] and dst[16] by D_n^F
        cx<R> b8[4] = {d[1], d[3], d[5], d[7]}, b9[2] = {d[2], d[6]};
        leaf::ot<V, 4, 1, R>(b8, kt, D4);
        leaf::ot<V, 2, 1, R>(b9, kt, D4);
        const cx<R> E10 = d[4];
        const cx<R> E9[4] = {zero<R>(), b9[0] + E10, b9[1], b9[0] - E10};
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            stc(w + chslot(8 + k), b8[k - 1] + E9[k]);
            stc(w + chslot(16 - k), b8[k - 1] - E9[k]);
        }
        stc(w + chslot(12), b8[3]);
    }
}

// ---------------------------------------------------------------------- F2
template <int V, int H, typename R>
__device__ __forceinline__ void f2_compute(cx<R>* w, const R* kf, const cx<R> (&v)[16], int P, int m0) {
    constexpr bool SW = variant_traits<V>::switches;
    const R* kw = kf + (m0 - 1);
    cx<R> cur[16][16];
#pragma unroll
    for (int r = 0; r < 16; ++r) cur[0][r] = v[r];
    sfor<0, 4>([&](auto tc) {
        constexpr int t = decltype(tc)::value;  // level 3 + t
        constexpr int K = 16 >> t;
        constexpr int rows = 1 << t;
        cx<R> nxt[16][16];
        sfor<0, rows>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int sg = H ^ (SW ? par(q) : 0);
#pragma unroll
            for (int r = 0; r < K / 2; ++r)
                bfly<sg, R>(cur[q][r], cur[q][K - 1 - r], kw[kf2_off(t) + 15 * r], nxt[2 * q][r], nxt[2 * q + 1][r]);
        });
#pragma unroll
        for (int q = 0; q < 2 * rows; ++q)
#pragma unroll
            for (int r = 0; r < K / 2; ++r) cur[q][r] = nxt[q][r];
    });
    sfor<0, 16>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int hq = H ^ (SW ? par(q) : 0);
        stc(w + hq * HS + 272 * P + 17 * q + m0, cur[q][0]);  // depth-7 row 16 P + q, slot m0
    });
}

// ---------------------------------------------------------------------- P3
template <int V, int H, typename R>
__device__ __forceinline__ void p3_row(cx<R>* w, const R* kt, int r7) {
    cx<R>* row = w + H * HS + 17 * r7;
    cx<R> s[15], o[15];
#pragma unroll
    for (int e = 0; e < 15; ++e) s[e] = ldc(row + e + 1);
    row16<V, H, R>(s, o, kt);
#pragma unroll
    for (int e = 0; e < 15; ++e) stc(row + e + 1, o[e]);
}

template <int V, typename S>
__global__ __launch_bounds__(THREADS4) void amqft_a4096_kernel(const S* __restrict__ in, S* __restrict__ out,
                                                                const typename storage<S>::R* __restrict__ ktab,
                                                                long long batch, int kshift, int flags,
                                                                const long long* __restrict__ offsets) {
    using R = typename storage<S>::R;
    constexpr bool SW = variant_traits<V>::switches;
    extern __shared__ __align__(16) unsigned char smem[];
    R* kt = reinterpret_cast<R*>(smem);
    R* kf = kt + Q4;
    cx<R>* w = reinterpret_cast<cx<R>*>(smem + (Q4 + KF2_ALLOC) * sizeof(R));
    const bool conj_in = flags & 1, conj_out = flags & 2, onthefly = flags & 4;
    const int tid = threadIdx.x;
    const long long sig = blockIdx.x;
    const long long base = offsets ? offsets[sig] : sig * (long long)N4;
    const S* x = in + base;
    S* y = out + base;
    const int h = tid >> 7;  // half (= arithmetic context) of the pass's rows
    const int u = tid & 127;

    // the signal's loads are issued first; the constant tables fill meanwhile
    cx<R> raw[16];
    f1_load<S, R>(x, tid, raw);

    // constants: p = 1..N/4-1 of the variant's family; p = N/8 is the base case
    auto kval = [&](int p) -> R {
        if (p == Q4 / 2) return cos_pi_4<R>();
        if (!onthefly) return ktab[(long)p << kshift];
        const double a = (double)p * 2.0 / (double)N4;
        constexpr int fam = const_family(V);
        const double d = fam == 1 ? 1.0 / (2.0 * cospi(a)) : 1.0 / (2.0 * sinpi(a));
        return p == 0 ? R(0) : R(d);
    };
    for (int p = tid; p < Q4; p += THREADS4) kt[p] = kval(p);
    if (tid < KF2) {
        const int t = tid < 120 ? 0 : tid < 180 ? 1 : tid < 210 ? 2 : 3;
        const int e = tid - kf2_off(t);
        const int r = e / 15, m0 = e - 15 * r + 1;
        const int mr = (r & 1) ? 16 * (r + 1) - m0 : m0 + 16 * r;  // orbit slot r of m0
        kf[tid] = kval(mr << (3 + t));
    }
    __syncthreads();

    // ------------------------------------------------------------------ F1
    if (tid > 0) f1_orbit<V, R>(w, kt, raw, tid, conj_in);
    else f1_chain<V, R>(w, kt, raw, conj_in);
    __syncthreads();

    // ------------------------------------------------------------------ F2
    {
        // 16-lane groups: lanes 0..14 of group P run the orbits m0 = 1..15 of
        // depth-3 row P; lane 15 finishes the row's slots 16 e (blocks 4..7)
        const int P = u >> 4;
        const int wl = u & 15;
        const bool orb = wl < 15;
        const int m0 = wl + 1;
        cx<R> v[16];
        const int rb = h * HS + 272 * P;
        if (orb) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                v[2 * i] = ldc(w + rb + m0 + 34 * i);                // slot m0 + 32 i
                v[2 * i + 1] = ldc(w + rb + 34 * (i + 1) - m0 - 1);  // slot 32 (i+1) - m0
            }
        } else {
#pragma unroll
            for (int e = 1; e < 16; ++e) v[e - 1] = ldc(w + rb + 17 * e);  // slot 16 e
        }
        __syncthreads();
        if (orb) {
            if (h == 0) f2_compute<V, 0, R>(w, kf, v, P, m0);
            else f2_compute<V, 1, R>(w, kf, v, P, m0);
        } else {
            cx<R> o[15];
            if (h == 0) row16<V, 0, R>(v, o, kt);
            else row16<V, 1, R>(v, o, kt);
#pragma unroll
            for (int i = 0; i < 15; ++i) stc(w + pslot(h, 16 * P + i), o[i]);
        }
    }
    __syncthreads();

    // ------------------------------------------------------------------ P3
    if (h == 0) p3_row<V, 0, R>(w, kt, u);
    else p3_row<V, 1, R>(w, kt, u);
    __syncthreads();

    // ------------------------------------------------------------------ B2
    {
        // 16-lane groups: lane w15 < 15 of group P handles block a, child index j
        const int P = u >> 4;
        const int w15 = u & 15;
        const bool blk = w15 < 15;
        const int a = w15 < 8 ? 0 : w15 < 12 ? 1 : w15 < 14 ? 2 : 3;
        const int j = w15 - (16 - (16 >> a));
        const int sp = 8 >> a;  // sub-block size of block a at depth 7
        cx<R> ext[16][3];
        if (blk) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int hq = h ^ (SW ? par(q) : 0);
                const int at = hq * HS + 272 * P + 17 * q + 1 + w15;
                const cx<R> lm = ldc(w + at - 1), lp = ldc(w + at + 1);
                ext[q][0] = j >= 1 ? lm : zero<R>();
                ext[q][1] = ldc(w + at);
                ext[q][2] = j + 1 < sp ? lp : zero<R>();
            }
        }
        __syncthreads();
        if (blk) {
            cx<R> o[16];
            if (h == 0) bwd_run<V, 0, 4, R>(ext, o);
            else bwd_run<V, 1, 4, R>(ext, o);
            cx<R>* dst = w + h * HS + 272 * P + 17 * (w15 + 1);  // block a at 16 + 16 w15 of the row
#pragma unroll
            for (int e = 0; e < 16; ++e) stc(dst + e, o[e]);
        }
    }
    __syncthreads();

    // ------------------------------------------------------------------ B1
    {
        const int p = tid;  // position in the depth-3 block layout
        int a, j;
        if (p < 16) {
            a = p <= 8 ? 4 : p <= 12 ? 5 : p <= 14 ? 6 : 7;
            j = p - (a == 4 ? 1 : a == 5 ? 9 : a == 6 ? 13 : 15);
        } else {
            const int pp = p - 16;
            a = pp < 128 ? 0 : pp < 192 ? 1 : pp < 224 ? 2 : 3;
            j = pp - (256 - (256 >> a));
        }
        const int sp = 128 >> a;  // sub-block size of block a at depth 3
        const bool act = p > 0;
        cx<R> ext[2][8][3];
        if (act) {
            // blocks 4..7 (p < 16) sit in pad slots 16 q + p - 1 (stride 17)
            const int o0 = p < 16 ? 17 * (p - 1) + 16 : pad(p);
            const int om = p < 16 ? (p > 1 ? o0 - 17 : o0) : pad(p - 1);
            const int op = p < 16 ? o0 + 17 : pad(p + 1);
#pragma unroll
            for (int side = 0; side < 2; ++side)
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int hq = side ^ (SW ? par(q) : 0);
                    const cx<R>* row = w + hq * HS + 272 * q;
                    const cx<R> lm = ldc(row + om), lp = ldc(row + op);
                    ext[side][q][0] = j >= 1 ? lm : zero<R>();
                    ext[side][q][1] = ldc(row + o0);
                    ext[side][q][2] = j + 1 < sp ? lp : zero<R>();
                }
        }
        __syncthreads();
        if (act) {
            const int ob = pad(2048 - (2048 >> a) + 8 * j);
            cx<R> o[8];
            bwd_run<V, 0, 3, R>(ext[0], o);
#pragma unroll
            for (int e = 0; e < 8; ++e) stc(w + ob + e, o[e]);
            bwd_run<V, 1, 3, R>(ext[1], o);
#pragma unroll
            for (int e = 0; e < 8; ++e) stc(w + HS + ob + e, o[e]);
        }
    }
    __syncthreads();

    // ------------------------------------------------------------------ C0
    {
        // O_a(k): DCT block a harmonic k; DST harmonics start at 1.  Block
        // bases are multiples of 16, so pad(base + k) = pad(base) + pad(k).
        auto bo = [](int a) { return 2048 - (2048 >> a) + ((2048 - (2048 >> a)) >> 4); };  // pad(base_a)
        auto st = [&](int k, cx<R> v) {
            if (conj_out) v = cconj(v);
            storage<S>::st(y + k, v);
        };
        if (tid > 0) {
            const int k0 = tid;
            // chain levels 3..7 along the reflection path of k0 (q_a = 1024 >> a):
            // the indices and weights depend on k0 only, so every read is issued
            // before any of them is used
            int ic[5], is[5];
            R wc[5], ws[5];
            {
                int kk = k0;
#pragma unroll
                for (int t = 0; t < 5; ++t) {
                    const int q = Q4 >> (3 + t);
                    const bool lt = kk < q, gt = kk > q;
                    kk = gt ? 2 * q - kk : kk;
                    ic[t] = kk;  // kk == q reads a slot past the block with weight 0
                    wc[t] = lt ? R(1) : gt ? R(-1) : R(0);
                }
            }
            int e8 = 0;
            {
                int kk = k0;
                R sgn = R(1);
                bool done = false;
#pragma unroll
                for (int t = 0; t < 5; ++t) {
                    const int q = Q4 >> (3 + t);
                    const bool gt = kk > q, eq = kk == q;
                    const int kn = gt ? 2 * q - kk : kk;
                    is[t] = done ? 1 : kn;
                    ws[t] = done ? R(0) : sgn;
                    sgn = (!done && gt) ? -sgn : sgn;
                    done = done || eq;
                    kk = kn;
                }
                e8 = done ? 0 : kk;  // D_8(kk), kk in 1..7, unless the path ended at a q_a
                const R wd = done ? R(0) : sgn;
                cx<R> accs = ldc(w + chslot(8 + e8)) * wd;
#pragma unroll
                for (int t = 0; t < 5; ++t) {
                    const cx<R> o = ldc(w + HS + bo(3 + t) + pad(is[t] - 1));
                    accs = cx<R>{accs.re + ws[t] * o.re, accs.im + ws[t] * o.im};
                }
                cx<R> accc = ldc(w + chslot(ic[4]));
#pragma unroll
                for (int t = 0; t < 5; ++t) {
                    const cx<R> o = ldc(w + bo(3 + t) + pad(ic[t]));
                    accc = cx<R>{accc.re + wc[t] * o.re, accc.im + wc[t] * o.im};
                }
                // levels 2, 1, 0 on the orbit {k0, 512-k0, 512+k0, 1024-k0, ...}
                const int kA = k0, kB = 512 - k0, kC = 512 + k0, kD = 1024 - k0;
                const int pA = pad(kA), pB = pad(kB), pC = pA + 544, pD = pB + 544;
                const int qA = pad(kA - 1), qB = pad(kB - 1), qC = qA + 544, qD = qB + 544;
                const cx<R> Ec3 = accc, Es3 = accs;
                const cx<R> oc2 = ldc(w + bo(2) + pA);
                const cx<R> c2a = Ec3 + oc2, c2b = Ec3 - oc2;  // E_2(k0), E_2(512-k0)
                const cx<R> o1a = ldc(w + bo(1) + pA), o1b = ldc(w + bo(1) + pB);
                const cx<R> c1[4] = {c2a + o1a, c2b + o1b, c2b - o1b, c2a - o1a};
                const int pk[4] = {pA, pB, pC, pD}, qk[4] = {qA, qB, qC, qD};
                cx<R> C[8];  // E_0 at kA, kB, kC, kD, 2048-kD, 2048-kC, 2048-kB, 2048-kA
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const cx<R> o0 = ldc(w + pk[i]);
                    C[i] = c1[i] + o0;
                    C[7 - i] = c1[i] - o0;
                }
                const cx<R> os2 = ldc(w + HS + bo(2) + qA);
                const cx<R> s2a = os2 + Es3, s2b = os2 - Es3;
                const cx<R> p1a = ldc(w + HS + bo(1) + qA), p1b = ldc(w + HS + bo(1) + qB);
                const cx<R> s1[4] = {p1a + s2a, p1b + s2b, p1b - s2b, p1a - s2a};
                cx<R> Dd[8];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const cx<R> o0 = ldc(w + HS + qk[i]);
                    Dd[i] = o0 + s1[i];
                    Dd[7 - i] = o0 - s1[i];
                }
                const int kk8[8] = {kA, kB, kC, kD, 2048 - kD, 2048 - kC, 2048 - kB, 2048 - kA};
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const cx<R> Cv = C[i], Dv = Dd[i];
                    st(kk8[i], cx<R>{Cv.re + Dv.im, Cv.im - Dv.re});
                    st(N4 - kk8[i], cx<R>{Cv.re - Dv.im, Cv.im + Dv.re});
                }
            }
        } else {
            auto Oc = [&](int a, int k) { return ldc(w + pad(2048 - (2048 >> a) + k)); };
            auto Os = [&](int a, int k) { return ldc(w + HS + pad(2048 - (2048 >> a) + k - 1)); };
            // harmonics 0, 256, ..., 2048
            const cx<R> e8_0 = ldc(w + chslot(0));
            const cx<R> E3_0 = e8_0 + Oc(3, 0) + Oc(4, 0) + Oc(5, 0) + Oc(6, 0) + Oc(7, 0);
            // E_3(256), the top harmonic of periodization 512: E_4(0) - O_3(0)
            const cx<R> E3_256 = e8_0 - Oc(3, 0) + Oc(4, 0) + Oc(5, 0) + Oc(6, 0) + Oc(7, 0);
            const cx<R> o2 = Oc(2, 0);
            const cx<R> E2_0 = E3_0 + o2, E2_512 = E3_0 - o2, E2_256 = E3_256;
            const cx<R> o1_0 = Oc(1, 0), o1_256 = Oc(1, 256);
            const cx<R> E1_0 = E2_0 + o1_0, E1_1024 = E2_0 - o1_0;
            const cx<R> E1_256 = E2_256 + o1_256, E1_768 = E2_256 - o1_256, E1_512 = E2_512;
            cx<R> C[9];  // k = 256 i
            const cx<R> E1v[4] = {E1_0, E1_256, E1_512, E1_768};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const cx<R> o0 = Oc(0, 256 * i);
                C[i] = E1v[i] + o0;
                C[8 - i] = E1v[i] - o0;
            }
            C[4] = E1_1024;
            // DST: D_2(256) = O_2(256); D_1 at 256, 768 and 512; D_0 at 256 i
            const cx<R> D2_256 = Os(2, 256);
            const cx<R> p1 = Os(1, 256);
            const cx<R> D1v[4] = {zero<R>(), p1 + D2_256, Os(1, 512), p1 - D2_256};
            cx<R> Dd[9];
            Dd[0] = zero<R>();
            Dd[8] = zero<R>();
#pragma unroll
            for (int i = 1; i < 4; ++i) {
                const cx<R> o0 = Os(0, 256 * i);
                Dd[i] = o0 + D1v[i];
                Dd[8 - i] = o0 - D1v[i];
            }
            Dd[4] = Os(0, 1024);
            st(0, C[0]);
            st(2048, C[8]);
#pragma unroll
            for (int i = 1; i < 8; ++i) {
                const cx<R> Cv = C[i], Dv = Dd[i];
                st(256 * i, cx<R>{Cv.re + Dv.im, Cv.im - Dv.re});
                st(N4 - 256 * i, cx<R>{Cv.re - Dv.im, Cv.im + Dv.re});
            }
        }
    }
}

template <typename R>
constexpr size_t a4096_lds() {
    return (Q4 + KF2_ALLOC) * sizeof(R) + WLEN * sizeof(cx<R>);
}

template <int V, typename S>
hipError_t launch_a4096_typed(const lds_launch& a, hipStream_t st) {
    using R = typename storage<S>::R;
    const int flags = (a.conj_in ? 1 : 0) | (a.conj_out ? 2 : 0) | (a.onthefly ? 4 : 0);
    hipLaunchKernelGGL((amqft_a4096_kernel<V, S>), dim3((unsigned)a.batch), dim3(THREADS4), a4096_lds<R>(), st,
                       static_cast<const S*>(a.in), static_cast<S*>(a.out), static_cast<const R*>(a.ktab),
                       (long long)a.batch, a.ktab_log2n - 12, flags, static_cast<const long long*>(a.offsets));
    return hipGetLastError();
}

}  // namespace

void a4096_shape(int dtype, int* threads, size_t* lds_bytes) {
    *threads = THREADS4;
    *lds_bytes = dtype == 0 ? a4096_lds<double>() : a4096_lds<float>();
}

bool a4096_supported(int variant, int logn, int dtype) {
    return logn == 12 && (variant == 4 || variant == 8) && (dtype == 1 || dtype == 0);
}

hipError_t prime_a4096(int variant, int dtype) {
    const void* k = nullptr;
    if (variant == 4) k = dtype == 0 ? reinterpret_cast<const void*>(&amqft_a4096_kernel<4, double2>)
                                     : reinterpret_cast<const void*>(&amqft_a4096_kernel<4, float2>);
    else if (variant == 8) k = dtype == 0 ? reinterpret_cast<const void*>(&amqft_a4096_kernel<8, double2>)
                                          : reinterpret_cast<const void*>(&amqft_a4096_kernel<8, float2>);
    if (!k || (dtype != 0 && dtype != 1)) return hipSuccess;
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

hipError_t launch_a4096(const lds_launch& a, hipStream_t st) {
    if (a.batch <= 0) return hipSuccess;
    if (a.variant == 4) return a.dtype == 0 ? launch_a4096_typed<4, double2>(a, st) : launch_a4096_typed<4, float2>(a, st);
    return a.dtype == 0 ? launch_a4096_typed<8, double2>(a, st) : launch_a4096_typed<8, float2>(a, st);
}

}  // namespace amqft
