// Skeleton-A AM-QFT for N = 4096 (variants 4 and 8), six passes over LDS.
//
// View of one side (DCT or DST, 2048 positions) used here: after the
// forward levels 0..l-1 of the dct_ot / dst_ot recursion, the data form 2^l
// "rows" of W_l = 2048 / 2^l slots; position = row * W_l + slot.  Slot m
// of a row holds the element of chain block a = v2(m) (the ot function of
// periodization N / 2^a) with odd index m / 2^a, at sub-block path "row".
// Every forward level pairs slot m with W_l - m (m < W_l / 2) inside a row
// and sends the sum/difference to rows 2P / 2P+1 at the same slot (the D_k
// split, eqs. of Table tab:elabora_relations_B), the hi half scaled by the
// M4 / M8 constant of index p = m * 2^l (Sec. 7.1; the L = 8 base case is
// p = N/8, whose table entry is set to cos(pi/4)).  After the backward phase
// of a block's sub-block, its spectrum value k sits at slot 2^a (2k+1).
//
// Passes (N = 4096, 320 threads = 5 waves per signal):
//   F1  load + D_c/D_r + levels 0..2 for the orbits {+-m0 + 512 j} (256
//       units); wave 4 handles the multiples of 256 completely (blocks of
//       <= 4 points and the chain up to dct[16] / dst[16]).
//   F2  levels 3..6 for the orbits {+-m0 + 32 j} inside each depth-3 row.
//   P3  every depth-7 row of 16 slots (blocks 0..3) and, on wave 4, the
//       multiples of 16 of every depth-3 row (blocks 4..7): whole
//       sub-blocks forward and backward in registers.
//   B2  backward levels 6..3 of blocks 0..3; B1 levels 2..0 of blocks 0..7:
//       a thread combines one child index j of 2^r descendant rows into 2^r
//       consecutive parent harmonics, with the +-1 neighbours of M4 / M8
//       read from the same rows.
//   C0  chain (D_n^F of dct/dst): levels 3..7 evaluated along each output's
//       reflection path, levels 0..2 on the orbit of 8 harmonics, then D_c
//       and the store.
#include <algorithm>

#include "amqft_device.h"
#include "amqft_internal.h"
#include "amqft_leaf.h"

namespace amqft {

namespace {

constexpr int N4 = 4096, H4 = 2048, D4 = 10, Q4 = 1024;
constexpr int THREADS4 = 320;

__device__ __forceinline__ int pad(int p) { return p + (p >> 4); }

template <typename R>
__device__ __forceinline__ cx<R> zero() { return cx<R>{R(0), R(0)}; }

// forward butterfly of context sg (0 = DCT, 1 = DST), hi scaled by k
template <typename R>
__device__ __forceinline__ void bfly(cx<R> x, cx<R> y, int sg, R k, cx<R>& lo, cx<R>& hi) {
    if (sg == 0) { lo = x + y; hi = (x - y) * k; }
    else { lo = x - y; hi = (x + y) * k; }
}

// M^F combine of one child index: parent context sg, hi child values around
// index i (hm = F[i-1], h0 = F[i], hp = F[i+1], zero outside the sub-block)
template <int V, typename R>
__device__ __forceinline__ cx<R> mf(int sg, cx<R> hm, cx<R> h0, cx<R> hp) {
    const cx<R> o = sg == 0 ? (V == 4 ? hp : hm) : (V == 4 ? hm : hp);
    return V == 4 ? h0 + o : h0 - o;  // M4: neighbour sum; M8: neighbour difference
}

// one backward level on extended runs: n = run length of the children;
// L, Hh: children arrays of n + 2 (index 0 = left halo, n + 1 = right halo),
// P: parent array of 2n + 2.  Out-of-reach halos come out as zero; the
// relations of M4 / M8 never read them (a hi child's halo is always a slot
// filled from its own lo child).
template <int V, int n, typename R>
__device__ __forceinline__ void combine(const cx<R>* L, const cx<R>* Hh, int sg, cx<R>* P) {
#pragma unroll
    for (int rho = -1; rho <= 2 * n; ++rho) {
        // child index feeding parent index rho: rho/2 (even) or (rho-1)/2 (odd)
        const bool even = ((rho + 2) & 1) == 0;
        const int i = even ? rho / 2 : (rho - 1) / 2;
        const cx<R> vl = (i >= -1 && i <= n) ? L[i + 1] : zero<R>();
        const cx<R> hm = (i - 1 >= -1 && i - 1 <= n) ? Hh[i] : zero<R>();
        const cx<R> h0 = (i >= -1 && i <= n) ? Hh[i + 1] : zero<R>();
        const cx<R> hp = (i + 1 >= -1 && i + 1 <= n) ? Hh[i + 2] : zero<R>();
        const cx<R> vh = mf<V, R>(sg, hm, h0, hp);
        // the lo child fills the even slots in DCT context, the odd ones in DST
        const bool from_lo = (sg == 0) == even;
        P[rho + 1] = cx<R>{from_lo ? vl.re : vh.re, from_lo ? vl.im : vh.im};
    }
}

// backward levels t .. r-1 of bwd_run: cur[q] holds the extended runs of
// the 2^(r-t) rows at this level (length 2^t + 2); pairs (2q, 2q+1) are the
// lo / hi children of parent q, whose global path is parent_row * 2^(r-t-1) + q
template <int V, int r, int t, typename R>
__device__ __forceinline__ void bwd_levels(cx<R> (&cur)[1 << r][(1 << r) + 2], int side, int parent_row) {
    if constexpr (t < r) {
        constexpr bool SW = variant_traits<V>::switches;
        constexpr int nrow = 1 << (r - t - 1);
        constexpr int n = 1 << t;
#pragma unroll
        for (int q = 0; q < nrow; ++q) {
            const int gp = (parent_row << (r - t - 1)) + q;
            const int sg = side ^ (SW ? (__popc(gp) & 1) : 0);
            cx<R> tmp[2 * n + 2];
            combine<V, n, R>(cur[2 * q], cur[2 * q + 1], sg, tmp);
#pragma unroll
            for (int e = 0; e < 2 * n + 2; ++e) cur[q][e] = tmp[e];
        }
        bwd_levels<V, r, t + 1, R>(cur, side, parent_row);
    }
}

// r backward levels from 2^r rows (paths q of r bits below parent_row) for
// one child index j: ext[q] = {F[j-1], F[j], F[j+1]} of row q (zero outside
// the sub-block); out = the 2^r parent values 2^r j .. 2^r j + 2^r - 1
template <int V, int r, typename R>
__device__ __forceinline__ void bwd_run(cx<R> (*ext)[3], int side, int parent_row, cx<R>* out) {
    cx<R> cur[1 << r][(1 << r) + 2];
#pragma unroll
    for (int q = 0; q < (1 << r); ++q) {
        cur[q][0] = ext[q][0];
        cur[q][1] = ext[q][1];
        cur[q][2] = ext[q][2];
    }
    bwd_levels<V, r, 0, R>(cur, side, parent_row);
#pragma unroll
    for (int e = 0; e < (1 << r); ++e) out[e] = cur[0][e + 1];
}

// whole sub-blocks of one 16-slot row (slot 0 untouched): blocks of 8, 4, 2
// and 1 points at the odd slots, slots 2 mod 4, slots 4 and 12, slot 8
template <int V, int SG, typename R>
__device__ __forceinline__ void row16(cx<R>* v, const R* kt) {
    cx<R> b0[8], b1[4], b2[2];
#pragma unroll
    for (int i = 0; i < 8; ++i) b0[i] = v[2 * i + 1];
#pragma unroll
    for (int i = 0; i < 4; ++i) b1[i] = v[4 * i + 2];
    b2[0] = v[4];
    b2[1] = v[12];
    leaf::ot<V, 8, SG, R>(b0, kt, D4);
    leaf::ot<V, 4, SG, R>(b1, kt, D4);
    leaf::ot<V, 2, SG, R>(b2, kt, D4);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[2 * i + 1] = b0[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[4 * i + 2] = b1[i];
    v[4] = b2[0];
    v[12] = b2[1];
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
    cx<R>* w = reinterpret_cast<cx<R>*>(smem + Q4 * sizeof(R));  // 2 sides x 2048 (+ pads)
    const bool conj_in = flags & 1, conj_out = flags & 2, onthefly = flags & 4;
    const int tid = threadIdx.x;
    const long long sig = blockIdx.x;
    const long long base = offsets ? offsets[sig] : sig * (long long)N4;
    const S* x = in + base;
    S* y = out + base;
    constexpr int SH = H4 + H4 / 16;  // padded side size

    // constants: p = 1..N/4-1 of the variant's family; p = N/8 is the base case
    for (int p = tid; p < Q4; p += THREADS4) {
        R v;
        if (p == Q4 / 2) v = cos_pi_4<R>();
        else if (!onthefly) v = ktab[(long)p << kshift];
        else {
            const double a = (double)p * 2.0 / (double)N4;
            constexpr int fam = const_family(V);
            double d = fam == 1 ? 1.0 / (2.0 * cospi(a)) : 1.0 / (2.0 * sinpi(a));
            v = p == 0 ? R(0) : R(d);
        }
        kt[p] = v;
    }
    __syncthreads();

    // ------------------------------------------------------------------ F1
    if (tid < 256) {
        if (tid > 0) {
            const int m0 = tid;
            cx<R> xa[8], xb[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                xa[j] = storage<S>::ld(x + m0 + 512 * j);
                xb[j] = storage<S>::ld(x + 512 * (j + 1) - m0);
                if (conj_in) { xa[j] = cconj(xa[j]); xb[j] = cconj(xb[j]); }
            }
            // orbit slots m_{2i} = m0 + 512 i, m_{2i+1} = 512 (i+1) - m0 (< 2048)
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
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                cx<R>* v = cd[side];
                cx<R> l1[2][4];  // rows 0, 1 at depth 1, slots m_0..m_3
#pragma unroll
                for (int r = 0; r < 4; ++r) bfly(v[r], v[7 - r], side, k0[r], l1[0][r], l1[1][r]);
                cx<R> l2[4][2];
#pragma unroll
                for (int P = 0; P < 2; ++P) {
                    const int sg = side ^ (SW ? P : 0);
#pragma unroll
                    for (int r = 0; r < 2; ++r) bfly(l1[P][r], l1[P][3 - r], sg, k1[r], l2[2 * P][r], l2[2 * P + 1][r]);
                }
#pragma unroll
                for (int P = 0; P < 4; ++P) {
                    const int sg = side ^ (SW ? (__popc(P) & 1) : 0);
                    cx<R> lo, hi;
                    bfly(l2[P][0], l2[P][1], sg, k2, lo, hi);
                    w[side * SH + pad(256 * (2 * P) + m0)] = lo;
                    w[side * SH + pad(256 * (2 * P + 1) + m0)] = hi;
                }
            }
        }
    } else if (tid == 256) {
        // multiples of 256: blocks of 4, 2, 1 points and dct[16] / dst[16]
        cx<R> xs[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            xs[k] = storage<S>::ld(x + 256 * k);
            if (conj_in) xs[k] = cconj(xs[k]);
        }
        cx<R> c[8], d[8];
        c[0] = xs[0];
        d[0] = zero<R>();
#pragma unroll
        for (int k = 1; k < 8; ++k) {
            c[k] = xs[k] + xs[16 - k];
            d[k] = xs[k] - xs[16 - k];
        }
        const cx<R> cN2 = xs[8];
        // DCT side: block 8 = slots 256*{1,3,5,7}, block 9 = {512,1536}, block 10 = {1024}
        {
            cx<R> b8[4] = {c[1], c[3], c[5], c[7]}, b9[2] = {c[2], c[6]};
            leaf::ot<V, 4, 0, R>(b8, kt, D4);
            leaf::ot<V, 2, 0, R>(b9, kt, D4);
            // dct[2] base, then D_n^F of dct[4], dct[8], dct[16]
            const cx<R> e0 = c[0] + cN2, e1 = c[0] - cN2;
            // E10 over k = 0..2
            const cx<R> O10 = c[4];
            cx<R> E10[3] = {e0 + O10, e1, e0 - O10};
            // E9 over k = 0..4 (q = 2), O9(k) = b9[k]
            cx<R> E9[5] = {E10[0] + b9[0], E10[1] + b9[1], E10[2], E10[1] - b9[1], E10[0] - b9[0]};
            // E8 over k = 0..8 (q = 4), O8(k) = b8[k]
            cx<R> E8[9];
#pragma unroll
            for (int k = 0; k < 4; ++k) E8[k] = E9[k] + b8[k];
            E8[4] = E9[4];
#pragma unroll
            for (int k = 1; k < 4; ++k) E8[8 - k] = E9[k] - b8[k];
            E8[8] = E9[0] - b8[0];
#pragma unroll
            for (int k = 0; k < 8; ++k) w[pad(256 * k)] = E8[k];
            w[SH + pad(0)] = E8[8];  // extra slot
        }
        // DST side: dst_ot of 4 and 2 points, dst[4] base
        {
            cx<R> b8[4] = {d[1], d[3], d[5], d[7]}, b9[2] = {d[2], d[6]};
            leaf::ot<V, 4, 1, R>(b8, kt, D4);
            leaf::ot<V, 2, 1, R>(b9, kt, D4);
            const cx<R> E10 = d[4];  // dst[4]: S(1) = s(1)
            // dst[8]: S(1) = O(1) + E(1), S(3) = O(1) - E(1), S(2) = O(2); O(k) = b9[k-1]
            cx<R> E9[4] = {zero<R>(), b9[0] + E10, b9[1], b9[0] - E10};
            // dst[16]: k = 1..7, q = 4, O(k) = b8[k-1]
            cx<R> E8[8];
            E8[0] = zero<R>();
#pragma unroll
            for (int k = 1; k < 4; ++k) {
                E8[k] = b8[k - 1] + E9[k];
                E8[8 - k] = b8[k - 1] - E9[k];
            }
            E8[4] = b8[3];
#pragma unroll
            for (int k = 1; k < 8; ++k) w[SH + pad(256 * k)] = E8[k];
        }
    }
    __syncthreads();

    // ------------------------------------------------------------------ F2
    {
        cx<R> v[16];
        int side = 0, P = 0, m0 = 0;
        const bool act = tid < 240;
        if (act) {
            side = tid / 120;
            const int u = tid - side * 120;
            P = u / 15;
            m0 = u - P * 15 + 1;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                v[2 * i] = w[side * SH + pad(256 * P + m0 + 32 * i)];
                v[2 * i + 1] = w[side * SH + pad(256 * P + 32 * (i + 1) - m0)];
            }
        }
        __syncthreads();
        if (act) {
            // slots m_r; level lev pairs (r, K-1-r) with K = 16 >> (lev-3)
            int mr[16];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                mr[2 * i] = m0 + 32 * i;
                mr[2 * i + 1] = 32 * (i + 1) - m0;
            }
            cx<R> cur[16][16];  // [row within pass][register]
#pragma unroll
            for (int r = 0; r < 16; ++r) cur[0][r] = v[r];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int K = 16 >> t;
                const int rows = 1 << t;
                cx<R> nxt[16][16];
#pragma unroll
                for (int q = 0; q < rows; ++q) {
                    const int gp = (P << t) + q;  // global row path at depth 3 + t
                    const int sg = side ^ (SW ? (__popc(gp) & 1) : 0);
#pragma unroll
                    for (int r = 0; r < K / 2; ++r) {
                        const R kk = kt[mr[r] << (3 + t)];
                        bfly(cur[q][r], cur[q][K - 1 - r], sg, kk, nxt[2 * q][r], nxt[2 * q + 1][r]);
                    }
                }
#pragma unroll
                for (int q = 0; q < 2 * rows; ++q)
#pragma unroll
                    for (int r = 0; r < K / 2; ++r) cur[q][r] = nxt[q][r];
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) w[side * SH + pad(16 * (16 * P + q) + m0)] = cur[q][0];
        }
    }
    __syncthreads();

    // ------------------------------------------------------------------ P3
    if (tid < 256) {
        const int side = tid >> 7, Rw = tid & 127;
        const int sg = side ^ (SW ? (__popc(Rw) & 1) : 0);
        const int b = side * SH;
        cx<R> v[16];
#pragma unroll
        for (int e = 1; e < 16; ++e) v[e] = w[b + pad(16 * Rw + e)];
        v[0] = zero<R>();
        if (sg == 0) row16<V, 0, R>(v, kt);
        else row16<V, 1, R>(v, kt);
#pragma unroll
        for (int e = 1; e < 16; ++e) w[b + pad(16 * Rw + e)] = v[e];
    } else if (tid < 272) {
        const int side = (tid - 256) >> 3, P = (tid - 256) & 7;
        const int sg = side ^ (SW ? (__popc(P) & 1) : 0);
        const int b = side * SH;
        cx<R> v[16];
#pragma unroll
        for (int e = 1; e < 16; ++e) v[e] = w[b + pad(256 * P + 16 * e)];
        v[0] = zero<R>();
        if (sg == 0) row16<V, 0, R>(v, kt);
        else row16<V, 1, R>(v, kt);
#pragma unroll
        for (int e = 1; e < 16; ++e) w[b + pad(256 * P + 16 * e)] = v[e];
    }
    __syncthreads();

    // ------------------------------------------------------------------ B2
    {
        const bool act = tid < 240;
        int side = 0, P = 0, a = 0, j = 0, sp = 1;
        cx<R> ext[16][3];
        if (act) {
            side = tid / 120;
            const int u = tid - side * 120;
            P = u / 15;
            const int w15 = u - P * 15;
            a = w15 < 8 ? 0 : w15 < 12 ? 1 : w15 < 14 ? 2 : 3;
            j = w15 - (a == 0 ? 0 : a == 1 ? 8 : a == 2 ? 12 : 14);
            sp = 8 >> a;  // sub-block size at depth 7
            const int b = side * SH;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int row = 16 * (16 * P + q);
                ext[q][0] = j >= 1 ? w[b + pad(row + ((2 * j - 1) << a))] : zero<R>();
                ext[q][1] = w[b + pad(row + ((2 * j + 1) << a))];
                ext[q][2] = j + 1 < sp ? w[b + pad(row + ((2 * j + 3) << a))] : zero<R>();
            }
        }
        __syncthreads();
        if (act) {
            cx<R> o[16];
            bwd_run<V, 4, R>(ext, side, P, o);
            const int b = side * SH;
#pragma unroll
            for (int e = 0; e < 16; ++e) w[b + pad(256 * P + ((2 * (16 * j + e) + 1) << a))] = o[e];
        }
    }
    __syncthreads();

    // ------------------------------------------------------------------ B1
    {
        const bool act = tid < 255;
        int a = 0, j = 0, sp = 1;
        cx<R> ext[2][8][3];
        if (act) {
            const int u1 = tid + 1;
            const int bb = 31 - __clz(u1);  // 0..7
            a = 7 - bb;
            j = u1 - (1 << bb);
            sp = 128 >> a;  // sub-block size at depth 3
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int b = side * SH;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int row = 256 * q;
                    ext[side][q][0] = j >= 1 ? w[b + pad(row + ((2 * j - 1) << a))] : zero<R>();
                    ext[side][q][1] = w[b + pad(row + ((2 * j + 1) << a))];
                    ext[side][q][2] = j + 1 < sp ? w[b + pad(row + ((2 * j + 3) << a))] : zero<R>();
                }
            }
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                cx<R> o[8];
                bwd_run<V, 3, R>(ext[side], side, 0, o);
                const int b = side * SH;
#pragma unroll
                for (int e = 0; e < 8; ++e) w[b + pad(((2 * (8 * j + e) + 1) << a))] = o[e];
            }
        }
    }
    __syncthreads();

    // ------------------------------------------------------------------ C0
    if (tid < 256) {
        // O_a(k): DCT at slot (2k+1) 2^a, DST at slot (2k-1) 2^a; E_8 at 256 k
        auto Oc = [&](int a, int k) { return w[pad((2 * k + 1) << a)]; };
        auto Os = [&](int a, int k) { return w[SH + pad((2 * k - 1) << a)]; };
        auto st = [&](int k, cx<R> v) {
            if (conj_out) v = cconj(v);
            storage<S>::st(y + k, v);
        };
        if (tid > 0) {
            const int k0 = tid;
            // chain levels 3..7 along the reflection path of k0 (q_a = 1024 >> a)
            cx<R> Ec3, Es3;
            {
                cx<R> acc = zero<R>();
                int kk = k0;
#pragma unroll
                for (int a = 3; a <= 7; ++a) {
                    const int q = Q4 >> a;
                    if (kk < q) acc = acc + Oc(a, kk);
                    else if (kk > q) { kk = 2 * q - kk; acc = acc - Oc(a, kk); }
                }
                const cx<R> e8 = kk < 8 ? w[pad(256 * kk)] : w[SH + pad(0)];
                Ec3 = acc + e8;
            }
            {
                cx<R> acc = zero<R>();
                R sgn = R(1);
                int kk = k0;
                bool done = false;
#pragma unroll
                for (int a = 3; a <= 7; ++a) {
                    const int q = Q4 >> a;
                    if (!done) {
                        if (kk < q) acc = acc + Os(a, kk) * sgn;
                        else if (kk > q) { kk = 2 * q - kk; acc = acc + Os(a, kk) * sgn; sgn = -sgn; }
                        else { acc = acc + Os(a, q) * sgn; done = true; }
                    }
                }
                if (!done) acc = acc + w[SH + pad(256 * kk)] * sgn;
                Es3 = acc;
            }
            // levels 2, 1, 0 on the orbit {k0, 512-k0, 512+k0, 1024-k0, ...}
            const int kA = k0, kB = 512 - k0, kC = 512 + k0, kD = 1024 - k0;
            // DCT
            const cx<R> oc2 = Oc(2, k0);
            const cx<R> c2a = Ec3 + oc2, c2b = Ec3 - oc2;  // E2(k0), E2(512-k0)
            const cx<R> o1a = Oc(1, kA), o1b = Oc(1, kB);
            const cx<R> c1[4] = {c2a + o1a, c2b + o1b, c2b - o1b, c2a - o1a};  // E1 at kA, kB, kC, kD
            cx<R> C[8];  // E0 at kA, kB, kC, kD, 2048-kD, 2048-kC, 2048-kB, 2048-kA
            const int ks[4] = {kA, kB, kC, kD};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const cx<R> o0 = Oc(0, ks[i]);
                C[i] = c1[i] + o0;
                C[7 - i] = c1[i] - o0;
            }
            // DST
            const cx<R> os2 = Os(2, k0);
            const cx<R> s2a = os2 + Es3, s2b = os2 - Es3;
            const cx<R> p1a = Os(1, kA), p1b = Os(1, kB);
            const cx<R> s1[4] = {p1a + s2a, p1b + s2b, p1b - s2b, p1a - s2a};
            cx<R> Dd[8];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const cx<R> o0 = Os(0, ks[i]);
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
        } else {
            // harmonics 0, 256, ..., 2048
            const cx<R> E3_0 = w[pad(0)] + Oc(3, 0) + Oc(4, 0) + Oc(5, 0) + Oc(6, 0) + Oc(7, 0);
            // E_3(256), the top harmonic of periodization 512: E_4(0) - O_3(0)
            const cx<R> E3_256 = w[pad(0)] - Oc(3, 0) + Oc(4, 0) + Oc(5, 0) + Oc(6, 0) + Oc(7, 0);
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
            const cx<R> D1_256 = p1 + D2_256, D1_768 = p1 - D2_256, D1_512 = Os(1, 512);
            cx<R> Dd[9];
            Dd[0] = zero<R>();
            Dd[8] = zero<R>();
            const cx<R> D1v[4] = {zero<R>(), D1_256, D1_512, D1_768};
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

template <int V, typename S>
hipError_t launch_a4096_typed(const lds_launch& a, hipStream_t st) {
    using R = typename storage<S>::R;
    constexpr size_t lds = Q4 * sizeof(R) + 2 * (H4 + H4 / 16) * sizeof(cx<R>);
    const int flags = (a.conj_in ? 1 : 0) | (a.conj_out ? 2 : 0) | (a.onthefly ? 4 : 0);
    hipLaunchKernelGGL((amqft_a4096_kernel<V, S>), dim3((unsigned)a.batch), dim3(THREADS4), lds, st,
                       static_cast<const S*>(a.in), static_cast<S*>(a.out), static_cast<const R*>(a.ktab),
                       (long long)a.batch, a.ktab_log2n - 12, flags, static_cast<const long long*>(a.offsets));
    return hipGetLastError();
}

}  // namespace

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
