// Device building blocks of the transposed (skeleton-B) program: the passes
// C0^T, FOLD, B0^T, B_k^T, P3^T, M_k^T, F1^T of amqft_kB.hip, shared by that
// kernel and by the large-N skeleton-B kernels (amqft_kLT.hip).  Included
// once per translation unit; everything lives in an unnamed namespace.
#pragma once
#include <type_traits>

#include "amqft_device.h"
#include "amqft_kA_passes.h"
#include "amqft_leaf.h"

namespace amqft {

namespace {

// skeleton-A variant whose transposed program is skeleton-B variant VB
template <int VB>
struct transposed_of;
template <> struct transposed_of<2> { static constexpr int V = 4; };
template <> struct transposed_of<6> { static constexpr int V = 8; };
template <> struct transposed_of<3> { static constexpr int V = 1; };
template <> struct transposed_of<7> { static constexpr int V = 5; };

// transposed butterfly of bfly<SG>: lo = x +- y, hi = (x -+ y) k
template <int SG, typename R>
__device__ __forceinline__ void bflyT(cx<R> lo, cx<R> hi, R k, cx<R>& x, cx<R>& y) {
    const cx<R> h = hi * k;
    x = lo + h;
    y = SG == 0 ? lo - h : h - lo;
}

// i z and -i z (exact)
template <typename R>
__device__ __forceinline__ cx<R> mul_i(cx<R> z) { return cx<R>{-z.im, z.re}; }

// transposed combine of one harmonic pair: X(k) = a = C - i D, X(N-k) = b =
// C + i D, so C' = a + b and D' = i (b - a)
template <typename R>
__device__ __forceinline__ void combineT(cx<R> a, cx<R> b, cx<R>& C, cx<R>& Dd) {
    C = a + b;
    Dd = mul_i(b - a);
}

// ---------------------------------------------------------------------------
// transposed backward levels: the transposes of combine / bwd_levels, on
// runs of the parent extended by a whole neighbouring run each side (those
// runs' contributions to the child index are exact; the rest is discarded)
// ---------------------------------------------------------------------------
// transposed M^F of one parent position in context SG: the parent value p
// (= P'[rho]) goes to the hi child entries it was formed from
template <int V, int SG, typename R>
__device__ __forceinline__ void mfT(cx<R> p, cx<R>& hm, cx<R>& h0, cx<R>& hp) {
    if constexpr (V == 4) {
        if (SG == 0) { h0 = h0 + p; hp = hp + p; }
        else { hm = hm + p; h0 = h0 + p; }
    } else {
        if (SG == 0) { h0 = h0 + p; hm = hm - p; }
        else { h0 = h0 + p; hp = hp - p; }
    }
}

// one transposed level on a parent run of 2n values (no halos: the caller's
// run is a whole window): L (n), Hh (n) out
template <int V, int SG, int n, typename R>
__device__ __forceinline__ void combineT_run(const cx<R>* P, cx<R>* L, cx<R>* Hh) {
#pragma unroll
    for (int i = 0; i < n; ++i) Hh[i] = zero<R>();
#pragma unroll
    for (int rho = 0; rho < 2 * n; ++rho) {
        const bool even = (rho & 1) == 0;
        const int i = even ? rho / 2 : (rho - 1) / 2;
        if ((SG == 0) == even) {
            L[i] = P[rho];
        } else {
            // forward: P[rho] = mf(H[i-1], H[i], H[i+1]) with H outside [0, n) zero
            cx<R> hm = zero<R>(), h0 = zero<R>(), hp = zero<R>();
            mfT<V, SG, R>(P[rho], hm, h0, hp);
            if (i - 1 >= 0) Hh[i - 1] = Hh[i - 1] + hm;
            Hh[i] = Hh[i] + h0;
            if (i + 1 < n) Hh[i + 1] = Hh[i + 1] + hp;
        }
    }
}

// r transposed levels below a parent of context SGB on a window of W runs
// of 2^r parent values: cur[0] holds the W 2^r parent values; after the
// levels, cur[q][w] = child q's value at run w of the window
template <int V, int SGB, int r, int t, int W, typename R>
__device__ __forceinline__ void fwd_levelsT(cx<R> (&cur)[1 << r][W << r]) {
    if constexpr (t < r) {
        constexpr bool SW = variant_traits<V>::switches;
        // before level t: 2^t rows, each a run of W 2^(r-t) values
        constexpr int nrow = 1 << t;
        constexpr int len = W << (r - t);
        cx<R> nxt[1 << r][W << r];
        sfor<0, nrow>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            // row q of depth t splits into rows 2q (lo) and 2q+1 (hi) of depth t+1;
            // in bwd_levels the parent of depth t is row q at level r-1-t counted
            // from the bottom, with context SGB ^ parity(q) for M8
            constexpr int sg = SGB ^ (SW ? par(q) : 0);
            combineT_run<V, sg, len / 2, R>(cur[q], nxt[2 * q], nxt[2 * q + 1]);
        });
#pragma unroll
        for (int q = 0; q < 2 * nrow; ++q)
#pragma unroll
            for (int e = 0; e < len / 2; ++e) cur[q][e] = nxt[q][e];
        fwd_levelsT<V, SGB, r, t + 1, W, R>(cur);
    }
}

// The window a child index needs: its own run and the runs whose parent
// values reach it through the time-side M2 / M6 terms.  M2 (from M4) in DCT
// context takes the neighbour before (H'[i] = P'[2i+1] + P'[2i-1]), in DST
// context the one after; M6 (from M8) switches context from row to row, so
// both.  OFF = first run relative to the child index, W = runs.
template <int VA, int SGB>
struct halo_window {
    static constexpr bool both = variant_traits<VA>::switches;
    static constexpr int W = both ? 3 : 2;
    static constexpr int OFF = both ? -1 : (SGB == 0 ? -1 : 0);
};

// ---------------------------------------------------------------------------
// C0^T: one thread per orbit of 16 outputs' positions (the F1 orbit); every
// entry of blocks 0..2 is written by exactly one thread (C0 read each of them
// once); the level-3 chain values go to FOLD.
//   depth-0 block a, entry i: unpadded position H - H / 2^a + i of its half
//   level-a chain of FOLD: DCT E(k) at H - 2 q_a + k (k < 2 q_a), E(2 q_a) in
//   the chain slot 8; DST S(k) at H - 2 q_a + k - 1 (k = 1 .. 2 q_a - 1);
//   q_a = N / 2^(a+2)
// ---------------------------------------------------------------------------
template <int LOGN>
__device__ __forceinline__ int hslot(int side, int p) {
    using G = kgeo<LOGN>;
    return side * G::HS + p + (p >> 4);
}

// Where C0^T and FOLD keep a side's depth-0 position p and the chain slots:
// the kernel's LDS image (padded halves, chain slots in pad slots) ...
template <int LOGN>
struct lds_lay {
    static __device__ __forceinline__ int at(int side, int p) { return hslot<LOGN>(side, p); }
    static __device__ __forceinline__ int ch(int c) { return lds_layout<LOGN>::chain(c); }
};
// ... or a global workspace (side after side, unpadded; chain slots in a
// buffer of 16 values of their own)
template <int LOGN>
struct glob_lay {
    static __device__ __forceinline__ int at(int side, int p) { return side * ((1 << LOGN) / 2) + p; }
    static __device__ __forceinline__ int ch(int c) { return c; }
};

template <int LOGN, typename R, typename LAY = lds_lay<LOGN>>
__device__ __forceinline__ void c0T(cx<R>* w, cx<R>* wc, const cx<R> (&raw)[16], int k0, bool conj_in) {
    using G = kgeo<LOGN>;
    constexpr int N = G::N, H = G::H, N8 = N / 8, N16 = N / 16;
    constexpr int B1 = H / 2, B2 = 3 * H / 4, C3 = H - N16;  // starts of blocks 1, 2 and of the level-3 chain
    cx<R> x[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = conj_in ? cconj(raw[e]) : raw[e];
    if (k0 > 0) {
        // res[] order of C0: pairs (lo, hi) = (X(k), X(N-k)) for C[c], Dd[c]
        constexpr int LO[8] = {0, 8, 1, 9, 2, 10, 3, 11}, HI[8] = {15, 7, 14, 6, 13, 5, 12, 4};
        cx<R> C[8], Dd[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) combineT(x[LO[c]], x[HI[c]], C[c], Dd[c]);
        const int kA = k0, kB = N8 - k0, kC = kA + N8, kD = kB + N8;
        // DCT: levels 0, 1, 2 of the chain's D_k^T
        cx<R> c1[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) c1[i] = C[i] + C[7 - i];
        stc(w + LAY::at(0, kA), C[0] - C[7]);
        stc(w + LAY::at(0, kB), C[1] - C[6]);
        stc(w + LAY::at(0, kC), C[2] - C[5]);
        stc(w + LAY::at(0, kD), C[3] - C[4]);
        const cx<R> c2a = c1[0] + c1[3], c2b = c1[1] + c1[2];
        stc(w + LAY::at(0, B1 + kA), c1[0] - c1[3]);
        stc(w + LAY::at(0, B1 + kB), c1[1] - c1[2]);
        stc(w + LAY::at(0, B2 + kA), c2a - c2b);
        stc(w + LAY::at(0, C3 + kA), c2a + c2b);  // E_3(k0)
        // DST
        cx<R> s1[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) s1[i] = Dd[i] - Dd[7 - i];
        stc(w + LAY::at(1, kA - 1), Dd[0] + Dd[7]);
        stc(w + LAY::at(1, kB - 1), Dd[1] + Dd[6]);
        stc(w + LAY::at(1, kC - 1), Dd[2] + Dd[5]);
        stc(w + LAY::at(1, kD - 1), Dd[3] + Dd[4]);
        const cx<R> s2a = s1[0] - s1[3], s2b = s1[1] - s1[2];
        stc(w + LAY::at(1, B1 + kA - 1), s1[0] + s1[3]);
        stc(w + LAY::at(1, B1 + kB - 1), s1[1] + s1[2]);
        stc(w + LAY::at(1, B2 + kA - 1), s2a + s2b);
        stc(w + LAY::at(1, C3 + kA - 1), s2a - s2b);  // S_3(k0)
    } else {
        // harmonics N/16 i: res[0] = C(0), res[8] = C(N/2), (res[i], res[16-i]) = (lo, hi) of (C, Dd)[i]
        cx<R> C[9], Dd[8];
        C[0] = x[0];
        C[8] = x[8];
#pragma unroll
        for (int i = 1; i < 8; ++i) combineT(x[i], x[16 - i], C[i], Dd[i]);
        cx<R> E1v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            E1v[i] = C[i] + C[8 - i];
            stc(w + LAY::at(0, N16 * i), C[i] - C[8 - i]);  // block 0 at N/16 i
        }
        const cx<R> E1_4 = C[4];
        const cx<R> E2_0 = E1v[0] + E1_4, E2_1 = E1v[1] + E1v[3], E2_2 = E1v[2];
        stc(w + LAY::at(0, B1), E1v[0] - E1_4);          // block 1 at 0
        stc(w + LAY::at(0, B1 + N16), E1v[1] - E1v[3]);  // block 1 at N/16
        stc(w + LAY::at(0, B2), E2_0 - E2_2);            // block 2 at 0
        stc(w + LAY::at(0, C3), E2_0 + E2_2);            // E_3(0)
        stc(wc + LAY::ch(8), E2_1);                          // E_3(N/16): the top of the level-3 chain
        // DST
        cx<R> D1v[4];
#pragma unroll
        for (int i = 1; i < 4; ++i) {
            stc(w + LAY::at(1, N16 * i - 1), Dd[i] + Dd[8 - i]);  // block 0 at N/16 i
            D1v[i] = Dd[i] - Dd[8 - i];
        }
        stc(w + LAY::at(1, 4 * N16 - 1), Dd[4]);                  // block 0 at N/4
        stc(w + LAY::at(1, B1 + N16 - 1), D1v[1] + D1v[3]);       // block 1 at N/16
        stc(w + LAY::at(1, B1 + 2 * N16 - 1), D1v[2]);            // block 1 at N/8
        stc(w + LAY::at(1, B2 + N16 - 1), D1v[1] - D1v[3]);       // block 2 at N/16
    }
}

// ---------------------------------------------------------------------------
// FOLD: D_k^T of the chain for levels a = 3 .. D-3 (C0 walked these levels
// along each harmonic's reflection path; here they are summed level by
// level).  A level of length L = 2 q_a folds E(k) with E(L - k) into the
// block entry E(k) - E(L - k) (k < q_a) and the next level's E(k) + E(L - k),
// E(q_a) becoming the next top; the DST side S(k) with S(L - k) into
// S(k) + S(L - k) and S(k) - S(L - k), S(q_a) staying a block entry.  The
// positions congruent to +-r modulo a power of two P stay among themselves
// under every fold down to L = P, so one lane takes each such orbit and walks
// those levels in registers with no barrier, storing its block entries as it
// goes and, after L = P, its values of the level L = P / 2.  The tail
// (L = P / 2 .. 16) is the same walk with P = 16 after a wave barrier: every
// orbit lane of a signal is a lane of the signal's first wave.  The last
// level writes the dct[16] / dst[16] values into the chain slots.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// orbit modulus of the first walk: at most 16 complex values a lane up to
// N = 2^13 (32 at 2^14), at most 64 lanes a signal
template <int LOGN>
constexpr int fold_p1() {
    constexpr int p = (1 << LOGN) / 128;
    return p < 16 ? 16 : p > 64 ? 64 : p;
}

// One walk on a side (DST: S values, else E values) from the level of length
// LS down to L = P, lane orbit r (0 = the orbit of the multiples of P / 2).
// The level of length L holds E(k) at H - L + k (k < L) with the top E(L) in
// chain slot 8, and S(k) at H - L + k - 1 (0 < k < L).  The lane's values v[i]
// of a level of length L = MP sit at k(i) = P floor(i / 2) + (i odd ? P - r :
// r) (orbit 0: k(i) = i P / 2, v[2M] the top); the fold pairs v[i] (i < M)
// with v[2M - 1 - i] (orbit 0: v[2M - i]), so every lane runs the same code
// (no divergence) and the values stay in registers.
template <int LOGN, int P, int LS, typename R, typename LAY = lds_lay<LOGN>>
struct fold_walk {
    using G = kgeo<LOGN>;
    static constexpr int M0 = LS / P;
    static constexpr int NV = 2 * M0 + 1;
    static constexpr int NL = ilog2c(M0) + 1;  // levels LS, LS / 2, .., P
    static constexpr bool LAST = P == 16;

    template <int Lv>
    static __device__ __forceinline__ int pos(bool dst, int k) {
        return LAY::at(dst, G::H - Lv + k - (dst ? 1 : 0));
    }
    static __device__ __forceinline__ int kpos(int i, int r) {
        return P * (i >> 1) + ((i & 1) ? (r > 0 ? P - r : P / 2) : r);
    }

    // the orbit's values of the level LS; slots a lane's orbit lacks (S(0),
    // and v[2 M0] outside the DCT orbit 0) read a position of its own orbit
    // (wc: the base of the chain slots)
    static __device__ __forceinline__ void load(const cx<R>* w, const cx<R>* wc, bool dst, int r, cx<R> (&v)[NV]) {
#pragma unroll
        for (int i = 0; i < 2 * M0; ++i) v[i] = ldc(w + pos<LS>(dst, kpos(i, r) + (dst && i == 0 && r == 0 ? P / 2 : 0)));
        v[2 * M0] = !dst && r == 0 ? ldc(wc + LAY::ch(8)) : ldc(w + pos<LS>(dst, kpos(1, r)));
    }

    // block entries go to w, the values of the level P / 2 to wo (the same
    // positions), the top and the last level's chain values to wc
    static __device__ __forceinline__ void walk(cx<R>* w, cx<R>* wo, cx<R>* wc, bool dst, int r, cx<R> (&v)[NV]) {
        const bool o0 = r == 0;
        sfor<0, NL>([&](auto lc) {
            constexpr int Lv = LS >> decltype(lc)::value;
            constexpr int M = Lv / P;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const cx<R> b = o0 ? v[2 * M - i] : v[2 * M - 1 - i];
                const cx<R> sb = dst ? cx<R>{-b.re, -b.im} : b;  // DCT: E -+ E', DST: S +- S'
                if (!(dst && o0 && i == 0)) stc(w + pos<Lv>(dst, kpos(i, r)), v[i] - sb);
                v[i] = v[i] + sb;
            }
            // orbit 0: E(L / 2) = v[M] becomes the next top; S(L / 2) stays a
            // block entry (in place on the first level)
            if constexpr (Lv != LS) {
                if (dst && o0) stc(w + pos<Lv>(true, Lv / 2), v[M]);
            }
        });
        // v[0]: index r of the level P / 2 (none for the DST orbit 0)
        if (!(dst && o0)) stc(LAST ? wc + LAY::ch((dst ? 8 : 0) + r) : wo + pos<P / 2>(dst, r), v[0]);
        if (!dst && o0) stc(wc + LAY::ch(8), v[1]);
    }
};

// The whole FOLD of one signal by one workgroup of NT threads, for chains
// longer than one wave folds alone: walks of at most 8 values a lane per
// side and orbit (P = LS / 8, at least 16), a barrier between walks.  w is
// the signal's image in layout LAY.
template <int LOGN, int NT, int LS, typename R, typename LAY>
__device__ __forceinline__ void fold_block(cx<R>* w, int tid) {
    constexpr int P = LS / 8 < 16 ? 16 : LS / 8;
    static_assert(P <= NT, "one lane per orbit");
    using F = fold_walk<LOGN, P, LS, R, LAY>;
    const bool act = tid < P, dst = tid >= P / 2;
    const int r = tid & (P / 2 - 1);
    cx<R> v[F::NV];
    if (act) F::load(w, w, dst, r, v);
    __syncthreads();  // the next level's values land where other lanes' loads were
    if (act) F::walk(w, w, w, dst, r, v);
    if constexpr (!F::LAST) {
        __syncthreads();
        fold_block<LOGN, NT, P / 2, R, LAY>(w, tid);
    }
}

template <int LOGN, typename R>
__device__ __forceinline__ void fold(cx<R>* wall, int tid) {
    using G = kgeo<LOGN>;
    constexpr int P1 = fold_p1<LOGN>(), L0 = G::N / 16;
    static_assert(P1 <= 64 && P1 <= G::T, "a signal's orbit lanes must fit its first wave");
    const int s = tid / G::T, k = tid - s * G::T;
    cx<R>* w = wall + s * G::SL;
    {
        using F = fold_walk<LOGN, P1, L0, R>;
        const bool act = k < P1, dst = k >= P1 / 2;
        const int r = k & (P1 / 2 - 1);
        cx<R> v[F::NV];
        if (act) F::load(w, w, dst, r, v);
        // the values of the level P1 / 2 land where other lanes' loads were
        // (the last level writes only chain slots and the lane's own orbit)
        if constexpr (!F::LAST) wave_sync();
        if (act) F::walk(w, w, w, dst, r, v);
    }
    if constexpr (P1 > 16) {
        using F = fold_walk<LOGN, 16, P1 / 2, R>;
        wave_sync();
        const bool act = k < 16, dst = k >= 8;
        const int r = k & 7;
        cx<R> v[F::NV];
        if (act) F::load(w, w, dst, r, v);
        if (act) F::walk(w, w, w, dst, r, v);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// B0^T: levels 0..2 of dct_to / dst_to on both sides; thread = position p of
// the depth-3 layout (as in B0): it reads the depth-0 runs of its child index
// j and of j -+ 1 (the neighbours' runs carry the +-1 neighbour terms of the
// time-side M2 / M6 relations) and writes its child index in the 8 rows.
// ---------------------------------------------------------------------------
template <int VA, int LOGN, typename R>
__device__ __forceinline__ void b0T_pass(cx<R>* wall, int tid) {
    using G = kgeo<LOGN>;
    constexpr bool SW = variant_traits<VA>::switches;
    constexpr int LW3 = ilog2c(G::W3);
    const int s = tid / G::T, p = tid - s * G::T;
    int a = 0, j = 0, sp = 1;
    int off1 = 0;
    if constexpr (G::NP == 0) {
        const int e = p - 1;
        const int b = e < 8 ? 0 : e < 12 ? 1 : e < 14 ? 2 : 3;
        sp = 8 >> b;
        j = e - (16 - 2 * sp);
        a = b;
        off1 = pad(p);
    } else {
        using M0 = mpass<LOGN, 0>;
        constexpr int r0 = M0::r, G0 = M0::GL;
        if (p < (1 << r0)) {
            const int e = p - 1;
            const int b = __clz(~(e << (32 - r0)));
            sp = (1 << (r0 - 1)) >> b;
            j = e - ((1 << r0) - 2 * sp);
            a = LW3 - r0 + b;
            off1 = 17 * ((e + 1) * (G0 / 16)) + 16;
        } else {
            const int pp = p - (1 << r0);
            a = __clz(~(pp << (32 - LW3)));
            j = pp - (G::W3 - (G::W3 >> a));
            sp = G::W3 >> (a + 1);
            off1 = pad(p);
        }
    }
    const bool act = p > 0;
    using W0 = halo_window<VA, 0>;
    using W1 = halo_window<VA, 1>;
    cx<R> cur0[8][W0::W * 8], cur1[8][W1::W * 8];
    if (act) {
        cx<R>* ws = wall + s * G::SL;
        auto load = [&](auto& cur, auto wc, int side) {
            using WW = decltype(wc);
#pragma unroll
            for (int d = 0; d < WW::W; ++d) {
                const int jj = j + WW::OFF + d;
                const bool in = jj >= 0 && jj < sp;
                const int ob = pad(G::H - (G::H >> a) + 8 * (in ? jj : j));
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const cx<R> v = ldc(ws + side * G::HS + ob + e);
                    cur[0][8 * d + e] = in ? v : zero<R>();
                }
            }
        };
        load(cur0, W0{}, 0);
        load(cur1, W1{}, 1);
    }
    __syncthreads();
    if (act) {
        fwd_levelsT<VA, 0, 3, 0, W0::W, R>(cur0);
        fwd_levelsT<VA, 1, 3, 0, W1::W, R>(cur1);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            stc(wall + s * G::SL + (0 ^ (SW ? par(q) : 0)) * G::HS + q * G::W3P + off1, cur0[q][-W0::OFF]);
            stc(wall + s * G::SL + (1 ^ (SW ? par(q) : 0)) * G::HS + q * G::W3P + off1, cur1[q][-W1::OFF]);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// B_K^T: forward levels l0 .. l0 + r - 1 of pass K (the transposed B_K)
// ---------------------------------------------------------------------------
template <int VA, int LOGN, int K, typename R>
__device__ __forceinline__ void bT_pass(cx<R>* wall, int tid) {
    using G = kgeo<LOGN>;
    using M = mpass<LOGN, K>;
    constexpr bool SW = variant_traits<VA>::switches;
    constexpr int NV = M::NV, IT = M::IT, LG = ilog2c(M::GL);
    // one window shape for both halves: a wave's tasks share a half, but the
    // compile-time window must cover both contexts
    constexpr int W = variant_traits<VA>::switches ? 3 : 2;
    cx<R> cur[IT][NV][W * NV];
    int off1[IT];
    task tk[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        tk[it] = mtask<LOGN, K>(it, tid);
        const task t = tk[it];
        off1[it] = 0;
        if (t.m > 0) {
            const int wm = t.m - 1;
            const int a = __clz(~(wm << (32 - LG)));
            const int j = wm - (M::GL - (M::GL >> a));
            const int sp = M::GL >> (a + 1);
            int off[3];
            child_offsets<LOGN, K>(a, j, sp, off);
            off1[it] = off[1];
            const cx<R>* src = wall + t.s * G::SL + t.h * G::HS + t.P * M::WP;
            // first run of the window relative to j: -1 (both neighbours, or
            // the one before in DCT context) or 0 (the one after, DST context)
            const int woff = W == 3 ? -1 : (t.h == 0 ? -1 : 0);
#pragma unroll
            for (int d = 0; d < W; ++d) {
                const int jj = j + woff + d;
                const bool in = jj >= 0 && jj < sp;
                const int base = pad(NV * (in ? t.m + woff + d : t.m));
#pragma unroll
                for (int e = 0; e < NV; ++e) {
                    const cx<R> v = ldc(src + base + e);
                    cur[it][0][NV * d + e] = in ? v : zero<R>();
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const task t = tk[it];
        if (t.m > 0) {
            // the half fixes the context of the levels and, for a window of
            // two runs, which of them is the child index's own (a compile-time
            // index keeps the window in registers)
            auto finish = [&](auto hc) {
                constexpr int h = decltype(hc)::value;
                constexpr int own = W == 3 ? 1 : (h == 0 ? 1 : 0);
                fwd_levelsT<VA, h, M::r, 0, W, R>(cur[it]);
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    const int hq = h ^ (SW ? par(q) : 0);
                    stc(wall + t.s * G::SL + hq * G::HS + (t.P * NV + q) * M::GP + off1[it], cur[it][q][own]);
                }
            };
            if (t.h == 0) finish(std::integral_constant<int, 0>{});
            else finish(std::integral_constant<int, 1>{});
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// M3 / M7: the transposes of the M1 / M5 recurrences.  With the sign pattern
// D = diag((-1)^i) of M1 and the halving Hv of the first term in scan order,
// the backward M^F of M1 / M5 is g = D T D Hv h (T an inclusive prefix or
// suffix sum along the hi child); its transpose is Hv D T^T D: the same lane
// scan run in the other direction, the halving applied after it.  That is
// the time-side recurrence of M3 / M7, the last term halved (Tables
// tab:DCT_odd_transformations, tab:DST_odd_transformations).
// ---------------------------------------------------------------------------
// one transposed level for one lane: parent entries P[0 .. 2n) -> lo child
// L[0 .. n), hi child Hh[0 .. n) (segment position pos of nl lanes)
template <int VA, int SG, int n, int MAXL, typename R>
__device__ __forceinline__ void rec_split(const cx<R>* P, cx<R>* L, cx<R>* Hh, int pos, int nl) {
    using RD = rec_dir<VA, SG>;
    constexpr bool TASC = !RD::asc;
    const int len = nl * n;
    cx<R> raw[n], u[n], loc[n];
#pragma unroll
    for (int e = 0; e < n; ++e) {
        L[e] = SG == 0 ? P[2 * e] : P[2 * e + 1];
        raw[e] = SG == 0 ? P[2 * e + 1] : P[2 * e];
        const int i = pos * n + e;
        u[e] = (RD::alt && (i & 1)) ? cx<R>{-raw[e].re, -raw[e].im} : raw[e];
    }
    cx<R> tot;
    if constexpr (TASC) {
        loc[0] = u[0];
#pragma unroll
        for (int e = 1; e < n; ++e) loc[e] = loc[e - 1] + u[e];
        tot = loc[n - 1];
    } else {
        loc[n - 1] = u[n - 1];
#pragma unroll
        for (int e = n - 2; e >= 0; --e) loc[e] = loc[e + 1] + u[e];
        tot = loc[0];
    }
    cx<R> carry, own = tot;
    if constexpr (n == 1) pair_excl<TASC, MAXL, R>(u[0], pos, nl, carry, own);
    else carry = seg_excl<TASC, MAXL, R>(tot, pos, nl);
#pragma unroll
    for (int e = 0; e < n; ++e) {
        const int i = pos * n + e;
        cx<R> g = (n == 1 ? own : loc[e]) + carry;
        if (RD::alt && (i & 1)) g = cx<R>{-g.re, -g.im};
        if (len > 1 && (RD::asc ? i == 0 : i == len - 1)) g = g * R(0.5);
        Hh[e] = len == 1 ? raw[e] : g;  // L = 8 base: no M step
    }
}

// r transposed recurrence levels below a parent of context SGB for one lane:
// cur[0][0 .. 2^r) = the lane's parent entries in; cur[q][0] = child q out
template <int VA, int SGB, int r, int t, int MAXL, typename R>
__device__ __forceinline__ void rec_levelsT(cx<R> (&cur)[1 << r][1 << r], int pos, int nl) {
    if constexpr (t < r) {
        constexpr bool SW = variant_traits<VA>::switches;
        constexpr int nrow = 1 << t, n = 1 << (r - 1 - t);
        cx<R> nxt[1 << r][1 << r];
        sfor<0, nrow>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int sg = SGB ^ (SW ? par(q) : 0);
            rec_split<VA, sg, n, MAXL, R>(cur[q], nxt[2 * q], nxt[2 * q + 1], pos, nl);
        });
#pragma unroll
        for (int q = 0; q < 2 * nrow; ++q)
#pragma unroll
            for (int e = 0; e < n; ++e) cur[q][e] = nxt[q][e];
        rec_levelsT<VA, SGB, r, t + 1, MAXL, R>(cur, pos, nl);
    }
}

// B_K^T for M3 / M7 (the transposed bpass_rec: same lane remapping)
template <int VA, int LOGN, int K, typename R>
__device__ __forceinline__ void bT_rec_pass(cx<R>* wall, int tid) {
    using G = kgeo<LOGN>;
    using M = mpass<LOGN, K>;
    constexpr bool SW = variant_traits<VA>::switches;
    constexpr int NV = M::NV, IT = M::IT, LG = ilog2c(M::GL), MAXL = M::GL / 2;
    cx<R> cur[IT][NV][NV];
    task tk[IT];
    int jj[IT], spp[IT], off1[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        tk[it] = mtask<LOGN, K>(it, tid);
        const task t = tk[it];
        const int wm = t.m;
        const int a = __clz(~(wm << (32 - LG)));
        const bool act = wm < M::GL - 1;
        const int j = act ? wm - (M::GL - (M::GL >> a)) : 0;
        const int sp = act ? M::GL >> (a + 1) : 0;
        jj[it] = j;
        spp[it] = sp;
        int off[3] = {0, 0, 0};
        if (act) child_offsets<LOGN, K>(a, j, sp, off);
        off1[it] = off[1];
        const cx<R>* src = wall + t.s * G::SL + t.h * G::HS + t.P * M::WP + pad(NV * (t.m + 1));
#pragma unroll
        for (int e = 0; e < NV; ++e) cur[it][0][e] = act ? ldc(src + e) : zero<R>();
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const task t = tk[it];
        if (t.h == 0) rec_levelsT<VA, 0, M::r, 0, MAXL, R>(cur[it], jj[it], spp[it]);
        else rec_levelsT<VA, 1, M::r, 0, MAXL, R>(cur[it], jj[it], spp[it]);
        if (t.m < M::GL - 1) {
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                const int hq = t.h ^ (SW ? par(q) : 0);
                stc(wall + t.s * G::SL + hq * G::HS + (t.P * NV + q) * M::GP + off1[it], cur[it][q][0]);
            }
        }
    }
    __syncthreads();
}

// B0^T for M3 / M7 (the transposed b0_pass_rec: same lane remapping, wave
// carries of segments longer than a wave through LDS, in the other direction)
template <int VA, int LOGN, typename R>
__device__ __forceinline__ void b0T_rec_pass(cx<R>* wall, cx<R>* scr, int tid) {
    using G = kgeo<LOGN>;
    constexpr bool SW = variant_traits<VA>::switches;
    constexpr int LW3 = ilog2c(G::W3);
    constexpr bool MULTI = G::W3 / 2 > 64;
    constexpr int MAXL = G::W3 / 2 < 64 ? G::W3 / 2 : 64;
    const int s = tid / G::T, L = tid - s * G::T;
    int a = 0, j = 0, sp = 0, p = 0;
    int off1 = 0;
    if constexpr (G::NP == 0) {
        p = L;
        if (p > 0) {
            const int e = p - 1;
            const int b = e < 8 ? 0 : e < 12 ? 1 : e < 14 ? 2 : 3;
            sp = 8 >> b;
            j = e - (16 - 2 * sp);
            a = b;
            off1 = pad(p);
        }
    } else {
        using M0 = mpass<LOGN, 0>;
        constexpr int r0 = M0::r, G0 = M0::GL, NS = 1 << r0;
        if (L < G::W3 - NS) {
            const int pp = L;
            p = pp + NS;
            a = __clz(~(pp << (32 - LW3)));
            j = pp - (G::W3 - (G::W3 >> a));
            sp = G::W3 >> (a + 1);
            off1 = pad(p);
        } else {
            p = L - (G::W3 - NS);
            if (p > 0) {
                const int e = p - 1;
                const int b = __clz(~(e << (32 - r0)));
                sp = (1 << (r0 - 1)) >> b;
                j = e - ((1 << r0) - 2 * sp);
                a = LW3 - r0 + b;
                off1 = 17 * ((e + 1) * (G0 / 16)) + 16;
            }
        }
    }
    const bool act = p > 0;
    cx<R> cur[2][8][8];
    {
        const int ob = pad(G::H - (G::H >> a) + 8 * j);
        const cx<R>* ws = wall + s * G::SL;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            cur[0][0][e] = act ? ldc(ws + ob + e) : zero<R>();
            cur[1][0][e] = act ? ldc(ws + G::HS + ob + e) : zero<R>();
        }
    }
    __syncthreads();
    const int wl = L & 63;
    const int wv = L >> 6;
    const int seg0 = L - j;
    const bool multi = MULTI && sp > 64;
    const int pw = multi ? wl : j, nw = multi ? 64 : sp;
    cx<R>* sc = scr + s * ((G::T / 64) * 8);
    sfor<0, 3>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        constexpr int NR = 1 << t, n = 1 << (2 - t);  // parent rows of depth t, child entries per lane
        cx<R> lo[2][NR][n], raw[2][NR][n], loc[2][NR][n], own[2][NR], car[2][NR];
        sfor<0, 2>([&](auto sc2) {
            constexpr int side = decltype(sc2)::value;
            sfor<0, NR>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int sg = side ^ (SW ? par(q) : 0);
                using RD = rec_dir<VA, sg>;
                constexpr bool TASC = !RD::asc;
                cx<R> u[n];
#pragma unroll
                for (int e = 0; e < n; ++e) {
                    lo[side][q][e] = sg == 0 ? cur[side][q][2 * e] : cur[side][q][2 * e + 1];
                    raw[side][q][e] = sg == 0 ? cur[side][q][2 * e + 1] : cur[side][q][2 * e];
                    const int i = j * n + e;
                    u[e] = (RD::alt && (i & 1)) ? cx<R>{-raw[side][q][e].re, -raw[side][q][e].im} : raw[side][q][e];
                }
                if constexpr (TASC) {
                    loc[side][q][0] = u[0];
#pragma unroll
                    for (int e = 1; e < n; ++e) loc[side][q][e] = loc[side][q][e - 1] + u[e];
                    own[side][q] = loc[side][q][n - 1];
                } else {
                    loc[side][q][n - 1] = u[n - 1];
#pragma unroll
                    for (int e = n - 2; e >= 0; --e) loc[side][q][e] = loc[side][q][e + 1] + u[e];
                    own[side][q] = loc[side][q][0];
                }
                if constexpr (n == 1) pair_excl<TASC, MAXL, R>(u[0], pw, nw, car[side][q], own[side][q]);
                else car[side][q] = seg_excl<TASC, MAXL, R>(own[side][q], pw, nw);
            });
        });
        if constexpr (MULTI) {
            sfor<0, 2>([&](auto sc2) {
                constexpr int side = decltype(sc2)::value;
                sfor<0, NR>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    constexpr int sg = side ^ (SW ? par(q) : 0);
                    constexpr bool TASC = !rec_dir<VA, sg>::asc;
                    if (multi && wl == (TASC ? 63 : 0)) stc(sc + wv * 8 + side * 4 + q, own[side][q] + car[side][q]);
                });
            });
            __syncthreads();
            if (multi) {
                const int w0 = seg0 >> 6, w1 = (seg0 + sp - 1) >> 6;
                sfor<0, 2>([&](auto sc2) {
                    constexpr int side = decltype(sc2)::value;
                    sfor<0, NR>([&](auto qc) {
                        constexpr int q = decltype(qc)::value;
                        constexpr int sg = side ^ (SW ? par(q) : 0);
                        constexpr bool TASC = !rec_dir<VA, sg>::asc;
                        cx<R> c = zero<R>();
                        if (TASC) {
                            for (int w = w0; w < wv; ++w) c = c + ldc(sc + w * 8 + side * 4 + q);
                        } else {
                            for (int w = wv + 1; w <= w1; ++w) c = c + ldc(sc + w * 8 + side * 4 + q);
                        }
                        car[side][q] = car[side][q] + c;
                    });
                });
            }
            __syncthreads();
        }
        cx<R> nxt[2][8][8];
        sfor<0, 2>([&](auto sc2) {
            constexpr int side = decltype(sc2)::value;
            sfor<0, NR>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int sg = side ^ (SW ? par(q) : 0);
                using RD = rec_dir<VA, sg>;
#pragma unroll
                for (int e = 0; e < n; ++e) {
                    const int i = j * n + e;
                    const int len = sp * n;
                    cx<R> g = (n == 1 ? own[side][q] : loc[side][q][e]) + car[side][q];
                    if (RD::alt && (i & 1)) g = cx<R>{-g.re, -g.im};
                    if (len > 1 && (RD::asc ? i == 0 : i == len - 1)) g = g * R(0.5);
                    nxt[side][2 * q][e] = lo[side][q][e];
                    nxt[side][2 * q + 1][e] = len == 1 ? raw[side][q][e] : g;
                }
            });
        });
#pragma unroll
        for (int side = 0; side < 2; ++side)
#pragma unroll
            for (int q = 0; q < 2 * NR; ++q)
#pragma unroll
                for (int e = 0; e < n; ++e) cur[side][q][e] = nxt[side][q][e];
    });
    if (act) {
#pragma unroll
        for (int side = 0; side < 2; ++side)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int hq = side ^ (SW ? par(q) : 0);
                stc(wall + s * G::SL + hq * G::HS + q * G::W3P + off1, cur[side][q][0]);
            }
    }
    __syncthreads();
}

// whole sub-blocks of a row of 2^r slots, transposed rowk: o = the blocks'
// time values, block-contiguous (block of sz points at 2^r - 2 sz); s[e-1] =
// slot e receives the spectra (dct_to / dst_to of variant VB)
template <int VB, int SG, int r, typename R>
__device__ __forceinline__ void rowkT(const cx<R>* o, cx<R>* s, const R* kt, int D) {
    sfor<0, r>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        constexpr int sz = 1 << (r - 1 - b);
        cx<R> blk[sz];
#pragma unroll
        for (int i = 0; i < sz; ++i) blk[i] = o[(1 << r) - 2 * sz + i];
        leaf::to<VB, sz, SG, R>(blk, kt, D);
#pragma unroll
        for (int i = 0; i < sz; ++i) s[((2 * i + 1) << b) - 1] = blk[i];
    });
}

// P3^T: rows of 16 at depth D-3, in place
template <int VB, int LOGN, typename R>
__device__ __forceinline__ void p3T_pass(cx<R>* wall, const R* kt, int tid) {
    using G = kgeo<LOGN>;
    constexpr int NR = 1 << (G::D - 3);
    const int h = tid / (G::SPW * NR);
    const int rem = tid - h * (G::SPW * NR);
    const int s = rem / NR, R7 = rem - s * NR;
    cx<R>* row = wall + s * G::SL + h * G::HS + 17 * R7;
    cx<R> in[15], o[15];
#pragma unroll
    for (int e = 0; e < 15; ++e) in[e] = ldc(row + e + 1);
    if (h == 0) rowkT<VB, 0, 4, R>(in, o, kt, G::D);
    else rowkT<VB, 1, 4, R>(in, o, kt, G::D);
#pragma unroll
    for (int e = 0; e < 15; ++e) stc(row + e + 1, o[e]);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// M_K^T: backward levels l0 + r - 1 .. l0 on the orbits of pass K
// ---------------------------------------------------------------------------
template <int VA, int LOGN, int K, int H, typename R>
__device__ __forceinline__ void orbitT_compute(const R* kf, const cx<R> (&c)[mpass<LOGN, K>::NV], int m0,
                                               cx<R> (&v)[mpass<LOGN, K>::NV]) {
    using G = kgeo<LOGN>;
    using M = mpass<LOGN, K>;
    constexpr bool SW = variant_traits<VA>::switches;
    constexpr int NV = M::NV, r = M::r;
    const R* kw = kf + G::kfbase(K) + (m0 - 1);
    // cur[q][rho]: after level t of orbit_compute row q holds entries rho < KK/2
    cx<R> cur[NV][NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) cur[q][0] = c[q];
    sfor<0, r>([&](auto tc) {
        constexpr int t = r - 1 - decltype(tc)::value;  // undo level t
        constexpr int KK = NV >> t;
        constexpr int rows = 1 << t;
        cx<R> prv[NV][NV];
        sfor<0, rows>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int sg = H ^ (SW ? par(q) : 0);
#pragma unroll
            for (int rho = 0; rho < KK / 2; ++rho)
                bflyT<sg, R>(cur[2 * q][rho], cur[2 * q + 1][rho], kw[G::kft(K, t) + (M::GL - 1) * rho], prv[q][rho],
                             prv[q][KK - 1 - rho]);
        });
#pragma unroll
        for (int q = 0; q < rows; ++q)
#pragma unroll
            for (int rho = 0; rho < KK; ++rho) cur[q][rho] = prv[q][rho];
    });
#pragma unroll
    for (int e = 0; e < NV; ++e) v[e] = cur[0][e];
}

template <int VA, int VB, int LOGN, int K, typename R>
__device__ __forceinline__ void orbitT_pass(cx<R>* wall, const R* kt, const R* kf, int tid) {
    using G = kgeo<LOGN>;
    using M = mpass<LOGN, K>;
    constexpr bool SW = variant_traits<VA>::switches;
    constexpr int NV = M::NV, IT = M::IT;
    cx<R> c[IT][NV];
    task tk[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        tk[it] = mtask<LOGN, K>(it, tid);
        const task t = tk[it];
        cx<R>* ws = wall + t.s * G::SL;
        if (t.m > 0) {
            const int pm = pad(t.m);
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                const int hq = t.h ^ (SW ? par(q) : 0);
                c[it][q] = ldc(ws + hq * G::HS + (t.P * NV + q) * M::GP + pm);  // child row P 2^r + q, slot m
            }
        } else {
            const cx<R>* pb = ws + t.h * G::HS + t.P * M::WP + 16;
#pragma unroll
            for (int i = 0; i < NV - 1; ++i) c[it][i] = ldc(pb + 17 * (i + 1) * (M::GL / 16));
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const task t = tk[it];
        cx<R>* base = wall + t.s * G::SL + t.h * G::HS + t.P * M::WP;
        const int m = t.m;
        if (m > 0) {
            cx<R> v[NV];
            if (t.h == 0) orbitT_compute<VA, LOGN, K, 0, R>(kf, c[it], m, v);
            else orbitT_compute<VA, LOGN, K, 1, R>(kf, c[it], m, v);
            const int pa = pad(m), pb = m + ((m + 15) >> 4);
#pragma unroll
            for (int i = 0; i < NV / 2; ++i) {
                stc(base + pa + 2 * M::GP * i, v[2 * i]);              // slot m + 2 G i
                stc(base + 2 * M::GP * (i + 1) - pb, v[2 * i + 1]);    // slot 2 G (i+1) - m
            }
        } else {
            cx<R> v[NV];
            if (t.h == 0) rowkT<VB, 0, M::r, R>(c[it], v, kt, G::D);
            else rowkT<VB, 1, M::r, R>(c[it], v, kt, G::D);
#pragma unroll
            for (int e = 1; e < NV; ++e) stc(base + e * M::GP, v[e - 1]);  // slot e G
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// F1^T: levels 2..0 backward on the orbit, transposed D_c / D_r, store
// ---------------------------------------------------------------------------
// levels 2..0 backward on the orbit of m0 of a 2^LOGN-point transform (kt:
// its constant table): d3of(side, P8) gives the depth-3 value of row P8 of a
// side at slot m0; cd[side][] comes out in the order of F1's c / d values
template <int VA, int LOGN, typename R, int KS = 0, typename LD>
__device__ __forceinline__ void f1T_levels(const R* kt, int m0, LD d3of, cx<R> (&cd)[2][8]) {
    constexpr bool SW = variant_traits<VA>::switches;
    constexpr int N8 = (1 << LOGN) / 8, N4 = (1 << LOGN) / 4;
    // KS: the table is that of a transform 2^KS times longer (read at stride 2^KS)
    const R k0[4] = {kt[m0 << KS], kt[(N8 - m0) << KS], kt[(N8 + m0) << KS], kt[(N4 - m0) << KS]};
    const R k1[2] = {kt[(2 * m0) << KS], kt[(N4 - 2 * m0) << KS]};
    const R k2 = kt[(4 * m0) << KS];
    sfor<0, 2>([&](auto sc) {
        constexpr int side = decltype(sc)::value;
        cx<R> d3[8];
        sfor<0, 8>([&](auto pc) { d3[decltype(pc)::value] = d3of(sc, pc); });
        cx<R> l2[4][2];
        sfor<0, 4>([&](auto pc) {
            constexpr int P = decltype(pc)::value;
            constexpr int sg = side ^ (SW ? par(P) : 0);
            bflyT<sg, R>(d3[2 * P], d3[2 * P + 1], k2, l2[P][0], l2[P][1]);
        });
        cx<R> l1[2][4];
        sfor<0, 2>([&](auto pc) {
            constexpr int P = decltype(pc)::value;
            constexpr int sg = side ^ (SW ? par(P) : 0);
#pragma unroll
            for (int r = 0; r < 2; ++r) bflyT<sg, R>(l2[2 * P][r], l2[2 * P + 1][r], k1[r], l1[P][r], l1[P][3 - r]);
        });
#pragma unroll
        for (int r = 0; r < 4; ++r) bflyT<side, R>(l1[0][r], l1[1][r], k0[r], cd[side][r], cd[side][7 - r]);
    });
}

// transposed D_c / D_r of an orbit: x(m) = c + d, x(N - m) = c - d at its slots
template <typename R>
__device__ __forceinline__ void f1T_combine(const cx<R> (&cd)[2][8], cx<R> (&res)[16]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        res[i] = cd[0][2 * i] + cd[1][2 * i];              // x(m0 + N8 i)
        res[8 + 7 - i] = cd[0][2 * i] - cd[1][2 * i];      // x(N8 (8 - i) - m0)
        res[8 + i] = cd[0][2 * i + 1] + cd[1][2 * i + 1];  // x(N8 (i + 1) - m0)
        res[7 - i] = cd[0][2 * i + 1] - cd[1][2 * i + 1];  // x(m0 + N8 (7 - i))
    }
}

// F1^T on the kernel's LDS image
template <int VA, int LOGN, typename R>
__device__ __forceinline__ void f1T_orbit(const cx<R>* w, const R* kt, int m0, cx<R> (&res)[16]) {
    using G = kgeo<LOGN>;
    constexpr bool SW = variant_traits<VA>::switches;
    const int pm = pad(m0);
    cx<R> cd[2][8];
    f1T_levels<VA, LOGN, R>(kt, m0, [&](auto sc, auto pc) {
        constexpr int hh = decltype(sc)::value ^ (SW ? par(decltype(pc)::value) : 0);
        return ldc(w + hh * G::HS + G::W3P * decltype(pc)::value + pm);
    }, cd);
    f1T_combine<R>(cd, res);
}

// thread 0: the chain from dct[16] / dst[16] (chain slots) with the blocks of
// 4, 2 and 1 points, then D_c / D_r transposed at the multiples of N/16
template <int VB, int LOGN, typename R>
__device__ __forceinline__ void f1T_chain(const cx<R> (&chs)[16], const R* kt, cx<R> (&res)[16]) {
    constexpr int D = LOGN - 2;
    cx<R> E8[9], P[16];
#pragma unroll
    for (int k = 0; k < 9; ++k) E8[k] = chs[k];
#pragma unroll
    for (int k = 9; k < 16; ++k) P[k] = chs[k];
    cx<R> c[9], d[8];
    {
        cx<R> E9[5], b8[4];
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            E9[k] = E8[k] + E8[8 - k];
            b8[k] = E8[k] - E8[8 - k];
        }
        E9[0] = E8[0] + E8[8];
        b8[0] = E8[0] - E8[8];
        E9[4] = E8[4];
        cx<R> b9[2];
        const cx<R> E10_0 = E9[0] + E9[4], E10_1 = E9[1] + E9[3], E10_2 = E9[2];
        b9[0] = E9[0] - E9[4];
        b9[1] = E9[1] - E9[3];
        const cx<R> e0 = E10_0 + E10_2, e1 = E10_1;
        c[4] = E10_0 - E10_2;  // O10
        c[0] = e0 + e1;
        c[8] = e0 - e1;        // c(N/2)
        leaf::to<VB, 4, 0, R>(b8, kt, D);
        leaf::to<VB, 2, 0, R>(b9, kt, D);
        c[1] = b8[0];
        c[3] = b8[1];
        c[5] = b8[2];
        c[7] = b8[3];
        c[2] = b9[0];
        c[6] = b9[1];
    }
    {
        cx<R> b8[4], E9[4];
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            b8[k - 1] = P[8 + k] + P[16 - k];
            E9[k] = P[8 + k] - P[16 - k];
        }
        b8[3] = P[12];
        cx<R> b9[2];
        b9[0] = E9[1] + E9[3];
        d[4] = E9[1] - E9[3];  // E10
        b9[1] = E9[2];
        leaf::to<VB, 4, 1, R>(b8, kt, D);
        leaf::to<VB, 2, 1, R>(b9, kt, D);
        d[1] = b8[0];
        d[3] = b8[1];
        d[5] = b8[2];
        d[7] = b8[3];
        d[2] = b9[0];
        d[6] = b9[1];
    }
    res[0] = c[0];
    res[8] = c[8];
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        res[k] = c[k] + d[k];
        res[16 - k] = c[k] - d[k];
    }
}

}  // namespace

}  // namespace amqft
