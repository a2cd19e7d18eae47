// Device building blocks of the compile-time skeleton-A kernel (the passes
// F1, M_k, P3, B_k, B0, C0 and their geometry, described in amqft_kA.hip),
// shared by amqft_kA.hip and by the transposed program in amqft_kB.hip.
// Included once per translation unit; everything lives in an unnamed
// namespace.
#pragma once
#include <type_traits>

#include "amqft_device.h"
#include "amqft_leaf.h"

namespace amqft {

namespace {


constexpr int par(int x) { return x ? ((x & 1) ^ par(x >> 1)) : 0; }
constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

__device__ __forceinline__ int pad(int p) { return p + (p >> 4); }

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

template <typename R>
__device__ __forceinline__ cx<R> zero() { return cx<R>{R(0), R(0)}; }

// One signal of S values seen through a buffer resource: a base address in
// scalar registers, element offsets split into a lane part and a scalar part,
// so that addressing costs no vector instructions (the base must be the same
// in every lane of the wave).
template <typename S>
struct sigbuf {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ sigbuf(const S* p, int n)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(p), (short)0, n * (int)sizeof(S), 0x00020000)) {}
    __device__ __forceinline__ S ld(int lane_elems, int scalar_elems) const {
        const int vo = lane_elems * (int)sizeof(S), so = scalar_elems * (int)sizeof(S);
        if constexpr (sizeof(S) == 16) return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
        else if constexpr (sizeof(S) == 8) return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
        else return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    __device__ __forceinline__ void st(int lane_elems, int scalar_elems, S v) const {
        const int vo = lane_elems * (int)sizeof(S), so = scalar_elems * (int)sizeof(S);
        if constexpr (sizeof(S) == 16) {
            // A VALU write to the data registers of a store of more than 8
            // bytes must wait one cycle; the compiler inserts that wait only
            // when the store has no scalar offset register (with one, the
            // next instruction may overwrite the data before it is read, and
            // the low word of the first value is stored wrong now and then).
            // So the scalar part joins the lane offset here.
            using U = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U, v), r, vo + so, 0, 0);
        } else if constexpr (sizeof(S) == 8) {
            using U = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, v), r, vo, so, 0);
        } else {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, 0);
        }
    }
};

// a value known to be the same in every lane, moved to scalar registers
__device__ __forceinline__ long long uniform64(long long v) {
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

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

// M^F of one child index in parent context SG (hm, h0, hp = F[i-1], F[i], F[i+1])
template <int V, int SG, typename R>
__device__ __forceinline__ cx<R> mf(cx<R> hm, cx<R> h0, cx<R> hp) {
    if constexpr (V == 4) return SG == 0 ? h0 + hp : hm + h0;
    else return SG == 0 ? h0 - hm : h0 - hp;
}

// one backward level on runs extended by one halo each side (L, Hh: n + 2
// children values; P: 2n + 2 parent values).  Halos out of reach come out as
// zero; M4 / M8 only consume a hi child's halo on the side its lo child fills.
template <int V, int SG, int n, typename R>
__device__ __forceinline__ void combine(const cx<R>* L, const cx<R>* Hh, cx<R>* P) {
#pragma unroll
    for (int rho = -1; rho <= 2 * n; ++rho) {
        const bool even = ((rho + 2) & 1) == 0;
        const int i = even ? rho / 2 : (rho - 1) / 2;
        if ((SG == 0) == even) {
            P[rho + 1] = L[i + 1];
        } else {
            const cx<R> hm = i >= 0 ? Hh[i] : zero<R>();
            const cx<R> hp = i + 1 <= n ? Hh[i + 2] : zero<R>();
            P[rho + 1] = mf<V, SG, R>(hm, Hh[i + 1], hp);
        }
    }
}

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

// r backward levels from 2^r rows below a parent of context SGB for one child
// index j: ext[q] = {F[j-1], F[j], F[j+1]}; out = parent values 2^r j ...
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

// whole sub-blocks of a row of 2^r slots in context SG: s[e-1] = slot e,
// e = 1 .. 2^r - 1 (blocks of 2^(r-1-b) points at slots (2i+1) 2^b);
// o = their spectra, block-contiguous, block of sz points at 2^r - 2 sz
template <int V, int SG, int r, typename R>
__device__ __forceinline__ void rowk(const cx<R>* s, cx<R>* o, const R* kt, int D) {
    sfor<0, r>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        constexpr int sz = 1 << (r - 1 - b);
        cx<R> blk[sz];
#pragma unroll
        for (int i = 0; i < sz; ++i) blk[i] = s[((2 * i + 1) << b) - 1];
        leaf::ot<V, sz, SG, R>(blk, kt, D);
#pragma unroll
        for (int i = 0; i < sz; ++i) o[(1 << r) - 2 * sz + i] = blk[i];
    });
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
template <int LOGN>
struct kgeo {
    static constexpr int N = 1 << LOGN, H = N / 2, D = LOGN - 2, Q = N / 4;
    static constexpr int T = N / 16;                 // threads per signal (= depth-3 row width W3)
    // threads per workgroup: one signal per workgroup from N = 4096 on; below,
    // several signals share a workgroup of 256 threads, or of one wave for
    // N <= 1024 (measured faster there for the fused loss and the FP64
    // latency case, and for N = 512)
    static constexpr int WG = T >= 256 ? T : LOGN <= 10 ? (T >= 64 ? T : 64) : 256;
    static constexpr int SPW = WG / T;               // signals per workgroup
    static constexpr int W3 = H / 8, W3P = W3 + W3 / 16;
    static constexpr int HS = H + H / 16;            // padded positions of one half
    static constexpr int GUARD = 32;
    static constexpr int SL = 2 * HS + GUARD;        // complex slots per signal
    static constexpr int NMID = D - 6;               // levels between F1 and P3
    static constexpr int NP = NMID > 0 ? (NMID + 3) / 4 : 0;
    static constexpr int rk(int k) { return NMID / NP + (k < NMID % NP ? 1 : 0); }
    static constexpr int lk(int k) { return k == 0 ? 3 : lk(k - 1) + rk(k - 1); }
    static constexpr int Wk(int k) { return H >> lk(k); }
    static constexpr int Gk(int k) { return Wk(k) >> rk(k); }
    // stride-1 constant tables of the middle passes: [t][rho][m - 1]
    static constexpr int kfsize(int k) { return (Gk(k) - 1) * ((1 << rk(k)) - 1); }
    static constexpr int kfbase(int k) { return k == 0 ? 0 : kfbase(k - 1) + kfsize(k - 1); }
    static constexpr int KF = NP > 0 ? kfbase(NP - 1) + kfsize(NP - 1) : 0;
    static constexpr int KF_ALLOC = (KF + 3) & ~3;
    static constexpr int kft(int k, int t) { return (Gk(k) - 1) * ((1 << rk(k)) - (1 << (rk(k) - t))); }
};

template <typename R, int LOGN>
constexpr size_t kA_lds_bytes() {
    using G = kgeo<LOGN>;
    return (size_t)(G::Q + G::KF_ALLOC) * sizeof(R) + (size_t)G::SPW * G::SL * sizeof(cx<R>);
}

// ---------------------------------------------------------------------------
// F1
// ---------------------------------------------------------------------------
// The 16 points of thread m0's orbit.  Workgroup slots past the end of the
// batch load signal 0 instead (valid memory; their results are never stored).
// WAVE_UNIFORM: x is the same in every lane of the wave (buffer addressing).
template <int LOGN, typename S, typename R, bool WAVE_UNIFORM = false>
__device__ __forceinline__ void f1_load(const S* x, int m0, cx<R> (&raw)[16]) {
    constexpr int N8 = (1 << LOGN) / 8, N16 = (1 << LOGN) / 16;
    if constexpr (WAVE_UNIFORM) {
        const sigbuf<S> b(x, 1 << LOGN);
        auto w = [](S v) { return storage<S>::ld(&v); };
        if (m0 > 0) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                raw[j] = w(b.ld(m0, N8 * j));
                raw[8 + j] = w(b.ld(N8 - m0, N8 * j));
            }
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) raw[k] = w(b.ld(0, N16 * k));
        }
        return;
    }
    if (m0 > 0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            raw[j] = storage<S>::ld(x + m0 + N8 * j);
            raw[8 + j] = storage<S>::ld(x + N8 * (j + 1) - m0);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) raw[k] = storage<S>::ld(x + N16 * k);
    }
}

// levels 0..2 on an orbit of 8 slots of two sides (cd[s][r], slots m_{2i} =
// m0 + (N/8) i, m_{2i+1} = (N/8)(i+1) - m0); put(s, P, v) receives the value
// of depth-3 row P of side s at slot m0.  kt: constant table of length N, or
// (KS > 0) of length 2^KS N, read at stride 2^KS.
template <int V, int LOGN, typename R, int KS = 0, typename PUT>
__device__ __forceinline__ void f1_levels(const R* kt, cx<R> (&cd)[2][8], int m0, PUT&& put) {
    constexpr bool SW = variant_traits<V>::switches;
    constexpr int N8 = (1 << LOGN) / 8, N4 = (1 << LOGN) / 4;
    const R k0[4] = {kt[m0 << KS], kt[(N8 - m0) << KS], kt[(N8 + m0) << KS], kt[(N4 - m0) << KS]};
    const R k1[2] = {kt[(2 * m0) << KS], kt[(N4 - 2 * m0) << KS]};
    const R k2 = kt[(4 * m0) << KS];
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
            cx<R> lo, hi;
            bfly<sg, R>(l2[P][0], l2[P][1], k2, lo, hi);
            put(std::integral_constant<int, side>{}, std::integral_constant<int, 2 * P>{}, lo);
            put(std::integral_constant<int, side>{}, std::integral_constant<int, 2 * P + 1>{}, hi);
        });
    });
}

// D_c / D_r on the orbit: c(m) = x(m) + x(N-m), d(m) = x(m) - x(N-m) at the
// orbit slots, from the 16 loaded points (raw[j] = x(m0 + (N/8) j),
// raw[8+j] = x((N/8)(j+1) - m0))
template <typename R>
__device__ __forceinline__ void f1_dc(const cx<R> (&raw)[16], bool conj_in, cx<R> (&cd)[2][8]) {
    cx<R> xa[8], xb[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        xa[j] = conj_in ? cconj(raw[j]) : raw[j];
        xb[j] = conj_in ? cconj(raw[8 + j]) : raw[8 + j];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        cd[0][2 * i] = xa[i] + xb[7 - i];
        cd[1][2 * i] = xa[i] - xb[7 - i];
        cd[0][2 * i + 1] = xb[i] + xa[7 - i];
        cd[1][2 * i + 1] = xb[i] - xa[7 - i];
    }
}

template <int V, int LOGN, typename R>
__device__ __forceinline__ void f1_orbit(cx<R>* w, const R* kt, const cx<R> (&raw)[16], int m0, bool conj_in) {
    using G = kgeo<LOGN>;
    constexpr bool SW = variant_traits<V>::switches;
    cx<R> cd[2][8];
    f1_dc<R>(raw, conj_in, cd);
    const int pm = pad(m0);
    f1_levels<V, LOGN, R>(kt, cd, m0, [&](auto sc, auto pc, cx<R> v) {
        constexpr int side = decltype(sc)::value, P8 = decltype(pc)::value;
        constexpr int hh = side ^ (SW ? par(P8) : 0);
        stc(w + hh * G::HS + G::W3P * P8 + pm, v);  // depth-3 row P8, slot m0
    });
}

// chain value c (E_{D-2}(0..8), then D_{D-2}(1..7)): first pad slot of depth-3 row c & 7
template <int LOGN>
__device__ __forceinline__ int chslot(int c) {
    using G = kgeo<LOGN>;
    return (c >> 3) * G::HS + (c & 7) * G::W3P + 16;
}

// multiples of N/16: blocks of 4, 2, 1 points and the chain to dct[16] / dst[16]
template <int V, int LOGN, typename R, typename PUT>
__device__ __forceinline__ void f1_chain_to(const R* kt, const cx<R> (&raw)[16], bool conj_in, PUT&& put) {
    constexpr int D = LOGN - 2;
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
        cx<R> b8[4] = {c[1], c[3], c[5], c[7]}, b9[2] = {c[2], c[6]};
        leaf::ot<V, 4, 0, R>(b8, kt, D);
        leaf::ot<V, 2, 0, R>(b9, kt, D);
        const cx<R> e0 = c[0] + cN2, e1 = c[0] - cN2;
        const cx<R> O10 = c[4];
        const cx<R> E10[3] = {e0 + O10, e1, e0 - O10};
        const cx<R> E9[5] = {E10[0] + b9[0], E10[1] + b9[1], E10[2], E10[1] - b9[1], E10[0] - b9[0]};
        cx<R> E8[9];
#pragma unroll
        for (int k = 0; k < 4; ++k) E8[k] = E9[k] + b8[k];
        E8[4] = E9[4];
#pragma unroll
        for (int k = 1; k < 4; ++k) E8[8 - k] = E9[k] - b8[k];
        E8[8] = E9[0] - b8[0];
#pragma unroll
        for (int k = 0; k < 9; ++k) put(k, E8[k]);
    }
    {
        cx<R> b8[4] = {d[1], d[3], d[5], d[7]}, b9[2] = {d[2], d[6]};
        leaf::ot<V, 4, 1, R>(b8, kt, D);
        leaf::ot<V, 2, 1, R>(b9, kt, D);
        const cx<R> E10 = d[4];
        const cx<R> E9[4] = {zero<R>(), b9[0] + E10, b9[1], b9[0] - E10};
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            put(8 + k, b8[k - 1] + E9[k]);
            put(16 - k, b8[k - 1] - E9[k]);
        }
        put(12, b8[3]);
    }
}

template <int V, int LOGN, typename R>
__device__ __forceinline__ void f1_chain(cx<R>* w, const R* kt, const cx<R> (&raw)[16], bool conj_in) {
    f1_chain_to<V, LOGN, R>(kt, raw, conj_in, [&](int c, cx<R> v) { stc(w + chslot<LOGN>(c), v); });
}

// ---------------------------------------------------------------------------
// middle orbit pass K
// ---------------------------------------------------------------------------
template <int LOGN, int K>
struct mpass {
    using G = kgeo<LOGN>;
    static constexpr int l0 = G::lk(K), r = G::rk(K), W = G::Wk(K), GL = G::Gk(K);
    static constexpr int WP = W + W / 16, GP = GL + GL / 16;
    static constexpr int NROW = 1 << l0;
    static constexpr int PERHALF = G::SPW * NROW * GL;
    static constexpr int IT = 16 >> r;
    static constexpr int NV = 1 << r;
};

struct task {
    int h, s, P, m;
};

template <int LOGN, int K>
__device__ __forceinline__ task mtask(int it, int tid) {
    using M = mpass<LOGN, K>;
    const int L = it * kgeo<LOGN>::WG + tid;
    task t;
    t.h = L / M::PERHALF;
    const int rem = L - t.h * M::PERHALF;
    t.s = rem / (M::NROW * M::GL);
    const int rem2 = rem - t.s * (M::NROW * M::GL);
    t.P = rem2 / M::GL;
    t.m = rem2 - t.P * M::GL;
    return t;
}

template <int V, int LOGN, int K, int H, typename R>
__device__ __forceinline__ void orbit_compute(cx<R>* ws, const R* kf, const cx<R> (&v)[mpass<LOGN, K>::NV], int P,
                                              int m0) {
    using G = kgeo<LOGN>;
    using M = mpass<LOGN, K>;
    constexpr bool SW = variant_traits<V>::switches;
    constexpr int NV = M::NV, r = M::r;
    const R* kw = kf + G::kfbase(K) + (m0 - 1);
    cx<R> cur[NV][NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) cur[0][e] = v[e];
    sfor<0, r>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        constexpr int KK = NV >> t;
        constexpr int rows = 1 << t;
        cx<R> nxt[NV][NV];
        sfor<0, rows>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int sg = H ^ (SW ? par(q) : 0);
#pragma unroll
            for (int rho = 0; rho < KK / 2; ++rho)
                bfly<sg, R>(cur[q][rho], cur[q][KK - 1 - rho], kw[G::kft(K, t) + (M::GL - 1) * rho], nxt[2 * q][rho],
                            nxt[2 * q + 1][rho]);
        });
#pragma unroll
        for (int q = 0; q < 2 * rows; ++q)
#pragma unroll
            for (int rho = 0; rho < KK / 2; ++rho) cur[q][rho] = nxt[q][rho];
    });
    const int pm = pad(m0);
    sfor<0, NV>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int hq = H ^ (SW ? par(q) : 0);
        stc(ws + hq * G::HS + (P * NV + q) * M::GP + pm, cur[q][0]);  // child row P 2^r + q, slot m0
    });
}

template <int V, int LOGN, int K, typename R>
__device__ __forceinline__ void orbit_pass(cx<R>* wall, const R* kt, const R* kf, int tid) {
    using G = kgeo<LOGN>;
    using M = mpass<LOGN, K>;
    constexpr int NV = M::NV, IT = M::IT;
    cx<R> v[IT][NV];
    task tk[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        tk[it] = mtask<LOGN, K>(it, tid);
        const cx<R>* base = wall + tk[it].s * G::SL + tk[it].h * G::HS + tk[it].P * M::WP;
        const int m = tk[it].m;
        if (m > 0) {
            const int pa = pad(m), pb = m + ((m + 15) >> 4);
#pragma unroll
            for (int i = 0; i < NV / 2; ++i) {
                v[it][2 * i] = ldc(base + pa + 2 * M::GP * i);              // slot m + 2 G i
                v[it][2 * i + 1] = ldc(base + 2 * M::GP * (i + 1) - pb);   // slot 2 G (i+1) - m
            }
        } else {
#pragma unroll
            for (int e = 1; e < NV; ++e) v[it][e - 1] = ldc(base + e * M::GP);  // slot e G
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const task t = tk[it];
        cx<R>* ws = wall + t.s * G::SL;
        if (t.m > 0) {
            if (t.h == 0) orbit_compute<V, LOGN, K, 0, R>(ws, kf, v[it], t.P, t.m);
            else orbit_compute<V, LOGN, K, 1, R>(ws, kf, v[it], t.P, t.m);
        } else {
            cx<R> o[NV];
            if (t.h == 0) rowk<V, 0, M::r, R>(v[it], o, kt, G::D);
            else rowk<V, 1, M::r, R>(v[it], o, kt, G::D);
            // first pad slot of child rows 1 .. 2^r - 1
            cx<R>* pb = ws + t.h * G::HS + t.P * M::WP + 16;
#pragma unroll
            for (int i = 0; i < NV - 1; ++i) stc(pb + 17 * (i + 1) * (M::GL / 16), o[i]);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// P3: rows of 16 at depth D-3
// ---------------------------------------------------------------------------
template <int V, int LOGN, typename R>
__device__ __forceinline__ void p3_pass(cx<R>* wall, const R* kt, int tid) {
    using G = kgeo<LOGN>;
    constexpr int NR = 1 << (G::D - 3);
    const int h = tid / (G::SPW * NR);
    const int rem = tid - h * (G::SPW * NR);
    const int s = rem / NR, R7 = rem - s * NR;
    cx<R>* row = wall + s * G::SL + h * G::HS + 17 * R7;
    cx<R> in[15], o[15];
#pragma unroll
    for (int e = 0; e < 15; ++e) in[e] = ldc(row + e + 1);
    if (h == 0) rowk<V, 0, 4, R>(in, o, kt, G::D);
    else rowk<V, 1, 4, R>(in, o, kt, G::D);
#pragma unroll
    for (int e = 0; e < 15; ++e) stc(row + e + 1, o[e]);
    __syncthreads();
}

// offsets (relative to the row's base) of index j-1, j, j+1 of a sub-block of
// sp values of block a inside a row of depth l1 = l0 + r of pass K
template <int LOGN, int K>
__device__ __forceinline__ void child_offsets(int a, int j, int sp, int (&off)[3]) {
    using G = kgeo<LOGN>;
    using M = mpass<LOGN, K>;
    if constexpr (K == G::NP - 1) {
        // P3 rows: block of sp points at 1 + 16 - 2 sp
        const int pos = 17 - 2 * sp + j;
        off[0] = pad(pos - 1);
        off[1] = pad(pos);
        off[2] = pad(pos + 1);
    } else {
        using M1 = mpass<LOGN, K + 1>;
        constexpr int r1 = M1::r, G1 = M1::GL;
        if (sp >= (1 << r1)) {
            const int pos = (1 << r1) + (M::GL - (M::GL >> a)) + j;  // main array of the child row
            off[0] = pad(pos - 1);
            off[1] = pad(pos);
            off[2] = pad(pos + 1);
        } else {
            const int e = (1 << r1) - 2 * sp + j;  // finished by pass K+1: pad slots
            off[0] = 17 * (e * (G1 / 16)) + 16;
            off[1] = 17 * ((e + 1) * (G1 / 16)) + 16;
            off[2] = 17 * ((e + 2) * (G1 / 16)) + 16;
        }
    }
}

// ---------------------------------------------------------------------------
// B_K: backward levels l0 + r - 1 .. l0 of pass K
// ---------------------------------------------------------------------------
template <int V, int LOGN, int K, typename R>
__device__ __forceinline__ void bpass(cx<R>* wall, int tid) {
    using G = kgeo<LOGN>;
    using M = mpass<LOGN, K>;
    constexpr bool SW = variant_traits<V>::switches;
    constexpr int NV = M::NV, IT = M::IT, LG = ilog2c(M::GL);
    cx<R> ext[IT][NV][3];
    task tk[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        tk[it] = mtask<LOGN, K>(it, tid);
        const task t = tk[it];
        if (t.m > 0) {
            const int wm = t.m - 1;
            const int a = __clz(~(wm << (32 - LG)));  // leading ones of wm in LG bits
            const int j = wm - (M::GL - (M::GL >> a));
            const int sp = M::GL >> (a + 1);         // sub-block size of block a at depth l0 + r
            int off[3];
            child_offsets<LOGN, K>(a, j, sp, off);
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                const int hq = t.h ^ (SW ? par(q) : 0);
                const cx<R>* row = wall + t.s * G::SL + hq * G::HS + (t.P * NV + q) * M::GP;
                const cx<R> lm = ldc(row + off[0]), lp = ldc(row + off[2]);
                ext[it][q][0] = j >= 1 ? lm : zero<R>();
                ext[it][q][1] = ldc(row + off[1]);
                ext[it][q][2] = j + 1 < sp ? lp : zero<R>();
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const task t = tk[it];
        if (t.m > 0) {
            cx<R> o[NV];
            if (t.h == 0) bwd_run<V, 0, M::r, R>(ext[it], o);
            else bwd_run<V, 1, M::r, R>(ext[it], o);
            cx<R>* dst = wall + t.s * G::SL + t.h * G::HS + t.P * M::WP + pad(NV * t.m);  // main array at 2^r m
#pragma unroll
            for (int e = 0; e < NV; ++e) stc(dst + e, o[e]);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// B0: levels 2..0, both sides; thread = position p in the depth-3 layout
// ---------------------------------------------------------------------------
template <int V, int LOGN, typename R>
__device__ __forceinline__ void b0_pass(cx<R>* wall, int tid) {
    using G = kgeo<LOGN>;
    constexpr bool SW = variant_traits<V>::switches;
    constexpr int LW3 = ilog2c(G::W3);
    const int s = tid / G::T, p = tid - s * G::T;
    int a = 0, j = 0, sp = 1;
    int off[3] = {0, 0, 0};
    if constexpr (G::NP == 0) {
        // depth 3 = P3 rows: [8 | 4 | 2 | 1] at slots 1..15
        const int e = p - 1;
        const int b = e < 8 ? 0 : e < 12 ? 1 : e < 14 ? 2 : 3;
        sp = 8 >> b;
        j = e - (16 - 2 * sp);
        a = b;
        off[0] = pad(p - 1);
        off[1] = pad(p);
        off[2] = pad(p + 1);
    } else {
        using M0 = mpass<LOGN, 0>;
        constexpr int r0 = M0::r, G0 = M0::GL;
        if (p < (1 << r0)) {
            const int e = p - 1;  // finished by pass 0: pad slots
            const int b = __clz(~(e << (32 - r0)));
            sp = (1 << (r0 - 1)) >> b;
            j = e - ((1 << r0) - 2 * sp);
            a = LW3 - r0 + b;  // block whose depth-3 sub-block has sp points
            off[0] = 17 * (e * (G0 / 16)) + 16;
            off[1] = 17 * ((e + 1) * (G0 / 16)) + 16;
            off[2] = 17 * ((e + 2) * (G0 / 16)) + 16;
        } else {
            const int pp = p - (1 << r0);
            a = __clz(~(pp << (32 - LW3)));
            j = pp - (G::W3 - (G::W3 >> a));
            sp = G::W3 >> (a + 1);
            off[0] = pad(p - 1);
            off[1] = pad(p);
            off[2] = pad(p + 1);
        }
    }
    const bool act = p > 0;
    cx<R> ext[2][8][3];
    if (act) {
#pragma unroll
        for (int side = 0; side < 2; ++side)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int hq = side ^ (SW ? par(q) : 0);
                const cx<R>* row = wall + s * G::SL + hq * G::HS + q * G::W3P;
                const cx<R> lm = ldc(row + off[0]), lp = ldc(row + off[2]);
                ext[side][q][0] = j >= 1 ? lm : zero<R>();
                ext[side][q][1] = ldc(row + off[1]);
                ext[side][q][2] = j + 1 < sp ? lp : zero<R>();
            }
    }
    __syncthreads();
    if (act) {
        const int ob = pad(G::H - (G::H >> a) + 8 * j);  // block a at H - H / 2^a at depth 0
        cx<R>* ws = wall + s * G::SL;
        cx<R> o[8];
        bwd_run<V, 0, 3, R>(ext[0], o);
#pragma unroll
        for (int e = 0; e < 8; ++e) stc(ws + ob + e, o[e]);
        bwd_run<V, 1, 3, R>(ext[1], o);
#pragma unroll
        for (int e = 0; e < 8; ++e) stc(ws + G::HS + ob + e, o[e]);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// M1 / M5: the backward M^F is a recurrence along each hi child, first term
// halved (Tables 5-6): M1 G(i) = H(i) - G(i -+ 1), M5 G(i) = H(i) + G(i -+ 1),
// ascending for (M1, DCT parent) and (M5, DST parent), descending otherwise.
// With G(i) = (-1)^i U(i) for M1 it is an inclusive prefix (suffix) sum U of
// u(k) = (-1)^k h'(k), h' the child with its first element halved.  Each lane
// holds n consecutive entries of the child; the sum runs in the lane, then
// across the lanes of the child as a segmented scan on lane shuffles.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ cx<R> shfl_up_c(cx<R> v, int d) {
    return cx<R>{__shfl_up(v.re, d), __shfl_up(v.im, d)};
}
template <typename R>
__device__ __forceinline__ cx<R> shfl_dn_c(cx<R> v, int d) {
    return cx<R>{__shfl_down(v.re, d), __shfl_down(v.im, d)};
}
__device__ __forceinline__ cx<fx32> shfl_up_c(cx<fx32> v, int d) {
    return cx<fx32>{fx32::raw(__shfl_up(v.re.v, d)), fx32::raw(__shfl_up(v.im.v, d))};
}
__device__ __forceinline__ cx<fx32> shfl_dn_c(cx<fx32> v, int d) {
    return cx<fx32>{fx32::raw(__shfl_down(v.re.v, d)), fx32::raw(__shfl_down(v.im.v, d))};
}

// lane i receives lane i - D (UP) or lane i + D inside its row of 16 lanes
// (data-parallel-primitive moves: a VALU operation, no LDS traffic)
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ fx32 dpp_mov(fx32 v) {
    return fx32::raw(__builtin_amdgcn_update_dpp(0, v.v, CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <bool UP, int D, typename R>
__device__ __forceinline__ cx<R> row_shift(cx<R> v) {
    constexpr int CTRL = UP ? 0x110 + D : 0x100 + D;  // row_shr:D / row_shl:D
    return cx<R>{dpp_mov<CTRL>(v.re), dpp_mov<CTRL>(v.im)};
}

// the value of lane l (the same l in every lane), in every lane
__device__ __forceinline__ float lane_value(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ fx32 lane_value(fx32 v, int l) { return fx32::raw(__builtin_amdgcn_readlane(v.v, l)); }
template <typename R>
__device__ __forceinline__ cx<R> lane_value_c(cx<R> v, int l) {
    return cx<R>{lane_value(v.re, l), lane_value(v.im, l)};
}

// a of i <= 0, b of 1, c of 2, d of 3 (per lane, from values: no array
// indexed at run time)
template <typename R>
__device__ __forceinline__ cx<R> pick4(cx<R> a, cx<R> b, cx<R> c, cx<R> d, int i) {
    const R re = i <= 0 ? a.re : i == 1 ? b.re : i == 2 ? c.re : d.re;
    const R im = i <= 0 ? a.im : i == 1 ? b.im : i == 2 ? c.im : d.im;
    return cx<R>{re, im};
}

// Carry of a segment longer than a row of 16 lanes (aligned to rows): the
// sum of the totals of the k rows before (ASC) / after this lane's row in its
// segment, ((T3 + T2) + T1) nearest row last; a row's total is `inc` at its
// last (ASC) / first lane.  Every lane of the wave must call it.
template <bool ASC, typename R>
__device__ __forceinline__ cx<R> rows_carry(cx<R> inc, int k) {
    const cx<R> T0 = lane_value_c(inc, ASC ? 15 : 0), T1 = lane_value_c(inc, ASC ? 31 : 16);
    const cx<R> T2 = lane_value_c(inc, ASC ? 47 : 32), T3 = lane_value_c(inc, ASC ? 63 : 48);
    const int r = (threadIdx.x >> 4) & 3;
    constexpr int d = ASC ? -1 : 1;
    const cx<R> p1 = pick4(T0, T1, T2, T3, r + d), p2 = pick4(T0, T1, T2, T3, r + 2 * d);
    const cx<R> p3 = pick4(T0, T1, T2, T3, r + 3 * d);
    cx<R> c = k >= 3 ? p3 + p2 : p2;
    c = k >= 2 ? c + p1 : p1;
    return k >= 1 ? c : zero<R>();
}

// lane i receives lane i - d (UP) or i + d; ROW: every use stays inside
// aligned rows of 16 lanes (then d <= 15 moves with DPP)
template <bool UP, bool ROW, int d, typename R>
__device__ __forceinline__ cx<R> lane_shift(cx<R> v) {
    if constexpr (ROW) return row_shift<UP, d, R>(v);
    else if constexpr (UP) return shfl_up_c(v, d);
    else return shfl_dn_c(v, d);
}

template <int V, int SG>
struct rec_dir {
    static constexpr bool asc = (V == 1) ? (SG == 0) : (SG != 0);
    static constexpr bool alt = variant_traits<V>::sign < 0;
};

// exclusive sum of t over the lanes before (ASC) or after this one in its
// segment of nl lanes (pos = index in the segment, segments of at most MAXL
// consecutive lanes inside one wave -- inside one row of 16 lanes when
// MAXL <= 16); every lane of the wave must call it
template <bool ASC, int MAXL, typename R>
__device__ __forceinline__ cx<R> seg_excl(cx<R> t, int pos, int nl) {
    constexpr bool ROW = MAXL <= 16;
    const cx<R> z = zero<R>();
    if constexpr (!ROW) {
        // segments longer than a row are aligned to rows: an inclusive scan
        // inside each row (DPP), shifted by one lane, plus the totals of the
        // segment's earlier (later) rows read from their lanes -- no LDS
        const int ip = pos & 15, lim = nl < 16 ? nl : 16;
        cx<R> inc = t;
        sfor<0, 4>([&](auto kc) {
            constexpr int d = 1 << decltype(kc)::value;
            const cx<R> u = row_shift<ASC, d, R>(inc);
            if (ASC ? ip >= d : ip + d < lim) inc = inc + u;
        });
        const cx<R> s1 = row_shift<ASC, 1, R>(inc);
        const cx<R> ex = (ASC ? ip >= 1 : ip + 1 < lim) ? s1 : z;
        return rows_carry<ASC, R>(inc, ASC ? pos >> 4 : (nl - 1 - pos) >> 4) + ex;
    }
    const cx<R> s1 = lane_shift<ASC, ROW, 1, R>(t);
    cx<R> w = (ASC ? pos >= 1 : pos + 1 < nl) ? s1 : z;
    sfor<0, ilog2c(MAXL)>([&](auto kc) {
        constexpr int d = 1 << decltype(kc)::value;
        const cx<R> u = lane_shift<ASC, ROW, d, R>(w);
        if (ASC ? pos >= d : pos + d < nl) w = w + u;
    });
    return w;
}

// One entry per lane (n = 1): the sums are formed over the index pairs
// {2m, 2m+1} first and then across pairs.  (Grouping the alternating terms
// the other way, {2m-1, 2m}, loses up to two decimal digits on these
// spectra.)  carry = exclusive sum over the pairs before (after) this lane's
// pair; own = the partial sum inside the pair up to this lane.
template <bool ASC, int MAXL, typename R>
__device__ __forceinline__ void pair_excl(cx<R> u, int pos, int nl, cx<R>& carry, cx<R>& own) {
    constexpr bool ROW = MAXL <= 16;
    const cx<R> z = zero<R>();
    // a pair never crosses a row: its partner moves with DPP in every case
    const cx<R> up = row_shift<true, 1, R>(u), dn = row_shift<false, 1, R>(u);
    const bool odd = pos & 1, paired = nl > 1;
    const cx<R> ps = !paired ? u : odd ? up + u : u + dn;  // u(2m) + u(2m+1)
    own = paired && (ASC ? odd : !odd) ? ps : u;
    const int pm = pos >> 1, np = paired ? nl >> 1 : 1;
    if constexpr (!ROW) {
        // as seg_excl over the pairs (8 to a row); both lanes of a pair hold its sums
        const int ipm = pm & 7, plim = np < 8 ? np : 8;
        cx<R> inc = ps;
        sfor<0, 3>([&](auto kc) {
            constexpr int d = 1 << decltype(kc)::value;
            const cx<R> a = row_shift<ASC, 2 * d, R>(inc);
            if (ASC ? ipm >= d : ipm + d < plim) inc = inc + a;
        });
        const cx<R> s2 = row_shift<ASC, 2, R>(inc);
        const cx<R> ex = (ASC ? ipm >= 1 : ipm + 1 < plim) ? s2 : z;
        carry = rows_carry<ASC, R>(inc, ASC ? pm >> 3 : (np - 1 - pm) >> 3) + ex;
        return;
    }
    const cx<R> a2 = lane_shift<ASC, ROW, 2, R>(ps);
    cx<R> w = (ASC ? pm >= 1 : pm + 1 < np) ? a2 : z;
    sfor<0, (ilog2c(MAXL) > 1 ? ilog2c(MAXL) - 1 : 0)>([&](auto kc) {
        constexpr int d = 1 << decltype(kc)::value;
        const cx<R> a = lane_shift<ASC, ROW, 2 * d, R>(w);
        if (ASC ? pm >= d : pm + d < np) w = w + a;
    });
    carry = w;
}

// first half of one recurrence level: local sums loc[] of the lane's n hi
// entries in scan order and their total
template <int V, int SG, int n, typename R>
__device__ __forceinline__ cx<R> rec_local(const cx<R>* Hh, int pos, int nl, cx<R> (&loc)[n]) {
    using RD = rec_dir<V, SG>;
    const int len = nl * n;
    cx<R> u[n];
#pragma unroll
    for (int e = 0; e < n; ++e) {
        const int i = pos * n + e;
        cx<R> v = Hh[e];
        if (len > 1 && (RD::asc ? i == 0 : i == len - 1)) v = v * R(0.5);
        if (RD::alt && (i & 1)) v = cx<R>{-v.re, -v.im};
        u[e] = v;
    }
    if constexpr (RD::asc) {
        loc[0] = u[0];
#pragma unroll
        for (int e = 1; e < n; ++e) loc[e] = loc[e - 1] + u[e];
        return loc[n - 1];
    } else {
        loc[n - 1] = u[n - 1];
#pragma unroll
        for (int e = n - 2; e >= 0; --e) loc[e] = loc[e + 1] + u[e];
        return loc[0];
    }
}

// second half: add the carry, undo the sign pattern, interleave with the lo
// child into the parent run P[0 .. 2n)
template <int V, int SG, int n, typename R>
__device__ __forceinline__ void rec_finish(const cx<R>* L, const cx<R>* Hh, const cx<R> (&loc)[n], cx<R> carry,
                                           cx<R> own, int pos, int nl, cx<R>* P) {
    using RD = rec_dir<V, SG>;
    const int len = nl * n;
#pragma unroll
    for (int e = 0; e < n; ++e) {
        const int i = pos * n + e;
        cx<R> g = (n == 1 ? own : loc[e]) + carry;
        if (RD::alt && (i & 1)) g = cx<R>{-g.re, -g.im};
        if (len == 1) g = Hh[e];  // L = 8 base: no M step
        if constexpr (SG == 0) {
            P[2 * e] = L[e];
            P[2 * e + 1] = g;
        } else {
            P[2 * e] = g;
            P[2 * e + 1] = L[e];
        }
    }
}

// r backward levels below a parent of context SGB for one lane (its segment
// position pos of nl lanes): cur[q][0] = child q's entry, cur[0][0 .. 2^r) out
template <int V, int SGB, int r, int t, int MAXL, typename R>
__device__ __forceinline__ void rec_levels(cx<R> (&cur)[1 << r][1 << r], int pos, int nl) {
    if constexpr (t < r) {
        constexpr bool SW = variant_traits<V>::switches;
        constexpr int nrow = 1 << (r - t - 1), n = 1 << t;
        sfor<0, nrow>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int sg = SGB ^ (SW ? par(q) : 0);
            constexpr bool ASC = rec_dir<V, sg>::asc;
            cx<R> loc[n];
            const cx<R> tot = rec_local<V, sg, n, R>(cur[2 * q + 1], pos, nl, loc);
            cx<R> carry, own = tot;
            if constexpr (n == 1) pair_excl<ASC, MAXL, R>(loc[0], pos, nl, carry, own);
            else carry = seg_excl<ASC, MAXL, R>(tot, pos, nl);
            cx<R> tmp[2 * n];
            rec_finish<V, sg, n, R>(cur[2 * q], cur[2 * q + 1], loc, carry, own, pos, nl, tmp);
#pragma unroll
            for (int e = 0; e < 2 * n; ++e) cur[q][e] = tmp[e];
        });
        rec_levels<V, SGB, r, t + 1, MAXL, R>(cur, pos, nl);
    }
}

// B_K for M1 / M5: lane wm = 0 .. GL - 2 of a row holds child index j of the
// block of its position (so that every child's lanes form an aligned group
// inside one wave); the last lane of each row idles
template <int V, int LOGN, int K, typename R>
__device__ __forceinline__ void bpass_rec(cx<R>* wall, int tid) {
    using G = kgeo<LOGN>;
    using M = mpass<LOGN, K>;
    constexpr bool SW = variant_traits<V>::switches;
    constexpr int NV = M::NV, IT = M::IT, LG = ilog2c(M::GL), MAXL = M::GL / 2;
    cx<R> cur[IT][NV][NV];
    task tk[IT];
    int jj[IT], spp[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        tk[it] = mtask<LOGN, K>(it, tid);
        const task t = tk[it];
        const int wm = t.m;
        const int a = __clz(~(wm << (32 - LG)));  // leading ones of wm in LG bits (LG: idle lane)
        const bool act = wm < M::GL - 1;
        const int j = act ? wm - (M::GL - (M::GL >> a)) : 0;
        const int sp = act ? M::GL >> (a + 1) : 0;
        jj[it] = j;
        spp[it] = sp;
        int off[3] = {0, 0, 0};
        if (act) child_offsets<LOGN, K>(a, j, sp, off);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const int hq = t.h ^ (SW ? par(q) : 0);
            const cx<R>* row = wall + t.s * G::SL + hq * G::HS + (t.P * NV + q) * M::GP;
            cur[it][q][0] = act ? ldc(row + off[1]) : zero<R>();
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const task t = tk[it];
        // t.h is the same in every lane of a wave (a half holds a multiple of 64 tasks)
        if (t.h == 0) rec_levels<V, 0, M::r, 0, MAXL, R>(cur[it], jj[it], spp[it]);
        else rec_levels<V, 1, M::r, 0, MAXL, R>(cur[it], jj[it], spp[it]);
        if (t.m < M::GL - 1) {
            cx<R>* dst = wall + t.s * G::SL + t.h * G::HS + t.P * M::WP + pad(NV * (t.m + 1));  // main array at 2^r m
#pragma unroll
            for (int e = 0; e < NV; ++e) stc(dst + e, cur[it][0][e]);
        }
    }
    __syncthreads();
}

// LDS scratch of the M1 / M5 backward passes: per signal, per wave, two sides
// times four rows of partial sums (segments longer than one wave)
template <int LOGN>
constexpr int kA_rec_scratch() {
    using G = kgeo<LOGN>;
    return G::W3 / 2 > 64 ? G::SPW * (G::T / 64) * 8 : 0;
}

// LDS of amqft_kA_kernel for variant V (M1 / M5 add the scratch above)
template <int V, typename R, int LOGN>
constexpr size_t kA_lds_bytes_v() {
    return kA_lds_bytes<R, LOGN>() + (variant_traits<V>::recurrence ? (size_t)kA_rec_scratch<LOGN>() * sizeof(cx<R>) : 0);
}

// B0 for M1 / M5: levels 2..0 of both sides.  Lanes are remapped so that the
// main-array blocks of the depth-3 rows start at lane 0 (aligned segments,
// those longer than a wave aligned to waves) and the small blocks of the
// first middle pass (or of P3) sit in the last lanes.
template <int V, int LOGN, typename R>
__device__ __forceinline__ void b0_pass_rec(cx<R>* wall, cx<R>* scr, int tid) {
    using G = kgeo<LOGN>;
    constexpr bool SW = variant_traits<V>::switches;
    constexpr int LW3 = ilog2c(G::W3);
    constexpr bool MULTI = G::W3 / 2 > 64;  // segments spanning several waves
    constexpr int MAXL = G::W3 / 2 < 64 ? G::W3 / 2 : 64;
    const int s = tid / G::T, L = tid - s * G::T;
    int a = 0, j = 0, sp = 0, p = 0;
    int off[3] = {0, 0, 0};
    if constexpr (G::NP == 0) {
        p = L;  // depth 3 = P3 rows: [8 | 4 | 2 | 1] at slots 1..15
        if (p > 0) {
            const int e = p - 1;
            const int b = e < 8 ? 0 : e < 12 ? 1 : e < 14 ? 2 : 3;
            sp = 8 >> b;
            j = e - (16 - 2 * sp);
            a = b;
            off[1] = pad(p);
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
            off[1] = pad(p);
        } else {
            p = L - (G::W3 - NS);
            if (p > 0) {
                const int e = p - 1;  // finished by pass 0: pad slots
                const int b = __clz(~(e << (32 - r0)));
                sp = (1 << (r0 - 1)) >> b;
                j = e - ((1 << r0) - 2 * sp);
                a = LW3 - r0 + b;
                off[1] = 17 * ((e + 1) * (G0 / 16)) + 16;
            }
        }
    }
    const bool act = p > 0;
    cx<R> cur[2][8][8];
#pragma unroll
    for (int side = 0; side < 2; ++side)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int hq = side ^ (SW ? par(q) : 0);
            const cx<R>* row = wall + s * G::SL + hq * G::HS + q * G::W3P;
            cur[side][q][0] = act ? ldc(row + off[1]) : zero<R>();
        }
    __syncthreads();
    const int wl = L & 63;                       // lane in the wave
    const int wv = L >> 6;                       // wave of the signal
    const int seg0 = L - j;                      // first lane of the segment
    const bool multi = MULTI && sp > 64;
    const int pw = multi ? wl : j, nw = multi ? 64 : sp;  // position / length inside this wave
    cx<R>* sc = scr + s * ((G::T / 64) * 8);
    sfor<0, 3>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        constexpr int n = 1 << t, NR = 1 << (2 - t);
        cx<R> loc[2][NR][n], own[2][NR], car[2][NR];
        sfor<0, 2>([&](auto sc2) {
            constexpr int side = decltype(sc2)::value;
            sfor<0, NR>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int sg = side ^ (SW ? par(q) : 0);
                constexpr bool ASC = rec_dir<V, sg>::asc;
                own[side][q] = rec_local<V, sg, n, R>(cur[side][2 * q + 1], j, sp, loc[side][q]);
                if constexpr (n == 1) pair_excl<ASC, MAXL, R>(loc[side][q][0], pw, nw, car[side][q], own[side][q]);
                else car[side][q] = seg_excl<ASC, MAXL, R>(own[side][q], pw, nw);
            });
        });
        if constexpr (MULTI) {
            // wave totals of the long segments, then the carry of the waves before (after)
            sfor<0, 2>([&](auto sc2) {
                constexpr int side = decltype(sc2)::value;
                sfor<0, NR>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    constexpr int sg = side ^ (SW ? par(q) : 0);
                    constexpr bool ASC = rec_dir<V, sg>::asc;
                    if (multi && wl == (ASC ? 63 : 0)) stc(sc + wv * 8 + side * 4 + q, own[side][q] + car[side][q]);
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
                        constexpr bool ASC = rec_dir<V, sg>::asc;
                        cx<R> c = zero<R>();
                        if (ASC) {
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
        sfor<0, 2>([&](auto sc2) {
            constexpr int side = decltype(sc2)::value;
            sfor<0, NR>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int sg = side ^ (SW ? par(q) : 0);
                cx<R> tmp[2 * n];
                rec_finish<V, sg, n, R>(cur[side][2 * q], cur[side][2 * q + 1], loc[side][q], car[side][q],
                                        own[side][q], j, sp, tmp);
#pragma unroll
                for (int e = 0; e < 2 * n; ++e) cur[side][q][e] = tmp[e];
            });
        });
    });
    if (act) {
        const int ob = pad(G::H - (G::H >> a) + 8 * j);  // block a at H - H / 2^a at depth 0
        cx<R>* ws = wall + s * G::SL;
#pragma unroll
        for (int e = 0; e < 8; ++e) stc(ws + ob + e, cur[0][0][e]);
#pragma unroll
        for (int e = 0; e < 8; ++e) stc(ws + G::HS + ob + e, cur[1][0][e]);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// C0: chain and D_c.  res[] comes out in the order of the thread's F1 orbit:
// res[j] = X(k0 + (N/8) j), res[8 + j] = X((N/8)(j+1) - k0), j = 0..7, or for
// k0 = 0, res[i] = X((N/16) i): the same 16 indices the thread loads in F1.
// ---------------------------------------------------------------------------
// LDS layout of a signal in the kA kernels: padded halves, chain in pad slots
template <int LOGN>
struct lds_layout {
    using G = kgeo<LOGN>;
    static constexpr int idx(int k) { return k + (k >> 4); }
    static constexpr int base(int side, int a) { return side * G::HS + idx(G::H - (G::H >> a)); }
    static constexpr int chain(int c) { return (c >> 3) * G::HS + (c & 7) * G::W3P + 16; }
};

// C0 of the chain thread k0 = 0 (harmonics N/16 i): Oc(a, k) / Os(a, k) read
// harmonic k of block a on the DCT / DST side (the DST side stores harmonic k
// at k - 1); e8_0 is chain value 0
template <int LOGN, typename R, typename OC, typename OS>
__device__ __forceinline__ void c0_zero(OC&& Oc, OS&& Os, cx<R> e8_0, cx<R> (&res)[16]) {
    using G = kgeo<LOGN>;
    constexpr int D = G::D, N16 = G::N / 16;
    auto lo = [](cx<R> Cv, cx<R> Dv) { return cx<R>{Cv.re + Dv.im, Cv.im - Dv.re}; };
    auto hi = [](cx<R> Cv, cx<R> Dv) { return cx<R>{Cv.re - Dv.im, Cv.im + Dv.re}; };
    // harmonics N16 i: E_3(0) and E_3(N16) (the top harmonic of periodization 32 q_3)
    cx<R> sum47 = zero<R>();
#pragma unroll
    for (int a = 4; a <= D - 3; ++a) sum47 = sum47 + Oc(a, 0);
    const cx<R> o3 = Oc(3, 0);
    const cx<R> E3_0 = e8_0 + sum47 + o3;
    const cx<R> E3_h = e8_0 + sum47 - o3;
    const cx<R> o2 = Oc(2, 0);
    const cx<R> E2_0 = E3_0 + o2, E2_2 = E3_0 - o2, E2_1 = E3_h;
    const cx<R> o1_0 = Oc(1, 0), o1_1 = Oc(1, N16);
    const cx<R> E1_0 = E2_0 + o1_0, E1_4 = E2_0 - o1_0;
    const cx<R> E1_1 = E2_1 + o1_1, E1_3 = E2_1 - o1_1, E1_2 = E2_2;
    cx<R> C[9];
    const cx<R> E1v[4] = {E1_0, E1_1, E1_2, E1_3};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const cx<R> o0 = Oc(0, N16 * i);
        C[i] = E1v[i] + o0;
        C[8 - i] = E1v[i] - o0;
    }
    C[4] = E1_4;
    const cx<R> D2_1 = Os(2, N16);
    const cx<R> p1 = Os(1, N16);
    const cx<R> D1v[4] = {zero<R>(), p1 + D2_1, Os(1, 2 * N16), p1 - D2_1};
    cx<R> Dd[9];
    Dd[0] = zero<R>();
    Dd[8] = zero<R>();
#pragma unroll
    for (int i = 1; i < 4; ++i) {
        const cx<R> o0 = Os(0, N16 * i);
        Dd[i] = o0 + D1v[i];
        Dd[8 - i] = o0 - D1v[i];
    }
    Dd[4] = Os(0, 4 * N16);
    res[0] = C[0];
#pragma unroll
    for (int i = 1; i < 8; ++i) res[i] = lo(C[i], Dd[i]);
    res[8] = C[8];
#pragma unroll
    for (int i = 9; i < 16; ++i) res[i] = hi(C[16 - i], Dd[16 - i]);
}

template <int LOGN, typename R, typename L>
__device__ __forceinline__ void c0_compute(const cx<R>* w, const cx<R>* chn, int k0, cx<R> (&res)[16]) {
    using G = kgeo<LOGN>;
    constexpr int N = G::N, H = G::H, Q = G::Q, D = G::D, N8 = N / 8, N4 = N / 4, N16 = N / 16;
    constexpr int NW = D - 5;  // walk levels a = 3 .. D-3
    // position of harmonic k of block a on a side = L::base(side, a) + L::idx(k)
    auto bo = [](int a) { return L::base(0, a); };
    constexpr int HSL = L::base(1, 0);
    // X(k) = C(k) - i D(k), X(N-k) = C(k) + i D(k)
    auto lo = [](cx<R> Cv, cx<R> Dv) { return cx<R>{Cv.re + Dv.im, Cv.im - Dv.re}; };
    auto hi = [](cx<R> Cv, cx<R> Dv) { return cx<R>{Cv.re - Dv.im, Cv.im + Dv.re}; };
    if (k0 > 0) {
        int ic[NW > 0 ? NW : 1], is[NW > 0 ? NW : 1];
        R wc[NW > 0 ? NW : 1], wsg[NW > 0 ? NW : 1];
        int kc = k0;
#pragma unroll
        for (int t = 0; t < NW; ++t) {
            const int q = Q >> (3 + t);
            const bool lt = kc < q, gt = kc > q;
            kc = gt ? 2 * q - kc : kc;
            // harmonic q of a level has no block term (weight 0); its read
            // goes to index 0 of the block, so that it never touches the
            // slot past the block's end (unwritten in a global workspace)
            ic[t] = lt || gt ? kc : 0;
            wc[t] = lt ? R(1) : gt ? R(-1) : R(0);
        }
        int ks = k0;
        R sgn = R(1);
        bool done = false;
#pragma unroll
        for (int t = 0; t < NW; ++t) {
            const int q = Q >> (3 + t);
            const bool gt = ks > q, eq = ks == q;
            const int kn = gt ? 2 * q - ks : ks;
            is[t] = done ? 1 : kn;
            wsg[t] = done ? R(0) : sgn;
            sgn = (!done && gt) ? -sgn : sgn;
            done = done || eq;
            ks = kn;
        }
        const int e8 = done ? 0 : ks;
        const R wd = done ? R(0) : sgn;
        cx<R> accs = ldc(chn + L::chain(8 + e8)) * wd;
#pragma unroll
        for (int t = 0; t < NW; ++t) {
            const cx<R> o = ldc(w + HSL + bo(3 + t) + L::idx(is[t] - 1));
            accs = cx<R>{accs.re + wsg[t] * o.re, accs.im + wsg[t] * o.im};
        }
        cx<R> accc = ldc(chn + L::chain(kc));
#pragma unroll
        for (int t = 0; t < NW; ++t) {
            const cx<R> o = ldc(w + bo(3 + t) + L::idx(ic[t]));
            accc = cx<R>{accc.re + wc[t] * o.re, accc.im + wc[t] * o.im};
        }
        const int kA = k0, kB = N8 - k0;
        constexpr int N8P = L::idx(N8);
        const int pA = L::idx(kA), pB = L::idx(kB), pC = pA + N8P, pD = pB + N8P;
        const int qA = L::idx(kA - 1), qB = L::idx(kB - 1), qC = qA + N8P, qD = qB + N8P;
        const cx<R> Ec3 = accc, Es3 = accs;
        const cx<R> oc2 = ldc(w + bo(2) + pA);
        const cx<R> c2a = Ec3 + oc2, c2b = Ec3 - oc2;
        const cx<R> o1a = ldc(w + bo(1) + pA), o1b = ldc(w + bo(1) + pB);
        const cx<R> c1[4] = {c2a + o1a, c2b + o1b, c2b - o1b, c2a - o1a};
        const int pk[4] = {pA, pB, pC, pD}, qk[4] = {qA, qB, qC, qD};
        cx<R> C[8];  // E_0 at kA, kB, kC, kD, H-kD, H-kC, H-kB, H-kA
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const cx<R> o0 = ldc(w + pk[i]);
            C[i] = c1[i] + o0;
            C[7 - i] = c1[i] - o0;
        }
        const cx<R> os2 = ldc(w + HSL + bo(2) + qA);
        const cx<R> s2a = os2 + Es3, s2b = os2 - Es3;
        const cx<R> p1a = ldc(w + HSL + bo(1) + qA), p1b = ldc(w + HSL + bo(1) + qB);
        const cx<R> s1[4] = {p1a + s2a, p1b + s2b, p1b - s2b, p1a - s2a};
        cx<R> Dd[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const cx<R> o0 = ldc(w + HSL + qk[i]);
            Dd[i] = o0 + s1[i];
            Dd[7 - i] = o0 - s1[i];
        }
        // harmonics kA, kB, kC, kD, H-kD, H-kC, H-kB, H-kA and N minus them, in
        // orbit order (both branches write res[0..15] in increasing order)
        res[0] = lo(C[0], Dd[0]);
        res[1] = lo(C[2], Dd[2]);
        res[2] = lo(C[4], Dd[4]);
        res[3] = lo(C[6], Dd[6]);
        res[4] = hi(C[7], Dd[7]);
        res[5] = hi(C[5], Dd[5]);
        res[6] = hi(C[3], Dd[3]);
        res[7] = hi(C[1], Dd[1]);
        res[8] = lo(C[1], Dd[1]);
        res[9] = lo(C[3], Dd[3]);
        res[10] = lo(C[5], Dd[5]);
        res[11] = lo(C[7], Dd[7]);
        res[12] = hi(C[6], Dd[6]);
        res[13] = hi(C[4], Dd[4]);
        res[14] = hi(C[2], Dd[2]);
        res[15] = hi(C[0], Dd[0]);
    } else {
        auto Oc = [&](int a, int k) { return ldc(w + bo(a) + L::idx(k)); };
        auto Os = [&](int a, int k) { return ldc(w + HSL + bo(a) + L::idx(k - 1)); };
        c0_zero<LOGN, R>(Oc, Os, ldc(chn + L::chain(0)), res);
    }
}

// store the 16 values of a thread at its orbit indices (the F1 load pattern)
template <int LOGN, typename S, typename R, bool WAVE_UNIFORM = false>
__device__ __forceinline__ void c0_store(S* y, int k0, const cx<R> (&res)[16], bool conj_out) {
    constexpr int N8 = (1 << LOGN) / 8, N16 = (1 << LOGN) / 16;
    auto c = [&](cx<R> v) { return conj_out ? cconj(v) : v; };
    if constexpr (WAVE_UNIFORM) {
        const sigbuf<S> b(y, 1 << LOGN);
        auto n = [](cx<R> v) {
            S o;
            storage<S>::st(&o, v);
            return o;
        };
        if (k0 > 0) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                b.st(k0, N8 * j, n(c(res[j])));
                b.st(N8 - k0, N8 * j, n(c(res[8 + j])));
            }
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) b.st(0, N16 * i, n(c(res[i])));
        }
        return;
    }
    if (k0 > 0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            storage<S>::st(y + k0 + N8 * j, c(res[j]));
            storage<S>::st(y + N8 * (j + 1) - k0, c(res[8 + j]));
        }
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) storage<S>::st(y + N16 * i, c(res[i]));
    }
}

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
template <int V, int LOGN, typename R>
__device__ __forceinline__ void fill_constants(R* kt, R* kf, const R* __restrict__ ktab, int kshift, bool onthefly,
                                               int tid) {
    using G = kgeo<LOGN>;
    auto kval = [&](int p) -> R {
        if (p == G::Q / 2) return cos_pi_4<R>();
        if (!onthefly) return ktab[(long)p << kshift];
        const double a = (double)p * 2.0 / (double)G::N;
        constexpr int fam = const_family(V);
        const double d = fam == 0 ? 2.0 * cospi(a)
                         : fam == 1 ? 1.0 / (2.0 * cospi(a))
                         : fam == 2 ? 2.0 * sinpi(a)
                                    : 1.0 / (2.0 * sinpi(a));
        return p == 0 ? R(0) : R(d);
    };
    for (int p = tid; p < G::Q; p += G::WG) kt[p] = kval(p);
    sfor<0, G::NP>([&](auto kc) {
        constexpr int K = decltype(kc)::value;
        using M = mpass<LOGN, K>;
        for (int e = tid; e < G::kfsize(K); e += G::WG) {
            // e = kft(t) + (GL-1) rho + (m-1)
            int t = 0;
#pragma unroll
            for (int tt = 1; tt < M::r; ++tt)
                if (e >= G::kft(K, tt)) t = tt;
            const int e1 = e - ((M::GL - 1) * ((1 << M::r) - (1 << (M::r - t))));
            const int rho = e1 / (M::GL - 1);
            const int m = e1 - rho * (M::GL - 1) + 1;
            const int mr = (rho & 1) ? M::GL * (rho + 1) - m : m + M::GL * rho;
            kf[G::kfbase(K) + e] = kval(mr << (M::l0 + t));
        }
    });
}

}  // namespace

}  // namespace amqft
