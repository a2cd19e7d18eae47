// Skeleton-B AM-QFT (variants 2 and 6) for signals larger than one
// workgroup's LDS: the transposed program of the large-N skeleton-A path
// (amqft_kL_* in amqft_kA.hip, variants 4 and 8), as amqft_kB_kernel is the
// transposed program of amqft_kA_kernel (the DFT matrix is symmetric, eq.
// qft_0A; transposing variant 4's program gives variant 2's, 8's gives 6's;
// Sec. 5).  The forward path runs top (F1 over global memory), rows, back
// and bchain (B0, the chain, C0); this one runs their transposes in reverse
// order over the same workspaces and layouts:
//   c0   C0^T over global memory: thread k0 loads the 16 points of its orbit,
//        D_c and -i D_r transposed, the chain's D_k^T for levels 0..2: depth-0
//        blocks 0..2 of both sides and the level-3 chain values -> ws2 (side
//        after side, unpadded), the top of the level-3 chain -> wsc
//   fold FOLD of each signal's level-3 chain in one workgroup: blocks 3 ..
//        D-3 of depth 0 back to ws2, dct[16] / dst[16] -> wsc
//   b0   B0^T for every position of the depth-3 block layout: the M2 / M6
//        neighbour sums across runs of depth-0 block entries (ws2) -> the
//        sixteen depth-3 rows (ws1, by side)
//   rows the transposed kB passes on every row pair (B0^T .. M_k^T of its
//        2^(log2 N - 3)-point transform) and the row's F1^T levels -> the
//        row's slots in ws1
//   top  F1^T over global memory: levels 2..0 on the orbit of m0 across the
//        sixteen rows, D_c / D_r transposed, the store; thread 0 runs the
//        chain from dct[16] / dst[16] (wsc)
// From N = 2^18 on (FP32 arithmetic, up to 2^20) a depth-3 row no longer fits
// one workgroup, and b0 is followed by rback (the row's levels 3..5
// transposed, to depth-6 rows), rows at depth 6 and rtop (the row's F1^T
// levels), the transposes of amqft_kL_rtop / rows<6> / rback.
// Sizes: N = 2^15 .. 2^20 with FP32 arithmetic, 2^14 .. 2^16 with FP64; from
// 2^11 when a plan forces the path (tests of its kernels at sizes where every
// variant is accurate).
#include <type_traits>

#include "amqft_device.h"
#include "amqft_internal.h"
#include "amqft_kB_passes.h"

namespace amqft {

namespace {

// the chain level of length LS of each side (positions [H - LS, H)) in LDS,
// padded, then the 16 chain slots
template <int LOGN, int LS>
struct fold_lay {
    static constexpr int H = (1 << LOGN) / 2, L0 = LS, CS = L0 + L0 / 16 + 1;
    static __device__ __forceinline__ int at(int side, int p) {
        const int i = p - (H - L0);
        return side * CS + i + (i >> 4);
    }
    static __device__ __forceinline__ int ch(int c) { return 2 * CS + c; }
    static constexpr int slots() { return 2 * CS + 16; }
};

// The level-3 chain has N/16 values a side.  Up to N = 2^17 one workgroup
// folds a signal's chain in LDS; from 2^18 on (too long for LDS) a first walk
// over global memory (orbits modulo N/128, eight values a lane and orbit, no
// exchange between lanes) takes it to the level of length N/256, which the
// workgroup folds on.
template <int LOGN>
constexpr int fold_ls() { return LOGN >= 18 ? (1 << LOGN) / 256 : (1 << LOGN) / 16; }

// threads of the fold workgroup: one lane per orbit of its first walk
template <int LOGN>
constexpr int fold_threads() {
    constexpr int p = fold_ls<LOGN>() / 8;
    return p < 256 ? 256 : p;
}

// ---------------------------------------------------------------------------
// c0: C0^T of every orbit of every signal of the chunk
// ---------------------------------------------------------------------------
template <int VB, typename S, int LOGN>
__global__ __launch_bounds__(256) void amqft_kLT_c0(const S* __restrict__ in, cx<typename storage<S>::R>* __restrict__ ws2,
                                                     cx<typename storage<S>::R>* __restrict__ wsc, long long sig0,
                                                     long long batch, int flags, const long long* __restrict__ offsets) {
    using R = typename storage<S>::R;
    constexpr int N = 1 << LOGN, W3 = N / 16;
    const int k0 = blockIdx.x * 256 + threadIdx.x;
    const long long sl = blockIdx.y, gs = sig0 + sl;
    if (gs >= batch || k0 >= W3) return;
    const long long base = uniform64(offsets ? offsets[gs] : gs * (long long)N);
    cx<R> raw[16];
    f1_load<LOGN, S, R, true>(in + base, k0, raw);
    c0T<LOGN, R, glob_lay<LOGN>>(ws2 + sl * N, wsc + sl * 16, raw, k0, (flags & 1) != 0);
}

// ---------------------------------------------------------------------------
// fold1 (N >= 2^18): the first walk over global memory, one lane per orbit;
// block entries in place in ws2, the level of length N/256 to ws1 (the same
// positions; ws1 is free until b0), the new top to wsc
// ---------------------------------------------------------------------------
template <typename R, int LOGN>
__global__ __launch_bounds__(256) void amqft_kLT_fold1(cx<R>* __restrict__ ws2, cx<R>* __restrict__ ws1,
                                                        cx<R>* __restrict__ wsc) {
    constexpr int N = 1 << LOGN, P = N / 128, L0 = N / 16;
    using F = fold_walk<LOGN, P, L0, R, glob_lay<LOGN>>;
    const int k = blockIdx.x * 256 + threadIdx.x;  // < P
    const bool dst = k >= P / 2;
    const int r = k & (P / 2 - 1);
    cx<R>* w = ws2 + (long long)blockIdx.y * N;
    cx<R>* wo = ws1 + (long long)blockIdx.y * N;
    cx<R>* wc = wsc + (long long)blockIdx.y * 16;
    cx<R> v[F::NV];
    F::load(w, wc, dst, r, v);
    F::walk(w, wo, wc, dst, r, v);
}

// ---------------------------------------------------------------------------
// fold: one workgroup per signal, from the level of length fold_ls (read
// from src: ws2, or ws1 after fold1) to dct[16] / dst[16]
// ---------------------------------------------------------------------------
template <typename R, int LOGN>
__global__ __launch_bounds__(fold_threads<LOGN>()) void amqft_kLT_fold(const cx<R>* __restrict__ src, cx<R>* __restrict__ ws2,
                                                                       cx<R>* __restrict__ wsc) {
    using FL = fold_lay<LOGN, fold_ls<LOGN>()>;
    constexpr int N = 1 << LOGN, H = N / 2, L0 = FL::L0, NT = fold_threads<LOGN>();
    extern __shared__ __align__(16) unsigned char smem[];
    cx<R>* w = reinterpret_cast<cx<R>*>(smem);
    const int tid = threadIdx.x;
    const cx<R>* gs = src + (long long)blockIdx.x * N;
    cx<R>* g = ws2 + (long long)blockIdx.x * N;
    cx<R>* gc = wsc + (long long)blockIdx.x * 16;
    for (int i = tid; i < L0; i += NT) {
        stc(w + FL::at(0, H - L0 + i), gs[H - L0 + i]);
        stc(w + FL::at(1, H - L0 + i), gs[H + H - L0 + i]);
    }
    if (tid == 0) stc(w + FL::ch(8), gc[8]);
    __syncthreads();
    fold_block<LOGN, NT, L0, R, FL>(w, tid);
    __syncthreads();
    for (int i = tid; i < L0; i += NT) {
        g[H - L0 + i] = ldc(w + FL::at(0, H - L0 + i));
        g[H + H - L0 + i] = ldc(w + FL::at(1, H - L0 + i));
    }
    if (tid < 16) gc[tid] = ldc(w + FL::ch(tid));
}

// ---------------------------------------------------------------------------
// b0: B0^T for position p of the depth-3 block layout (block a, index j): the
// window of depth-0 runs of 8 that the time-side M2 / M6 terms reach, three
// transposed levels per side, child q -> row (side, q) at p.  Run j of
// depth-0 block a starts at 8p (depth-0 blocks sit at H - H / 2^a = 8 (W3 -
// W3 / 2^a)), so the 256 positions of a workgroup read one contiguous range
// of 8 (256 + 2) values per side: staged in LDS with coalesced loads, one pad
// slot per run of 8 against bank conflicts.
// ---------------------------------------------------------------------------
constexpr int kB0Pos = 256;                      // depth-3 positions per workgroup
constexpr int kB0Runs = kB0Pos + 2;              // with one run before and after
__device__ __forceinline__ int b0_slot(int i) { return i + (i >> 3); }
template <typename R>
constexpr size_t kLT_b0_lds() { return 2 * (size_t)(9 * kB0Runs) * sizeof(cx<R>); }

template <int VB, typename R, int LOGN>
__global__ __launch_bounds__(kB0Pos) void amqft_kLT_b0(const cx<R>* __restrict__ ws2, cx<R>* __restrict__ ws1) {
    constexpr int VA = transposed_of<VB>::V;
    constexpr int N = 1 << LOGN, H = N / 2, W3 = N / 16, LW3 = ilog2c(W3), RS = 9 * kB0Runs;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<R>* st = reinterpret_cast<cx<R>*>(smem);  // [side][b0_slot(depth-0 position - 8 (p0 - 1))]
    const int p0 = blockIdx.x * kB0Pos, tid = threadIdx.x;
    const cx<R>* g = ws2 + (long long)blockIdx.y * N;
    cx<R>* rows = ws1 + (long long)blockIdx.y * N;
    const int lo = 8 * (p0 - 1);
    for (int i = tid; i < 8 * kB0Runs; i += kB0Pos) {
        const int d0 = lo + i;
        const bool in = d0 >= 0 && d0 < H;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const cx<R> v = g[side * H + (in ? d0 : 0)];
            stc(st + side * RS + b0_slot(i), in ? v : zero<R>());
        }
    }
    __syncthreads();
    const int p = p0 + tid;
    if (p >= W3 - 1) return;
    const int a = __clz(~(p << (32 - LW3)));
    const int j = p - (W3 - (W3 >> a));
    const int sp = W3 >> (a + 1);
    sfor<0, 2>([&](auto sc) {
        constexpr int side = decltype(sc)::value;
        using WW = halo_window<VA, side>;
        cx<R> cur[8][WW::W * 8];
#pragma unroll
        for (int d = 0; d < WW::W; ++d) {
            const int jj = j + WW::OFF + d;
            const bool in = jj >= 0 && jj < sp;  // runs outside block a count as zero
            const int r0 = 8 * (tid + 1 + WW::OFF + d);  // the run's first value in the staged range
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const cx<R> v = ldc(st + side * RS + b0_slot(r0 + e));
                cur[0][8 * d + e] = in ? v : zero<R>();
            }
        }
        fwd_levelsT<VA, side, 3, 0, WW::W, R>(cur);
#pragma unroll
        for (int q = 0; q < 8; ++q) rows[(side * 8 + q) * W3 + p] = cur[q][-WW::OFF];
    });
}

// ---------------------------------------------------------------------------
// rows: the transposed passes of amqft_kL_rows on a row pair (the two sides
// of a 2^(log2 N - DEP)-point transform; at depth 3 half hh holds the row of
// side hh ^ parity(P) for M6 / M8, at depth 6 the row of context hh)
// ---------------------------------------------------------------------------
template <int VB, typename R, int LOGN, int DEP>
__global__ __launch_bounds__(kgeo<LOGN - DEP>::WG) void amqft_kLT_rows(cx<R>* __restrict__ ws1,
                                                                       const R* __restrict__ ktab) {
    constexpr int VA = transposed_of<VB>::V;
    constexpr int LR = LOGN - DEP;
    using G = kgeo<LR>;
    constexpr bool SW = variant_traits<VA>::switches;
    constexpr int W3 = (1 << LOGN) >> (DEP + 1);  // row width (= G::H)
    constexpr int N8r = G::N / 8;
    extern __shared__ __align__(16) unsigned char smem[];
    R* kt = reinterpret_cast<R*>(smem);
    R* kf = kt + G::Q;
    cx<R>* wall = reinterpret_cast<cx<R>*>(smem + (G::Q + G::KF_ALLOC) * sizeof(R));
    const int tid = threadIdx.x;
    const int fs = tid / G::T, m0 = tid - fs * G::T;
    const int P = blockIdx.x * G::SPW + fs;
    cx<R>* w = wall + fs * G::SL;
    cx<R>* sig = ws1 + (long long)blockIdx.y * (1 << LOGN);
    cx<R>* row[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
        row[hh] = DEP == 3 ? sig + ((hh ^ (SW ? par(P) : 0)) * 8 + P) * W3 : sig + (2 * P + hh) * W3;
    // the row's block layout into LDS; the blocks of 4, 2 and 1 points (the
    // last seven slots of each row) into the chain slots, which no pass of a
    // row touches (keeping them in registers would cost occupancy)
    using L = lds_layout<LR>;
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
        for (int pos = m0; pos < W3 - 8; pos += G::T) stc(w + hh * G::HS + pad(pos), row[hh][pos]);
    if (m0 < 14) stc(w + L::chain(m0), row[m0 / 7][W3 - 8 + m0 % 7]);
    fill_constants<VA, LR, R>(kt, kf, ktab, DEP, false, tid);
    __syncthreads();
    b0T_pass<VA, LR, R>(wall, tid);
    sfor<0, G::NP>([&](auto kc) { bT_pass<VA, LR, decltype(kc)::value, R>(wall, tid); });
    p3T_pass<VB, LR, R>(wall, kt, tid);
    sfor<0, G::NP>([&](auto kc) { orbitT_pass<VA, VB, LR, G::NP - 1 - decltype(kc)::value, R>(wall, kt, kf, tid); });
    if (m0 > 0) {
        const int pm = pad(m0);
        cx<R> cd[2][8];
        f1T_levels<VA, LR, R>(kt, m0, [&](auto sc, auto pc) {
            constexpr int h2 = decltype(sc)::value ^ (SW ? par(decltype(pc)::value) : 0);
            return ldc(w + h2 * G::HS + G::W3P * decltype(pc)::value + pm);
        }, cd);
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                row[hh][m0 + N8r * i] = cd[hh][2 * i];
                row[hh][N8r * (i + 1) - m0] = cd[hh][2 * i + 1];
            }
    } else {
        // the transposes of the row's blocks of 4, 2 and 1 points
        sfor<0, 2>([&](auto hc) {
            constexpr int hh = decltype(hc)::value;
            cx<R> small[7];
#pragma unroll
            for (int i = 0; i < 7; ++i) small[i] = ldc(w + L::chain(7 * hh + i));
            cx<R> b4[4] = {small[0], small[1], small[2], small[3]};
            cx<R> b2[2] = {small[4], small[5]};
            leaf::to<VB, 4, hh, R>(b4, kt, G::D);
            leaf::to<VB, 2, hh, R>(b2, kt, G::D);
            row[hh][(W3 / 8) * 1] = b4[0];
            row[hh][(W3 / 8) * 3] = b4[1];
            row[hh][(W3 / 8) * 5] = b4[2];
            row[hh][(W3 / 8) * 7] = b4[3];
            row[hh][(W3 / 8) * 2] = b2[0];
            row[hh][(W3 / 8) * 6] = b2[1];
            row[hh][(W3 / 8) * 4] = small[6];
        });
    }
}

// ---------------------------------------------------------------------------
// N >= 2^18 (depth-3 rows above one workgroup's LDS): rback^T -- levels 3..5
// of every depth-3 row transposed (the row's B0^T: its block layout, staged
// as in b0, to the eight depth-6 rows of each context in ws2) -- and rtop^T
// -- the row's F1^T levels from the depth-6 rows back to the depth-3 row's
// slots, with the row's blocks of 4, 2 and 1 points.
// ---------------------------------------------------------------------------
template <int VB, typename R, int LOGN>
__global__ __launch_bounds__(kB0Pos) void amqft_kLT_rback(const cx<R>* __restrict__ ws1, cx<R>* __restrict__ ws2) {
    constexpr int VA = transposed_of<VB>::V;
    constexpr bool SW = variant_traits<VA>::switches;
    constexpr int N = 1 << LOGN, W3 = N / 16, W6 = N / 128, LW6 = ilog2c(W6), RS = 9 * kB0Runs;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<R>* st = reinterpret_cast<cx<R>*>(smem);
    const int p0 = blockIdx.x * kB0Pos, tid = threadIdx.x;
    const int P = blockIdx.y >> 1, hh = blockIdx.y & 1;  // depth-3 row of path P and context hh
    const cx<R>* row = ws1 + (long long)blockIdx.z * N + ((hh ^ (SW ? par(P) : 0)) * 8 + P) * W3;
    cx<R>* sig2 = ws2 + (long long)blockIdx.z * N;
    const int lo = 8 * (p0 - 1);
    for (int i = tid; i < 8 * kB0Runs; i += kB0Pos) {
        const int d0 = lo + i;
        const bool in = d0 >= 0 && d0 < W3;
        const cx<R> v = row[in ? d0 : 0];
        stc(st + b0_slot(i), in ? v : zero<R>());
    }
    __syncthreads();
    const int p = p0 + tid;
    if (p >= W6 - 1) return;
    const int a = __clz(~(p << (32 - LW6)));
    const int j = p - (W6 - (W6 >> a));
    const int sp = W6 >> (a + 1);
    auto levels = [&](auto hc) {
        constexpr int h = decltype(hc)::value;
        using WW = halo_window<VA, h>;
        cx<R> cur[8][WW::W * 8];
#pragma unroll
        for (int d = 0; d < WW::W; ++d) {
            const int jj = j + WW::OFF + d;
            const bool in = jj >= 0 && jj < sp;
            const int r0 = 8 * (tid + 1 + WW::OFF + d);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const cx<R> v = ldc(st + b0_slot(r0 + e));
                cur[0][8 * d + e] = in ? v : zero<R>();
            }
        }
        fwd_levelsT<VA, h, 3, 0, WW::W, R>(cur);
#pragma unroll
        for (int q = 0; q < 8; ++q)
            sig2[(2 * (8 * P + q) + (h ^ (SW ? par(q) : 0))) * W6 + p] = cur[q][-WW::OFF];
    };
    (void)RS;
    if (hh == 0) levels(std::integral_constant<int, 0>{});
    else levels(std::integral_constant<int, 1>{});
}

template <int VB, typename R, int LOGN>
__global__ __launch_bounds__(256) void amqft_kLT_rtop(const cx<R>* __restrict__ ws2, cx<R>* __restrict__ ws1,
                                                       const R* __restrict__ ktab) {
    constexpr int VA = transposed_of<VB>::V;
    constexpr int LR = LOGN - 3;
    constexpr bool SW = variant_traits<VA>::switches;
    constexpr int N = 1 << LOGN, W3 = N / 16, W6 = N / 128, N8r = (1 << LR) / 8;
    const int m0 = blockIdx.x * 256 + threadIdx.x;  // < W6 (a multiple of 256)
    const int P = blockIdx.y;                       // depth-3 path
    cx<R>* sig1 = ws1 + (long long)blockIdx.z * N;
    const cx<R>* sig2 = ws2 + (long long)blockIdx.z * N;
    cx<R>* row[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) row[hh] = sig1 + ((hh ^ (SW ? par(P) : 0)) * 8 + P) * W3;
    // thread 0 reads the row's blocks of 4, 2 and 1 points before threads
    // 2 .. 8 of this workgroup overwrite those slots with their orbits' values
    cx<R> small[2][7];
    if (m0 == 0) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
#pragma unroll
            for (int i = 0; i < 7; ++i) small[hh][i] = row[hh][W3 - 8 + i];
    }
    __syncthreads();
    if (m0 > 0) {
        cx<R> cd[2][8];
        f1T_levels<VA, LR, R, 3>(ktab, m0, [&](auto sc, auto pc) {
            constexpr int h2 = decltype(sc)::value ^ (SW ? par(decltype(pc)::value) : 0);
            return sig2[(2 * (8 * P + decltype(pc)::value) + h2) * W6 + m0];
        }, cd);
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                row[hh][m0 + N8r * i] = cd[hh][2 * i];
                row[hh][N8r * (i + 1) - m0] = cd[hh][2 * i + 1];
            }
    } else {
        sfor<0, 2>([&](auto hc) {
            constexpr int hh = decltype(hc)::value;
            cx<R> b4[4] = {small[hh][0], small[hh][1], small[hh][2], small[hh][3]};
            cx<R> b2[2] = {small[hh][4], small[hh][5]};
            leaf::to<VB, 4, hh, R>(b4, ktab, LOGN - 2);
            leaf::to<VB, 2, hh, R>(b2, ktab, LOGN - 2);
            row[hh][(W3 / 8) * 1] = b4[0];
            row[hh][(W3 / 8) * 3] = b4[1];
            row[hh][(W3 / 8) * 5] = b4[2];
            row[hh][(W3 / 8) * 7] = b4[3];
            row[hh][(W3 / 8) * 2] = b2[0];
            row[hh][(W3 / 8) * 6] = b2[1];
            row[hh][(W3 / 8) * 4] = small[hh][6];
        });
    }
}

// ---------------------------------------------------------------------------
// top: F1^T over global memory and the store
// ---------------------------------------------------------------------------
template <int VB, typename S, int LOGN>
__global__ __launch_bounds__(256) void amqft_kLT_top(const cx<typename storage<S>::R>* __restrict__ ws1,
                                                      const cx<typename storage<S>::R>* __restrict__ wsc,
                                                      S* __restrict__ out, const typename storage<S>::R* __restrict__ ktab,
                                                      long long sig0, long long batch, int flags,
                                                      const long long* __restrict__ offsets) {
    using R = typename storage<S>::R;
    constexpr int VA = transposed_of<VB>::V;
    constexpr int N = 1 << LOGN, W3 = N / 16;
    const int m0 = blockIdx.x * 256 + threadIdx.x;
    const long long sl = blockIdx.y, gs = sig0 + sl;
    if (gs >= batch || m0 >= W3) return;
    const cx<R>* rows = ws1 + sl * N;
    cx<R> res[16];
    if (m0 > 0) {
        cx<R> cd[2][8];
        f1T_levels<VA, LOGN, R>(ktab, m0, [&](auto sc, auto pc) {
            return rows[(decltype(sc)::value * 8 + decltype(pc)::value) * W3 + m0];
        }, cd);
        f1T_combine<R>(cd, res);
    } else {
        cx<R> chs[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) chs[k] = wsc[sl * 16 + k];
        f1T_chain<VB, LOGN, R>(chs, ktab, res);
    }
    const long long base = uniform64(offsets ? offsets[gs] : gs * (long long)N);
    c0_store<LOGN, S, R, true>(out + base, m0, res, (flags & 2) != 0);
}

template <int VB, typename S, int LOGN>
hipError_t launch_kLT_n(const kl_launch& a, hipStream_t st) {
    using R = typename storage<S>::R;
    constexpr int VA = transposed_of<VB>::V;
    constexpr int N = 1 << LOGN, W3 = N / 16;
    constexpr int DEP = LOGN >= 18 ? 6 : 3;  // depth of the rows that fit one workgroup's LDS
    using GR = kgeo<LOGN - DEP>;
    const int flags = (a.conj_in ? 1 : 0) | (a.conj_out ? 2 : 0);
    const size_t lds_rows = kA_lds_bytes_v<VA, R, LOGN - DEP>();
    const size_t lds_fold = (size_t)fold_lay<LOGN, fold_ls<LOGN>()>::slots() * sizeof(cx<R>);
    cx<R>* ws1 = static_cast<cx<R>*>(a.ws1);
    cx<R>* ws2 = static_cast<cx<R>*>(a.ws2);
    cx<R>* wsc = static_cast<cx<R>*>(a.wsc);
    const R* kt = static_cast<const R*>(a.ktab);
    for (long long s0 = 0; s0 < a.batch; s0 += a.chunk) {
        const long long nb = a.batch - s0 < a.chunk ? a.batch - s0 : a.chunk;
        const dim3 gw((W3 + 255) / 256, (unsigned)nb);
        hipLaunchKernelGGL((amqft_kLT_c0<VB, S, LOGN>), gw, dim3(256), 0, st, static_cast<const S*>(a.in), ws2, wsc,
                           s0, (long long)a.batch, flags, static_cast<const long long*>(a.offsets));
        if constexpr (LOGN >= 18)
            hipLaunchKernelGGL((amqft_kLT_fold1<R, LOGN>), dim3(N / 128 / 256, (unsigned)nb), dim3(256), 0, st, ws2, ws1,
                               wsc);
        hipLaunchKernelGGL((amqft_kLT_fold<R, LOGN>), dim3((unsigned)nb), dim3(fold_threads<LOGN>()), lds_fold, st,
                           static_cast<const cx<R>*>(LOGN >= 18 ? ws1 : ws2), ws2, wsc);
        hipLaunchKernelGGL((amqft_kLT_b0<VB, R, LOGN>), dim3((W3 - 1 + kB0Pos - 1) / kB0Pos, (unsigned)nb), dim3(kB0Pos),
                           kLT_b0_lds<R>(), st, static_cast<const cx<R>*>(ws2), ws1);
        if constexpr (DEP == 3) {
            hipLaunchKernelGGL((amqft_kLT_rows<VB, R, LOGN, 3>), dim3(8 / GR::SPW, (unsigned)nb), dim3(GR::WG), lds_rows,
                               st, ws1, kt);
        } else {
            constexpr int W6 = N / 128;
            static_assert(GR::SPW == 1, "depth-6 rows are at least 2^12 points");
            hipLaunchKernelGGL((amqft_kLT_rback<VB, R, LOGN>), dim3((W6 - 1 + kB0Pos - 1) / kB0Pos, 16, (unsigned)nb),
                               dim3(kB0Pos), kLT_b0_lds<R>() / 2, st, static_cast<const cx<R>*>(ws1), ws2);
            hipLaunchKernelGGL((amqft_kLT_rows<VB, R, LOGN, 6>), dim3(64, (unsigned)nb), dim3(GR::WG), lds_rows, st, ws2,
                               kt);
            hipLaunchKernelGGL((amqft_kLT_rtop<VB, R, LOGN>), dim3(W6 / 256, 8, (unsigned)nb), dim3(256), 0, st,
                               static_cast<const cx<R>*>(ws2), ws1, kt);
        }
        hipLaunchKernelGGL((amqft_kLT_top<VB, S, LOGN>), gw, dim3(256), 0, st, static_cast<const cx<R>*>(ws1),
                           static_cast<const cx<R>*>(wsc), static_cast<S*>(a.out), kt, s0, (long long)a.batch, flags,
                           static_cast<const long long*>(a.offsets));
    }
    return hipGetLastError();
}

template <int VB, typename S>
hipError_t launch_kLT_s(const kl_launch& a, hipStream_t st) {
    switch (a.logn) {
    case 11: return launch_kLT_n<VB, S, 11>(a, st);
    case 12: return launch_kLT_n<VB, S, 12>(a, st);
    case 13: return launch_kLT_n<VB, S, 13>(a, st);
    case 14: return launch_kLT_n<VB, S, 14>(a, st);
    case 15: return launch_kLT_n<VB, S, 15>(a, st);
    default:
        if constexpr (std::is_same<S, double2>::value) {
            return launch_kLT_n<VB, S, 16>(a, st);
        } else {
            switch (a.logn) {
            case 16: return launch_kLT_n<VB, S, 16>(a, st);
            case 17: return launch_kLT_n<VB, S, 17>(a, st);
            case 18: return launch_kLT_n<VB, S, 18>(a, st);
            case 19: return launch_kLT_n<VB, S, 19>(a, st);
            default: return launch_kLT_n<VB, S, 20>(a, st);
            }
        }
    }
}

template <int VB>
hipError_t launch_kLT_v(const kl_launch& a, hipStream_t st) {
    switch (a.dtype) {
    case 0: return launch_kLT_s<VB, double2>(a, st);
    case 1: return launch_kLT_s<VB, float2>(a, st);
    case 2: return launch_kLT_s<VB, __half2>(a, st);
    default: return launch_kLT_s<VB, bf16x2>(a, st);
    }
}

template <int VB, typename R, int LOGN, int LMAX>
hipError_t prime_kLT_n() {
    constexpr int DEP = LOGN >= 18 ? 6 : 3;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amqft_kLT_rows<VB, R, LOGN, DEP>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if constexpr (DEP == 6) {
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amqft_kLT_rback<VB, R, LOGN>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    }
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amqft_kLT_fold<R, LOGN>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amqft_kLT_b0<VB, R, LOGN>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if constexpr (LOGN < LMAX) {
        if (e == hipSuccess) e = prime_kLT_n<VB, R, LOGN + 1, LMAX>();
    }
    return e;
}

}  // namespace

bool kLT_supported(int variant, int logn, int dtype) {
    if (variant != 2 && variant != 6) return false;
    if (dtype == 0) return logn >= 14 && logn <= 16;
    if (dtype == 1 || dtype == 2 || dtype == 3) return logn >= 15 && logn <= 20;
    return false;
}

bool kLT_supported_forced(int variant, int logn, int dtype) {
    if (variant != 2 && variant != 6) return false;
    if (dtype == 0) return logn >= 11 && logn <= 16;
    if (dtype == 1) return logn >= 11 && logn <= 20;
    return kLT_supported(variant, logn, dtype);
}

hipError_t prime_kLT(int variant, int dtype) {
    // the rows and fold kernels depend on the arithmetic type only
    if (variant == 2) return dtype == 0 ? prime_kLT_n<2, double, 11, 16>() : prime_kLT_n<2, float, 11, 20>();
    if (variant == 6) return dtype == 0 ? prime_kLT_n<6, double, 11, 16>() : prime_kLT_n<6, float, 11, 20>();
    return hipSuccess;
}

hipError_t launch_kLT(const kl_launch& a, hipStream_t st) {
    if (a.batch <= 0) return hipSuccess;
    if (!kLT_supported_forced(a.variant, a.logn, a.dtype)) return hipErrorInvalidValue;
    return a.variant == 2 ? launch_kLT_v<2>(a, st) : launch_kLT_v<6>(a, st);
}

}  // namespace amqft
