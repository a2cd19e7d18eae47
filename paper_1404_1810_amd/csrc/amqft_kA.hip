// Skeleton-A AM-QFT (variants 1, 4, 5, 8) for N = 2^8 .. 2^14 with the whole
// dataflow fixed at compile time: a handful of passes over LDS, each reading
// everything it needs, waiting at a barrier and writing, every thread
// holding 16 complex values per pass.  Further down: the fused loss/gradient
// kernel on the same passes, and the global-memory kernels for N = 2^15 ..
// 2^20 (variants 4 and 8) that reuse them on the rows of a larger transform.
//
// View of one side (DCT or DST, H = N/2 positions): after the forward levels
// 0..l-1 of dct_ot / dst_ot the data form 2^l rows of W_l = H / 2^l slots;
// slot m of a row holds the element of chain block a = v2(m) (the ot
// function of periodization N / 2^a) with odd index m / 2^a.  A forward level
// pairs slot m with W_l - m inside a row and sends sum / difference to rows
// 2P / 2P+1 at the same slot (D_k, Table tab:elabora_relations_B), the hi half
// scaled by the M4 / M8 constant of index p = m * 2^l (Sec. 7.1; table entry
// N/8 is set to cos(pi/4), the L = 8 base case).
//
// Passes (D = log2 N - 2):
//   F1   load, D_c / D_r, levels 0..2 on the orbits {+-m0 + (N/8) j}; thread
//        m0 = 0 of a signal does the blocks of 4, 2, 1 points and the chain
//        up to dct[16] / dst[16].
//   M_k  middle levels in one or two orbit passes of r <= 4 levels on the
//        orbits {+-m0 + 2G j} of each row (G = W / 2^r lanes per row); lane
//        m0 = 0 of a row finishes the slots that are multiples of G (whole
//        sub-blocks of at most 2^(r-1) points) in registers.
//   P3   rows of 16 slots at depth D-3: sub-blocks of 8, 4, 2, 1 points,
//        forward and backward in registers.
//   B_k  mirror of M_k: a thread combines one child index j of 2^r rows into
//        2^r consecutive parent harmonics, with the +-1 neighbours M4 / M8 read
//        (M1 / M5: a segmented scan across the lanes of each child instead).
//   B0   mirror of F1 (levels 2..0), both sides per thread.
//   C0   chain D_n^F: levels 3..D-3 along each output's reflection path,
//        levels 0..2 on an orbit of 8 harmonics, D_c and the store.
//
// Storage per signal: two LDS halves (contexts: row (side, path) lives in
// half side ^ parity(path) for M8, in half side for M4), positions padded by
// one slot per 16.  The pad slots (index k at 17 k + 16) hold what the orbit
// passes finish early: row R of pass k stores its values at the first pad
// slot of its child rows 1 .. 2^r - 1, so no two passes collide; the first
// pad slot of the eight depth-3 rows of each half holds the chain values.
#include <type_traits>

#include "amqft_device.h"
#include "amqft_internal.h"
#include "amqft_kA_passes.h"
#include "amqft_leaf.h"

namespace amqft {

namespace {

template <int V, typename S, int LOGN>
__global__ __launch_bounds__(kgeo<LOGN>::WG) void amqft_kA_kernel(const S* __restrict__ in, S* __restrict__ out,
                                                                   const typename storage<S>::R* __restrict__ ktab,
                                                                   long long batch, int kshift, int flags,
                                                                   const long long* __restrict__ offsets) {
    using R = typename storage<S>::R;
    using G = kgeo<LOGN>;
    extern __shared__ __align__(16) unsigned char smem[];
    R* kt = reinterpret_cast<R*>(smem);
    R* kf = kt + G::Q;
    cx<R>* wall = reinterpret_cast<cx<R>*>(smem + (G::Q + G::KF_ALLOC) * sizeof(R));
    const bool conj_in = flags & 1, conj_out = flags & 2, onthefly = flags & 4;
    const int tid = threadIdx.x;
    const int fs = tid / G::T, m0 = tid - fs * G::T;  // signal of this thread in F1 / B0 / C0, orbit index
    const long long gs = (long long)blockIdx.x * G::SPW + fs;
    const bool live = gs < batch;
    long long base = !live ? 0 : offsets ? offsets[gs] : gs * (long long)G::N;
    // at least one wave per signal: the signal's offset is the same in every
    // lane, so loads and stores address it from scalar registers
    constexpr bool WU = G::T >= 64;
    if constexpr (WU) base = uniform64(base);

    cx<R> raw[16];
    f1_load<LOGN, S, R, WU>(in + base, m0, raw);
    fill_constants<V, LOGN, R>(kt, kf, ktab, kshift, onthefly, tid);
    __syncthreads();

    cx<R>* w = wall + fs * G::SL;
    if (m0 > 0) f1_orbit<V, LOGN, R>(w, kt, raw, m0, conj_in);
    else f1_chain<V, LOGN, R>(w, kt, raw, conj_in);
    __syncthreads();

    sfor<0, G::NP>([&](auto kc) { orbit_pass<V, LOGN, decltype(kc)::value, R>(wall, kt, kf, tid); });
    p3_pass<V, LOGN, R>(wall, kt, tid);
    if constexpr (variant_traits<V>::recurrence) {
        sfor<0, G::NP>([&](auto kc) { bpass_rec<V, LOGN, G::NP - 1 - decltype(kc)::value, R>(wall, tid); });
        b0_pass_rec<V, LOGN, R>(wall, wall + G::SPW * G::SL, tid);
    } else {
        sfor<0, G::NP>([&](auto kc) { bpass<V, LOGN, G::NP - 1 - decltype(kc)::value, R>(wall, tid); });
        b0_pass<V, LOGN, R>(wall, tid);
    }
    if (live) {
        cx<R> res[16];
        c0_compute<LOGN, R, lds_layout<LOGN>>(w, w, m0, res);
        c0_store<LOGN, S, R, WU>(out + base, m0, res, conj_out);
    }
}

// Fused loss and gradient: y = F x, loss = sum_k |W(k) y(k)|^2 per signal,
// grad = F^H (2 |W|^2 y) = conj(F conj(g)).  The forward transform's C0
// leaves each thread with y at exactly the 16 indices its F1 of the second
// transform needs, so the weighting happens in registers between the two.
template <typename R, int LOGN>
constexpr size_t kA_loss_lds_bytes() {
    using G = kgeo<LOGN>;
    return (size_t)(G::Q + G::KF_ALLOC + 16) * sizeof(R) + (size_t)G::SPW * G::SL * sizeof(cx<R>);
}

template <int V, typename S, int LOGN>
__global__ __launch_bounds__(kgeo<LOGN>::WG) void amqft_kA_loss_kernel(const S* __restrict__ xin,
                                                                        const S* __restrict__ win,
                                                                        S* __restrict__ grad,
                                                                        typename storage<S>::R* __restrict__ loss,
                                                                        const typename storage<S>::R* __restrict__ ktab,
                                                                        long long batch, int kshift, int flags) {
    using R = typename storage<S>::R;
    using G = kgeo<LOGN>;
    extern __shared__ __align__(16) unsigned char smem[];
    R* kt = reinterpret_cast<R*>(smem);
    R* kf = kt + G::Q;
    R* red = kf + G::KF_ALLOC;  // per-wave partial losses
    cx<R>* wall = reinterpret_cast<cx<R>*>(smem + (G::Q + G::KF_ALLOC + 16) * sizeof(R));
    const bool onthefly = flags & 4;
    const int tid = threadIdx.x;
    const int fs = tid / G::T, m0 = tid - fs * G::T;
    const long long gs = (long long)blockIdx.x * G::SPW + fs;
    const bool live = gs < batch;
    constexpr bool WU = G::T >= 64;  // one signal per wave or more: uniform offsets
    long long base = live ? gs * (long long)G::N : 0;
    if constexpr (WU) base = uniform64(base);
    cx<R>* w = wall + fs * G::SL;

    cx<R> raw[16];
    f1_load<LOGN, S, R, WU>(xin + base, m0, raw);
    fill_constants<V, LOGN, R>(kt, kf, ktab, kshift, onthefly, tid);
    __syncthreads();

    // forward transform
    if (m0 > 0) f1_orbit<V, LOGN, R>(w, kt, raw, m0, false);
    else f1_chain<V, LOGN, R>(w, kt, raw, false);
    __syncthreads();
    sfor<0, G::NP>([&](auto kc) { orbit_pass<V, LOGN, decltype(kc)::value, R>(wall, kt, kf, tid); });
    p3_pass<V, LOGN, R>(wall, kt, tid);
    sfor<0, G::NP>([&](auto kc) { bpass<V, LOGN, G::NP - 1 - decltype(kc)::value, R>(wall, tid); });
    b0_pass<V, LOGN, R>(wall, tid);
    cx<R> y[16];
    c0_compute<LOGN, R, lds_layout<LOGN>>(w, w, m0, y);

    // weighting: g = 2 |W|^2 y at the thread's 16 indices; loss partial
    cx<R> wt[16];
    f1_load<LOGN, S, R, WU>(win + base, m0, wt);
    R part = R(0);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const R m2 = wt[i].re * wt[i].re + wt[i].im * wt[i].im;
        part += m2 * (y[i].re * y[i].re + y[i].im * y[i].im);
        raw[i] = y[i] * (R(2) * m2);
    }
    // per-signal loss, reduced in a fixed order
    constexpr int GRP = G::T < 64 ? G::T : 64;
#pragma unroll
    for (int o = 1; o < GRP; o <<= 1) part += __shfl_xor(part, o);
    if constexpr (G::T <= 64) {
        if (m0 == 0 && live) loss[gs] = part;
    } else {
        if ((tid & 63) == 0) red[tid >> 6] = part;
    }
    __syncthreads();  // C0's LDS reads (and the partials) are complete
    if constexpr (G::T > 64) {
        if (m0 == 0 && live) {
            R sum = R(0);
            for (int u = 0; u < G::T / 64; ++u) sum += red[fs * (G::T / 64) + u];
            loss[gs] = sum;
        }
    }

    // adjoint: grad = conj(F conj(g))
    if (m0 > 0) f1_orbit<V, LOGN, R>(w, kt, raw, m0, true);
    else f1_chain<V, LOGN, R>(w, kt, raw, true);
    __syncthreads();
    sfor<0, G::NP>([&](auto kc) { orbit_pass<V, LOGN, decltype(kc)::value, R>(wall, kt, kf, tid); });
    p3_pass<V, LOGN, R>(wall, kt, tid);
    sfor<0, G::NP>([&](auto kc) { bpass<V, LOGN, G::NP - 1 - decltype(kc)::value, R>(wall, tid); });
    b0_pass<V, LOGN, R>(wall, tid);
    if (live) {
        c0_compute<LOGN, R, lds_layout<LOGN>>(w, w, m0, y);
        c0_store<LOGN, S, R, WU>(grad + base, m0, y, true);
    }
}

template <int V, typename S, int LOGN>
hipError_t launch_kA_loss_n(const loss_launch& a, hipStream_t st) {
    using R = typename storage<S>::R;
    using G = kgeo<LOGN>;
    const long long grid = (a.batch + G::SPW - 1) / G::SPW;
    const size_t lds = kA_loss_lds_bytes<R, LOGN>();
    hipLaunchKernelGGL((amqft_kA_loss_kernel<V, S, LOGN>), dim3((unsigned)grid), dim3(G::WG), lds, st,
                       static_cast<const S*>(a.x), static_cast<const S*>(a.w), static_cast<S*>(a.grad),
                       static_cast<R*>(a.loss), static_cast<const R*>(a.ktab), (long long)a.batch,
                       a.ktab_log2n - LOGN, a.onthefly ? 4 : 0);
    return hipGetLastError();
}

template <int V, typename S>
hipError_t launch_kA_loss_s(const loss_launch& a, hipStream_t st) {
    switch (a.logn) {
    case 8: return launch_kA_loss_n<V, S, 8>(a, st);
    case 9: return launch_kA_loss_n<V, S, 9>(a, st);
    case 10: return launch_kA_loss_n<V, S, 10>(a, st);
    case 11: return launch_kA_loss_n<V, S, 11>(a, st);
    case 12: return launch_kA_loss_n<V, S, 12>(a, st);
    case 13: return launch_kA_loss_n<V, S, 13>(a, st);
    default: return launch_kA_loss_n<V, S, 14>(a, st);
    }
}

template <int V, typename S, int LOGN>
hipError_t prime_kA_loss_n() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amqft_kA_loss_kernel<V, S, LOGN>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if constexpr (LOGN < 14) {
        if (e == hipSuccess) e = prime_kA_loss_n<V, S, LOGN + 1>();
    }
    return e;
}

template <int V, typename S, int LOGN>
hipError_t launch_kA_n(const lds_launch& a, hipStream_t st) {
    using R = typename storage<S>::R;
    using G = kgeo<LOGN>;
    const int flags = (a.conj_in ? 1 : 0) | (a.conj_out ? 2 : 0) | (a.onthefly ? 4 : 0);
    const long long grid = (a.batch + G::SPW - 1) / G::SPW;
    const size_t lds = kA_lds_bytes_v<V, R, LOGN>();
    hipLaunchKernelGGL((amqft_kA_kernel<V, S, LOGN>), dim3((unsigned)grid), dim3(G::WG), lds, st,
                       static_cast<const S*>(a.in), static_cast<S*>(a.out), static_cast<const R*>(a.ktab),
                       (long long)a.batch, a.ktab_log2n - LOGN, flags, static_cast<const long long*>(a.offsets));
    return hipGetLastError();
}

template <int V, typename S>
hipError_t launch_kA_s(const lds_launch& a, hipStream_t st) {
    switch (a.logn) {
    case 8: return launch_kA_n<V, S, 8>(a, st);
    case 9: return launch_kA_n<V, S, 9>(a, st);
    case 10: return launch_kA_n<V, S, 10>(a, st);
    case 11: return launch_kA_n<V, S, 11>(a, st);
    case 12: return launch_kA_n<V, S, 12>(a, st);
    case 13: return launch_kA_n<V, S, 13>(a, st);
    default: return launch_kA_n<V, S, 14>(a, st);
    }
}

template <int V, typename S, int LOGN>
hipError_t prime_kA_n() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amqft_kA_kernel<V, S, LOGN>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if constexpr (LOGN < 14) {
        if (e == hipSuccess) e = prime_kA_n<V, S, LOGN + 1>();
    }
    return e;
}

// ---------------------------------------------------------------------------
// Signals larger than one workgroup's LDS (N = 2^15 .. 2^20): four kernels
// over a global workspace (six from 2^18 on, see amqft_kL_rtop / rback).  A depth-3 row of an N-point transform (W3 = N/16
// slots) is one side of the dct_ot / dst_ot recursion of an N/8-point
// transform, with the constant table subsampled by 8, so the row pass runs
// the kernels above at log2 N - 3.
//   top    D_c / D_r + levels 0..2 (F1): depth-3 rows -> ws1, chain -> wsc
//   rows   two rows (one per context) per workgroup through every level
//          below depth 3 and back; each row -> ws1 in block layout (block a
//          at W3 - W3 / 2^a)
//   back   levels 2..0 (B0 over global rows) for the blocks a >= 3 and the
//          few groups of blocks 0..2 that harmonics N/16 i read -> ws2, depth 0
//          in block layout per side (block a at H - H / 2^a)
//   bchain B0 of the blocks 0..2 that a workgroup's chain threads read, into
//          LDS; then the chain, D_c and the store (C0)
// ---------------------------------------------------------------------------
template <int LOGN>
struct global_layout {
    static constexpr int H = (1 << LOGN) / 2;
    static constexpr int idx(int k) { return k; }
    static constexpr int base(int side, int a) { return side * H + H - (H >> a); }
    static constexpr int chain(int c) { return c; }
};

// member(r, o) of the in-place path: the position of row r's value in orbit o
// (the orbit of a first-kernel thread: o + j N/8 and (j+1) N/8 - o)
template <int LOGN>
__device__ __forceinline__ int ip_member(int r, int o) {
    constexpr int N8 = (1 << LOGN) / 8;
    return r < 8 ? r * N8 + o : (r - 7) * N8 - o;
}

template <int V, typename S, int LOGN>
__global__ __launch_bounds__(256) void amqft_kL_top(const S* __restrict__ in, cx<typename storage<S>::R>* __restrict__ ws1,
                                                     cx<typename storage<S>::R>* __restrict__ wsc,
                                                     const typename storage<S>::R* __restrict__ ktab, long long sig0,
                                                     long long batch, int flags, const long long* __restrict__ offsets) {
    using R = typename storage<S>::R;
    constexpr int N = 1 << LOGN, W3 = N / 16;
    const int m0 = blockIdx.x * 256 + threadIdx.x;
    const long long sl = blockIdx.y, gs = sig0 + sl;
    if (gs >= batch || m0 >= W3) return;
    const bool conj_in = flags & 1;
    const long long base = uniform64(offsets ? offsets[gs] : gs * (long long)N);
    cx<R> raw[16];
    f1_load<LOGN, S, R, true>(in + base, m0, raw);
    cx<R>* rows = ws1 + sl * N;
    if (m0 > 0) {
        cx<R> cd[2][8];
        f1_dc<R>(raw, conj_in, cd);
        f1_levels<V, LOGN, R>(ktab, cd, m0, [&](auto sc, auto pc, cx<R> v) {
            constexpr int side = decltype(sc)::value, P8 = decltype(pc)::value;
            rows[(side * 8 + P8) * W3 + m0] = v;  // depth-3 row (side, P8), slot m0
        });
    } else {
        f1_chain_to<V, LOGN, R>(ktab, raw, conj_in, [&](int c, cx<R> v) { wsc[sl * 16 + c] = v; });
    }
}

// In place: thread m0 writes the sixteen row values of slot m0 to the sixteen
// positions of orbit m0 it read (row r at ip_member(r, m0)); thread 0 reads
// orbit 0 (the positions N/16 k) and writes the chain values to wsc.
template <int V, typename S, int LOGN>
__global__ __launch_bounds__(256) void amqft_kL_top_ip(S* x, cx<typename storage<S>::R>* __restrict__ wsc,
                                                        const typename storage<S>::R* __restrict__ ktab,
                                                        long long sig0, long long batch, int flags) {
    using R = typename storage<S>::R;
    constexpr int N = 1 << LOGN, W3 = N / 16;
    const int m0 = blockIdx.x * 256 + threadIdx.x;
    const long long sl = blockIdx.y, gs = sig0 + sl;
    if (gs >= batch || m0 >= W3) return;
    const bool conj_in = flags & 1;
    const long long base = uniform64(gs * (long long)N);
    cx<R> raw[16];
    f1_load<LOGN, S, R, true>(x + base, m0, raw);
    cx<R>* sig = reinterpret_cast<cx<R>*>(x + base);
    if (m0 > 0) {
        cx<R> cd[2][8];
        f1_dc<R>(raw, conj_in, cd);
        f1_levels<V, LOGN, R>(ktab, cd, m0, [&](auto sc, auto pc, cx<R> v) {
            constexpr int side = decltype(sc)::value, P8 = decltype(pc)::value;
            xst(sig + ip_member<LOGN>(side * 8 + P8, m0), v);
        });
    } else {
        f1_chain_to<V, LOGN, R>(ktab, raw, conj_in, [&](int c, cx<R> v) { wsc[sl * 16 + c] = v; });
    }
}

// Rows at depth DEP (3, or 6 for N >= 2^18): a pair of rows of the two
// contexts is the pair of sides of a 2^(log2 N - DEP)-point transform.  Depth-3
// rows live in ws by side (row (side, P) at (8 side + P) W), depth-6 rows by
// context (row (P, h) at (2 P + h) W); either way the pair leaves in the
// block layout of the row (block a at W - W / 2^a).
//
// IP (in place, depth 3): ws1 is the signal buffer; slot s of row r is read
// at ip_member(r, s) and written at ip_member(r, orb[s]).  The workgroup
// reads all of its rows before its first barrier.
template <int V, typename R, int LOGN, int DEP, bool IP = false>
__global__ __launch_bounds__(kgeo<LOGN - DEP>::WG) void amqft_kL_rows(cx<R>* __restrict__ ws1,
                                                                      const R* __restrict__ ktab,
                                                                      const int* __restrict__ orb) {
    constexpr int LR = LOGN - DEP;  // rows = sides of a 2^LR-point transform
    using G = kgeo<LR>;
    constexpr bool SW = variant_traits<V>::switches;
    constexpr int W3 = (1 << LOGN) >> (DEP + 1);  // row width (= G::H)
    constexpr int N8r = G::N / 8;
    extern __shared__ __align__(16) unsigned char smem[];
    R* kt = reinterpret_cast<R*>(smem);
    R* kf = kt + G::Q;
    cx<R>* wall = reinterpret_cast<cx<R>*>(smem + (G::Q + G::KF_ALLOC) * sizeof(R));
    const int tid = threadIdx.x;
    // rows shorter than 2^12 points share a workgroup, as signals do in the
    // LDS kernel: slot fs of the workgroup takes the row pair of path P
    const int fs = tid / G::T, m0 = tid - fs * G::T;
    const int P = blockIdx.x * G::SPW + fs;  // path of the row pair
    cx<R>* w = wall + fs * G::SL;
    cx<R>* sig = ws1 + (long long)blockIdx.y * (1 << LOGN);
    // half hh (= context) holds the row of side hh ^ parity(P) (depth 3) or
    // the row of context hh (depth 6)
    static_assert(!IP || DEP == 3, "the in-place layout is that of depth-3 rows");
    cx<R>* row[2];
    int rid[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        rid[hh] = (hh ^ (SW ? par(P) : 0)) * 8 + P;
        row[hh] = DEP == 3 ? sig + rid[hh] * W3 : sig + (2 * P + hh) * W3;
    }
    // slot q of the row in half hh: the input layout, and the output layout
    auto rd = [&](int hh, int q) {
        if constexpr (IP) return xld(sig + ip_member<LOGN>(rid[hh], q));
        else return row[hh][q];
    };
    auto wr = [&](int hh, int q, cx<R> v) {
        if constexpr (IP) xst(sig + ip_member<LOGN>(rid[hh], orb[q]), v);
        else row[hh][q] = v;
    };
    cx<R> cd[2][8];
    if (m0 > 0) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                cd[hh][2 * i] = rd(hh, m0 + N8r * i);
                cd[hh][2 * i + 1] = rd(hh, N8r * (i + 1) - m0);
            }
    } else {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
#pragma unroll
            for (int k = 1; k < 8; ++k) cd[hh][k] = rd(hh, (W3 / 8) * k);
    }
    fill_constants<V, LR, R>(kt, kf, ktab, DEP, false, tid);
    __syncthreads();
    if (m0 > 0) {
        const int pm = pad(m0);
        f1_levels<V, LR, R>(kt, cd, m0, [&](auto sc, auto pc, cx<R> v) {
            constexpr int hh = decltype(sc)::value, P8 = decltype(pc)::value;
            constexpr int h2 = hh ^ (SW ? par(P8) : 0);
            stc(w + h2 * G::HS + G::W3P * P8 + pm, v);
        });
    } else {
        // the row's blocks of 4, 2 and 1 points (slots (W3/8) k), straight to the output layout
        sfor<0, 2>([&](auto hc) {
            constexpr int hh = decltype(hc)::value;
            cx<R> b4[4] = {cd[hh][1], cd[hh][3], cd[hh][5], cd[hh][7]}, b2[2] = {cd[hh][2], cd[hh][6]};
            leaf::ot<V, 4, hh, R>(b4, kt, G::D);
            leaf::ot<V, 2, hh, R>(b2, kt, G::D);
#pragma unroll
            for (int i = 0; i < 4; ++i) wr(hh, W3 - 8 + i, b4[i]);
            wr(hh, W3 - 4, b2[0]);
            wr(hh, W3 - 3, b2[1]);
            wr(hh, W3 - 2, cd[hh][4]);
        });
    }
    __syncthreads();
    sfor<0, G::NP>([&](auto kc) { orbit_pass<V, LR, decltype(kc)::value, R>(wall, kt, kf, tid); });
    p3_pass<V, LR, R>(wall, kt, tid);
    sfor<0, G::NP>([&](auto kc) { bpass<V, LR, G::NP - 1 - decltype(kc)::value, R>(wall, tid); });
    b0_pass<V, LR, R>(wall, tid);
    // blocks with at least 8 points: LDS block layout -> the row
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
        for (int pos = m0; pos < W3 - 8; pos += G::T) wr(hh, pos, ldc(w + hh * G::HS + pad(pos)));
}

// N >= 2^18: levels 3..5 of every depth-3 row pair (the F1 levels of its
// 2^(log2 N - 3)-point transform, constants at stride 8 in the table of N):
// depth-6 rows -> ws2 by context; the slots that are multiples of W3 / 8 (the
// row's blocks of 4, 2 and 1 points) are finished in place in ws1, at the
// positions the row's block layout gives them.
template <int V, typename R, int LOGN>
__global__ __launch_bounds__(256) void amqft_kL_rtop(cx<R>* __restrict__ ws1, cx<R>* __restrict__ ws2,
                                                      const R* __restrict__ ktab) {
    constexpr int LR = LOGN - 3;
    constexpr bool SW = variant_traits<V>::switches;
    constexpr int N = 1 << LOGN, W3 = N / 16, W6 = N / 128, N8r = (1 << LR) / 8;
    const int m0 = blockIdx.x * 256 + threadIdx.x;  // < W6 (a multiple of 256)
    const int P = blockIdx.y;                       // depth-3 path
    cx<R>* sig1 = ws1 + (long long)blockIdx.z * N;
    cx<R>* sig2 = ws2 + (long long)blockIdx.z * N;
    cx<R>* row[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) row[hh] = sig1 + ((hh ^ (SW ? par(P) : 0)) * 8 + P) * W3;
    cx<R> cd[2][8];
    if (m0 > 0) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                cd[hh][2 * i] = row[hh][m0 + N8r * i];
                cd[hh][2 * i + 1] = row[hh][N8r * (i + 1) - m0];
            }
    } else {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            cd[hh][0] = zero<R>();
#pragma unroll
            for (int k = 1; k < 8; ++k) cd[hh][k] = row[hh][(W3 / 8) * k];
        }
    }
    // the slots that thread m0 = 0 overwrites below are read only by threads
    // of this workgroup (m0 = 2 .. 8 of their orbits' last pair)
    __syncthreads();
    if (m0 > 0) {
        f1_levels<V, LR, R, 3>(ktab, cd, m0, [&](auto sc, auto pc, cx<R> v) {
            constexpr int hh = decltype(sc)::value, P8 = decltype(pc)::value;
            constexpr int h2 = hh ^ (SW ? par(P8) : 0);
            sig2[(2 * (8 * P + P8) + h2) * W6 + m0] = v;  // depth-6 row (8 P + P8) of context h2, slot m0
        });
    } else {
        sfor<0, 2>([&](auto hc) {
            constexpr int hh = decltype(hc)::value;
            cx<R> b4[4] = {cd[hh][1], cd[hh][3], cd[hh][5], cd[hh][7]}, b2[2] = {cd[hh][2], cd[hh][6]};
            leaf::ot<V, 4, hh, R>(b4, ktab, LOGN - 2);
            leaf::ot<V, 2, hh, R>(b2, ktab, LOGN - 2);
#pragma unroll
            for (int i = 0; i < 4; ++i) row[hh][W3 - 8 + i] = b4[i];
            row[hh][W3 - 4] = b2[0];
            row[hh][W3 - 3] = b2[1];
            row[hh][W3 - 2] = cd[hh][4];
        });
    }
}

// N >= 2^18: levels 5..3 -- the eight depth-6 children of every depth-3 row
// (in their block layout in ws2) back to that row's block layout in ws1
// (blocks of at least 8 points; the smaller ones are already there)
template <int V, typename R, int LOGN>
__global__ __launch_bounds__(256) void amqft_kL_rback(const cx<R>* __restrict__ ws2, cx<R>* __restrict__ ws1) {
    constexpr bool SW = variant_traits<V>::switches;
    constexpr int N = 1 << LOGN, W3 = N / 16, W6 = N / 128, LW6 = ilog2c(W6);
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= W6 - 1) return;
    const int P = blockIdx.y >> 1, hh = blockIdx.y & 1;  // depth-3 row of path P and context hh
    const cx<R>* sig2 = ws2 + (long long)blockIdx.z * N;
    const int a = __clz(~(p << (32 - LW6)));  // block of position p in the child rows' block layout
    const int j = p - (W6 - (W6 >> a));
    const int sp = W6 >> (a + 1);
    const int pm = p > 0 ? p - 1 : 0;
    cx<R> ext[8][3];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const cx<R>* row = sig2 + (2 * (8 * P + q) + (hh ^ (SW ? par(q) : 0))) * W6;
        const cx<R> lm = row[pm], lp = row[p + 1];
        ext[q][0] = j >= 1 ? lm : zero<R>();
        ext[q][1] = row[p];
        ext[q][2] = j + 1 < sp ? lp : zero<R>();
    }
    cx<R>* out = ws1 + (long long)blockIdx.z * N + ((hh ^ (SW ? par(P) : 0)) * 8 + P) * W3 + (W3 - (W3 >> a)) + 8 * j;
    cx<R> o[8];
    if (hh == 0) bwd_run<V, 0, 3, R>(ext, o);
    else bwd_run<V, 1, 3, R>(ext, o);
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = o[e];
}

// B0 of one position p of the depth-3 block layout (block a, index j): the
// eight rows of each side at p - 1, p, p + 1 (neighbours outside the block
// count as zero) give harmonics 8j .. 8j + 7 of depth-0 block a of both sides.
// B0 (levels 2..0) of the group of depth-3 slot p of the sixteen rows: the
// eight harmonics per side it expands to.  ld(r, s) reads slot s of row
// (side, q) = r / 8, r % 8.  The neighbour slots p - 1, p + 1 are read always
// and discarded where the group has no neighbour in its block; OWN: such a
// discarded read goes to slot p instead (the in-place path, whose slots past
// a block's ends may belong to another workgroup).
template <int V, typename R, int LOGN, bool OWN = false, typename LD>
__device__ __forceinline__ void b0_group(LD&& ld, int p, cx<R> (&o)[2][8]) {
    constexpr int N = 1 << LOGN, W3 = N / 16, LW3 = ilog2c(W3);
    const int a = __clz(~(p << (32 - LW3)));  // block of position p in the row's block layout
    const int j = p - (W3 - (W3 >> a));
    const int sp = W3 >> (a + 1);
    const int pm = OWN ? (j >= 1 ? p - 1 : p) : (p > 0 ? p - 1 : 0);
    const int pp = OWN ? (j + 1 < sp ? p + 1 : p) : p + 1;
    cx<R> ext[2][8][3];
#pragma unroll
    for (int side = 0; side < 2; ++side)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int r = side * 8 + q;
            const cx<R> lm = ld(r, pm), lp = ld(r, pp);
            ext[side][q][0] = j >= 1 ? lm : zero<R>();
            ext[side][q][1] = ld(r, p);
            ext[side][q][2] = j + 1 < sp ? lp : zero<R>();
        }
    bwd_run<V, 0, 3, R>(ext[0], o[0]);
    bwd_run<V, 1, 3, R>(ext[1], o[1]);
}

// B0 into ws2 (depth-0 block layout per side) for the blocks a >= 3, which
// the chain reads at folded indices from every part of the signal, and for
// the 14 groups of blocks 0..2 that the harmonics N/16 i (thread k0 = 0 of
// the chain) read: block 0 at harmonics 0, N/16 i - 1, N/16 i (i = 1..3) and
// N/4 - 1; block 1 at 0, N/16 - 1, N/16, N/8 - 1; block 2 at 0, N/16 - 1.
template <int V, typename R, int LOGN>
__global__ __launch_bounds__(64) void amqft_kL_back(const cx<R>* __restrict__ ws1, cx<R>* __restrict__ ws2) {
    constexpr int N = 1 << LOGN, H = N / 2, W3 = N / 16, NB3 = W3 / 8 - 1, GA = N / 128;
    const int i = blockIdx.x * 64 + threadIdx.x;  // one-wave workgroups: few threads per signal
    if (i >= NB3 + 14) return;
    int p;
    if (i < NB3) {
        p = W3 - W3 / 8 + i;
    } else {
        const int x = i - NB3;
        const int a = x < 8 ? 0 : x < 12 ? 1 : 2;
        const int y = x - (x < 8 ? 0 : x < 12 ? 8 : 12);
        const int g = ((y + 1) >> 1) * GA - (y & 1);  // 0, GA - 1, GA, 2 GA - 1, 2 GA, ...
        p = W3 - (W3 >> a) + g;
    }
    constexpr int LW3 = ilog2c(W3);
    const int a = __clz(~(p << (32 - LW3)));
    const int j = p - (W3 - (W3 >> a));
    cx<R> o[2][8];
    const cx<R>* sig = ws1 + (long long)blockIdx.y * N;
    b0_group<V, R, LOGN>([&](int r, int q) { return sig[r * W3 + q]; }, p, o);
    cx<R>* out = ws2 + (long long)blockIdx.y * N + (H - (H >> a)) + 8 * j;
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = o[0][e];
#pragma unroll
    for (int e = 0; e < 8; ++e) out[H + e] = o[1][e];
}

// In place: the same groups read from the signal buffer x (slot s of row r at
// ip_member(r, orb[s])); blocks >= 3 -> ws2 at side H/8 + (block a of side 0
// at H/8 - H/2^a), the fourteen groups -> the one value of each that thread
// k0 = 0 reads (DCT side at element 0 of the even groups, DST side at element
// 7 of the odd ones) at ws2 + N/8; and the slots that two workgroups of the
// chain kernel read -> ws3, row-major (row r of shared slot k at r nsh + k, so
// that neighbouring shared slots are neighbouring words).
template <int V, typename R, int LOGN>
__global__ __launch_bounds__(64) void amqft_kL_back_ip(const cx<R>* x, cx<R>* __restrict__ ws2,
                                                        cx<R>* __restrict__ ws3, const int* __restrict__ iptab,
                                                        int nsh, long long sig0) {
    constexpr int N = 1 << LOGN, H = N / 2, W3 = N / 16, NB3 = W3 / 8 - 1, GA = N / 128;
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= NB3 + 14 + nsh) return;
    const long long sl = blockIdx.y;
    const cx<R>* sig = x + (sig0 + sl) * N;
    const int* orb = iptab;
    auto ld = [&](int r, int q) { return xld(sig + ip_member<LOGN>(r, orb[q])); };
    cx<R>* w2 = ws2 + sl * (N / 8 + 16);
    if (i >= NB3 + 14) {
        const int k = i - NB3 - 14, q = iptab[2 * W3 + k];
#pragma unroll
        for (int r = 0; r < 16; ++r) ws3[(sl * 16 + r) * nsh + k] = ld(r, q);
        return;
    }
    int p, y = 0;
    if (i < NB3) {
        p = W3 - W3 / 8 + i;
    } else {
        const int xg = i - NB3;
        const int a = xg < 8 ? 0 : xg < 12 ? 1 : 2;
        y = xg - (xg < 8 ? 0 : xg < 12 ? 8 : 12);
        const int g = ((y + 1) >> 1) * GA - (y & 1);
        p = W3 - (W3 >> a) + g;
    }
    cx<R> o[2][8];
    b0_group<V, R, LOGN, true>(ld, p, o);
    if (i < NB3) {
        constexpr int LW3 = ilog2c(W3);
        const int a = __clz(~(p << (32 - LW3)));
        const int j = p - (W3 - (W3 >> a));
        cx<R>* out = w2 + (H / 8 - (H >> a)) + 8 * j;
#pragma unroll
        for (int e = 0; e < 8; ++e) out[e] = o[0][e];
#pragma unroll
        for (int e = 0; e < 8; ++e) out[H / 8 + e] = o[1][e];
    } else {
        w2[N / 8 + i - NB3] = (y & 1) ? o[1][7] : o[0][0];
    }
}

// B0 for blocks 0..2 and the chain in one kernel.  Workgroup K/256 serves
// the chain threads k0 = K .. K + 255, whose harmonics in blocks 0..2 lie in
// seven windows of 34 groups of eight (block 0 at k0, N/8 - k0, N/8 + k0,
// N/4 - k0; block 1 at k0, N/8 - k0; block 2 at k0; the DST side one index
// lower); the workgroup runs B0 for those groups into LDS, then the chain
// reads them there and blocks >= 3 and the chain values from ws2 / wsc.
// Thread k0 = 0 (harmonics N/16 i) reads everything from ws2.
template <typename R>
constexpr size_t kL_bchain_lds() { return 2 * 7 * 34 * 8 * sizeof(cx<R>); }

// The kernel body; IP: the in-place path, where ws1 is the signal buffer
// itself (rows at member(r, orb[s]), the slots two workgroups read taken from
// ws3), ws2 holds only the blocks >= 3 of each side (H/8 values a side) and
// then the fourteen values thread k0 = 0 reads from blocks 0..2.
template <int V, typename S, int LOGN, bool IP>
__device__ __forceinline__ void kL_bchain_body(const cx<typename storage<S>::R>* ws1,
                                               const cx<typename storage<S>::R>* ws2,
                                               const cx<typename storage<S>::R>* ws3,
                                               const cx<typename storage<S>::R>* wsc, S* out, const int* iptab,
                                               int nsh, long long sig0, long long batch, int flags,
                                               const long long* offsets) {
    using R = typename storage<S>::R;
    constexpr int N = 1 << LOGN, H = N / 2, Q = N / 4, W3 = N / 16, N8 = N / 8, D = LOGN - 2;
    constexpr int NG = 34, NWIN = 7, WS = NG * 8, NW = D - 5;
    // ws2 per signal and the offset of block a of side s in it
    constexpr long long W2 = IP ? N / 8 + 16 : N;
    constexpr int GOFF = IP ? H - H / 8 : 0, SIDE2 = IP ? H / 8 : H;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<R>(*blk)[NWIN * WS] = reinterpret_cast<cx<R>(*)[NWIN * WS]>(smem);  // [side][slot]
    // Every workgroup of a signal reads the signal's blocks >= 3 (ws2) at
    // folded indices.  Workgroups are dealt to the eight XCDs (each with its
    // own L2) round-robin by launch order, so the launch order is remapped to
    // put all of a signal's workgroups on one XCD: ws2 then comes from HBM
    // once per signal rather than once per XCD.
    const unsigned gx = gridDim.x, total = gx * gridDim.y;
    unsigned lid = blockIdx.x + blockIdx.y * gx;
    if (total % 8 == 0) lid = (lid % 8) * (total / 8) + lid / 8;
    const int K = (int)(lid % gx) * 256, tid = threadIdx.x;
    const long long sl = lid / gx, gs = sig0 + sl;
    if (gs >= batch) return;
    // first group of window r (block 0: r = 0..3, block 1: r = 4, 5, block 2: r = 6)
    auto wg0 = [&](int r) {
        return (r == 0 || r == 4 || r == 6) ? K / 8 - 1
               : (r == 1 || r == 5)         ? (N8 - K) / 8 - 33
               : r == 2                     ? (N8 + K) / 8 - 1
                                            : (Q - K) / 8 - 33;
    };
    if (tid < NWIN * NG) {
        const int r = tid / NG;
        const int a = r < 4 ? 0 : r < 6 ? 1 : 2;
        const int g = wg0(r) + (tid - r * NG);
        if (g >= 0 && g < (W3 >> (a + 1))) {
            cx<R> o[2][8];
            if constexpr (IP) {
                const long long gsb = gs * (long long)N;
                const int* orb = iptab;
                const int* shx = iptab + W3;
                // one load a row through the selected address (no branch
                // around loads: those would wait for each other)
                b0_group<V, R, LOGN, true>(
                    [&](int r, int q) {
                        const int x = shx[q], ob = orb[q];
                        const cx<R>* src = x >= 0 ? ws3 + (sl * 16 + r) * nsh + x : ws1 + gsb + ip_member<LOGN>(r, ob);
                        return xld(src);
                    },
                    W3 - (W3 >> a) + g, o);
            } else {
                const cx<R>* sig = ws1 + sl * N;
                b0_group<V, R, LOGN>([&](int r, int q) { return sig[r * W3 + q]; }, W3 - (W3 >> a) + g, o);
            }
#pragma unroll
            for (int side = 0; side < 2; ++side)
#pragma unroll
                for (int e = 0; e < 8; ++e) stc(&blk[side][tid * 8 + e], o[side][e]);
        }
    }
    __syncthreads();
    const int k0 = K + tid;
    if (k0 >= W3) return;  // N < 2^12: fewer chain threads than the workgroup has
    const cx<R>* w2 = ws2 + sl * W2;
    const cx<R>* chn = wsc + sl * 16;
    cx<R> res[16];
    if (k0 == 0) {
        if constexpr (IP) {
            // blocks >= 3 at harmonic 0; blocks 0..2 at the harmonics N/16 i
            // (DCT side) and N/16 i - 1 (DST side), in the order the back
            // kernel stores them: block 0 i = 0..3 / 1..4, block 1 i = 0, 1 /
            // 1, 2, block 2 i = 0 / 1
            constexpr int N16 = N / 16;
            const cx<R>* z = w2 + N / 8;
            auto zb = [](int a) { return a == 0 ? 0 : a == 1 ? 8 : 12; };
            c0_zero<LOGN, R>(
                [&](int a, int k) { return a >= 3 ? w2[H / 8 - (H >> a) + k] : z[zb(a) + 2 * (k / N16)]; },
                [&](int a, int k) { return z[zb(a) + 2 * (k / N16) - 1]; }, chn[0], res);
        } else {
            c0_compute<LOGN, R, global_layout<LOGN>>(w2, chn, 0, res);
        }
    } else {
        // harmonic k of window r, side s
        auto lw = [&](int s, int r, int k) { return ldc(&blk[s][r * WS + k - 8 * wg0(r)]); };
        auto gb = [](int a) { return H - (H >> a) - GOFF; };  // block a of side 0 in ws2
        auto lo = [](cx<R> Cv, cx<R> Dv) { return cx<R>{Cv.re + Dv.im, Cv.im - Dv.re}; };
        auto hi = [](cx<R> Cv, cx<R> Dv) { return cx<R>{Cv.re - Dv.im, Cv.im + Dv.re}; };
        // the chain walk: folded indices and signs, as in the LDS kernel's C0
        int ic[NW], is[NW];
        R wc[NW], wsg[NW];
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
        cx<R> accs = ldc(chn + 8 + e8) * wd;
#pragma unroll
        for (int t = 0; t < NW; ++t) {
            const cx<R> o = ldc(w2 + SIDE2 + gb(3 + t) + is[t] - 1);
            accs = cx<R>{accs.re + wsg[t] * o.re, accs.im + wsg[t] * o.im};
        }
        cx<R> accc = ldc(chn + kc);
#pragma unroll
        for (int t = 0; t < NW; ++t) {
            const cx<R> o = ldc(w2 + gb(3 + t) + ic[t]);
            accc = cx<R>{accc.re + wc[t] * o.re, accc.im + wc[t] * o.im};
        }
        const int kA = k0, kB = N8 - k0, kC = kA + N8, kD = kB + N8;
        const cx<R> oc2 = lw(0, 6, kA);
        const cx<R> c2a = accc + oc2, c2b = accc - oc2;
        const cx<R> o1a = lw(0, 4, kA), o1b = lw(0, 5, kB);
        const cx<R> c1[4] = {c2a + o1a, c2b + o1b, c2b - o1b, c2a - o1a};
        const cx<R> o0[4] = {lw(0, 0, kA), lw(0, 1, kB), lw(0, 2, kC), lw(0, 3, kD)};
        cx<R> C[8];  // E_0 at kA, kB, kC, kD, H-kD, H-kC, H-kB, H-kA
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            C[i] = c1[i] + o0[i];
            C[7 - i] = c1[i] - o0[i];
        }
        const cx<R> os2 = lw(1, 6, kA - 1);
        const cx<R> s2a = os2 + accs, s2b = os2 - accs;
        const cx<R> p1a = lw(1, 4, kA - 1), p1b = lw(1, 5, kB - 1);
        const cx<R> s1[4] = {p1a + s2a, p1b + s2b, p1b - s2b, p1a - s2a};
        const cx<R> q0[4] = {lw(1, 0, kA - 1), lw(1, 1, kB - 1), lw(1, 2, kC - 1), lw(1, 3, kD - 1)};
        cx<R> Dd[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            Dd[i] = q0[i] + s1[i];
            Dd[7 - i] = q0[i] - s1[i];
        }
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
    }
    const long long base = uniform64(offsets ? offsets[gs] : gs * (long long)N);
    c0_store<LOGN, S, R, true>(out + base, k0, res, (flags & 2) != 0);
}

template <int V, typename S, int LOGN>
__global__ __launch_bounds__(256) void amqft_kL_bchain(const cx<typename storage<S>::R>* __restrict__ ws1,
                                                        const cx<typename storage<S>::R>* __restrict__ ws2,
                                                        const cx<typename storage<S>::R>* __restrict__ wsc,
                                                        S* __restrict__ out, long long sig0, long long batch, int flags,
                                                        const long long* __restrict__ offsets) {
    kL_bchain_body<V, S, LOGN, false>(ws1, ws2, nullptr, wsc, out, nullptr, 0, sig0, batch, flags, offsets);
}

// in place: x is read (rows) and written (the transform) by the same
// workgroup only, its reads before a barrier and its writes after
template <int V, typename S, int LOGN>
__global__ __launch_bounds__(256) void amqft_kL_bchain_ip(S* x, const cx<typename storage<S>::R>* __restrict__ ws2,
                                                           const cx<typename storage<S>::R>* __restrict__ ws3,
                                                           const cx<typename storage<S>::R>* __restrict__ wsc,
                                                           const int* __restrict__ iptab, int nsh, long long sig0,
                                                           long long batch, int flags) {
    using R = typename storage<S>::R;
    kL_bchain_body<V, S, LOGN, true>(reinterpret_cast<const cx<R>*>(x), ws2, ws3, wsc, x, iptab, nsh, sig0, batch,
                                     flags, nullptr);
}

// The in-place path (N/16 rows of depth 3; FP32 and FP64 storage): the
// signal buffer a.out (= a.in) holds the rows between the kernels; ws2 holds
// N/8 + 16 values a signal, ws3 16 per shared slot, wsc 16.
template <int V, typename S, int LOGN>
hipError_t launch_kL_ip_n(const kl_launch& a, hipStream_t st) {
    using R = typename storage<S>::R;
    constexpr int N = 1 << LOGN, W3 = N / 16, NB3 = W3 / 8 - 1;
    using GR = kgeo<LOGN - 3>;
    const int flags = (a.conj_in ? 1 : 0) | (a.conj_out ? 2 : 0);
    const size_t lds = kA_lds_bytes<R, LOGN - 3>();
    S* x = static_cast<S*>(a.out);
    cx<R>* ws2 = static_cast<cx<R>*>(a.ws2);
    cx<R>* ws3 = static_cast<cx<R>*>(a.ws3);
    cx<R>* wsc = static_cast<cx<R>*>(a.wsc);
    const R* kt = static_cast<const R*>(a.ktab);
    for (long long s0 = 0; s0 < a.batch; s0 += a.chunk) {
        const long long nb = a.batch - s0 < a.chunk ? a.batch - s0 : a.chunk;
        const dim3 gw((W3 + 255) / 256, (unsigned)nb);
        hipLaunchKernelGGL((amqft_kL_top_ip<V, S, LOGN>), gw, dim3(256), 0, st, x, wsc, kt, s0, (long long)a.batch,
                           flags);
        hipLaunchKernelGGL((amqft_kL_rows<V, R, LOGN, 3, true>), dim3(8 / GR::SPW, (unsigned)nb), dim3(GR::WG), lds, st,
                           reinterpret_cast<cx<R>*>(x + s0 * N), kt, a.iptab);
        hipLaunchKernelGGL((amqft_kL_back_ip<V, R, LOGN>), dim3((NB3 + 14 + a.ipnsh + 63) / 64, (unsigned)nb), dim3(64),
                           0, st, reinterpret_cast<const cx<R>*>(x), ws2, ws3, a.iptab, a.ipnsh, s0);
        hipLaunchKernelGGL((amqft_kL_bchain_ip<V, S, LOGN>), gw, dim3(256), kL_bchain_lds<R>(), st, x,
                           static_cast<const cx<R>*>(ws2), static_cast<const cx<R>*>(ws3),
                           static_cast<const cx<R>*>(wsc), a.iptab, a.ipnsh, s0, (long long)a.batch, flags);
    }
    return hipGetLastError();
}

template <int V, typename S, int LOGN>
hipError_t launch_kL_n(const kl_launch& a, hipStream_t st) {
    constexpr int DEP_ = (1 << LOGN) >= (1 << 18) ? 6 : 3;
    if constexpr (DEP_ == 3 && (std::is_same<S, float2>::value || std::is_same<S, double2>::value)) {
        if (a.inplace) return launch_kL_ip_n<V, S, LOGN>(a, st);
    } else {
        if (a.inplace) return hipErrorInvalidValue;
    }
    using R = typename storage<S>::R;
    constexpr int N = 1 << LOGN, W3 = N / 16;
    constexpr int DEP = LOGN >= 18 ? 6 : 3;  // depth of the rows that fit one workgroup's LDS
    using GR = kgeo<LOGN - DEP>;
    const int flags = (a.conj_in ? 1 : 0) | (a.conj_out ? 2 : 0);
    const size_t lds = kA_lds_bytes<R, LOGN - DEP>();
    cx<R>* ws1 = static_cast<cx<R>*>(a.ws1);
    cx<R>* ws2 = static_cast<cx<R>*>(a.ws2);
    cx<R>* wsc = static_cast<cx<R>*>(a.wsc);
    const R* kt = static_cast<const R*>(a.ktab);
    for (long long s0 = 0; s0 < a.batch; s0 += a.chunk) {
        const long long nb = a.batch - s0 < a.chunk ? a.batch - s0 : a.chunk;
        const dim3 gw((W3 + 255) / 256, (unsigned)nb);
        hipLaunchKernelGGL((amqft_kL_top<V, S, LOGN>), gw, dim3(256), 0, st, static_cast<const S*>(a.in), ws1, wsc, kt,
                           s0, (long long)a.batch, flags, static_cast<const long long*>(a.offsets));
        if constexpr (DEP == 3) {
            hipLaunchKernelGGL((amqft_kL_rows<V, R, LOGN, 3>), dim3(8 / GR::SPW, (unsigned)nb), dim3(GR::WG), lds, st, ws1,
                               kt, nullptr);
        } else {
            constexpr int W6 = N / 128;
            hipLaunchKernelGGL((amqft_kL_rtop<V, R, LOGN>), dim3(W6 / 256, 8, (unsigned)nb), dim3(256), 0, st, ws1, ws2,
                               kt);
            static_assert(GR::SPW == 1, "depth-6 rows are at least 2^12 points");
            hipLaunchKernelGGL((amqft_kL_rows<V, R, LOGN, 6>), dim3(64, (unsigned)nb), dim3(GR::WG), lds, st, ws2, kt,
                               nullptr);
            hipLaunchKernelGGL((amqft_kL_rback<V, R, LOGN>), dim3(W6 / 256, 16, (unsigned)nb), dim3(256), 0, st,
                               static_cast<const cx<R>*>(ws2), ws1);
        }
        const dim3 gb((W3 / 8 - 1 + 14 + 63) / 64, (unsigned)nb);
        hipLaunchKernelGGL((amqft_kL_back<V, R, LOGN>), gb, dim3(64), 0, st, static_cast<const cx<R>*>(ws1), ws2);
        hipLaunchKernelGGL((amqft_kL_bchain<V, S, LOGN>), gw, dim3(256), kL_bchain_lds<R>(), st, static_cast<const cx<R>*>(ws1),
                           static_cast<const cx<R>*>(ws2), static_cast<const cx<R>*>(wsc), static_cast<S*>(a.out), s0,
                           (long long)a.batch, flags, static_cast<const long long*>(a.offsets));
    }
    return hipGetLastError();
}

// 2^11 .. 2^14 (2^13 in FP64) fit one workgroup's LDS; the path runs there
// only when a plan forces it (tests of its kernels at sizes where every
// variant is accurate), for FP64 and FP32 storage
template <int V, typename S>
hipError_t launch_kL_s(const kl_launch& a, hipStream_t st) {
    if constexpr (std::is_same<S, double2>::value) {
        switch (a.logn) {
        case 11: return launch_kL_n<V, S, 11>(a, st);
        case 12: return launch_kL_n<V, S, 12>(a, st);
        case 13: return launch_kL_n<V, S, 13>(a, st);
        case 14: return launch_kL_n<V, S, 14>(a, st);
        case 15: return launch_kL_n<V, S, 15>(a, st);
        default: return launch_kL_n<V, S, 16>(a, st);
        }
    } else {
        if constexpr (std::is_same<S, float2>::value) {
            switch (a.logn) {
            case 11: return launch_kL_n<V, S, 11>(a, st);
            case 12: return launch_kL_n<V, S, 12>(a, st);
            case 13: return launch_kL_n<V, S, 13>(a, st);
            case 14: return launch_kL_n<V, S, 14>(a, st);
            default: break;
            }
        }
        if (a.logn < 15) return hipErrorInvalidValue;
        switch (a.logn) {
        case 15: return launch_kL_n<V, S, 15>(a, st);
        case 16: return launch_kL_n<V, S, 16>(a, st);
        case 17: return launch_kL_n<V, S, 17>(a, st);
        case 18: return launch_kL_n<V, S, 18>(a, st);
        case 19: return launch_kL_n<V, S, 19>(a, st);
        default: return launch_kL_n<V, S, 20>(a, st);
        }
    }
}

template <int V, typename R, int LOGN, int LMAX>
hipError_t prime_kL_n() {
    constexpr int DEP = LOGN >= 18 ? 6 : 3;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amqft_kL_rows<V, R, LOGN, DEP>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if constexpr (DEP == 3) {
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amqft_kL_rows<V, R, LOGN, 3, true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    }
    if constexpr (LOGN < LMAX) {
        if (e == hipSuccess) e = prime_kL_n<V, R, LOGN + 1, LMAX>();
    }
    return e;
}

}  // namespace

bool kA_supported(int variant, int logn, int dtype) {
    if (variant != 1 && variant != 4 && variant != 5 && variant != 8) return false;
    if (dtype == 0) return logn >= 8 && logn <= 13;
    // fixed point: the variants whose constants (2cos, 2sin) have a Q2.29 form
    if (dtype == 4) return (variant == 1 || variant == 5) && logn >= 8 && logn <= 14;
    return logn >= 8 && logn <= 14;  // FP32 arithmetic: FP32, FP16 and BF16 storage
}

template <int V>
static size_t kA_lds_v(int logn, int dtype) {
    switch (logn) {
    case 8: return dtype == 0 ? kA_lds_bytes_v<V, double, 8>() : kA_lds_bytes_v<V, float, 8>();
    case 9: return dtype == 0 ? kA_lds_bytes_v<V, double, 9>() : kA_lds_bytes_v<V, float, 9>();
    case 10: return dtype == 0 ? kA_lds_bytes_v<V, double, 10>() : kA_lds_bytes_v<V, float, 10>();
    case 11: return dtype == 0 ? kA_lds_bytes_v<V, double, 11>() : kA_lds_bytes_v<V, float, 11>();
    case 12: return dtype == 0 ? kA_lds_bytes_v<V, double, 12>() : kA_lds_bytes_v<V, float, 12>();
    case 13: return dtype == 0 ? kA_lds_bytes_v<V, double, 13>() : kA_lds_bytes_v<V, float, 13>();
    default: return dtype == 0 ? kA_lds_bytes_v<V, double, 14>() : kA_lds_bytes_v<V, float, 14>();
    }
}

size_t kA_lds(int variant, int logn, int dtype) {
    return (variant == 1 || variant == 5) ? kA_lds_v<1>(logn, dtype) : kA_lds_v<4>(logn, dtype);
}

void kA_shape(int logn, int dtype, int* threads, int* signals_per_wg, size_t* lds_bytes) {
    const int N = 1 << logn, T = N / 16, WG = T >= 256 ? T : logn <= 10 ? (T >= 64 ? T : 64) : 256;
    *threads = WG;
    *signals_per_wg = WG / T;
    size_t b = 0;
    switch (logn) {
    case 8: b = dtype == 0 ? kA_lds_bytes<double, 8>() : kA_lds_bytes<float, 8>(); break;
    case 9: b = dtype == 0 ? kA_lds_bytes<double, 9>() : kA_lds_bytes<float, 9>(); break;
    case 10: b = dtype == 0 ? kA_lds_bytes<double, 10>() : kA_lds_bytes<float, 10>(); break;
    case 11: b = dtype == 0 ? kA_lds_bytes<double, 11>() : kA_lds_bytes<float, 11>(); break;
    case 12: b = dtype == 0 ? kA_lds_bytes<double, 12>() : kA_lds_bytes<float, 12>(); break;
    case 13: b = dtype == 0 ? kA_lds_bytes<double, 13>() : kA_lds_bytes<float, 13>(); break;
    default: b = dtype == 0 ? kA_lds_bytes<double, 14>() : kA_lds_bytes<float, 14>(); break;
    }
    *lds_bytes = b;
}

template <int V>
static hipError_t prime_kA_v(int dtype) {
    constexpr bool LOSS = !variant_traits<V>::recurrence;  // the fused loss kernel: M4 / M8
    switch (dtype) {
    case 0: {
        const hipError_t e = prime_kA_n<V, double2, 8>();
        if constexpr (LOSS) return e == hipSuccess ? prime_kA_loss_n<V, double2, 8>() : e;
        return e;
    }
    case 1: {
        const hipError_t e = prime_kA_n<V, float2, 8>();
        if constexpr (LOSS) return e == hipSuccess ? prime_kA_loss_n<V, float2, 8>() : e;
        return e;
    }
    case 2: return prime_kA_n<V, __half2, 8>();
    case 4:
        if constexpr (V == 1 || V == 5) return prime_kA_n<V, int2, 8>();
        else return hipErrorInvalidValue;
    default: return prime_kA_n<V, bf16x2, 8>();
    }
}

hipError_t prime_kA(int variant, int dtype) {
    switch (variant) {
    case 1: return prime_kA_v<1>(dtype);
    case 4: return prime_kA_v<4>(dtype);
    case 5: return prime_kA_v<5>(dtype);
    case 8: return prime_kA_v<8>(dtype);
    default: return hipSuccess;
    }
}

bool kA_loss_supported(int variant, int logn, int dtype) {
    return (variant == 4 || variant == 8) && (dtype == 0 || dtype == 1) && kA_supported(variant, logn, dtype);
}

hipError_t launch_kA_loss(const loss_launch& a, hipStream_t st) {
    if (a.batch <= 0) return hipSuccess;
    if (a.variant == 4) return a.dtype == 0 ? launch_kA_loss_s<4, double2>(a, st) : launch_kA_loss_s<4, float2>(a, st);
    return a.dtype == 0 ? launch_kA_loss_s<8, double2>(a, st) : launch_kA_loss_s<8, float2>(a, st);
}

bool kL_supported(int variant, int logn, int dtype) {
    if (variant == 2 || variant == 6) return kLT_supported(variant, logn, dtype);
    if (variant != 4 && variant != 8) return false;
    if (dtype == 0) return logn >= 14 && logn <= 16;
    return logn >= 15 && logn <= 20;  // FP32 arithmetic: FP32, FP16 and BF16 storage
}

bool kL_supported_forced(int variant, int logn, int dtype) {
    if (variant == 2 || variant == 6) return kLT_supported_forced(variant, logn, dtype);
    if (variant != 4 && variant != 8) return false;
    if (dtype == 0) return logn >= 11 && logn <= 16;
    if (dtype == 1) return logn >= 11 && logn <= 20;
    return kL_supported(variant, logn, dtype);
}

bool kL_inplace_supported(int variant, int logn, int dtype, bool forced) {
    if (variant != 4 && variant != 8) return false;
    if (dtype == 0) return logn >= (forced ? 11 : 14) && logn <= 16;
    if (dtype == 1) return logn >= (forced ? 11 : 15) && logn <= 17;
    return false;  // FP16 / BF16 storage would round the rows kept in the buffer
}

size_t kL_ws_bytes_per_signal(int logn, int dtype) { return ((size_t)1 << logn) * (dtype == 0 ? 16 : 8); }

hipError_t prime_kL(int variant, int dtype) {
    if (variant == 2 || variant == 6) return prime_kLT(variant, dtype);
    // the rows kernels depend on the arithmetic type only (float for dtypes 1..3)
    if (variant == 4) return dtype == 0 ? prime_kL_n<4, double, 11, 16>() : prime_kL_n<4, float, 11, 20>();
    if (variant == 8) return dtype == 0 ? prime_kL_n<8, double, 11, 16>() : prime_kL_n<8, float, 11, 20>();
    return hipSuccess;
}

template <int V>
static hipError_t launch_kL_t(const kl_launch& a, hipStream_t st) {
    switch (a.dtype) {
    case 0: return launch_kL_s<V, double2>(a, st);
    case 1: return launch_kL_s<V, float2>(a, st);
    case 2: return launch_kL_s<V, __half2>(a, st);
    default: return launch_kL_s<V, bf16x2>(a, st);
    }
}

hipError_t launch_kL(const kl_launch& a, hipStream_t st) {
    if (a.batch <= 0) return hipSuccess;
    if (a.inplace && (a.in != a.out || !kL_inplace_supported(a.variant, a.logn, a.dtype, true)))
        return hipErrorInvalidValue;
    if (a.variant == 2 || a.variant == 6) return launch_kLT(a, st);
    if (a.variant == 4) return launch_kL_t<4>(a, st);
    return launch_kL_t<8>(a, st);
}

template <int V>
static hipError_t launch_kA_t(const lds_launch& a, hipStream_t st) {
    switch (a.dtype) {
    case 0: return launch_kA_s<V, double2>(a, st);
    case 1: return launch_kA_s<V, float2>(a, st);
    case 2: return launch_kA_s<V, __half2>(a, st);
    case 4:
        if constexpr (V == 1 || V == 5) return launch_kA_s<V, int2>(a, st);
        else return hipErrorInvalidValue;
    default: return launch_kA_s<V, bf16x2>(a, st);
    }
}

hipError_t launch_kA(const lds_launch& a, hipStream_t st) {
    if (a.batch <= 0) return hipSuccess;
    switch (a.variant) {
    case 1: return launch_kA_t<1>(a, st);
    case 4: return launch_kA_t<4>(a, st);
    case 5: return launch_kA_t<5>(a, st);
    default: return launch_kA_t<8>(a, st);
    }
}

}  // namespace amqft
