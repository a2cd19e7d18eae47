// Multi-pass AM-QFT for signals larger than one workgroup's LDS.
//
// The signal lives in a global workspace with the same layout as the LDS
// engine (amqft_levels.h).  Chain blocks bigger than S = 2^sb points run their
// top recursion levels as position-parallel "gather" kernels (each output
// element computed from the level's inputs; ping-pong between two buffers;
// positions a level does not touch are copied).  Once every big block has
// been split into sub-blocks of S points, the sub-blocks -- independent
// dct_ot/dst_ot (or dct_to/dst_to) problems -- are finished by the LDS engine,
// two per workgroup, and so is the tail of the chain (all blocks of at most S
// points), which occupies positions [0, 2S) of each side exactly as a whole
// signal of 4S points would.  The upper chain levels and the D_c combine
// run as gather kernels again.
#include "amqft_device.h"
#include "amqft_internal.h"
#include "amqft_levels.h"

namespace amqft {

using namespace lv;

namespace {

enum { K_A_FWD = 0, K_A_BWD, K_B_FWD, K_B_BWD, K_A_CHAIN, K_B_CHAIN_FWD, K_B_CHAIN_BWD };

struct mp_geo {
    int logn, D, H, sb;
};

// sub-block of an active big block containing side position p (p >= 2), depth l
struct sub {
    int base, s, h, u, hb, P, sigma;
};

__device__ __forceinline__ sub locate(int p, int l, int side, bool sw) {
    sub r;
    const int bp = 31 - __clz(p);  // block of size 2^bp at [2^bp, 2^(bp+1))
    const int Mb = 1 << bp;
    const int sl = bp - l;         // log2 of the sub-block size
    r.s = 1 << sl;
    r.h = r.s >> 1;
    r.hb = sl - 1;
    r.P = (p - Mb) >> sl;
    r.u = (p - Mb) & (r.s - 1);
    r.base = Mb + r.P * r.s;
    r.sigma = side ^ (sw ? (__popc(r.P) & 1) : 0);
    return r;
}

// ---------------------------------------------------------------------------
// position-parallel level kernel: dst[p] for every position of every signal
// ---------------------------------------------------------------------------
template <int V, int KIND, typename R>
__global__ __launch_bounds__(256) void mp_level_kernel(const cx<R>* __restrict__ src, cx<R>* __restrict__ dst,
                                                       const cx<R>* __restrict__ tmp, const R* __restrict__ kt,
                                                       int logn, int sb, int lev, long long nsig) {
    constexpr bool SW = variant_traits<V>::switches;
    const int N = 1 << logn, H = N >> 1, D = logn - 2;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nsig * N) return;
    const long long sig = gid >> logn;
    const int pos = (int)(gid & (N - 1));
    const cx<R>* s = src + sig * N;
    const cx<R>* tp = tmp + sig * N;
    const int side = pos >= H;
    const int p = pos - side * H;
    const int off = side * H;
    cx<R> out = s[pos];

    if constexpr (KIND == K_A_FWD || KIND == K_A_BWD || KIND == K_B_FWD || KIND == K_B_BWD) {
        if (p >= (2 << (sb + lev))) {
            const sub b = locate(p, lev, side, SW);
            const int kpos = off + b.base;
            if constexpr (KIND == K_A_FWD) {
                // D_k^T and M^T (M1, M4, M5, M8) of dct_ot / dst_ot
                const int i = b.u < b.h ? b.u : b.u - b.h;
                const cx<R> xa = s[kpos + i], xb = s[kpos + b.s - 1 - i];
                if (b.u < b.h) {
                    out = (b.sigma == 0) ? xa + xb : xa - xb;
                } else {
                    const cx<R> hi = (b.sigma == 0) ? xa - xb : xa + xb;
                    out = hi * kt[kidx(i, b.hb, D)];
                }
            } else if constexpr (KIND == K_B_BWD) {
                // M^F (M2, M3, M6, M7) and D_n^F of dct_to / dst_to
                const int i = b.u < b.h ? b.u : b.s - 1 - b.u;
                const cx<R> e = s[kpos + i];
                const cx<R> O = s[kpos + b.h + i] * kt[kidx(i, b.hb, D)];
                if (b.u < b.h) out = (b.sigma == 0) ? e + O : O + e;
                else out = (b.sigma == 0) ? e - O : O - e;
            } else if constexpr (KIND == K_A_BWD) {
                const int j = b.u >> 1, par = b.u & 1;
                const bool lo_slot = (b.sigma == 0) ? (par == 0) : (par == 1);
                if (lo_slot) {
                    out = s[kpos + j];
                } else if constexpr (variant_traits<V>::recurrence) {
                    out = tp[kpos + b.h + j];  // M1 / M5 recurrence, from the scan kernel
                } else {
                    const cx<R> f = s[kpos + b.h + j];
                    bool up = (V == 4) ? (b.sigma == 0) : (b.sigma != 0);
                    const int jn = up ? j + 1 : j - 1;
                    const cx<R> fn = (jn >= 0 && jn < b.h) ? s[kpos + b.h + jn] : cx<R>{R(0), R(0)};
                    out = (V == 4) ? f + fn : f - fn;
                }
            } else {  // K_B_FWD
                const bool dctc = (b.sigma == 0);
                if (b.u < b.h) {
                    const int i = b.u;
                    out = s[kpos + (dctc ? 2 * i : 2 * i + 1)];
                } else if constexpr (variant_traits<V>::recurrence) {
                    out = tp[kpos + b.u];  // M3 / M7 recurrence, from the scan kernel
                } else {
                    const int i = b.u - b.h;
                    const cx<R> xo = s[kpos + (dctc ? 2 * i + 1 : 2 * i)];
                    bool up = (V == 2) ? !dctc : dctc;
                    const int in = up ? i + 1 : i - 1;
                    const cx<R> xn = (in >= 0 && in < b.h) ? s[kpos + (dctc ? 2 * in + 1 : 2 * in)]
                                                          : cx<R>{R(0), R(0)};
                    out = (V == 2) ? xo + xn : xo - xn;
                }
            }
        }
    } else if constexpr (KIND == K_A_CHAIN) {
        // D_n^F of dct[L] / dst[L] at chain level lev, q = 2^(D-lev)
        const int q = 1 << (D - lev);
        if (side == 0 && p < 2 * q) {
            if (p < q) out = s[p] + s[q + p];
            else if (p == q) out = s[H];
            else out = s[2 * q - p] - s[q + 2 * q - p];
        } else if (side == 1 && p == 0) {
            out = s[0] - s[q];  // S(L/2) of the DCT chain in the extra slot
        } else if (side == 1 && p < 2 * q) {
            if (p < q) out = s[H + q + p - 1] + s[H + p];
            else if (p == q) out = s[H + 2 * q - 1];
            else { const int k = 2 * q - p; out = s[H + q + k - 1] - s[H + k]; }
        }
    } else if constexpr (KIND == K_B_CHAIN_FWD) {
        // D_k^T of dct[L] / dst[L] at chain level lev
        const int q = 1 << (D - lev);
        if (side == 0 && p < 2 * q) {
            const int n = p < q ? p : p - q;
            const cx<R> a = s[n], bb = (n == 0) ? s[H] : s[2 * q - n];
            out = (p < q) ? a + bb : a - bb;
        } else if (side == 1 && p == 0) {
            out = s[q];  // e(q) = s(q) of the DCT chain
        } else if (side == 1 && p < 2 * q) {
            if (p < q) out = s[H + p] - s[H + 2 * q - p];
            else if (p < 2 * q - 1) { const int n = p - q + 1; out = s[H + n] + s[H + 2 * q - n]; }
            else out = s[H + q];
        }
    } else if constexpr (KIND == K_B_CHAIN_BWD) {
        const int q = 1 << (D - lev);
        if (p < 2 * q && !(side == 1 && p == 0)) {
            if ((p & 1) == 0) out = s[off + p / 2];
            else out = s[off + q + (p - 1) / 2];
        }
    }
    dst[sig * N + pos] = out;
}

// ---------------------------------------------------------------------------
// recurrences of M1/M5 (skeleton A backward) and M3/M7 (skeleton B forward)
// over the hi halves of the active big sub-blocks: one workgroup per segment.
// Y_r = a_r + c Y_{r-1} along the recurrence direction (c = +-1) in tiles of
// 256 K values: coalesced loads into LDS, K consecutive values a thread,
// the carries of the threads by a workgroup prefix sum (K is even, so a
// chunk's carry passes through with weight c^K = 1), coalesced stores from
// LDS; the last value of a tile carries into the next.
// ---------------------------------------------------------------------------
constexpr int kScanK = 8, kScanT = 256;

// exclusive prefix sum of v over the workgroup's 256 threads; total: the sum
template <typename R>
__device__ __forceinline__ cx<R> wg_excl_sum(cx<R> v, cx<R>* wsum, int tid, cx<R>& total) {
    const int lane = tid & 63, wave = tid >> 6;
    cx<R> incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const cx<R> u = shfl_up_cx(incl, d);
        if (lane >= d) incl = incl + u;
    }
    if (lane == 63) stc(wsum + wave, incl);
    __syncthreads();
    cx<R> before = {R(0), R(0)}, all = {R(0), R(0)};
#pragma unroll
    for (int w = 0; w < kScanT / 64; ++w) {
        const cx<R> t = ldc(wsum + w);
        if (w < wave) before = before + t;
        all = all + t;
    }
    __syncthreads();
    total = all;
    return before + incl - v;
}

template <int V, bool SKEL_A, typename R>
__global__ __launch_bounds__(kScanT) void mp_scan_kernel(const cx<R>* __restrict__ src, cx<R>* __restrict__ tmp,
                                                         int logn, int sb, int lev, int nseg_side) {
    constexpr R c = R(variant_traits<V>::sign);
    constexpr bool SW = variant_traits<V>::switches;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<R>* tile = reinterpret_cast<cx<R>*>(smem);  // kScanT * kScanK values, then the wave sums
    cx<R>* wsum = tile + kScanT * kScanK;
    const int N = 1 << logn, H = N >> 1, D = logn - 2;
    const long long sig = blockIdx.y;
    int sidx = blockIdx.x;
    const int side = sidx >= nseg_side;
    sidx -= side * nseg_side;
    const int j = sidx >> lev;              // block index, block size 2^(D-j)
    const int P = sidx & ((1 << lev) - 1);  // sub-block path
    const int Mb = 1 << (D - j);
    const int s = Mb >> lev, h = s >> 1;
    const int base = side * H + Mb + P * s;
    const int sigma = side ^ (SW ? (__popc(P) & 1) : 0);
    const cx<R>* x = src + sig * N;
    cx<R>* y = tmp + sig * N;
    bool fwd;
    if (SKEL_A) fwd = (V == 1) ? (sigma == 0) : (sigma != 0);
    else fwd = (V == 3) ? (sigma != 0) : (sigma == 0);
    const bool dctc = (sigma == 0);
    // position of the r-th value along the recurrence direction
    auto idx = [&](int r) { return fwd ? r : h - 1 - r; };
    auto val = [&](int r) -> cx<R> {
        const int i = idx(r);
        cx<R> a = SKEL_A ? x[base + h + i] : x[base + (dctc ? 2 * i + 1 : 2 * i)];
        if (SKEL_A && r == 0) a = a * R(0.5);
        return a;
    };
    const int tid = threadIdx.x;
    const int K = h < kScanK ? h : kScanK;           // values a thread (even: h >= 2)
    const int TS = h < kScanT * K ? h : kScanT * K;  // values a tile
    cx<R> carry = {R(0), R(0)};                     // Y before the tile
    for (int t0 = 0; t0 < h; t0 += TS) {
        for (int u = tid; u < TS; u += kScanT) stc(tile + u, val(t0 + u));
        __syncthreads();
        const bool part = tid * K < TS;
        cx<R> Y = {R(0), R(0)};
        if (part)
            for (int k = 0; k < K; ++k) Y = ldc(tile + tid * K + k) + Y * c;
        cx<R> total;
        const cx<R> before = wg_excl_sum(part ? Y : cx<R>{R(0), R(0)}, wsum, tid, total);
        if (part) {
            Y = carry + before;
            for (int k = 0; k < K; ++k) {
                Y = ldc(tile + tid * K + k) + Y * c;
                stc(tile + tid * K + k, Y);
            }
        }
        carry = carry + total;
        __syncthreads();
        for (int u = tid; u < TS; u += kScanT) {
            const int r = t0 + u;
            cx<R> o = ldc(tile + u);
            if (!SKEL_A && r == h - 1) o = o * R(0.5);
            y[base + h + idx(r)] = o;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// LDS tasks: a workgroup finishes either two big sub-blocks of S points (the
// one in the DCT context in region 0, the other in region 1, both at
// [S, 2S)) or the tail [0, 2S) of both sides, on a virtual signal of 4S points
// ---------------------------------------------------------------------------
template <int V, typename R>
__global__ __launch_bounds__(1024) void mp_lds_kernel(cx<R>* __restrict__ ws, const R* __restrict__ ktab, int logn,
                                                      int sb, int kshift, int ntask, int onthefly) {
    using VT = variant_traits<V>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = 1 << logn, H = N >> 1, D = logn - 2;
    const int S = 1 << sb;
    const int Dv = sb, Hv = 2 * S, Qv = S, Nv = 4 * S;
    const int T = blockDim.x;
    const int tid = threadIdx.x;
    const long long sig = blockIdx.y;
    const int task = blockIdx.x;
    R* kt = reinterpret_cast<R*>(smem);
    const size_t kt_bytes = ((size_t)Qv * sizeof(R) + 15) & ~(size_t)15;
    cx<R>* w = reinterpret_cast<cx<R>*>(smem + kt_bytes);
    cx<R>* scr = w + Nv;
    cx<R>* g = ws + sig * N;
    load_constants<V, R>(kt, ktab, Qv, kshift, onthefly != 0, sb + 2);
    const bool tail = (task == ntask - 1);
    int gpos[2] = {0, 0};  // start of the sub-block in region 0 / 1 (type a)
    if (tail) {
        for (int v = tid; v < 2 * S; v += T) {
            w[v] = g[v];
            w[Hv + v] = g[H + v];
        }
    } else {
        // task -> (block j, path P): block j has 2^(D-sb-j) sub-blocks
        int t = task, j = 0;
        while (t >= (1 << (D - sb - j))) { t -= 1 << (D - sb - j); ++j; }
        const int P = t;
        const int Mb = 1 << (D - j);
        const int par = VT::switches ? (__popc(P) & 1) : 0;
        // side 0 sub-block has context par, side 1 has 1 - par
        gpos[par] = Mb + P * S;
        gpos[1 - par] = H + Mb + P * S;
        for (int v = tid; v < S; v += T) {
            w[S + v] = g[gpos[0] + v];
            w[Hv + S + v] = g[gpos[1] + v];
            w[v] = cx<R>{R(0), R(0)};
            w[Hv + v] = cx<R>{R(0), R(0)};
        }
    }
    __syncthreads();
    if (tail) {
        core<V, R>(w, kt, scr, tid, T, Dv, Hv);
    } else if constexpr (VT::skel_a) {
        // only the virtual signal's top block [S, 2S) of each side holds the
        // sub-block; the levels skip the smaller (zero) blocks: at level l
        // that block's sub-blocks have half-size 2^(sb - 1 - l)
        // (the scan levels give each of the T = 2^(sb-2) threads four of the
        // top block's 2^sb items, so that every thread has work)
        for (int l = 0; l < Dv; ++l) a_fwd_level<V, R>(w, kt, tid, T, Dv, Hv, l, Dv - 1 - l);
        for (int l = Dv - 1; l >= 0; --l) {
            if constexpr (VT::recurrence) a_bwd_scan_level<V, R, ad_identity, 4, true>(w, scr, tid, T, Dv, Hv, l, Dv - 1 - l);
            else a_bwd_level<V, R>(w, tid, T, Dv, Hv, l, Dv - 1 - l);
        }
    } else {
        for (int l = 0; l < Dv; ++l) {
            if constexpr (VT::recurrence) b_fwd_scan_level<V, R, ad_identity, 4, true>(w, scr, tid, T, Dv, Hv, l, Dv - 1 - l);
            else b_fwd_level<V, R>(w, tid, T, Dv, Hv, l, Dv - 1 - l);
        }
        for (int l = Dv - 1; l >= 0; --l) b_bwd_level<V, R>(w, kt, tid, T, Dv, Hv, l, Dv - 1 - l);
    }
    if (tail) {
        for (int v = tid; v < 2 * S; v += T) {
            g[v] = w[v];
            g[H + v] = w[Hv + v];
        }
    } else {
        for (int v = tid; v < S; v += T) {
            g[gpos[0] + v] = w[S + v];
            g[gpos[1] + v] = w[Hv + S + v];
        }
    }
}

// load with D_c/D_r (placement of skeleton A or natural order of B)
template <bool SKEL_A, typename S>
__global__ __launch_bounds__(256) void mp_load_kernel(const S* __restrict__ in, cx<typename storage<S>::R>* __restrict__ ws,
                                                      int logn, long long nsig, int conj,
                                                      const long long* __restrict__ offsets) {
    using R = typename storage<S>::R;
    const int N = 1 << logn, H = N >> 1, D = logn - 2;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nsig * H) return;
    const long long sig = gid / H;
    const int m = (int)(gid - sig * H);
    const S* x = in + (offsets ? offsets[sig] : sig * N);
    cx<R>* w = ws + sig * N;
    cx<R> a = storage<S>::ld(x + (m == 0 ? 0 : m));
    cx<R> b = storage<S>::ld(x + (m == 0 ? H : N - m));
    if (conj) { a = cconj(a); b = cconj(b); }
    if (m == 0) {
        w[0] = a;
        w[H] = b;
    } else {
        int pos = m;
        if (SKEL_A) {
            const int j = __ffs(m) - 1;
            pos = (1 << (D - j)) + (m >> (j + 1));
        }
        w[pos] = a + b;
        w[H + pos] = a - b;
    }
}

// D_c combine and store
template <typename S>
__global__ __launch_bounds__(256) void mp_store_kernel(const cx<typename storage<S>::R>* __restrict__ ws, S* __restrict__ out,
                                                       int logn, long long nsig, int conj,
                                                       const long long* __restrict__ offsets) {
    using R = typename storage<S>::R;
    const int N = 1 << logn, H = N >> 1;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nsig * H) return;
    const long long sig = gid / H;
    const int k = (int)(gid - sig * H);
    const cx<R>* w = ws + sig * N;
    S* y = out + (offsets ? offsets[sig] : sig * N);
    if (k == 0) {
        cx<R> a = w[0], b = w[H];
        if (conj) { a = cconj(a); b = cconj(b); }
        storage<S>::st(y, a);
        storage<S>::st(y + H, b);
    } else {
        const cx<R> C = w[k], Dd = w[H + k];
        cx<R> xk = {C.re + Dd.im, C.im - Dd.re};
        cx<R> xnk = {C.re - Dd.im, C.im + Dd.re};
        if (conj) { xk = cconj(xk); xnk = cconj(xnk); }
        storage<S>::st(y + k, xk);
        storage<S>::st(y + N - k, xnk);
    }
}

template <int V, int KIND, typename R>
hipError_t level(cx<R>*& a, cx<R>*& b, const cx<R>* tmp, const R* kt, int logn, int sb, int lev, long long nsig,
                 hipStream_t st) {
    const long long total = nsig << logn;
    const unsigned grid = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL((mp_level_kernel<V, KIND, R>), dim3(grid), dim3(256), 0, st, a, b, tmp, kt, logn, sb, lev,
                       nsig);
    std::swap(a, b);
    return hipGetLastError();
}

template <int V, typename R>
hipError_t scan(const cx<R>* a, cx<R>* tmp, int logn, int sb, int lev, long long nsig, hipStream_t st) {
    const int D = logn - 2;
    const int active = D - sb - lev;  // big blocks still splitting at this level
    const int nseg_side = active << lev;
    hipLaunchKernelGGL((mp_scan_kernel<V, variant_traits<V>::skel_a, R>), dim3(2 * nseg_side, (unsigned)nsig),
                       dim3(kScanT), (kScanT * kScanK + kScanT / 64) * sizeof(cx<R>), st, a, tmp, logn, sb, lev,
                       nseg_side);
    return hipGetLastError();
}

template <int V, typename S>
hipError_t run_typed(const mp_launch& m, hipStream_t st) {
    using R = typename storage<S>::R;
    using VT = variant_traits<V>;
    const int logn = m.logn, D = logn - 2, sb = m.sb;
    const int js = D - sb;  // chain levels above the tail (blocks bigger than S)
    const int Dv = sb;
    const int kshift = m.ktab_log2n - (sb + 2);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mp_lds_kernel<V, R>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int Tv = ((4 << sb) >> 4) > 1 ? ((4 << sb) >> 4) : 1;
    const size_t lds = ((((size_t)1 << Dv) * sizeof(R) + 15) & ~(size_t)15) +
                       ((size_t)(4 << sb) + Tv) * sizeof(cx<R>);
    const int ntask = (2 << (D - sb)) - 2 + 1;
    const R* kt = static_cast<const R*>(m.ktab);
    hipError_t e;
    for (long long s0 = 0; s0 < m.batch; s0 += m.chunk) {
        const long long ns = std::min<long long>(m.chunk, m.batch - s0);
        const long long* offs = m.offsets ? static_cast<const long long*>(m.offsets) + s0 : nullptr;
        const S* in = static_cast<const S*>(m.in) + (offs ? 0 : (s0 << logn));
        S* out = static_cast<S*>(m.out) + (offs ? 0 : (s0 << logn));
        cx<R>* a = static_cast<cx<R>*>(m.ws0);
        cx<R>* b = static_cast<cx<R>*>(m.ws1);
        cx<R>* tmp = static_cast<cx<R>*>(m.ws2);
        {
            const long long total = ns << (logn - 1);
            hipLaunchKernelGGL((mp_load_kernel<VT::skel_a, S>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                               st, in, a, logn, ns, m.conj_in, offs);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if constexpr (VT::skel_a) {
            for (int l = 0; l < js; ++l)
                if ((e = level<V, K_A_FWD, R>(a, b, tmp, kt, logn, sb, l, ns, st)) != hipSuccess) return e;
        } else {
            for (int j = 0; j < js; ++j)
                if ((e = level<V, K_B_CHAIN_FWD, R>(a, b, tmp, kt, logn, sb, j, ns, st)) != hipSuccess) return e;
            for (int l = 0; l < js; ++l) {
                if (VT::recurrence && (e = scan<V, R>(a, tmp, logn, sb, l, ns, st)) != hipSuccess) return e;
                if ((e = level<V, K_B_FWD, R>(a, b, tmp, kt, logn, sb, l, ns, st)) != hipSuccess) return e;
            }
        }
        hipLaunchKernelGGL((mp_lds_kernel<V, R>), dim3(ntask, (unsigned)ns), dim3(Tv), lds, st, a, kt, logn, sb,
                           kshift, ntask, m.onthefly);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if constexpr (VT::skel_a) {
            for (int l = js - 1; l >= 0; --l) {
                if (VT::recurrence && (e = scan<V, R>(a, tmp, logn, sb, l, ns, st)) != hipSuccess) return e;
                if ((e = level<V, K_A_BWD, R>(a, b, tmp, kt, logn, sb, l, ns, st)) != hipSuccess) return e;
            }
            for (int j = js - 1; j >= 0; --j)
                if ((e = level<V, K_A_CHAIN, R>(a, b, tmp, kt, logn, sb, j, ns, st)) != hipSuccess) return e;
        } else {
            for (int l = js - 1; l >= 0; --l)
                if ((e = level<V, K_B_BWD, R>(a, b, tmp, kt, logn, sb, l, ns, st)) != hipSuccess) return e;
            for (int j = js - 1; j >= 0; --j)
                if ((e = level<V, K_B_CHAIN_BWD, R>(a, b, tmp, kt, logn, sb, j, ns, st)) != hipSuccess) return e;
        }
        {
            const long long total = ns << (logn - 1);
            hipLaunchKernelGGL((mp_store_kernel<S>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a,
                               out, logn, ns, m.conj_out, offs);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

template <int V>
hipError_t run_v(const mp_launch& m, hipStream_t st) {
    switch (m.dtype) {
    case 0: return run_typed<V, double2>(m, st);
    case 1: return run_typed<V, float2>(m, st);
    case 2: return run_typed<V, __half2>(m, st);
    default: return run_typed<V, bf16x2>(m, st);
    }
}

}  // namespace

int multipass_sb(int dtype) { return dtype == 0 ? kMaxLdsLog2F64 - 2 : kMaxLdsLog2F32 - 2; }

size_t multipass_ws_bytes_per_signal(int logn, int dtype) {
    const size_t r = dtype == 0 ? 16 : 8;
    return ((size_t)1 << logn) * r;
}

template <int V>
static hipError_t prime_mp_v(int dtype) {
    const void* k = dtype == 0 ? reinterpret_cast<const void*>(&mp_lds_kernel<V, double>)
                               : reinterpret_cast<const void*>(&mp_lds_kernel<V, float>);
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

hipError_t prime_multipass(int variant, int dtype) {
    switch (variant) {
    case 1: return prime_mp_v<1>(dtype);
    case 2: return prime_mp_v<2>(dtype);
    case 3: return prime_mp_v<3>(dtype);
    case 4: return prime_mp_v<4>(dtype);
    case 5: return prime_mp_v<5>(dtype);
    case 6: return prime_mp_v<6>(dtype);
    case 7: return prime_mp_v<7>(dtype);
    default: return prime_mp_v<8>(dtype);
    }
}

hipError_t launch_multipass(const mp_launch& m, hipStream_t st) {
    if (m.batch <= 0) return hipSuccess;
    switch (m.variant) {
    case 1: return run_v<1>(m, st);
    case 2: return run_v<2>(m, st);
    case 3: return run_v<3>(m, st);
    case 4: return run_v<4>(m, st);
    case 5: return run_v<5>(m, st);
    case 6: return run_v<6>(m, st);
    case 7: return run_v<7>(m, st);
    default: return run_v<8>(m, st);
    }
}

}  // namespace amqft
