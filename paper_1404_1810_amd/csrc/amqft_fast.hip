// Fast LDS-resident AM-QFT for N = 64 .. 4096 with the geometry fixed at
// compile time.  Same layout and level functions as the generic engine
// (amqft_levels.h, with one pad slot per 16 points), but the recursion stops
// its level-synchronous passes at sub-blocks of 16 points: every such
// sub-block -- on each side the positions [16c, 16c + 16), c >= 1 -- is
// finished forward and backward in registers by one thread (amqft_leaf.h).
// Thread c = 0 of each side finishes the blocks of at most 8 points and the
// bottom four levels of the D_n / D_k chain in registers as well.
#include <algorithm>

#include "amqft_device.h"
#include "amqft_internal.h"
#include "amqft_leaf.h"
#include "amqft_levels.h"

namespace amqft {

using namespace lv;

namespace {

using AD = ad_pad16;

template <int V, int SG, typename R>
__device__ __forceinline__ void leaf16(cx<R>* v, const R* kt, int D) {
    if constexpr (variant_traits<V>::skel_a) leaf::ot<V, 16, SG, R>(v, kt, D);
    else leaf::to<V, 16, SG, R>(v, kt, D);
}

// blocks of 8, 4, 2, 1 points and the chain levels of periodization 4..32
// (positions [0, 16) of one side, plus the extra slot for the DCT side)
template <int V, typename R>
__device__ void small_blocks_and_chain(cx<R>* w, const R* kt, int D, int H, int side) {
    constexpr bool A = variant_traits<V>::skel_a;
    cx<R> u[16], t[16];
    const int off = side * H;
    for (int e = (side ? 1 : 0); e < 16; ++e) u[e] = w[AD::at(off + e)];
    cx<R> X = side == 0 ? w[AD::at(H)] : cx<R>{R(0), R(0)};
    if (side == 0) {
        if constexpr (A) {
            leaf::ot<V, 8, 0, R>(u + 8, kt, D);
            leaf::ot<V, 4, 0, R>(u + 4, kt, D);
            leaf::ot<V, 2, 0, R>(u + 2, kt, D);
            // dct[2] base, then D_n^F of dct[4], dct[8], dct[16], dct[32]
            const cx<R> e0 = u[0] + X, e1 = u[0] - X;
            u[0] = e0;
            X = e1;
#pragma unroll
            for (int q = 1; q <= 8; q *= 2) {
#pragma unroll
                for (int k = 0; k < 16; ++k) t[k] = u[k];
#pragma unroll
                for (int k = 0; k < q; ++k) {
                    t[k] = u[k] + u[q + k];
                    if (k > 0) t[2 * q - k] = u[k] - u[q + k];
                }
                t[q] = X;
                X = u[0] - u[q];
#pragma unroll
                for (int k = 0; k < 16; ++k) u[k] = t[k];
            }
        } else {
            // D_k^T of dct[32], dct[16], dct[8], dct[4]
#pragma unroll
            for (int q = 8; q >= 1; q /= 2) {
#pragma unroll
                for (int k = 0; k < 16; ++k) t[k] = u[k];
                t[0] = u[0] + X;
                t[q] = u[0] - X;
                const cx<R> xn = u[q];
#pragma unroll
                for (int n = 1; n < q; ++n) {
                    t[n] = u[n] + u[2 * q - n];
                    t[q + n] = u[n] - u[2 * q - n];
                }
                X = xn;
#pragma unroll
                for (int k = 0; k < 16; ++k) u[k] = t[k];
            }
            leaf::to<V, 8, 0, R>(u + 8, kt, D);
            leaf::to<V, 4, 0, R>(u + 4, kt, D);
            leaf::to<V, 2, 0, R>(u + 2, kt, D);
            // dct[2] base, then the harmonic interleave of dct[4] .. dct[32]
            const cx<R> e0 = u[0] + X, e1 = u[0] - X;
            u[0] = e0;
            X = e1;
#pragma unroll
            for (int q = 1; q <= 8; q *= 2) {
#pragma unroll
                for (int k = 0; k < 16; ++k) t[k] = u[k];
#pragma unroll
                for (int i = 0; i < q; ++i) {
                    t[2 * i] = u[i];
                    t[2 * i + 1] = u[q + i];
                }
#pragma unroll
                for (int k = 0; k < 16; ++k) u[k] = t[k];
            }
        }
        for (int e = 0; e < 16; ++e) w[AD::at(e)] = u[e];
        w[AD::at(H)] = X;
    } else {
        u[0] = cx<R>{R(0), R(0)};
        if constexpr (A) {
            leaf::ot<V, 8, 1, R>(u + 8, kt, D);
            leaf::ot<V, 4, 1, R>(u + 4, kt, D);
            leaf::ot<V, 2, 1, R>(u + 2, kt, D);
            // D_n^F of dst[8], dst[16], dst[32] (dst[4] is its own base)
#pragma unroll
            for (int q = 2; q <= 8; q *= 2) {
#pragma unroll
                for (int k = 0; k < 16; ++k) t[k] = u[k];
#pragma unroll
                for (int k = 1; k < q; ++k) {
                    t[k] = u[q + k - 1] + u[k];
                    t[2 * q - k] = u[q + k - 1] - u[k];
                }
                t[q] = u[2 * q - 1];
#pragma unroll
                for (int k = 0; k < 16; ++k) u[k] = t[k];
            }
        } else {
            // D_k^T of dst[32], dst[16], dst[8]
#pragma unroll
            for (int q = 8; q >= 2; q /= 2) {
#pragma unroll
                for (int k = 0; k < 16; ++k) t[k] = u[k];
#pragma unroll
                for (int n = 1; n < q; ++n) {
                    t[n] = u[n] - u[2 * q - n];
                    t[q + n - 1] = u[n] + u[2 * q - n];
                }
                t[2 * q - 1] = u[q];
#pragma unroll
                for (int k = 0; k < 16; ++k) u[k] = t[k];
            }
            leaf::to<V, 8, 1, R>(u + 8, kt, D);
            leaf::to<V, 4, 1, R>(u + 4, kt, D);
            leaf::to<V, 2, 1, R>(u + 2, kt, D);
#pragma unroll
            for (int q = 2; q <= 8; q *= 2) {
#pragma unroll
                for (int k = 0; k < 16; ++k) t[k] = u[k];
#pragma unroll
                for (int i = 0; i < q; ++i) {
                    if (i > 0) t[2 * i] = u[i];
                    t[2 * i + 1] = u[q + i];
                }
#pragma unroll
                for (int k = 0; k < 16; ++k) u[k] = t[k];
            }
        }
        for (int e = 1; e < 16; ++e) w[AD::at(off + e)] = u[e];
    }
}

template <int V, typename R>
__device__ void leaf_pass(cx<R>* w, const R* kt, int ltid, int T, int D, int H) {
    constexpr bool SW = variant_traits<V>::switches;
    const int half = T >> 1;  // chunks per side
    const int side = ltid >= half;
    const int c = ltid - side * half;
    if (c == 0) {
        small_blocks_and_chain<V, R>(w, kt, D, H, side);
    } else {
        const int p0 = c << 4;
        const int Mb = 1 << (31 - __clz(p0));
        const int P = (p0 - Mb) >> 4;
        const int sigma = side ^ (SW ? (__popc(P) & 1) : 0);
        const int base = side * H + p0;
        cx<R> v[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = w[AD::at(base + e)];
        if (sigma == 0) leaf16<V, 0, R>(v, kt, D);
        else leaf16<V, 1, R>(v, kt, D);
#pragma unroll
        for (int e = 0; e < 16; ++e) w[AD::at(base + e)] = v[e];
    }
    __syncthreads();
}

template <int V, typename S, int LOGN>
__global__ __launch_bounds__(256) void amqft_fast_kernel(const S* __restrict__ in, S* __restrict__ out,
                                                          const typename storage<S>::R* __restrict__ ktab,
                                                          long long batch, int kshift, int flags,
                                                          const long long* __restrict__ offsets) {
    using R = typename storage<S>::R;
    using VT = variant_traits<V>;
    constexpr int N = 1 << LOGN, H = N / 2, D = LOGN - 2, Q = 1 << D;
    constexpr int T = N / 16;            // 16-point chunks of both sides
    constexpr int SPW = 256 / T;         // signals per workgroup
    constexpr int LW = N + N / 16;       // padded signal region
    constexpr int LMAX = D - 4;          // last level with sub-blocks above 16 points
    extern __shared__ __align__(16) unsigned char smem[];
    const bool conj_in = flags & 1, conj_out = flags & 2, onthefly = flags & 4;
    const int slot = threadIdx.x / T;
    const int ltid = threadIdx.x - slot * T;
    const long long sig = (long long)blockIdx.x * SPW + slot;
    const bool valid = sig < batch;
    R* kt = reinterpret_cast<R*>(smem);
    constexpr size_t kt_bytes = ((size_t)Q * sizeof(R) + 15) & ~(size_t)15;
    cx<R>* w = reinterpret_cast<cx<R>*>(smem + kt_bytes) + (size_t)slot * (LW + T);
    cx<R>* scr = w + LW;
    const long long base = valid ? (offsets ? offsets[sig] : sig * (long long)N) : 0;

    load_constants<V, R>(kt, ktab, Q, kshift, onthefly, LOGN);
    load_signal<VT::skel_a, S, R, AD>(w, in + base, ltid, T, D, H, conj_in, valid);
    __syncthreads();
    if constexpr (VT::skel_a) {
#pragma unroll 1
        for (int l = 0; l < LMAX; ++l) a_fwd_level<V, R, AD>(w, kt, ltid, T, D, H, l, 4);
        leaf_pass<V, R>(w, kt, ltid, T, D, H);
#pragma unroll 1
        for (int l = LMAX - 1; l >= 0; --l) {
            if constexpr (VT::recurrence) a_bwd_scan_level<V, R, AD>(w, scr, ltid, T, D, H, l, 4);
            else a_bwd_level<V, R, AD>(w, ltid, T, D, H, l, 4);
        }
        a_chain<R, AD>(w, ltid, T, D, H, LMAX, false);
    } else {
        b_chain_fwd<R, AD>(w, ltid, T, D, H, LMAX);
#pragma unroll 1
        for (int l = 0; l < LMAX; ++l) {
            if constexpr (VT::recurrence) b_fwd_scan_level<V, R, AD>(w, scr, ltid, T, D, H, l, 4);
            else b_fwd_level<V, R, AD>(w, ltid, T, D, H, l, 4);
        }
        leaf_pass<V, R>(w, kt, ltid, T, D, H);
#pragma unroll 1
        for (int l = LMAX - 1; l >= 0; --l) b_bwd_level<V, R, AD>(w, kt, ltid, T, D, H, l, 4);
        b_chain_bwd<R, AD>(w, ltid, T, D, H, LMAX, false);
    }
    store_signal<S, R, AD>(w, out + base, ltid, T, H, conj_out, valid);
}

template <int V, typename S, int LOGN>
hipError_t launch_fast_n(const lds_launch& a, hipStream_t st) {
    using R = typename storage<S>::R;
    constexpr int N = 1 << LOGN, T = N / 16, SPW = 256 / T, Q = N / 4;
    constexpr size_t kt_bytes = ((size_t)Q * sizeof(R) + 15) & ~(size_t)15;
    constexpr size_t lds = kt_bytes + (size_t)SPW * (N + N / 16 + T) * sizeof(cx<R>);
    const int flags = (a.conj_in ? 1 : 0) | (a.conj_out ? 2 : 0) | (a.onthefly ? 4 : 0);
    const long long grid = (a.batch + SPW - 1) / SPW;
    hipLaunchKernelGGL((amqft_fast_kernel<V, S, LOGN>), dim3((unsigned)grid), dim3(256), lds, st,
                       static_cast<const S*>(a.in), static_cast<S*>(a.out), static_cast<const R*>(a.ktab),
                       (long long)a.batch, a.ktab_log2n - LOGN, flags, static_cast<const long long*>(a.offsets));
    return hipGetLastError();
}

template <int V, typename S>
hipError_t launch_fast_s(const lds_launch& a, hipStream_t st) {
    switch (a.logn) {
    case 6: return launch_fast_n<V, S, 6>(a, st);
    case 7: return launch_fast_n<V, S, 7>(a, st);
    case 8: return launch_fast_n<V, S, 8>(a, st);
    case 9: return launch_fast_n<V, S, 9>(a, st);
    case 10: return launch_fast_n<V, S, 10>(a, st);
    case 11: return launch_fast_n<V, S, 11>(a, st);
    default: return launch_fast_n<V, S, 12>(a, st);
    }
}

template <int V>
hipError_t launch_fast_v(const lds_launch& a, hipStream_t st) {
    if (a.dtype == 0) return launch_fast_s<V, double2>(a, st);
    return launch_fast_s<V, float2>(a, st);
}

}  // namespace

template <int V, typename S, int LOGN>
static hipError_t prime_fast_n() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amqft_fast_kernel<V, S, LOGN>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess || LOGN == 12) return e;
    return prime_fast_n<V, S, (LOGN < 12 ? LOGN + 1 : 12)>();
}

template <int V>
static hipError_t prime_fast_v(int dtype) {
    if (dtype == 0) return prime_fast_n<V, double2, 6>();
    if (dtype == 1) return prime_fast_n<V, float2, 6>();
    return hipSuccess;
}

hipError_t prime_fast(int variant, int dtype) {
    switch (variant) {
    case 1: return prime_fast_v<1>(dtype);
    case 2: return prime_fast_v<2>(dtype);
    case 3: return prime_fast_v<3>(dtype);
    case 4: return prime_fast_v<4>(dtype);
    case 5: return prime_fast_v<5>(dtype);
    case 6: return prime_fast_v<6>(dtype);
    case 7: return prime_fast_v<7>(dtype);
    default: return prime_fast_v<8>(dtype);
    }
}

void fast_shape(int logn, int dtype, int* threads, int* spw, size_t* lds_bytes) {
    const int N = 1 << logn, T = N / 16, Q = N / 4;
    const size_t r = dtype == 0 ? 8 : 4;
    *threads = 256;
    *spw = 256 / T;
    *lds_bytes = ((Q * r + 15) & ~(size_t)15) + (size_t)(256 / T) * (N + N / 16 + T) * 2 * r;
}

bool fast_supported(int logn, int dtype) { return logn >= 6 && logn <= 12 && (dtype == 0 || dtype == 1); }

hipError_t launch_fast(const lds_launch& a, hipStream_t st) {
    if (a.batch <= 0) return hipSuccess;
    switch (a.variant) {
    case 1: return launch_fast_v<1>(a, st);
    case 2: return launch_fast_v<2>(a, st);
    case 3: return launch_fast_v<3>(a, st);
    case 4: return launch_fast_v<4>(a, st);
    case 5: return launch_fast_v<5>(a, st);
    case 6: return launch_fast_v<6>(a, st);
    case 7: return launch_fast_v<7>(a, st);
    default: return launch_fast_v<8>(a, st);
    }
}

}  // namespace amqft
