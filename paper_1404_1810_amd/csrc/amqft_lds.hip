// LDS-resident AM-QFT engine: one signal (or several short ones) per
// workgroup, the whole recursion of Sec. 4 and 6 flattened into
// level-synchronous passes over the signal held in LDS (layout and level
// functions in amqft_levels.h).
#include <stdio.h>

#include <algorithm>

#include "amqft_device.h"
#include "amqft_internal.h"
#include "amqft_levels.h"

namespace amqft {

using namespace lv;

// ---------------------------------------------------------------------------
// the kernel: blockDim.x = spw * T threads, spw signals per workgroup
// ---------------------------------------------------------------------------
template <int V, typename S>
__global__ __launch_bounds__(1024) void amqft_lds_kernel(const S* __restrict__ in, S* __restrict__ out,
                                                          const typename storage<S>::R* __restrict__ ktab,
                                                          int logn, long long batch, int kshift, int flags,
                                                          const long long* __restrict__ offsets) {
    using R = typename storage<S>::R;
    using VT = variant_traits<V>;
    extern __shared__ __align__(16) unsigned char smem[];
    const bool conj_in = flags & 1, conj_out = flags & 2, onthefly = flags & 4;
    const int N = 1 << logn;
    const int H = N >> 1;
    const int D = logn - 2;
    const int Q = 1 << D;
    const int T = (N >> 4) > 1 ? (N >> 4) : 1;
    const int spw = blockDim.x / T;
    const int slot = threadIdx.x / T;
    const int ltid = threadIdx.x - slot * T;
    const long long sig = (long long)blockIdx.x * spw + slot;
    const bool valid = sig < batch;
    R* kt = reinterpret_cast<R*>(smem);
    const size_t kt_bytes = ((size_t)Q * sizeof(R) + 15) & ~(size_t)15;
    cx<R>* w = reinterpret_cast<cx<R>*>(smem + kt_bytes) + (size_t)slot * (N + T);
    cx<R>* scr = w + N;
    const long long base = valid ? (offsets ? offsets[sig] : sig * (long long)N) : 0;
    const S* x = in + base;
    S* y = out + base;

    load_constants<V, R>(kt, ktab, Q, kshift, onthefly, logn);
    load_signal<VT::skel_a, S, R>(w, x, ltid, T, D, H, conj_in, valid);
    __syncthreads();
    core<V, R>(w, kt, scr, ltid, T, D, H);
    store_signal<S, R>(w, y, ltid, T, H, conj_out, valid);
}

// ---------------------------------------------------------------------------
// Real transforms on the same recursion (Sec. 3.1 and Sec. 7.4: the CDFT is
// D_c / D_r, a DCT-0 and a DST-0 and the combine; the RDFT, the DCT-0 and the
// DST-0 are that code minus some of these steps).  Since every coefficient of
// the recursion is real, a complex lane carries two real signals: slot s of
// the batch runs real signals 2s (real part) and 2s + 1 (imaginary part).
//   REAL_RDFT  in: n reals per signal; D_c / D_r, dct and dst, then
//              X(k) = C(k) - i D(k) for k = 0 .. n/2: n/2 + 1 complex out
//   REAL_DCT0  in: s(0 .. n/2) (n/2 + 1 reals); out S(k) = sum_n s(n)
//              cos(2 pi n k / n), k = 0 .. n/2 (the dct[n] function)
//   REAL_DST0  in: s(1 .. n/2 - 1) (n/2 - 1 reals); out S(k) = sum_n s(n)
//              sin(2 pi n k / n), k = 1 .. n/2 - 1 (the dst[n] function)
// ---------------------------------------------------------------------------
template <int V, typename R, int KIND>
__global__ __launch_bounds__(1024) void amqft_real_kernel(const R* __restrict__ in, R* __restrict__ out,
                                                           const R* __restrict__ ktab, int logn, long long nreal,
                                                           int kshift, int onthefly) {
    using VT = variant_traits<V>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = 1 << logn;
    const int H = N >> 1;
    const int D = logn - 2;
    const int Q = 1 << D;
    const int T = (N >> 4) > 1 ? (N >> 4) : 1;
    const int spw = blockDim.x / T;
    const int slot = threadIdx.x / T;
    const int ltid = threadIdx.x - slot * T;
    const long long sig = (long long)blockIdx.x * spw + slot;  // complex slot: real signals 2 sig, 2 sig + 1
    const bool va = 2 * sig < nreal, vb = 2 * sig + 1 < nreal;
    R* kt = reinterpret_cast<R*>(smem);
    const size_t kt_bytes = ((size_t)Q * sizeof(R) + 15) & ~(size_t)15;
    cx<R>* w = reinterpret_cast<cx<R>*>(smem + kt_bytes) + (size_t)slot * (N + T);
    cx<R>* scr = w + N;
    const int in_len = KIND == REAL_RDFT ? N : KIND == REAL_DCT0 ? H + 1 : H - 1;
    const int out_len = KIND == REAL_RDFT ? 2 * (H + 1) : KIND == REAL_DCT0 ? H + 1 : H - 1;
    const R* xa = in + (va ? 2 * sig : 0) * (long long)in_len;
    const R* xb = in + (vb ? 2 * sig + 1 : 0) * (long long)in_len;
    // lane pair (signal a, signal b) of one real index; zero for a missing signal
    auto pair = [&](int i) { return cx<R>{va ? xa[i] : R(0), vb ? xb[i] : R(0)}; };
    const cx<R> z0 = {R(0), R(0)};

    load_constants<V, R>(kt, ktab, Q, kshift, onthefly != 0, logn);
    for (int m = ltid; m < H; m += T) {
        int pos = m;
        if (VT::skel_a && m > 0) {
            const int j = __ffs(m) - 1;
            pos = (1 << (D - j)) + (m >> (j + 1));
        }
        if (KIND == REAL_RDFT) {
            const cx<R> a = pair(m), b = pair(m == 0 ? H : N - m);
            if (m == 0) {
                w[0] = a;  // c(0)
                w[H] = b;  // c(N/2)
            } else {
                w[pos] = a + b;
                w[H + pos] = a - b;
            }
        } else if (KIND == REAL_DCT0) {
            if (m == 0) {
                w[0] = pair(0);
                w[H] = pair(H);
            } else {
                w[pos] = pair(m);
                w[H + pos] = z0;
            }
        } else {
            if (m == 0) {
                w[0] = z0;
                w[H] = z0;
            } else {
                w[pos] = z0;
                w[H + pos] = pair(m - 1);
            }
        }
    }
    __syncthreads();
    core<V, R>(w, kt, scr, ltid, T, D, H);
    R* ya = out + (va ? 2 * sig : 0) * (long long)out_len;
    R* yb = out + (vb ? 2 * sig + 1 : 0) * (long long)out_len;
    for (int k = ltid; k <= H; k += T) {
        const cx<R> C = k == 0 ? w[0] : w[k];
        const cx<R> Dd = (k == 0 || k == H) ? z0 : w[H + k];
        if (KIND == REAL_RDFT) {
            if (va) { ya[2 * k] = C.re; ya[2 * k + 1] = -Dd.re; }
            if (vb) { yb[2 * k] = C.im; yb[2 * k + 1] = -Dd.im; }
        } else if (KIND == REAL_DCT0) {
            if (va) ya[k] = C.re;
            if (vb) yb[k] = C.im;
        } else if (k >= 1 && k < H) {
            if (va) ya[k - 1] = Dd.re;
            if (vb) yb[k - 1] = Dd.im;
        }
    }
}

// ---------------------------------------------------------------------------
// fused loss and gradient, loss_b = sum_k |w(k) (F x_b)(k)|^2,
// grad_b = 2 F^H(|w|^2 F x_b) = conj(F conj(2 |w|^2 F x_b)):
// forward recursion, then the D_c combine of the forward fused with the
// weighting and the D_r split of the adjoint, the recursion again, and the
// final D_c combine with conjugation on store.
// ---------------------------------------------------------------------------
template <int V, typename S>
__global__ __launch_bounds__(1024) void amqft_loss_kernel(const S* __restrict__ xin, const S* __restrict__ win,
                                                           S* __restrict__ grad,
                                                           typename storage<S>::R* __restrict__ loss,
                                                           const typename storage<S>::R* __restrict__ ktab,
                                                           int logn, long long batch, int kshift, int flags) {
    using R = typename storage<S>::R;
    using VT = variant_traits<V>;
    extern __shared__ __align__(16) unsigned char smem[];
    const bool onthefly = flags & 4;
    const int N = 1 << logn;
    const int H = N >> 1;
    const int D = logn - 2;
    const int Q = 1 << D;
    const int T = (N >> 4) > 1 ? (N >> 4) : 1;
    const int spw = blockDim.x / T;
    const int slot = threadIdx.x / T;
    const int ltid = threadIdx.x - slot * T;
    const long long sig = (long long)blockIdx.x * spw + slot;
    const bool valid = sig < batch;
    R* kt = reinterpret_cast<R*>(smem);
    const size_t kt_bytes = ((size_t)Q * sizeof(R) + 15) & ~(size_t)15;
    cx<R>* w = reinterpret_cast<cx<R>*>(smem + kt_bytes) + (size_t)slot * (N + T);
    cx<R>* scr = w + N;
    const S* x = xin + (valid ? sig : 0) * (long long)N;
    const S* wt = win + (valid ? sig : 0) * (long long)N;
    S* g = grad + (valid ? sig : 0) * (long long)N;

    load_constants<V, R>(kt, ktab, Q, kshift, onthefly, logn);
    load_signal<VT::skel_a, S, R>(w, x, ltid, T, D, H, false, valid);
    __syncthreads();
    core<V, R>(w, kt, scr, ltid, T, D, H);
    // combine + weight + split for the adjoint (conj of the weighted spectrum)
    R part = R(0);
    cx<R> a[KMAX], b[KMAX];
    int kk[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int kidx0 = ltid + k * T;
        kk[k] = kidx0;
        if (kidx0 < H && valid) {
            cx<R> y0, y1;
            if (kidx0 == 0) {
                y0 = w[0];
                y1 = w[H];
            } else {
                const cx<R> C = w[kidx0], Dd = w[H + kidx0];
                y0 = {C.re + Dd.im, C.im - Dd.re};  // Y(k)
                y1 = {C.re - Dd.im, C.im + Dd.re};  // Y(N-k)
            }
            const cx<R> w0 = storage<S>::ld(wt + kidx0);
            const cx<R> w1 = storage<S>::ld(wt + (kidx0 == 0 ? H : N - kidx0));
            const R m0 = w0.re * w0.re + w0.im * w0.im;
            const R m1 = w1.re * w1.re + w1.im * w1.im;
            part += m0 * (y0.re * y0.re + y0.im * y0.im) + m1 * (y1.re * y1.re + y1.im * y1.im);
            a[k] = cconj(y0 * (R(2) * m0));  // conj of g(k)
            b[k] = cconj(y1 * (R(2) * m1));  // conj of g(N-k)
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int m = kk[k];
        if (m < H && valid) {
            if (m == 0) {
                w[0] = a[k];
                w[H] = b[k];
            } else {
                int pos = m;
                if (VT::skel_a) {
                    const int j = __ffs(m) - 1;
                    pos = (1 << (D - j)) + (m >> (j + 1));
                }
                w[pos] = a[k] + b[k];
                w[H + pos] = a[k] - b[k];
            }
        }
    }
    // per-signal loss: reduce the partial sums of the T threads of the signal
    cx<R>* red = scr;
    red[ltid] = {part, R(0)};
    __syncthreads();
    if (ltid == 0 && valid) {
        R s = R(0);
        for (int u = 0; u < T; ++u) s += red[u].re;
        loss[sig] = s;
    }
    __syncthreads();
    core<V, R>(w, kt, scr, ltid, T, D, H);
    store_signal<S, R>(w, g, ltid, T, H, true, valid);
}

// N = 1 (identity) and N = 2 (direct definition of the CDFT, Sec. 4)
template <typename S>
__device__ void tiny_one(const S* x, S* y, int logn, bool conj_in, bool conj_out) {
    using R = typename storage<S>::R;
    if (logn == 0) {
        cx<R> a = storage<S>::ld(x);
        if (conj_in != conj_out) a = cconj(a);
        storage<S>::st(y, a);
    } else {
        cx<R> a = storage<S>::ld(x), c = storage<S>::ld(x + 1);
        if (conj_in) { a = cconj(a); c = cconj(c); }
        cx<R> s0 = a + c, s1 = a - c;
        if (conj_out) { s0 = cconj(s0); s1 = cconj(s1); }
        storage<S>::st(y, s0);
        storage<S>::st(y + 1, s1);
    }
}

template <typename S>
__global__ void amqft_tiny_kernel(const S* __restrict__ in, S* __restrict__ out, int logn, long long batch,
                                  int flags, const long long* __restrict__ offsets) {
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const long long base = offsets ? offsets[b] : (b << logn);
    tiny_one<S>(in + base, out + base, logn, flags & 1, flags & 2);
}

// ---------------------------------------------------------------------------
// persistent kernel for many signals of different lengths (N <= 4096): the
// work list holds items (log2 N, first entry of the offset list, count);
// workgroup g takes items g, g + gridDim.x, ... (the list is sorted by cost,
// largest first, so the static round robin balances like longest-first).
// Each item is up to 256/T signals of one length, T = max(1, N/16).
// ---------------------------------------------------------------------------
template <int V, typename S>
__global__ __launch_bounds__(256) void amqft_persistent_kernel(const S* __restrict__ in, S* __restrict__ out,
                                                                const typename storage<S>::R* __restrict__ ktab,
                                                                int ktab_log2n, const int4* __restrict__ items,
                                                                int nitems, const long long* __restrict__ offsets,
                                                                int flags) {
    using R = typename storage<S>::R;
    using VT = variant_traits<V>;
    extern __shared__ __align__(16) unsigned char smem[];
    const bool conj_in = flags & 1, conj_out = flags & 2, onthefly = flags & 4;
    int kt_logn = -1;  // length whose constants the LDS table holds (items run longest first)
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 w4 = items[it];
        const int logn = w4.x, first = w4.y, count = w4.z;
        if (logn <= 1) {
            for (int u = threadIdx.x; u < count; u += blockDim.x) {
                const long long o = offsets[first + u];
                tiny_one<S>(in + o, out + o, logn, conj_in, conj_out);
            }
            continue;
        }
        const int N = 1 << logn, H = N >> 1, D = logn - 2, Q = 1 << D;
        const int T = (N >> 4) > 1 ? (N >> 4) : 1;
        const int slot = threadIdx.x / T;
        const int ltid = threadIdx.x - slot * T;
        const bool valid = slot < count;
        R* kt = reinterpret_cast<R*>(smem);
        const size_t kt_bytes = ((size_t)(1 << 10) * sizeof(R) + 15) & ~(size_t)15;  // up to N = 4096
        cx<R>* w = reinterpret_cast<cx<R>*>(smem + kt_bytes) + (size_t)slot * (N + T);
        cx<R>* scr = w + N;
        const long long o = valid ? offsets[first + slot] : 0;
        // the previous item's last barrier ended every read of the table
        if (logn != kt_logn) load_constants<V, R>(kt, ktab, Q, ktab_log2n - logn, onthefly, logn);
        kt_logn = logn;
        load_signal<VT::skel_a, S, R>(w, in + o, ltid, T, D, H, conj_in, valid);
        __syncthreads();
        core<V, R>(w, kt, scr, ltid, T, D, H);
        store_signal<S, R>(w, out + o, ltid, T, H, conj_out, valid);
        __syncthreads();
    }
}

void lds_shape(int logn, int dtype, int* threads, int* spw, size_t* lds_bytes) {
    const int N = 1 << logn;
    const int T = (N >> 4) > 1 ? (N >> 4) : 1;
    const int s = T >= 256 ? 1 : 256 / T;
    const size_t rsz = dtype == 0 ? 8 : 4;
    const int Q = logn >= 2 ? (1 << (logn - 2)) : 1;
    const size_t kt_bytes = ((size_t)Q * rsz + 15) & ~(size_t)15;
    *threads = s * T;
    *spw = s;
    *lds_bytes = kt_bytes + (size_t)s * (N + T) * 2 * rsz;
}

template <int V, typename S>
static hipError_t launch_typed(const lds_launch& a, hipStream_t stream) {
    using R = typename storage<S>::R;
    const int flags = (a.conj_in ? 1 : 0) | (a.conj_out ? 2 : 0) | (a.onthefly ? 4 : 0);
    if (a.batch <= 0) return hipSuccess;
    if (a.logn <= 1) {
        const int tpb = 256;
        const long long grid = (a.batch + tpb - 1) / tpb;
        hipLaunchKernelGGL(amqft_tiny_kernel<S>, dim3((unsigned)grid), dim3(tpb), 0, stream,
                           static_cast<const S*>(a.in), static_cast<S*>(a.out), a.logn, (long long)a.batch, flags,
                           static_cast<const long long*>(a.offsets));
        return hipGetLastError();
    }
    int threads, spw;
    size_t lds;
    lds_shape(a.logn, a.dtype, &threads, &spw, &lds);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amqft_lds_kernel<V, S>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const long long grid = (a.batch + spw - 1) / spw;
    const int kshift = a.ktab_log2n - a.logn;
    hipLaunchKernelGGL((amqft_lds_kernel<V, S>), dim3((unsigned)grid), dim3(threads), lds, stream,
                       static_cast<const S*>(a.in), static_cast<S*>(a.out), static_cast<const R*>(a.ktab), a.logn,
                       (long long)a.batch, kshift, flags, static_cast<const long long*>(a.offsets));
    return hipGetLastError();
}

template <int V, typename R, int KIND>
static hipError_t launch_real_k(const real_launch& a, hipStream_t stream) {
    int threads, spw;
    size_t lds;
    lds_shape(a.logn, a.dtype, &threads, &spw, &lds);
    const long long slots = (a.nreal + 1) / 2;
    const long long grid = (slots + spw - 1) / spw;
    hipLaunchKernelGGL((amqft_real_kernel<V, R, KIND>), dim3((unsigned)grid), dim3(threads), lds, stream,
                       static_cast<const R*>(a.in), static_cast<R*>(a.out), static_cast<const R*>(a.ktab), a.logn,
                       (long long)a.nreal, a.ktab_log2n - a.logn, a.onthefly);
    return hipGetLastError();
}

template <int V, typename R>
static hipError_t launch_real_r(const real_launch& a, hipStream_t s) {
    switch (a.kind) {
    case REAL_RDFT: return launch_real_k<V, R, REAL_RDFT>(a, s);
    case REAL_DCT0: return launch_real_k<V, R, REAL_DCT0>(a, s);
    default: return launch_real_k<V, R, REAL_DST0>(a, s);
    }
}

template <int V>
static hipError_t launch_real_v(const real_launch& a, hipStream_t s) {
    return a.dtype == 0 ? launch_real_r<V, double>(a, s) : launch_real_r<V, float>(a, s);
}

hipError_t launch_real(const real_launch& a, hipStream_t s) {
    if (a.nreal <= 0) return hipSuccess;
    switch (a.variant) {
    case 1: return launch_real_v<1>(a, s);
    case 2: return launch_real_v<2>(a, s);
    case 3: return launch_real_v<3>(a, s);
    case 4: return launch_real_v<4>(a, s);
    case 5: return launch_real_v<5>(a, s);
    case 6: return launch_real_v<6>(a, s);
    case 7: return launch_real_v<7>(a, s);
    default: return launch_real_v<8>(a, s);
    }
}

template <int V, typename S>
static hipError_t launch_loss_typed(const loss_launch& a, hipStream_t stream) {
    using R = typename storage<S>::R;
    if (a.batch <= 0) return hipSuccess;
    int threads, spw;
    size_t lds;
    lds_shape(a.logn, a.dtype, &threads, &spw, &lds);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amqft_loss_kernel<V, S>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const long long grid = (a.batch + spw - 1) / spw;
    const int kshift = a.ktab_log2n - a.logn;
    hipLaunchKernelGGL((amqft_loss_kernel<V, S>), dim3((unsigned)grid), dim3(threads), lds, stream,
                       static_cast<const S*>(a.x), static_cast<const S*>(a.w), static_cast<S*>(a.grad),
                       static_cast<R*>(a.loss), static_cast<const R*>(a.ktab), a.logn, (long long)a.batch, kshift,
                       a.onthefly ? 4 : 0);
    return hipGetLastError();
}

template <int V>
static hipError_t launch_loss_v(const loss_launch& a, hipStream_t s) {
    switch (a.dtype) {
    case 0: return launch_loss_typed<V, double2>(a, s);
    case 1: return launch_loss_typed<V, float2>(a, s);
    case 2: return launch_loss_typed<V, __half2>(a, s);
    default: return launch_loss_typed<V, bf16x2>(a, s);
    }
}

hipError_t launch_loss(const loss_launch& a, hipStream_t s) {
    if (kA_loss_supported(a.variant, a.logn, a.dtype)) return launch_kA_loss(a, s);
    switch (a.variant) {
    case 1: return launch_loss_v<1>(a, s);
    case 2: return launch_loss_v<2>(a, s);
    case 3: return launch_loss_v<3>(a, s);
    case 4: return launch_loss_v<4>(a, s);
    case 5: return launch_loss_v<5>(a, s);
    case 6: return launch_loss_v<6>(a, s);
    case 7: return launch_loss_v<7>(a, s);
    default: return launch_loss_v<8>(a, s);
    }
}

size_t persistent_lds_bytes(int dtype) {
    const size_t rsz = dtype == 0 ? 8 : 4;
    const size_t kt_bytes = ((size_t)(1 << 10) * rsz + 15) & ~(size_t)15;
    size_t m = 0;
    for (int logn = 2; logn <= kPersistentMaxLog2; ++logn) {
        const int N = 1 << logn, T = (N >> 4) > 1 ? (N >> 4) : 1, spw = 256 / T;
        m = std::max(m, (size_t)spw * (N + T) * 2 * rsz);
    }
    return kt_bytes + m;
}

template <int V, typename S>
static hipError_t launch_persistent_typed(const persistent_launch& a, hipStream_t stream) {
    using R = typename storage<S>::R;
    if (a.nitems <= 0) return hipSuccess;
    const size_t lds = persistent_lds_bytes(a.dtype);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amqft_persistent_kernel<V, S>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int flags = (a.conj_in ? 1 : 0) | (a.conj_out ? 2 : 0) | (a.onthefly ? 4 : 0);
    hipLaunchKernelGGL((amqft_persistent_kernel<V, S>), dim3((unsigned)a.grid), dim3(256), lds, stream,
                       static_cast<const S*>(a.in), static_cast<S*>(a.out), static_cast<const R*>(a.ktab),
                       a.ktab_log2n, static_cast<const int4*>(a.items), a.nitems,
                       static_cast<const long long*>(a.offsets), flags);
    return hipGetLastError();
}

template <int V>
static hipError_t launch_persistent_v(const persistent_launch& a, hipStream_t s) {
    switch (a.dtype) {
    case 0: return launch_persistent_typed<V, double2>(a, s);
    case 1: return launch_persistent_typed<V, float2>(a, s);
    case 2: return launch_persistent_typed<V, __half2>(a, s);
    default: return launch_persistent_typed<V, bf16x2>(a, s);
    }
}

hipError_t launch_persistent(const persistent_launch& a, hipStream_t s) {
    switch (a.variant) {
    case 1: return launch_persistent_v<1>(a, s);
    case 2: return launch_persistent_v<2>(a, s);
    case 3: return launch_persistent_v<3>(a, s);
    case 4: return launch_persistent_v<4>(a, s);
    case 5: return launch_persistent_v<5>(a, s);
    case 6: return launch_persistent_v<6>(a, s);
    case 7: return launch_persistent_v<7>(a, s);
    default: return launch_persistent_v<8>(a, s);
    }
}

template <int V>
static hipError_t launch_v(const lds_launch& a, hipStream_t s) {
    switch (a.dtype) {
    case 0: return launch_typed<V, double2>(a, s);
    case 1: return launch_typed<V, float2>(a, s);
    case 2: return launch_typed<V, __half2>(a, s);
    default: return launch_typed<V, bf16x2>(a, s);
    }
}

// set the dynamic-LDS limit of every kernel a plan may launch (before any
// graph capture, since attribute calls are not stream work)
template <int V, typename S>
static hipError_t prime_typed() {
    using R = typename storage<S>::R;
    const void* ks[6] = {reinterpret_cast<const void*>(&amqft_lds_kernel<V, S>),
                         reinterpret_cast<const void*>(&amqft_loss_kernel<V, S>),
                         reinterpret_cast<const void*>(&amqft_persistent_kernel<V, S>),
                         reinterpret_cast<const void*>(&amqft_real_kernel<V, R, REAL_RDFT>),
                         reinterpret_cast<const void*>(&amqft_real_kernel<V, R, REAL_DCT0>),
                         reinterpret_cast<const void*>(&amqft_real_kernel<V, R, REAL_DST0>)};
    for (const void* k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int V>
static hipError_t prime_v(int dtype) {
    switch (dtype) {
    case 0: return prime_typed<V, double2>();
    case 1: return prime_typed<V, float2>();
    case 2: return prime_typed<V, __half2>();
    default: return prime_typed<V, bf16x2>();
    }
}

hipError_t prime_lds(int variant, int dtype) {
    hipError_t e = prime_fast(variant, dtype);
    if (e == hipSuccess) e = prime_kA(variant, dtype);
    if (e == hipSuccess) e = prime_kB(variant, dtype);
    if (e != hipSuccess) return e;
    switch (variant) {
    case 1: return prime_v<1>(dtype);
    case 2: return prime_v<2>(dtype);
    case 3: return prime_v<3>(dtype);
    case 4: return prime_v<4>(dtype);
    case 5: return prime_v<5>(dtype);
    case 6: return prime_v<6>(dtype);
    case 7: return prime_v<7>(dtype);
    default: return prime_v<8>(dtype);
    }
}

// constants of family fam for length 2^logn, entries p < N/4, computed on the
// device in FP64 (cospi / sinpi) and rounded once to R (the same values the
// kernels generate per workgroup under AMQFT_FLAG_ONTHEFLY_CONSTANTS)
template <typename R>
__global__ __launch_bounds__(256) void amqft_fill_table_kernel(R* __restrict__ kt, int fam, int logn) {
    const long long q = 1ll << (logn - 2);
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= q) return;
    const double x = (double)p * 2.0 / (double)(1ll << logn);
    double v;
    if (fam == 0) v = 2.0 * cospi(x);
    else if (fam == 1) v = 1.0 / (2.0 * cospi(x));
    else if (fam == 2) v = 2.0 * sinpi(x);
    else v = 1.0 / (2.0 * sinpi(x));
    kt[p] = p == 0 ? R(0) : R(v);
}

hipError_t fill_table_device(void* ktab, int variant, int dtype, int logn, hipStream_t st) {
    const long long q = 1ll << (logn - 2);
    const dim3 grid((unsigned)((q + 255) / 256));
    if (dtype == 0)
        hipLaunchKernelGGL((amqft_fill_table_kernel<double>), grid, dim3(256), 0, st, static_cast<double*>(ktab),
                           const_family(variant), logn);
    else if (dtype == 4)
        hipLaunchKernelGGL((amqft_fill_table_kernel<fx32>), grid, dim3(256), 0, st, static_cast<fx32*>(ktab),
                           const_family(variant), logn);
    else
        hipLaunchKernelGGL((amqft_fill_table_kernel<float>), grid, dim3(256), 0, st, static_cast<float*>(ktab),
                           const_family(variant), logn);
    return hipGetLastError();
}

void describe_lds(const lds_launch& a, char* buf, size_t len) {
    static const char* st[5] = {"double2", "float2", "__half2", "bf16x2", "int2"};
    const char* sname = st[a.dtype >= 0 && a.dtype <= 4 ? a.dtype : 1];
    int threads = 0, spw = 1;
    size_t lds = 0;
    if (!a.generic && kA_supported(a.variant, a.logn, a.dtype)) {
        kA_shape(a.logn, a.dtype, &threads, &spw, &lds);
        lds = kA_lds(a.variant, a.logn, a.dtype);
        snprintf(buf, len, "amqft_kA_kernel<%d, %s, %d> grid=%lld block=%d lds=%zu", a.variant, sname, a.logn,
                 (long long)((a.batch + spw - 1) / spw), threads, lds);
    } else if (!a.generic && kB_supported(a.variant, a.logn, a.dtype)) {
        kA_shape(a.logn, a.dtype, &threads, &spw, &lds);  // the geometry and LDS of its skeleton-A transpose
        lds = kA_lds(a.variant == 2 ? 4 : a.variant == 6 ? 8 : a.variant == 3 ? 1 : 5, a.logn, a.dtype);
        snprintf(buf, len, "amqft_kB_kernel<%d, %s, %d> grid=%lld block=%d lds=%zu", a.variant, sname, a.logn,
                 (long long)((a.batch + spw - 1) / spw), threads, lds);
    } else if (!a.generic && fast_supported(a.logn, a.dtype)) {
        fast_shape(a.logn, a.dtype, &threads, &spw, &lds);
        snprintf(buf, len, "amqft_fast_kernel<%d, %s, %d> grid=%lld block=%d lds=%zu", a.variant, sname, a.logn,
                 (long long)((a.batch + spw - 1) / spw), threads, lds);
    } else if (a.logn <= 1) {
        snprintf(buf, len, "amqft_tiny_kernel<%s> n=%d", sname, 1 << a.logn);
    } else {
        lds_shape(a.logn, a.dtype, &threads, &spw, &lds);
        snprintf(buf, len, "amqft_lds_kernel<%d, %s> grid=%lld block=%d lds=%zu", a.variant, sname,
                 (long long)((a.batch + spw - 1) / spw), threads, lds);
    }
}

hipError_t launch_lds(const lds_launch& a, hipStream_t s) {
    if (!a.generic && kA_supported(a.variant, a.logn, a.dtype)) return launch_kA(a, s);
    if (!a.generic && kB_supported(a.variant, a.logn, a.dtype)) return launch_kB(a, s);
    if (!a.generic && fast_supported(a.logn, a.dtype)) return launch_fast(a, s);
    switch (a.variant) {
    case 1: return launch_v<1>(a, s);
    case 2: return launch_v<2>(a, s);
    case 3: return launch_v<3>(a, s);
    case 4: return launch_v<4>(a, s);
    case 5: return launch_v<5>(a, s);
    case 6: return launch_v<6>(a, s);
    case 7: return launch_v<7>(a, s);
    default: return launch_v<8>(a, s);
    }
}

}  // namespace amqft
