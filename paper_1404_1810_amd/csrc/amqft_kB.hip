// Skeleton-B AM-QFT (variants 2, 3, 6, 7) for N = 2^8 .. 2^14 as the transposed
// program of the compile-time skeleton-A kernel (amqft_kA.hip).
//
// The DFT matrix is symmetric (eq. qft_0A), so the transposed program of any
// algorithm for F computes F again.  Transposing the skeleton-A program of
// variant 4 step by step gives exactly the program of variant 2 (8 gives 6,
// 1 gives 3, 5 gives 7): the reflections of D_k^T become the reflections of D_n^F and back,
// time splits become harmonic interleaves, the multiply of M4 / M8 by
// 1/(2cos) / 1/(2sin) of theta*n moves to the frequency side, where M2 / M6
// put it, and their neighbour sums / differences move to the time side
// (Tables tab:DCT_odd_transformations, tab:DST_odd_transformations); the
// dct / dst chain's D_n^F becomes the D_k^T that skeleton B applies first
// (Sec. 5).  The combine X(k) = C(k) -+ i D(k) transposes into D_c plus
// -i times D_r, and D_c / D_r into the combine: the factor -i rides through
// the (real-coefficient) DST side exactly.  Every 2-term sum of one program
// is a 2-term fan-out of the other, so the rounding is that of variant 2
// (6) evaluated in this order.
//
// The kernel therefore runs the passes of amqft_kA.hip in reverse order,
// each transposed, on the same LDS layouts:
//   C0^T   load the 16 outputs' positions of the thread's orbit, D_c and -i D_r
//          of the combine, the three top levels of the chain's D_k^T: blocks
//          0..2 of both sides into the depth-0 block layout, the level-3 chain
//          values into the places of blocks 3.. (FOLD's input).
//   FOLD   the chain's D_k^T for levels 3 .. D-3, one lane per orbit of
//          positions that the reflections keep together, in registers:
//          blocks 3..D-3 and the values of dct[16] / dst[16] (the chain slots).
//   B0^T   levels 0..2 of dct_to / dst_to: time splits with the M2 / M6
//          neighbour sums (the transposed B0: the +-1 neighbours of a child
//          index come from the neighbouring threads' runs, read as a window).
//   B_k^T  the same for the middle levels.
//   P3^T   rows of 16 slots, forward and backward in registers (dct_to leaves).
//   M_k^T  the backward D_n^F butterflies with the 1/(2cos) / 1/(2sin) multiply
//          on the orbits of the middle passes.
//   F1^T   the last backward levels on the thread's orbit, the combine of
//          D_c / D_r transposed, and the store; thread 0 of a signal runs the
//          chain from dct[16] / dst[16] with the blocks of 4, 2 and 1 points.
#include <type_traits>

#include "amqft_device.h"
#include "amqft_internal.h"
#include "amqft_kB_passes.h"

namespace amqft {

namespace {

// ---------------------------------------------------------------------------
// the kernel (same launch geometry and LDS as amqft_kA_kernel)
// ---------------------------------------------------------------------------
template <int VB, typename S, int LOGN>
__global__ __launch_bounds__(kgeo<LOGN>::WG) void amqft_kB_kernel(const S* __restrict__ in, S* __restrict__ out,
                                                                   const typename storage<S>::R* __restrict__ ktab,
                                                                   long long batch, int kshift, int flags,
                                                                   const long long* __restrict__ offsets) {
    using R = typename storage<S>::R;
    using G = kgeo<LOGN>;
    constexpr int VA = transposed_of<VB>::V;
    extern __shared__ __align__(16) unsigned char smem[];
    R* kt = reinterpret_cast<R*>(smem);
    R* kf = kt + G::Q;
    cx<R>* wall = reinterpret_cast<cx<R>*>(smem + (G::Q + G::KF_ALLOC) * sizeof(R));
    const bool conj_in = flags & 1, conj_out = flags & 2, onthefly = flags & 4;
    const int tid = threadIdx.x;
    const int fs = tid / G::T, m0 = tid - fs * G::T;
    const long long gs = (long long)blockIdx.x * G::SPW + fs;
    const bool live = gs < batch;
    long long base = !live ? 0 : offsets ? offsets[gs] : gs * (long long)G::N;
    constexpr bool WU = G::T >= 64;
    if constexpr (WU) base = uniform64(base);

    cx<R> raw[16];
    f1_load<LOGN, S, R, WU>(in + base, m0, raw);
    fill_constants<VA, LOGN, R>(kt, kf, ktab, kshift, onthefly, tid);
    cx<R>* w = wall + fs * G::SL;
    c0T<LOGN, R>(w, w, raw, m0, conj_in);
    __syncthreads();
    fold<LOGN, R>(wall, tid);
    if constexpr (variant_traits<VB>::recurrence) {
        b0T_rec_pass<VA, LOGN, R>(wall, wall + G::SPW * G::SL, tid);
        sfor<0, G::NP>([&](auto kc) { bT_rec_pass<VA, LOGN, decltype(kc)::value, R>(wall, tid); });
    } else {
        b0T_pass<VA, LOGN, R>(wall, tid);
        sfor<0, G::NP>([&](auto kc) { bT_pass<VA, LOGN, decltype(kc)::value, R>(wall, tid); });
    }
    p3T_pass<VB, LOGN, R>(wall, kt, tid);
    sfor<0, G::NP>([&](auto kc) { orbitT_pass<VA, VB, LOGN, G::NP - 1 - decltype(kc)::value, R>(wall, kt, kf, tid); });
    if (live) {
        cx<R> res[16];
        if (m0 > 0) f1T_orbit<VA, LOGN, R>(w, kt, m0, res);
        else {
            cx<R> chs[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) chs[k] = ldc(w + lds_layout<LOGN>::chain(k));
            f1T_chain<VB, LOGN, R>(chs, kt, res);
        }
        c0_store<LOGN, S, R, WU>(out + base, m0, res, conj_out);
    }
}

template <int VB, typename S, int LOGN>
hipError_t launch_kB_n(const lds_launch& a, hipStream_t st) {
    using R = typename storage<S>::R;
    using G = kgeo<LOGN>;
    const int flags = (a.conj_in ? 1 : 0) | (a.conj_out ? 2 : 0) | (a.onthefly ? 4 : 0);
    const long long grid = (a.batch + G::SPW - 1) / G::SPW;
    const size_t lds = kA_lds_bytes_v<transposed_of<VB>::V, R, LOGN>();
    hipLaunchKernelGGL((amqft_kB_kernel<VB, S, LOGN>), dim3((unsigned)grid), dim3(G::WG), lds, st,
                       static_cast<const S*>(a.in), static_cast<S*>(a.out), static_cast<const R*>(a.ktab),
                       (long long)a.batch, a.ktab_log2n - LOGN, flags, static_cast<const long long*>(a.offsets));
    return hipGetLastError();
}

template <int VB, typename S>
hipError_t launch_kB_s(const lds_launch& a, hipStream_t st) {
    switch (a.logn) {
    case 8: return launch_kB_n<VB, S, 8>(a, st);
    case 9: return launch_kB_n<VB, S, 9>(a, st);
    case 10: return launch_kB_n<VB, S, 10>(a, st);
    case 11: return launch_kB_n<VB, S, 11>(a, st);
    case 12: return launch_kB_n<VB, S, 12>(a, st);
    case 13: return launch_kB_n<VB, S, 13>(a, st);
    default:
        if constexpr (std::is_same<S, double2>::value) return hipErrorInvalidValue;
        else return launch_kB_n<VB, S, 14>(a, st);
    }
}

template <int VB, typename S, int LOGN>
hipError_t prime_kB_n() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&amqft_kB_kernel<VB, S, LOGN>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    constexpr int LMAX = std::is_same<S, double2>::value ? 13 : 14;
    if constexpr (LOGN < LMAX) {
        if (e == hipSuccess) e = prime_kB_n<VB, S, LOGN + 1>();
    }
    return e;
}

template <int VB>
hipError_t launch_kB_v(const lds_launch& a, hipStream_t st) {
    switch (a.dtype) {
    case 0: return launch_kB_s<VB, double2>(a, st);
    case 1: return launch_kB_s<VB, float2>(a, st);
    case 2: return launch_kB_s<VB, __half2>(a, st);
    case 4:
        if constexpr (VB == 3 || VB == 7) return launch_kB_s<VB, int2>(a, st);
        else return hipErrorInvalidValue;
    default: return launch_kB_s<VB, bf16x2>(a, st);
    }
}

template <int VB>
hipError_t prime_kB_v(int dtype) {
    switch (dtype) {
    case 0: return prime_kB_n<VB, double2, 8>();
    case 1: return prime_kB_n<VB, float2, 8>();
    case 2: return prime_kB_n<VB, __half2, 8>();
    case 4:
        if constexpr (VB == 3 || VB == 7) return prime_kB_n<VB, int2, 8>();
        else return hipErrorInvalidValue;
    default: return prime_kB_n<VB, bf16x2, 8>();
    }
}

}  // namespace

bool kB_supported(int variant, int logn, int dtype) {
    if (variant != 2 && variant != 3 && variant != 6 && variant != 7) return false;
    if (dtype == 0) return logn >= 8 && logn <= 13;
    // fixed point: the variants whose constants (2cos, 2sin) have a Q2.29 form
    if (dtype == 4) return (variant == 3 || variant == 7) && logn >= 8 && logn <= 14;
    return logn >= 8 && logn <= 14;
}

hipError_t launch_kB(const lds_launch& a, hipStream_t st) {
    if (a.batch <= 0) return hipSuccess;
    if (!kB_supported(a.variant, a.logn, a.dtype)) return hipErrorInvalidValue;
    switch (a.variant) {
    case 2: return launch_kB_v<2>(a, st);
    case 3: return launch_kB_v<3>(a, st);
    case 6: return launch_kB_v<6>(a, st);
    default: return launch_kB_v<7>(a, st);
    }
}

hipError_t prime_kB(int variant, int dtype) {
    switch (variant) {
    case 2: return prime_kB_v<2>(dtype);
    case 3: return prime_kB_v<3>(dtype);
    case 6: return prime_kB_v<6>(dtype);
    case 7: return prime_kB_v<7>(dtype);
    default: return hipSuccess;
    }
}

}  // namespace amqft
