// Host-side interface between the C ABI (amqft_api.cpp) and the kernel
// launchers (amqft_lds.hip, ...).  Not installed; not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace amqft {

// Largest log2(N) a single workgroup keeps resident in LDS, per arithmetic
// precision (FP32 compute: 2^14 points = 128 KiB; FP64: 2^13).
constexpr int kMaxLdsLog2F32 = 14;
constexpr int kMaxLdsLog2F64 = 13;

struct lds_launch {
    int variant;       // 1..8
    int dtype;         // amqft_dtype
    int logn;          // log2 N, 0..kMaxLds*
    int64_t batch;     // signals (stride N)
    const void* in;    // device
    void* out;         // device
    const void* ktab;  // device constant table (R values), entries (1<<ktab_log2n)/4
    int ktab_log2n;    // log2 of the length the table was built for
    int conj_in;       // conjugate the input on load
    int conj_out;      // conjugate the output on store
    int onthefly;      // generate constants on the device (FP64) instead
    const void* offsets = nullptr;  // device int64 offsets (complex elements) per signal, or NULL = stride N
    int generic = 0;                // 1: always use the generic engine (tests of that path)
};

// Largest log2(N) handled by the persistent many-length kernel (256 threads).
constexpr int kPersistentMaxLog2 = 12;

struct persistent_launch {
    int variant, dtype;
    const void* in;
    void* out;
    const void* ktab;
    int ktab_log2n;
    const void* items;    // device int4 {log2 N, first offset index, count, 0}
    int nitems;
    const void* offsets;  // device int64 signal offsets, grouped per item
    int grid;             // persistent workgroups
    int conj_in, conj_out, onthefly;
};
hipError_t launch_persistent(const persistent_launch& a, hipStream_t stream);
size_t persistent_lds_bytes(int dtype);

struct loss_launch {
    int variant, dtype, logn;  // logn >= 2
    int64_t batch;
    const void* x;     // device, (batch, N) storage type
    const void* w;     // device, (batch, N) storage type
    void* grad;        // device, (batch, N) storage type
    void* loss;        // device, batch values of the arithmetic type
    const void* ktab;
    int ktab_log2n;
    int onthefly;
};

// Real transforms (RDFT, DCT-0, DST-0) on the LDS engine: two real signals
// per complex lane.
enum { REAL_RDFT = 0, REAL_DCT0 = 1, REAL_DST0 = 2 };
struct real_launch {
    int variant, dtype, logn, kind;  // dtype 0 (FP64) or 1 (FP32); 2 <= logn <= kMaxLds*
    int64_t nreal;                   // real signals
    const void* in;                  // device reals, stride n / n/2+1 / n/2-1 per kind
    void* out;                       // device: n/2+1 complex / n/2+1 reals / n/2-1 reals per signal
    const void* ktab;
    int ktab_log2n;
    int onthefly;
};
hipError_t launch_real(const real_launch& a, hipStream_t stream);

// Fused loss/gradient kernel (forward, |w|^2 weighting, adjoint).
hipError_t launch_loss(const loss_launch& a, hipStream_t stream);
hipError_t launch_kA_loss(const loss_launch& a, hipStream_t stream);

// Fast kernels with compile-time geometry (N = 64 .. 4096, FP32 / FP64).
bool fast_supported(int logn, int dtype);
hipError_t launch_fast(const lds_launch& a, hipStream_t stream);
hipError_t prime_fast(int variant, int dtype);
void fast_shape(int logn, int dtype, int* threads, int* signals_per_wg, size_t* lds_bytes);

// Skeleton-A kernels for N = 2^8 .. 2^14 (variants 1, 4, 5, 8; FP64 up to 2^13)
// with the dataflow fixed at compile time (amqft_kA.hip).
bool kA_supported(int variant, int logn, int dtype);
hipError_t launch_kA(const lds_launch& a, hipStream_t stream);
hipError_t prime_kA(int variant, int dtype);
void kA_shape(int logn, int dtype, int* threads, int* signals_per_wg, size_t* lds_bytes);
// dynamic LDS bytes of the compile-time kernel for one variant
size_t kA_lds(int variant, int logn, int dtype);
// N = 2^15 .. 2^20 (FP64 2^14 .. 2^16), variants 4 and 8: four kernels over a
// global workspace (top levels, rows through the kA kernels, back levels,
// chain); signals run in chunks of `chunk`.
struct kl_launch {
    int variant, dtype, logn;
    int64_t batch, chunk;
    const void* in;
    void* out;
    void* ws1;  // chunk * N complex values of the arithmetic type
    void* ws2;  // chunk * N
    void* wsc;  // chunk * 16
    const void* ktab;  // table built for exactly N
    int conj_in, conj_out;
    const void* offsets = nullptr;
    // in place (in == out; variants 4, 8, N = 2^11 .. 2^17, FP32 / FP64
    // storage): ws1 unused, ws2 chunk * (N/8 + 16), ws3 chunk * 16 * ipnsh,
    // iptab the slot table of amqft_iplayout.h on the device
    int inplace = 0;
    void* ws3 = nullptr;
    const int* iptab = nullptr;
    int ipnsh = 0;
};
bool kL_supported(int variant, int logn, int dtype);
// sizes and types the in-place path takes
bool kL_inplace_supported(int variant, int logn, int dtype, bool forced);
// variants 2 and 6 on the transposed program of that path (amqft_kLT.hip):
// N = 2^15 .. 2^17 (FP64 2^14 .. 2^16), forced from 2^11; kL_* below
// dispatch to these for those variants
bool kLT_supported(int variant, int logn, int dtype);
bool kLT_supported_forced(int variant, int logn, int dtype);
hipError_t prime_kLT(int variant, int dtype);
hipError_t launch_kLT(const kl_launch& a, hipStream_t stream);
// sizes a plan may force onto that path (from 2^11; tests)
bool kL_supported_forced(int variant, int logn, int dtype);
size_t kL_ws_bytes_per_signal(int logn, int dtype);
hipError_t prime_kL(int variant, int dtype);
hipError_t launch_kL(const kl_launch& a, hipStream_t stream);

// Skeleton-B kernels for N = 2^8 .. 2^14 (variants 2, 3, 6, 7; FP64 up to
// 2^13): the transposed program of the skeleton-A kernels (amqft_kB.hip).
bool kB_supported(int variant, int logn, int dtype);
hipError_t launch_kB(const lds_launch& a, hipStream_t stream);
hipError_t prime_kB(int variant, int dtype);

// fused loss / gradient on the same kernels (forward, weighting, adjoint)
bool kA_loss_supported(int variant, int logn, int dtype);

// Name and launch shape of the kernel launch_lds picks for a (for reports).
void describe_lds(const lds_launch& a, char* buf, size_t len);

// Launch the LDS-resident engine; returns the hipError_t of the launch.
hipError_t launch_lds(const lds_launch& a, hipStream_t stream);

// Multi-pass engine for signals larger than LDS (amqft_multipass.hip).
struct mp_launch {
    int variant, dtype, logn;
    int sb;             // log2 of the sub-block size finished in LDS (2..12)
    int64_t batch;
    int64_t chunk;      // signals per round (workspace capacity)
    const void* in;
    void* out;
    void* ws0;          // workspaces: chunk * N complex values of the
    void* ws1;          // arithmetic type each
    void* ws2;
    const void* ktab;
    int ktab_log2n;
    int conj_in, conj_out, onthefly;
    const void* offsets = nullptr;  // device int64 per-signal offsets, or NULL = stride N
};
hipError_t launch_multipass(const mp_launch& m, hipStream_t stream);
// default sub-block exponent for a storage type (largest the LDS engine holds)
int multipass_sb(int dtype);
// bytes of one workspace buffer per signal
size_t multipass_ws_bytes_per_signal(int logn, int dtype);

// Raise the dynamic-LDS limit of the kernels of a variant/dtype (done at plan
// creation so that no attribute call happens during graph capture).
hipError_t prime_lds(int variant, int dtype);
// Overwrite a plan's constant table (N/4 entries of the arithmetic type,
// log2 N >= 2) with values generated on the device in FP64.
hipError_t fill_table_device(void* ktab, int variant, int dtype, int logn, hipStream_t stream);
hipError_t prime_multipass(int variant, int dtype);

// Record a failed HIP call as the calling thread's last HIP error (read by
// amqft_last_hip_error) and return the amqft_status it maps to.
int record_hip_failure(hipError_t e);

// Bytes of dynamic LDS and threads per workgroup the LDS engine uses.
void lds_shape(int logn, int dtype, int* threads, int* signals_per_wg, size_t* lds_bytes);

}  // namespace amqft
