// amqft_exec_noalloc: the transform of amqft_exec without a plan and without
// any allocation, for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops).  The workspace and the constant
// table of the paths that need them live in one file-scope device array per
// GPU, `scratch`, of AMQFT_NOALLOC_SCRATCH_BYTES; its device address is
// resolved once per device with hipGetSymbolAddress and only that address is
// handed to kernels.  Same kernels and constants as a plan made with
// AMQFT_FLAG_ONTHEFLY_CONSTANTS, so the results are the same bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/amqft.h"
#include "amqft_internal.h"

namespace amqft {
namespace {

constexpr size_t kScratchBytes = AMQFT_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
struct device_state {
    void* scratch = nullptr;  // device address of `scratch` on this device
    unsigned primed = 0;      // bit 4 (variant - 1) + dtype: kernel attributes set
};
std::mutex g_mu;
device_state g_dev[kMaxDevices];

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

int log2_exact(int64_t n) {
    if (n < 1 || (n & (n - 1)) != 0) return -1;
    int l = 0;
    while ((int64_t(1) << l) < n) ++l;
    return l;
}

// which path a length takes (the same choice a plan makes without flags)
enum path_kind { PATH_LDS, PATH_LARGE, PATH_MULTIPASS };

path_kind choose(int variant, int logn, int dtype) {
    const int maxlds = dtype == AMQFT_C128 ? kMaxLdsLog2F64 : kMaxLdsLog2F32;
    if (logn <= maxlds) return PATH_LDS;
    return kL_supported(variant, logn, dtype) ? PATH_LARGE : PATH_MULTIPASS;
}

size_t real_bytes(int dtype) { return dtype == AMQFT_C128 ? sizeof(double) : sizeof(float); }

// scratch bytes of the constant table and per signal of workspace
void scratch_need(path_kind pk, int logn, int dtype, size_t* table, size_t* per_signal) {
    *table = pk == PATH_LDS ? 0 : round256((size_t(1) << (logn - 2)) * real_bytes(dtype));
    if (pk == PATH_LARGE) *per_signal = 2 * kL_ws_bytes_per_signal(logn, dtype) + 16 * 2 * real_bytes(dtype);
    else if (pk == PATH_MULTIPASS) *per_signal = 3 * multipass_ws_bytes_per_signal(logn, dtype);
    else *per_signal = 0;
}

// device address of this device's scratch and the kernel attributes of
// (variant, dtype), set up on the first call on a device
hipError_t setup(int dev, int variant, int dtype, void** out) {
    std::lock_guard<std::mutex> g(g_mu);
    device_state& st = g_dev[dev];
    if (!st.scratch) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        st.scratch = ptr;
    }
    const unsigned bit = 1u << (4 * (variant - 1) + dtype);
    if (!(st.primed & bit)) {
        hipError_t e = prime_lds(variant, dtype);
        if (e == hipSuccess) e = prime_multipass(variant, dtype);
        if (e == hipSuccess) e = prime_kL(variant, dtype);
        if (e != hipSuccess) return e;
        st.primed |= bit;
    }
    *out = st.scratch;
    return hipSuccess;
}

}  // namespace
}  // namespace amqft

using namespace amqft;

extern "C" amqft_status amqft_exec_noalloc(int64_t n, int64_t batch, amqft_variant variant, amqft_dtype dtype,
                                           int adjoint, const void* in_dev, void* out_dev, void* stream) {
    const int v = (int)variant, t = (int)dtype;
    if (v < 1 || v > 8 || t < 0 || t > 3 || batch < 0) return AMQFT_ERR_INVALID_ARG;
    const int logn = log2_exact(n);
    if (logn < 0) return AMQFT_ERR_NOT_POW2;
    if (logn > AMQFT_MAX_LOG2N) return AMQFT_ERR_UNSUPPORTED;
    const path_kind pk = choose(v, logn, t);
    size_t table = 0, per = 0;
    scratch_need(pk, logn, t, &table, &per);
    if (table + per > kScratchBytes) return AMQFT_ERR_UNSUPPORTED;  // one signal does not fit the scratch
    if (batch == 0) return AMQFT_OK;
    if (!in_dev || !out_dev) return AMQFT_ERR_INVALID_ARG;

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (amqft_status)record_hip_failure(e);
    if (dev < 0 || dev >= kMaxDevices) return AMQFT_ERR_UNSUPPORTED;
    void* base = nullptr;
    e = setup(dev, v, t, &base);
    if (e != hipSuccess) return (amqft_status)record_hip_failure(e);
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned char* sp = static_cast<unsigned char*>(base);

    if (pk == PATH_LDS) {
        lds_launch a{};
        a.variant = v;
        a.dtype = t;
        a.logn = logn;
        a.batch = batch;
        a.in = in_dev;
        a.out = out_dev;
        a.ktab = sp;  // never read: constants are generated in every workgroup
        a.ktab_log2n = logn;
        a.conj_in = adjoint != 0;
        a.conj_out = adjoint != 0;
        a.onthefly = 1;
        e = launch_lds(a, st);
        return e == hipSuccess ? AMQFT_OK : (amqft_status)record_hip_failure(e);
    }
    // constant table of length n, generated on the device in FP64 (the values
    // the LDS kernels generate per workgroup)
    e = fill_table_device(sp, v, t, logn, st);
    if (e != hipSuccess) return (amqft_status)record_hip_failure(e);
    const int64_t chunk = std::min<int64_t>(batch, (int64_t)((kScratchBytes - table) / per));
    if (pk == PATH_LARGE) {
        const size_t ws = (size_t)chunk * kL_ws_bytes_per_signal(logn, t);
        kl_launch k{};
        k.variant = v;
        k.dtype = t;
        k.logn = logn;
        k.batch = batch;
        k.chunk = chunk;
        k.in = in_dev;
        k.out = out_dev;
        k.ws1 = sp + table;
        k.ws2 = sp + table + ws;
        k.wsc = sp + table + 2 * ws;
        k.ktab = sp;
        k.conj_in = adjoint != 0;
        k.conj_out = adjoint != 0;
        e = launch_kL(k, st);
    } else {
        const size_t ws = (size_t)chunk * multipass_ws_bytes_per_signal(logn, t);
        mp_launch m{};
        m.variant = v;
        m.dtype = t;
        m.logn = logn;
        m.sb = std::min(multipass_sb(t), logn - 3);
        m.batch = batch;
        m.chunk = chunk;
        m.in = in_dev;
        m.out = out_dev;
        m.ws0 = sp + table;
        m.ws1 = sp + table + ws;
        m.ws2 = sp + table + 2 * ws;
        m.ktab = sp;
        m.ktab_log2n = logn;
        m.conj_in = adjoint != 0;
        m.conj_out = adjoint != 0;
        m.onthefly = 1;
        e = launch_multipass(m, st);
    }
    return e == hipSuccess ? AMQFT_OK : (amqft_status)record_hip_failure(e);
}
