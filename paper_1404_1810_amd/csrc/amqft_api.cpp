// C ABI of the AM-QFT library (declarations and documentation in
// include/amqft.h).  Validation happens before any HIP call so that every
// error path can be exercised without a GPU.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/amqft.h"
#include "amqft_device.h"
#include "amqft_internal.h"

using namespace amqft;

struct amqft_plan_s {
    int variant = 4;
    int dtype = 1;
    unsigned flags = 0;
    int64_t n = 0;
    int logn = 0;
    int64_t batch = 0;
    // constant table for length 2^ktab_log2n, working precision, on device
    void* ktab = nullptr;
    int ktab_log2n = 2;
    std::vector<double> ktab_host;  // FP64 values as rounded to working precision
    int device = 0;
    // multi-pass (signals larger than LDS)
    bool multipass = false;
    int sb = 0;
    int64_t chunk = 0;
    void* ws[3] = {nullptr, nullptr, nullptr};
    size_t ws_bytes = 0;
};

namespace {

thread_local std::string g_hip_error;

amqft_status hip_fail(hipError_t e) {
    g_hip_error = hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? AMQFT_ERR_ALLOC : AMQFT_ERR_HIP;
}

bool valid_variant(int v) { return v >= 1 && v <= 8; }
bool valid_dtype(int t) { return t >= 0 && t <= 3; }

int log2_exact(int64_t n) {
    if (n < 1 || (n & (n - 1)) != 0) return -1;
    int l = 0;
    while ((int64_t(1) << l) < n) ++l;
    return l;
}

int max_lds_log2(int dtype) { return dtype == AMQFT_C128 ? kMaxLdsLog2F64 : kMaxLdsLog2F32; }

// f(2 pi p / n) for the variant's family (Sec. 7.1), evaluated in long double
// and rounded to double; the caller rounds once more to the working type.
double family_value(int fam, int64_t p, int64_t n) {
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double a = 2.0L * pi * (long double)p / (long double)n;
    long double v;
    switch (fam) {
    case 0: v = 2.0L * cosl(a); break;
    case 1: v = 1.0L / (2.0L * cosl(a)); break;
    case 2: v = 2.0L * sinl(a); break;
    default: v = 1.0L / (2.0L * sinl(a)); break;
    }
    return (double)v;
}

amqft_status build_constants(amqft_plan_s* p, int log2n) {
    const int64_t n = int64_t(1) << (log2n < 2 ? 2 : log2n);
    const int64_t q = n / 4;
    const int fam = const_family(p->variant);
    p->ktab_log2n = log2n < 2 ? 2 : log2n;
    p->ktab_host.assign((size_t)q, 0.0);
    const bool f64 = p->dtype == AMQFT_C128;
    std::vector<float> tf;
    if (!f64) tf.assign((size_t)q, 0.f);
    for (int64_t i = 1; i < q; ++i) {
        const double v = family_value(fam, i, n);
        if (f64) {
            p->ktab_host[i] = v;
        } else {
            tf[i] = (float)v;
            p->ktab_host[i] = (double)tf[i];
        }
    }
    const size_t bytes = (size_t)q * (f64 ? sizeof(double) : sizeof(float));
    hipError_t e = hipMalloc(&p->ktab, bytes < 16 ? 16 : bytes);
    if (e != hipSuccess) { p->ktab = nullptr; return hip_fail(e); }
    e = hipMemcpy(p->ktab, f64 ? (const void*)p->ktab_host.data() : (const void*)tf.data(), bytes,
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
    return AMQFT_OK;
}

amqft_status exec_common(amqft_plan p, const void* in, void* out, void* stream, bool adjoint) {
    if (!p) return AMQFT_ERR_INVALID_ARG;
    if (p->batch == 0) return AMQFT_OK;  // nothing to read or write; pointers may be NULL
    if (!in || !out) return AMQFT_ERR_INVALID_ARG;
    if (p->multipass) {
        mp_launch m{};
        m.variant = p->variant;
        m.dtype = p->dtype;
        m.logn = p->logn;
        m.sb = p->sb;
        m.batch = p->batch;
        m.chunk = p->chunk;
        m.in = in;
        m.out = out;
        m.ws0 = p->ws[0];
        m.ws1 = p->ws[1];
        m.ws2 = p->ws[2];
        m.ktab = p->ktab;
        m.ktab_log2n = p->ktab_log2n;
        m.conj_in = adjoint;
        m.conj_out = adjoint;
        m.onthefly = (p->flags & AMQFT_FLAG_ONTHEFLY_CONSTANTS) != 0;
        hipError_t e = launch_multipass(m, static_cast<hipStream_t>(stream));
        return e == hipSuccess ? AMQFT_OK : hip_fail(e);
    }
    lds_launch a{};
    a.variant = p->variant;
    a.dtype = p->dtype;
    a.logn = p->logn;
    a.batch = p->batch;
    a.in = in;
    a.out = out;
    a.ktab = p->ktab;
    a.ktab_log2n = p->ktab_log2n;
    a.conj_in = adjoint;
    a.conj_out = adjoint;
    a.onthefly = (p->flags & AMQFT_FLAG_ONTHEFLY_CONSTANTS) != 0;
    hipError_t e = launch_lds(a, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? AMQFT_OK : hip_fail(e);
}

}  // namespace

extern "C" {

const char* amqft_version(void) { return "amqft 0.1.0 (gfx950)"; }

const char* amqft_last_hip_error(void) { return g_hip_error.c_str(); }

const char* amqft_status_string(amqft_status st) {
    switch (st) {
    case AMQFT_OK: return "ok";
    case AMQFT_ERR_INVALID_ARG: return "invalid argument";
    case AMQFT_ERR_NOT_POW2: return "length is not a power of two";
    case AMQFT_ERR_UNSUPPORTED: return "unsupported length or option";
    case AMQFT_ERR_ALLOC: return "allocation failed";
    case AMQFT_ERR_HIP: return "HIP error";
    }
    return "unknown status";
}

amqft_status amqft_plan_create(amqft_plan* out, int64_t n, int64_t batch, amqft_variant variant,
                               amqft_dtype dtype, unsigned flags) {
    if (!out) return AMQFT_ERR_INVALID_ARG;
    *out = nullptr;
    if (!valid_variant((int)variant) || !valid_dtype((int)dtype) || batch < 0) return AMQFT_ERR_INVALID_ARG;
    if (flags & ~(unsigned)(AMQFT_FLAG_ONTHEFLY_CONSTANTS | AMQFT_FLAG_NO_AUTOTUNE | AMQFT_FLAG_FORCE_MULTIPASS))
        return AMQFT_ERR_INVALID_ARG;
    const int logn = log2_exact(n);
    if (logn < 0) return AMQFT_ERR_NOT_POW2;
    if (logn > AMQFT_MAX_LOG2N) return AMQFT_ERR_UNSUPPORTED;
    const bool mp = logn > max_lds_log2((int)dtype) || (flags & AMQFT_FLAG_FORCE_MULTIPASS);
    if (mp && logn < 5) return AMQFT_ERR_UNSUPPORTED;  // multi-pass needs a block of at least 8 points
    if (batch > (int64_t(1) << 40)) return AMQFT_ERR_UNSUPPORTED;
    amqft_plan_s* p = new (std::nothrow) amqft_plan_s();
    if (!p) return AMQFT_ERR_ALLOC;
    p->variant = (int)variant;
    p->dtype = (int)dtype;
    p->flags = flags;
    p->n = n;
    p->logn = logn;
    p->batch = batch;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { delete p; return hip_fail(e); }
    amqft_status st = build_constants(p, logn);
    if (st != AMQFT_OK) { amqft_plan_destroy(p); return st; }
    if (mp) {
        p->multipass = true;
        // forced (test) plans use small sub-blocks so that several global levels run
        p->sb = (flags & AMQFT_FLAG_FORCE_MULTIPASS) ? std::max(2, std::min(multipass_sb((int)dtype), logn - 5))
                                                     : std::min(multipass_sb((int)dtype), logn - 3);
        const size_t per = multipass_ws_bytes_per_signal(logn, (int)dtype);
        const size_t cap = size_t(1) << 30;  // bytes per workspace buffer
        p->chunk = std::max<int64_t>(1, std::min<int64_t>(batch, (int64_t)(cap / per)));
        p->ws_bytes = 3 * (size_t)p->chunk * per;
        for (int i = 0; i < 3 && batch > 0; ++i) {
            hipError_t e = hipMalloc(&p->ws[i], (size_t)p->chunk * per);
            if (e != hipSuccess) { p->ws[i] = nullptr; amqft_plan_destroy(p); return hip_fail(e); }
        }
    }
    *out = p;
    return AMQFT_OK;
}

amqft_status amqft_plan_create_many(amqft_plan* out, int64_t count, const int64_t* lengths_host,
                                    const int64_t* offsets_host, amqft_variant variant, amqft_dtype dtype,
                                    unsigned flags) {
    if (!out) return AMQFT_ERR_INVALID_ARG;
    *out = nullptr;
    if (!valid_variant((int)variant) || !valid_dtype((int)dtype) || count < 0) return AMQFT_ERR_INVALID_ARG;
    if (count > 0 && (!lengths_host || !offsets_host)) return AMQFT_ERR_INVALID_ARG;
    if (flags & ~(unsigned)(AMQFT_FLAG_ONTHEFLY_CONSTANTS | AMQFT_FLAG_NO_AUTOTUNE | AMQFT_FLAG_FORCE_MULTIPASS))
        return AMQFT_ERR_INVALID_ARG;
    for (int64_t i = 0; i < count; ++i) {
        const int l = log2_exact(lengths_host[i]);
        if (l < 0) return AMQFT_ERR_NOT_POW2;
        if (l > AMQFT_MAX_LOG2N) return AMQFT_ERR_UNSUPPORTED;
    }
    if (count > 0 && offsets_host[0] < 0) return AMQFT_ERR_INVALID_ARG;
    for (int64_t i = 0; i < count; ++i)
        if (offsets_host[i + 1] - offsets_host[i] < lengths_host[i]) return AMQFT_ERR_INVALID_ARG;
    return AMQFT_ERR_UNSUPPORTED;
}

amqft_status amqft_exec(amqft_plan p, const void* in, void* out, void* stream) {
    return exec_common(p, in, out, stream, false);
}

amqft_status amqft_exec_adjoint(amqft_plan p, const void* in, void* out, void* stream) {
    return exec_common(p, in, out, stream, true);
}

amqft_status amqft_power_loss_grad(amqft_plan p, const void* x, const void* w, void* grad, void* loss,
                                   void* stream) {
    if (!p) return AMQFT_ERR_INVALID_ARG;
    if (p->batch == 0) return AMQFT_OK;
    if (!x || !w || !grad || !loss) return AMQFT_ERR_INVALID_ARG;
    if (p->logn < 2 || p->multipass) return AMQFT_ERR_UNSUPPORTED;
    loss_launch a{};
    a.variant = p->variant;
    a.dtype = p->dtype;
    a.logn = p->logn;
    a.batch = p->batch;
    a.x = x;
    a.w = w;
    a.grad = grad;
    a.loss = loss;
    a.ktab = p->ktab;
    a.ktab_log2n = p->ktab_log2n;
    a.onthefly = (p->flags & AMQFT_FLAG_ONTHEFLY_CONSTANTS) != 0;
    hipError_t e = launch_loss(a, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? AMQFT_OK : hip_fail(e);
}

amqft_status amqft_exec_graph(amqft_plan p, const void* in, void* out, int adjoint, void* stream) {
    if (!p || !in || !out) return AMQFT_ERR_INVALID_ARG;
    (void)adjoint; (void)stream;
    return AMQFT_ERR_UNSUPPORTED;
}

amqft_status amqft_plan_destroy(amqft_plan p) {
    if (!p) return AMQFT_OK;
    if (p->ktab) (void)hipFree(p->ktab);
    for (void* w : p->ws)
        if (w) (void)hipFree(w);
    delete p;
    return AMQFT_OK;
}

amqft_status amqft_plan_workspace_size(amqft_plan p, size_t* bytes) {
    if (!p || !bytes) return AMQFT_ERR_INVALID_ARG;
    *bytes = p->ws_bytes;
    return AMQFT_OK;
}

amqft_status amqft_plan_constants(amqft_plan p, int64_t n, double* table_host, int64_t entries) {
    if (!p || !table_host) return AMQFT_ERR_INVALID_ARG;
    const int logn = log2_exact(n);
    if (logn < 2 || logn > p->ktab_log2n) return AMQFT_ERR_INVALID_ARG;
    if (entries < n / 4) return AMQFT_ERR_INVALID_ARG;
    const int shift = p->ktab_log2n - logn;
    for (int64_t i = 0; i < n / 4; ++i) table_host[i] = p->ktab_host[(size_t)(i << shift)];
    return AMQFT_OK;
}

}  // extern "C"
