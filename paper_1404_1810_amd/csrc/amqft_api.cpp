// C ABI of the AM-QFT library (declarations and documentation in
// include/amqft.h).  Validation happens before any HIP call so that every
// error path can be exercised without a GPU.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/amqft.h"
#include "amqft_device.h"
#include "amqft_internal.h"
#include "amqft_iplayout.h"

using namespace amqft;

namespace {

// one length class of a many-length plan
struct length_class {
    int logn = 0;
    int64_t count = 0;
    amqft_plan sub = nullptr;     // single-length plan (LDS or multi-pass), NULL = persistent kernel
    void* offsets_dev = nullptr;  // int64 offsets of the class's signals
};

struct graph_entry {
    const void* in;
    void* out;
    int adjoint;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

}  // namespace

struct amqft_plan_s {
    int variant = 4;
    int dtype = 1;
    unsigned flags = 0;
    int64_t n = 0;
    int logn = 0;
    int64_t batch = 0;
    int real_kind = -1;  // amqft_real_kind of a real-transform plan, -1 for the CDFT
    // constant table for length 2^ktab_log2n, working precision, on device
    void* ktab = nullptr;
    int ktab_log2n = 2;
    std::vector<double> ktab_host;  // FP64 values as rounded to working precision
    int device = 0;
    // multi-pass (signals larger than LDS)
    bool multipass = false;
    bool large = false;  // the four-kernel path of amqft_kA.hip (uses ws[0..2] and chunk)
    int sb = 0;
    int64_t chunk = 0;
    void* ws[3] = {nullptr, nullptr, nullptr};
    // in-place large path: shared-slot workspace and slot table (device)
    bool inplace = false;
    void* ws3 = nullptr;
    int* iptab = nullptr;
    int ipnsh = 0;
    size_t ws_bytes = 0;
    const void* offsets = nullptr;  // per-signal offsets (sub-plans of a many-length plan)
    // many-length plans
    bool many = false;
    int64_t count = 0;
    std::vector<length_class> classes;
    void* items_dev = nullptr;     // persistent work list (int4 per item)
    void* poffsets_dev = nullptr;  // offsets in work-list order
    int nitems = 0;
    int grid = 0;  // persistent workgroups
    bool tuned = false;
    // captured graphs
    std::vector<graph_entry> graphs;
    // many-length plans with classes above one workgroup's LDS: those run on
    // a second stream forked from (and joined back into) the caller's stream
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace {

thread_local std::string g_hip_error;

amqft_status hip_fail(hipError_t e) {
    g_hip_error = hipGetErrorString(e);
    (void)hipGetLastError();  // a failed allocation must not resurface at the next launch check
    return e == hipErrorOutOfMemory ? AMQFT_ERR_ALLOC : AMQFT_ERR_HIP;
}

bool valid_variant(int v) { return v >= 1 && v <= 8; }
bool valid_dtype(int t) { return t >= 0 && t <= 4; }
constexpr unsigned kAllFlags = AMQFT_FLAG_ONTHEFLY_CONSTANTS | AMQFT_FLAG_NO_AUTOTUNE | AMQFT_FLAG_FORCE_MULTIPASS |
                               AMQFT_FLAG_FORCE_LARGE | AMQFT_FLAG_TRANSPOSED_ADJOINT | AMQFT_FLAG_IN_PLACE;

// the variant whose program is the transpose of variant v's (skeleton A <-> B)
int dual_variant(int v) {
    static const int d[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    return d[v];
}

// both compile-time kernels exist for v and its dual at this size
bool transposed_adjoint_supported(int v, int logn, int dtype) {
    const int a = (v == 1 || v == 4 || v == 5 || v == 8) ? v : dual_variant(v);
    return kA_supported(a, logn, dtype) && kB_supported(dual_variant(a), logn, dtype);
}
constexpr unsigned kForceFlags = AMQFT_FLAG_FORCE_MULTIPASS | AMQFT_FLAG_FORCE_LARGE;

int log2_exact(int64_t n) {
    if (n < 1 || (n & (n - 1)) != 0) return -1;
    int l = 0;
    while ((int64_t(1) << l) < n) ++l;
    return l;
}

int max_lds_log2(int dtype) { return dtype == AMQFT_C128 ? kMaxLdsLog2F64 : kMaxLdsLog2F32; }

// signals per chunk of a path with chunked workspaces: at most cap, and the
// chunks as equal as they can be (no small last chunk whose launches would
// be all latency)
int64_t balanced_chunk(int64_t batch, int64_t cap) {
    cap = std::max<int64_t>(1, cap);
    if (batch <= cap) return std::max<int64_t>(1, batch);
    const int64_t chunks = (batch + cap - 1) / cap;
    return (batch + chunks - 1) / chunks;
}

// f(2 pi p / n) for the variant's family (Sec. 7.1), evaluated in long double
long double family_value_ld(int fam, int64_t p, int64_t n) {
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double a = 2.0L * pi * (long double)p / (long double)n;
    long double v;
    switch (fam) {
    case 0: v = 2.0L * cosl(a); break;
    case 1: v = 1.0L / (2.0L * cosl(a)); break;
    case 2: v = 2.0L * sinl(a); break;
    default: v = 1.0L / (2.0L * sinl(a)); break;
    }
    return v;
}

// the same rounded to double; the caller rounds once more to the working type
double family_value(int fam, int64_t p, int64_t n) { return (double)family_value_ld(fam, p, n); }

// fixed point: the constant's Q2.29 integer round(f 2^29), ties away from zero
int32_t q29_value(int fam, int64_t p, int64_t n) {
    return (int32_t)llroundl(family_value_ld(fam, p, n) * (long double)(1 << 29));
}

amqft_status build_constants(amqft_plan_s* p, int log2n) {
    const int64_t n = int64_t(1) << (log2n < 2 ? 2 : log2n);
    const int64_t q = n / 4;
    const int fam = const_family(p->variant);
    p->ktab_log2n = log2n < 2 ? 2 : log2n;
    p->ktab_host.assign((size_t)q, 0.0);
    const bool f64 = p->dtype == AMQFT_C128;
    if (p->dtype == AMQFT_C32I) {
        // the kernels read the Q2.29 integers; the host copy holds their values
        std::vector<int32_t> ti((size_t)q, 0);
        for (int64_t i = 1; i < q; ++i) {
            ti[i] = q29_value(fam, i, n);
            p->ktab_host[i] = ldexp((double)ti[i], -29);
        }
        const size_t bytes = (size_t)q * sizeof(int32_t);
        hipError_t e = hipMalloc(&p->ktab, bytes < 16 ? 16 : bytes);
        if (e != hipSuccess) { p->ktab = nullptr; return hip_fail(e); }
        e = hipMemcpy(p->ktab, ti.data(), bytes, hipMemcpyHostToDevice);
        return e == hipSuccess ? AMQFT_OK : hip_fail(e);
    }
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

amqft_status prime(int variant, int dtype) {
    if (dtype == AMQFT_C32I) {
        // fixed point runs on the compile-time kernels only
        hipError_t e = prime_kA(variant, dtype);
        if (e == hipSuccess) e = prime_kB(variant, dtype);
        return e == hipSuccess ? AMQFT_OK : hip_fail(e);
    }
    hipError_t e = prime_lds(variant, dtype);
    if (e == hipSuccess) e = prime_multipass(variant, dtype);
    if (e == hipSuccess) e = prime_kL(variant, dtype);
    return e == hipSuccess ? AMQFT_OK : hip_fail(e);
}

// ---------------------------------------------------------------------------
// tuning cache: JSON lines {"key": "...", "value": N} in $AMQFT_TUNE_CACHE
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

std::string arch_name(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    return a.substr(0, a.find(':'));
}

void tune_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("AMQFT_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        char key[400];
        int v;
        if (sscanf(line, " {\"key\": \"%399[^\"]\", \"value\": %d}", key, &v) == 2) g_tune[key] = v;
    }
    fclose(f);
}

bool tune_get(const std::string& key, int* v) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load();
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *v = it->second;
    return true;
}

void tune_put(const std::string& key, int v) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load();
    g_tune[key] = v;
    const char* path = getenv("AMQFT_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "{\"key\": \"%s\", \"value\": %d}\n", key.c_str(), v);
    fclose(f);
}

amqft_status exec_single(amqft_plan p, const void* in, void* out, hipStream_t stream, bool adjoint) {
    if (p->batch == 0) return AMQFT_OK;
    if (p->real_kind >= 0) {
        // the DCT-0 and DST-0 matrices are symmetric and real: their adjoint is the transform itself
        if (adjoint && p->real_kind == AMQFT_RDFT) return AMQFT_ERR_UNSUPPORTED;
        real_launch r{};
        r.variant = p->variant;
        r.dtype = p->dtype;
        r.logn = p->logn;
        r.kind = p->real_kind;
        r.nreal = p->batch;
        r.in = in;
        r.out = out;
        r.ktab = p->ktab;
        r.ktab_log2n = p->ktab_log2n;
        r.onthefly = (p->flags & AMQFT_FLAG_ONTHEFLY_CONSTANTS) != 0;
        hipError_t e = launch_real(r, stream);
        return e == hipSuccess ? AMQFT_OK : hip_fail(e);
    }
    if (p->large) {
        kl_launch k{};
        k.variant = p->variant;
        k.dtype = p->dtype;
        k.logn = p->logn;
        k.batch = p->batch;
        k.chunk = p->chunk;
        k.in = in;
        k.out = out;
        k.ws1 = p->ws[0];
        k.ws2 = p->ws[1];
        k.wsc = p->ws[2];
        k.ktab = p->ktab;
        k.conj_in = adjoint;
        k.conj_out = adjoint;
        k.offsets = p->offsets;
        k.inplace = p->inplace;
        k.ws3 = p->ws3;
        k.iptab = p->iptab;
        k.ipnsh = p->ipnsh;
        hipError_t e = launch_kL(k, stream);
        return e == hipSuccess ? AMQFT_OK : hip_fail(e);
    }
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
        m.offsets = p->offsets;
        hipError_t e = launch_multipass(m, stream);
        return e == hipSuccess ? AMQFT_OK : hip_fail(e);
    }
    lds_launch a{};
    // the transposed flow graph of variant v: its dual variant's program with
    // the sign of i flipped, i.e. conjugated on load and store
    a.variant = adjoint && (p->flags & AMQFT_FLAG_TRANSPOSED_ADJOINT) ? dual_variant(p->variant) : p->variant;
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
    a.offsets = p->offsets;
    hipError_t e = launch_lds(a, stream);
    return e == hipSuccess ? AMQFT_OK : hip_fail(e);
}

amqft_status exec_many(amqft_plan p, const void* in, void* out, hipStream_t stream, bool adjoint,
                       bool persistent = true, bool classes = true) {
    if (persistent && p->nitems > 0) {
        persistent_launch a{};
        a.variant = p->variant;
        a.dtype = p->dtype;
        a.in = in;
        a.out = out;
        a.ktab = p->ktab;
        a.ktab_log2n = p->ktab_log2n;
        a.items = p->items_dev;
        a.nitems = p->nitems;
        a.offsets = p->poffsets_dev;
        a.grid = p->grid;
        a.conj_in = adjoint;
        a.conj_out = adjoint;
        a.onthefly = (p->flags & AMQFT_FLAG_ONTHEFLY_CONSTANTS) != 0;
        hipError_t e = launch_persistent(a, stream);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (!classes) return AMQFT_OK;
    // long classes (global-memory paths) on the side stream, concurrently with
    // the rest; every class writes only its own signals
    const bool fork = p->side != nullptr;
    if (fork) {
        hipError_t e = hipEventRecord(p->ev_fork, stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->ev_fork, 0);
        if (e != hipSuccess) return hip_fail(e);
    }
    for (const length_class& c : p->classes) {
        if (!c.sub) continue;
        const bool long_class = c.sub->large || c.sub->multipass;
        amqft_status st = exec_single(c.sub, in, out, fork && long_class ? p->side : stream, adjoint);
        if (st != AMQFT_OK) return st;
    }
    if (fork) {
        hipError_t e = hipEventRecord(p->ev_join, p->side);
        if (e == hipSuccess) e = hipStreamWaitEvent(stream, p->ev_join, 0);
        if (e != hipSuccess) return hip_fail(e);
    }
    return AMQFT_OK;
}

amqft_status exec_any(amqft_plan p, const void* in, void* out, hipStream_t stream, bool adjoint) {
    return p->many ? exec_many(p, in, out, stream, adjoint) : exec_single(p, in, out, stream, adjoint);
}

// time one run of fn on stream s (ms), after one warm-up run
template <typename F>
amqft_status time_it(F fn, hipStream_t s, float* ms) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return AMQFT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return AMQFT_ERR_HIP; }
    amqft_status st = fn();
    (void)hipEventRecord(e0, s);
    if (st == AMQFT_OK) st = fn();
    (void)hipEventRecord(e1, s);
    hipError_t e = hipEventSynchronize(e1);
    if (st == AMQFT_OK && e != hipSuccess) st = hip_fail(e);
    if (st == AMQFT_OK) (void)hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

// Autotuning of a many-length plan on its first out-of-place execution: the
// number of persistent workgroups, the sub-block size of each multi-pass
// length class and the chunk (signals per round of kernels) of each large-N
// length class.  Every candidate computes the same transform, so the
// buffers hold a valid result whichever candidate ran last.  Results are
// cached per process and, with AMQFT_TUNE_CACHE set, in that file.
amqft_status autotune(amqft_plan p, const void* in, void* out, hipStream_t user, bool adjoint) {
    if (p->flags & AMQFT_FLAG_NO_AUTOTUNE) {
        p->tuned = true;
        return AMQFT_OK;
    }
    if (in == out) return AMQFT_OK;  // tuning runs overwrite the output: wait for an out-of-place call
    hipError_t e = hipStreamSynchronize(user);
    if (e != hipSuccess) return hip_fail(e);
    hipStream_t s;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e);
    const std::string arch = arch_name(p->device);
    char buf[400];
    amqft_status st = AMQFT_OK;
    if (p->nitems > 0) {
        std::string hist;
        for (const length_class& c : p->classes)
            if (!c.sub) hist += std::to_string(c.logn) + ":" + std::to_string(c.count) + ",";
        snprintf(buf, sizeof buf, "%s/v%d/t%d/persistent/%s", arch.c_str(), p->variant, p->dtype, hist.c_str());
        int g;
        if (tune_get(buf, &g)) {
            p->grid = g;
        } else {
            int cus = 256;
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) cus = prop.multiProcessorCount;
            const int cand[5] = {cus, 2 * cus, 4 * cus, 8 * cus, 16 * cus};
            float best = 1e30f;
            int bestg = p->grid;
            for (int g2 : cand) {
                p->grid = std::max(1, std::min(g2, p->nitems));
                float ms = 0;
                st = time_it([&] { return exec_many(p, in, out, s, adjoint, true, false); }, s, &ms);
                if (st != AMQFT_OK) break;
                if (ms < best) { best = ms; bestg = p->grid; }
            }
            p->grid = bestg;
            if (st == AMQFT_OK) tune_put(buf, bestg);
        }
    }
    for (length_class& c : p->classes) {
        if (st != AMQFT_OK) break;
        if (!c.sub || !c.sub->multipass) continue;
        amqft_plan q = c.sub;
        snprintf(buf, sizeof buf, "%s/v%d/t%d/multipass/logn%d", arch.c_str(), p->variant, p->dtype, c.logn);
        int sbv;
        if (tune_get(buf, &sbv)) {
            q->sb = sbv;
            continue;
        }
        const int hi = std::min(multipass_sb(q->dtype), q->logn - 3);
        float best = 1e30f;
        int bestsb = q->sb;
        for (int cand = std::max(2, hi - 2); cand <= hi; ++cand) {
            q->sb = cand;
            float ms = 0;
            st = time_it([&] { return exec_single(q, in, out, s, adjoint); }, s, &ms);
            if (st != AMQFT_OK) break;
            if (ms < best) { best = ms; bestsb = cand; }
        }
        q->sb = bestsb;
        if (st == AMQFT_OK) tune_put(buf, bestsb);
    }
    // large-N classes: signals per chunk (the workspaces were sized for the
    // largest candidate; smaller chunks keep more of them in the last-level
    // cache between the kernels, larger ones launch fewer kernels)
    for (length_class& c : p->classes) {
        if (st != AMQFT_OK) break;
        if (!c.sub || !c.sub->large) continue;
        amqft_plan q = c.sub;
        snprintf(buf, sizeof buf, "%s/v%d/t%d/large/logn%d/count%lld", arch.c_str(), p->variant, p->dtype, c.logn,
                 (long long)c.count);
        const int64_t cap = q->chunk;
        int ch;
        if (tune_get(buf, &ch)) {
            if (ch >= 1 && ch <= cap) q->chunk = ch;
            continue;
        }
        float best = 1e30f;
        int64_t bestc = cap, prev = 0;
        for (int d = 1; d <= 4; d *= 2) {
            const int64_t cand = balanced_chunk(q->batch, cap / d);
            if (cand == prev) continue;
            prev = cand;
            q->chunk = cand;
            float ms = 0;
            st = time_it([&] { return exec_single(q, in, out, s, adjoint); }, s, &ms);
            if (st != AMQFT_OK) break;
            if (ms < best) { best = ms; bestc = cand; }
        }
        q->chunk = bestc;
        if (st == AMQFT_OK) tune_put(buf, (int)bestc);
    }
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (st == AMQFT_OK) p->tuned = true;
    return st;
}

amqft_status exec_common(amqft_plan p, const void* in, void* out, void* stream, bool adjoint) {
    if (!p) return AMQFT_ERR_INVALID_ARG;
    if ((p->many ? p->count : p->batch) == 0) return AMQFT_OK;  // nothing to read or write
    if (!in || !out) return AMQFT_ERR_INVALID_ARG;
    if ((p->flags & AMQFT_FLAG_IN_PLACE) && in != out) return AMQFT_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->many && !p->tuned) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
            amqft_status st = autotune(p, in, out, s, adjoint);
            if (st != AMQFT_OK) return st;
        }
    }
    return exec_any(p, in, out, s, adjoint);
}

amqft_status create_single(amqft_plan* out, int64_t n, int64_t batch, int variant, int dtype, unsigned flags) {
    const int logn = log2_exact(n);
    const bool force_large = (flags & AMQFT_FLAG_FORCE_LARGE) != 0;
    const bool mp = logn > max_lds_log2(dtype) || (flags & kForceFlags);
    amqft_plan_s* p = new (std::nothrow) amqft_plan_s();
    if (!p) return AMQFT_ERR_ALLOC;
    p->variant = variant;
    p->dtype = dtype;
    p->flags = flags;
    p->n = n;
    p->logn = logn;
    p->batch = batch;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { delete p; return hip_fail(e); }
    amqft_status st = build_constants(p, logn);
    if (st == AMQFT_OK) st = prime(variant, dtype);
    if (st == AMQFT_OK && (flags & AMQFT_FLAG_ONTHEFLY_CONSTANTS) && logn >= 2) {
        // the table that kernels read from global memory (the multi-pass and
        // large-N paths) is generated on the device as well
        e = fill_table_device(p->ktab, variant, dtype, logn, nullptr);
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) st = hip_fail(e);
    }
    if (st != AMQFT_OK) { amqft_plan_destroy(p); return st; }
    if (mp && (flags & AMQFT_FLAG_IN_PLACE)) {
        // the rows stay in the signal buffer; workspaces for the blocks the
        // chain reads at folded indices, the shared slots and the chain
        p->large = true;
        p->inplace = true;
        std::vector<int> tab;
        p->ipnsh = ip_layout_build(logn, tab);
        if (p->ipnsh < 0) { amqft_plan_destroy(p); return AMQFT_ERR_UNSUPPORTED; }
        e = hipMalloc(&p->iptab, tab.size() * sizeof(int));
        if (e == hipSuccess) e = hipMemcpy(p->iptab, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e != hipSuccess) { amqft_plan_destroy(p); return hip_fail(e); }
        const size_t esz = dtype == AMQFT_C128 ? 16 : 8;
        const size_t per2 = ((size_t(1) << logn) / 8 + 16) * esz, per3 = (size_t)p->ipnsh * 16 * esz, perc = 16 * esz;
        size_t cap = size_t(128) << 20;
        if (const char* env = getenv("AMQFT_LARGE_WS_MB")) {
            const long mb = atol(env);
            if (mb >= 1 && mb <= (1l << 20)) cap = size_t(mb) << 20;
        }
        p->chunk = balanced_chunk(batch, (int64_t)(cap / per2));
        p->ws_bytes = (size_t)p->chunk * (per2 + per3 + perc);
        if (batch > 0) {
            e = hipMalloc(&p->ws[1], (size_t)p->chunk * per2);
            if (e == hipSuccess) e = hipMalloc(&p->ws[2], (size_t)p->chunk * perc);
            if (e == hipSuccess) e = hipMalloc(&p->ws3, std::max<size_t>(1, (size_t)p->chunk * per3));
            if (e != hipSuccess) { amqft_plan_destroy(p); return hip_fail(e); }
        }
    } else if (mp && !(flags & AMQFT_FLAG_FORCE_MULTIPASS) &&
        (force_large ? kL_supported_forced(variant, logn, dtype) : kL_supported(variant, logn, dtype))) {
        // workspaces sized so that both stay within the last-level cache
        p->large = true;
        const size_t per = kL_ws_bytes_per_signal(logn, dtype);
        size_t cap = size_t(128) << 20;  // bytes per workspace buffer
        if (const char* env = getenv("AMQFT_LARGE_WS_MB")) {
            const long mb = atol(env);
            if (mb >= 1 && mb <= (1l << 20)) cap = size_t(mb) << 20;
        }
        p->chunk = balanced_chunk(batch, (int64_t)(cap / per));
        const size_t chain = (size_t)p->chunk * 16 * (dtype == AMQFT_C128 ? 16 : 8);
        p->ws_bytes = 2 * (size_t)p->chunk * per + chain;
        for (int i = 0; i < 3 && batch > 0; ++i) {
            e = hipMalloc(&p->ws[i], i < 2 ? (size_t)p->chunk * per : chain);
            if (e != hipSuccess) { p->ws[i] = nullptr; amqft_plan_destroy(p); return hip_fail(e); }
        }
    } else if (mp) {
        p->multipass = true;
        // forced (test) plans use small sub-blocks so that several global levels run
        p->sb = (flags & AMQFT_FLAG_FORCE_MULTIPASS) ? std::max(2, std::min(multipass_sb(dtype), logn - 5))
                                                     : std::min(multipass_sb(dtype), logn - 3);
        const size_t per = multipass_ws_bytes_per_signal(logn, dtype);
        const size_t cap = size_t(1) << 30;  // bytes per workspace buffer
        p->chunk = balanced_chunk(batch, (int64_t)(cap / per));
        p->ws_bytes = 3 * (size_t)p->chunk * per;
        for (int i = 0; i < 3 && batch > 0; ++i) {
            e = hipMalloc(&p->ws[i], (size_t)p->chunk * per);
            if (e != hipSuccess) { p->ws[i] = nullptr; amqft_plan_destroy(p); return hip_fail(e); }
        }
    }
    *out = p;
    return AMQFT_OK;
}

}  // namespace

int amqft::record_hip_failure(hipError_t e) { return (int)hip_fail(e); }

extern "C" {

const char* amqft_version(void) { return "amqft 0.2.0 (gfx950)"; }

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
    if (flags & ~kAllFlags) return AMQFT_ERR_INVALID_ARG;
    const int logn = log2_exact(n);
    if (logn < 0) return AMQFT_ERR_NOT_POW2;
    if (logn > AMQFT_MAX_LOG2N) return AMQFT_ERR_UNSUPPORTED;
    if ((flags & kForceFlags) == kForceFlags) return AMQFT_ERR_UNSUPPORTED;
    if (dtype == AMQFT_C32I &&
        ((flags & kForceFlags) || !(kA_supported((int)variant, logn, AMQFT_C32I) ||
                                    kB_supported((int)variant, logn, AMQFT_C32I))))
        return AMQFT_ERR_UNSUPPORTED;
    if ((flags & AMQFT_FLAG_TRANSPOSED_ADJOINT) &&
        ((flags & kForceFlags) || !transposed_adjoint_supported((int)variant, logn, (int)dtype)))
        return AMQFT_ERR_UNSUPPORTED;
    if ((flags & AMQFT_FLAG_FORCE_LARGE) && !kL_supported_forced((int)variant, logn, (int)dtype))
        return AMQFT_ERR_UNSUPPORTED;
    const bool mp = logn > max_lds_log2((int)dtype) || (flags & kForceFlags);
    if ((flags & AMQFT_FLAG_IN_PLACE) && mp &&
        ((flags & AMQFT_FLAG_FORCE_MULTIPASS) ||
         !kL_inplace_supported((int)variant, logn, (int)dtype, (flags & AMQFT_FLAG_FORCE_LARGE) != 0)))
        return AMQFT_ERR_UNSUPPORTED;
    if (mp && logn < 5) return AMQFT_ERR_UNSUPPORTED;  // multi-pass needs a block of at least 8 points
    if (batch > (int64_t(1) << 40)) return AMQFT_ERR_UNSUPPORTED;
    return create_single(out, n, batch, (int)variant, (int)dtype, flags);
}

amqft_status amqft_plan_create_real(amqft_plan* out, int64_t n, int64_t batch, amqft_real_kind kind,
                                    amqft_variant variant, amqft_dtype dtype, unsigned flags) {
    if (!out) return AMQFT_ERR_INVALID_ARG;
    *out = nullptr;
    if (!valid_variant((int)variant) || !valid_dtype((int)dtype) || batch < 0) return AMQFT_ERR_INVALID_ARG;
    if ((int)kind < AMQFT_RDFT || (int)kind > AMQFT_DST0) return AMQFT_ERR_INVALID_ARG;
    if (flags & ~kAllFlags) return AMQFT_ERR_INVALID_ARG;
    const int logn = log2_exact(n);
    if (logn < 0) return AMQFT_ERR_NOT_POW2;
    if (flags & (kForceFlags | AMQFT_FLAG_TRANSPOSED_ADJOINT | AMQFT_FLAG_IN_PLACE)) return AMQFT_ERR_UNSUPPORTED;
    if (dtype != AMQFT_C128 && dtype != AMQFT_C64) return AMQFT_ERR_UNSUPPORTED;  // also no fixed point
    if (logn < 2 || logn > max_lds_log2((int)dtype)) return AMQFT_ERR_UNSUPPORTED;
    if (batch > (int64_t(1) << 40)) return AMQFT_ERR_UNSUPPORTED;
    amqft_plan_s* p = new (std::nothrow) amqft_plan_s();
    if (!p) return AMQFT_ERR_ALLOC;
    p->variant = (int)variant;
    p->dtype = (int)dtype;
    p->flags = flags;
    p->n = n;
    p->logn = logn;
    p->batch = batch;
    p->real_kind = (int)kind;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { delete p; return hip_fail(e); }
    amqft_status st = build_constants(p, logn);
    if (st == AMQFT_OK) st = prime((int)variant, (int)dtype);
    if (st != AMQFT_OK) { amqft_plan_destroy(p); return st; }
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
    if (flags & ~kAllFlags) return AMQFT_ERR_INVALID_ARG;
    if (flags & (AMQFT_FLAG_TRANSPOSED_ADJOINT | AMQFT_FLAG_IN_PLACE)) return AMQFT_ERR_UNSUPPORTED;
    if (dtype == AMQFT_C32I) return AMQFT_ERR_UNSUPPORTED;
    int maxlog = 2;
    for (int64_t i = 0; i < count; ++i) {
        const int l = log2_exact(lengths_host[i]);
        if (l < 0) return AMQFT_ERR_NOT_POW2;
        if (l > AMQFT_MAX_LOG2N) return AMQFT_ERR_UNSUPPORTED;
        maxlog = std::max(maxlog, l);
    }
    if (count > 0 && offsets_host[0] < 0) return AMQFT_ERR_INVALID_ARG;
    for (int64_t i = 0; i < count; ++i)
        if (offsets_host[i + 1] - offsets_host[i] < lengths_host[i]) return AMQFT_ERR_INVALID_ARG;

    amqft_plan_s* p = new (std::nothrow) amqft_plan_s();
    if (!p) return AMQFT_ERR_ALLOC;
    p->variant = (int)variant;
    p->dtype = (int)dtype;
    p->flags = flags & ~kForceFlags;
    p->many = true;
    p->count = count;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { delete p; return hip_fail(e); }
    amqft_status st = build_constants(p, maxlog);
    if (st == AMQFT_OK) st = prime((int)variant, (int)dtype);
    if (st == AMQFT_OK && (flags & AMQFT_FLAG_ONTHEFLY_CONSTANTS) && maxlog >= 2) {
        // the same FP64 device values the persistent kernel generates per workgroup
        e = fill_table_device(p->ktab, (int)variant, (int)dtype, p->ktab_log2n, nullptr);
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) st = hip_fail(e);
    }
    if (st != AMQFT_OK) { amqft_plan_destroy(p); return st; }

    // group the signals by length
    std::vector<std::vector<int64_t>> by(AMQFT_MAX_LOG2N + 1);
    for (int64_t i = 0; i < count; ++i) by[log2_exact(lengths_host[i])].push_back(offsets_host[i]);
    // persistent work list: the lengths without a compile-time kernel (up to
    // kPersistentMaxLog2, or below 2^8 where one exists), items of up to 256/T
    // signals of one length, longest length first
    const int pmax = (kA_supported(p->variant, 8, p->dtype) || kB_supported(p->variant, 8, p->dtype))
                         ? 7 : kPersistentMaxLog2;
    std::vector<int> items;  // 4 ints per item
    std::vector<long long> poffs;
    for (int l = pmax; l >= 0; --l) {
        const std::vector<int64_t>& v = by[l];
        if (v.empty()) continue;
        length_class c;
        c.logn = l;
        c.count = (int64_t)v.size();
        p->classes.push_back(c);
        const int N = 1 << l;
        const int T = (N >> 4) > 1 ? (N >> 4) : 1;
        const int spw = l <= 1 ? 256 : 256 / T;
        for (size_t s0 = 0; s0 < v.size(); s0 += spw) {
            const int cnt = (int)std::min<size_t>(spw, v.size() - s0);
            items.push_back(l);
            items.push_back((int)poffs.size());
            items.push_back(cnt);
            items.push_back(0);
            for (int u = 0; u < cnt; ++u) poffs.push_back(v[s0 + u]);
        }
    }
    p->nitems = (int)(items.size() / 4);
    if (p->nitems > 0) {
        e = hipMalloc(&p->items_dev, items.size() * sizeof(int));
        if (e == hipSuccess)
            e = hipMemcpy(p->items_dev, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc(&p->poffsets_dev, poffs.size() * sizeof(long long));
        if (e == hipSuccess)
            e = hipMemcpy(p->poffsets_dev, poffs.data(), poffs.size() * sizeof(long long), hipMemcpyHostToDevice);
        if (e != hipSuccess) { amqft_plan_destroy(p); return hip_fail(e); }
        int cus = 256;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) cus = prop.multiProcessorCount;
        p->grid = std::max(1, std::min(4 * cus, p->nitems));
    }
    // longer lengths: one single-length plan per class over the packed buffer
    for (int l = pmax + 1; l <= AMQFT_MAX_LOG2N; ++l) {
        const std::vector<int64_t>& v = by[l];
        if (v.empty()) continue;
        length_class c;
        c.logn = l;
        c.count = (int64_t)v.size();
        st = create_single(&c.sub, int64_t(1) << l, c.count, p->variant, p->dtype, p->flags);
        if (st == AMQFT_OK) {
            e = hipMalloc(&c.offsets_dev, v.size() * sizeof(int64_t));
            if (e == hipSuccess)
                e = hipMemcpy(c.offsets_dev, v.data(), v.size() * sizeof(int64_t), hipMemcpyHostToDevice);
            if (e != hipSuccess) st = hip_fail(e);
            else c.sub->offsets = c.offsets_dev;
        }
        p->classes.push_back(c);
        if (st != AMQFT_OK) { amqft_plan_destroy(p); return st; }
        p->ws_bytes += c.sub->ws_bytes;
    }
    bool has_long = false, has_short = p->nitems > 0;
    for (const length_class& c : p->classes) {
        if (!c.sub) continue;
        if (c.sub->large || c.sub->multipass) has_long = true;
        else has_short = true;
    }
    if (has_long && has_short) {
        e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);  // default priority
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
        if (e != hipSuccess) { amqft_plan_destroy(p); return hip_fail(e); }
    }
    *out = p;
    return AMQFT_OK;
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
    if (p->many) return AMQFT_ERR_UNSUPPORTED;
    if (p->batch == 0) return AMQFT_OK;
    if (!x || !w || !grad || !loss) return AMQFT_ERR_INVALID_ARG;
    if (p->logn < 2 || p->multipass || p->large || p->real_kind >= 0) return AMQFT_ERR_UNSUPPORTED;
    if (p->dtype == AMQFT_C32I) return AMQFT_ERR_UNSUPPORTED;
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
    if (!p) return AMQFT_ERR_INVALID_ARG;
    if ((p->many ? p->count : p->batch) == 0) return AMQFT_OK;
    if (!in || !out) return AMQFT_ERR_INVALID_ARG;
    if ((p->flags & AMQFT_FLAG_IN_PLACE) && in != out) return AMQFT_ERR_INVALID_ARG;
    hipStream_t user = static_cast<hipStream_t>(stream);
    graph_entry* g = nullptr;
    for (graph_entry& ge : p->graphs)
        if (ge.in == in && ge.out == out && ge.adjoint == (adjoint != 0)) g = &ge;
    if (!g) {
        // tuning synchronises and times candidates, so it happens before capture
        if (p->many && !p->tuned) {
            amqft_status st = autotune(p, in, out, user, adjoint != 0);
            if (st != AMQFT_OK) return st;
        }
        hipStream_t cs;
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e);
        graph_entry ne{in, out, adjoint != 0, nullptr, nullptr};
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        amqft_status st = AMQFT_OK;
        if (e == hipSuccess) {
            st = exec_any(p, in, out, cs, adjoint != 0);
            hipError_t e2 = hipStreamEndCapture(cs, &ne.graph);
            if (st == AMQFT_OK && e2 != hipSuccess) st = hip_fail(e2);
        } else {
            st = hip_fail(e);
        }
        if (st == AMQFT_OK) {
            e = hipGraphInstantiate(&ne.exec, ne.graph, nullptr, nullptr, 0);
            if (e != hipSuccess) st = hip_fail(e);
        }
        (void)hipStreamDestroy(cs);
        if (st != AMQFT_OK) {
            if (ne.exec) (void)hipGraphExecDestroy(ne.exec);
            if (ne.graph) (void)hipGraphDestroy(ne.graph);
            return st;
        }
        p->graphs.push_back(ne);
        g = &p->graphs.back();
    }
    hipError_t e = hipGraphLaunch(g->exec, user);
    return e == hipSuccess ? AMQFT_OK : hip_fail(e);
}

amqft_status amqft_plan_destroy(amqft_plan p) {
    if (!p) return AMQFT_OK;
    for (graph_entry& g : p->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    for (length_class& c : p->classes) {
        if (c.sub) amqft_plan_destroy(c.sub);
        if (c.offsets_dev) (void)hipFree(c.offsets_dev);
    }
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->side) (void)hipStreamDestroy(p->side);
    if (p->items_dev) (void)hipFree(p->items_dev);
    if (p->poffsets_dev) (void)hipFree(p->poffsets_dev);
    if (p->ktab) (void)hipFree(p->ktab);
    for (void* w : p->ws)
        if (w) (void)hipFree(w);
    if (p->ws3) (void)hipFree(p->ws3);
    if (p->iptab) (void)hipFree(p->iptab);
    delete p;
    return AMQFT_OK;
}

amqft_status amqft_plan_describe(amqft_plan p, char* buf, size_t len) {
    if (!p || !buf || len == 0) return AMQFT_ERR_INVALID_ARG;
    if (p->real_kind >= 0) {
        static const char* kinds[3] = {"REAL_RDFT", "REAL_DCT0", "REAL_DST0"};
        int threads = 0, spw = 1;
        size_t lds = 0;
        lds_shape(p->logn, p->dtype, &threads, &spw, &lds);
        snprintf(buf, len, "amqft_real_kernel<%d, %s, %s> grid=%lld block=%d lds=%zu", p->variant,
                 p->dtype == AMQFT_C128 ? "double" : "float", kinds[p->real_kind],
                 (long long)(((p->batch + 1) / 2 + spw - 1) / spw), threads, lds);
    } else if (p->many) {
        int nclass = 0;
        for (auto& c : p->classes) nclass += c.sub ? 1 : 0;
        snprintf(buf, len, "many-length plan: %lld signals, persistent kernel grid=%d items=%d, %d long-length classes",
                 (long long)p->count, p->grid, p->nitems, nclass);
    } else if (p->inplace) {
        snprintf(buf, len, "amqft_kL_{top_ip,rows,back_ip,bchain_ip}<%d> in place n=%lld chunk=%lld shared=%d",
                 p->variant, (long long)p->n, (long long)p->chunk, p->ipnsh);
    } else if (p->large) {
        const bool transposed = p->variant == 2 || p->variant == 6;
        snprintf(buf, len, transposed       ? (p->logn >= 18 ? "amqft_kLT_{c0,fold,b0,rback,rows,rtop,top}<%d> n=%lld chunk=%lld"
                                                             : "amqft_kLT_{c0,fold,b0,rows,top}<%d> n=%lld chunk=%lld")
                           : p->logn >= 18 ? "amqft_kL_{top,rtop,rows,rback,back,bchain}<%d> n=%lld chunk=%lld"
                                           : "amqft_kL_{top,rows,back,bchain}<%d> n=%lld chunk=%lld",
                 p->variant, (long long)p->n, (long long)p->chunk);
    } else if (p->multipass) {
        snprintf(buf, len, "multi-pass engine n=%lld sb=%d chunk=%lld", (long long)p->n, p->sb, (long long)p->chunk);
    } else {
        lds_launch a{};
        a.variant = p->variant;
        a.dtype = p->dtype;
        a.logn = p->logn;
        a.batch = p->batch;
        describe_lds(a, buf, len);
    }
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
    if (!(p->flags & AMQFT_FLAG_ONTHEFLY_CONSTANTS)) {
        for (int64_t i = 0; i < n / 4; ++i) table_host[i] = p->ktab_host[(size_t)(i << shift)];
        return AMQFT_OK;
    }
    // generated on the device: copy the table back as the kernels read it
    const size_t q = size_t(1) << (p->ktab_log2n - 2);
    if (p->dtype == AMQFT_C32I) {
        std::vector<int32_t> ti(q);
        hipError_t e = hipMemcpy(ti.data(), p->ktab, q * sizeof(int32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e);
        for (int64_t i = 0; i < n / 4; ++i) table_host[i] = ldexp((double)ti[(size_t)(i << shift)], -29);
        return AMQFT_OK;
    }
    const bool f64 = p->dtype == AMQFT_C128;
    std::vector<double> td;
    std::vector<float> tf;
    if (f64) td.resize(q);
    else tf.resize(q);
    hipError_t e = hipMemcpy(f64 ? (void*)td.data() : (void*)tf.data(), p->ktab, q * (f64 ? sizeof(double) : sizeof(float)),
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    for (int64_t i = 0; i < n / 4; ++i) {
        const size_t j = (size_t)(i << shift);
        table_host[i] = f64 ? td[j] : (double)tf[j];
    }
    return AMQFT_OK;
}

}  // extern "C"
