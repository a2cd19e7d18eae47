// Driver of the CPU emulation of the amqft kernels (test infrastructure):
//   amqft_emu PATH VARIANT DTYPE LOGN BATCH CONJ IN OUT
// PATH: lds (the dispatch of launch_lds: compile-time kernels where they
// exist), generic (the level engine), large (the top/rows/back/bchain
// kernels of variants 4 and 8 over malloc'd workspaces), large_ip (the
// in-place form of that path: the input is copied to the output buffer, which
// the path then transforms in place; with EMU_TRACK_GLOBAL=1 the shim checks
// that no workgroup touches a word another workgroup of the same launch
// writes), large_ip_naive (the same with a slot layout that ignores which
// workgroup reads a slot: the checker's own test), tkernel (the transposed
// compile-time kernel), multipass (the multi-pass engine, sub-blocks as a
// forced plan takes them).  DTYPE 0 = complex FP64, 1 = complex FP32,
// 4 = complex int32 fixed point (Q2.29 constants).
// IN / OUT: raw interleaved complex arrays of BATCH x 2^LOGN values.
// The constant table is built on the host in long double and rounded once.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "amqft_device.h"
#include "amqft_internal.h"
#include "amqft_iplayout.h"

using namespace amqft;

static long double family_value(int fam, long p, long n) {
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

int main(int argc, char** argv) {
    if (argc != 9) {
        std::fprintf(stderr, "usage: %s PATH VARIANT DTYPE LOGN BATCH CONJ IN OUT\n", argv[0]);
        return 2;
    }
    const std::string path = argv[1];
    const int variant = std::atoi(argv[2]), dtype = std::atoi(argv[3]), logn = std::atoi(argv[4]);
    const long batch = std::atol(argv[5]);
    const int conj = std::atoi(argv[6]);
    const long n = 1L << logn;
    const size_t esz = dtype == 0 ? 16 : 8, rsz = esz / 2;
    std::vector<unsigned char> in((size_t)batch * n * esz), out(in.size(), 0xFF);
    FILE* f = std::fopen(argv[7], "rb");
    if (!f || std::fread(in.data(), 1, in.size(), f) != in.size()) { std::fprintf(stderr, "bad input\n"); return 2; }
    std::fclose(f);
    const long q = n / 4 > 1 ? n / 4 : 1;
    std::vector<unsigned char> kt((size_t)q * rsz, 0);
    for (long p = 1; p < q; ++p) {
        const long double lv = family_value(const_family(variant), p, n);
        const double v = (double)lv;
        if (dtype == 0) std::memcpy(&kt[p * rsz], &v, 8);
        else if (dtype == 4) { const int32_t k = (int32_t)llroundl(lv * (long double)(1 << 29)); std::memcpy(&kt[p * rsz], &k, 4); }
        else { const float fv = (float)v; std::memcpy(&kt[p * rsz], &fv, 4); }
    }
    hipError_t e = hipSuccess;
    if (path == "lds" || path == "generic" || path == "tkernel") {
        lds_launch a{};
        a.variant = variant;
        a.dtype = dtype;
        a.logn = logn;
        a.batch = batch;
        a.in = in.data();
        a.out = out.data();
        a.ktab = kt.data();
        a.ktab_log2n = logn;
        a.conj_in = conj;
        a.conj_out = conj;
        a.generic = path == "generic";
        e = path == "tkernel" ? launch_kB(a, nullptr) : launch_lds(a, nullptr);
    } else if (path == "large") {
        kl_launch k{};
        k.variant = variant;
        k.dtype = dtype;
        k.logn = logn;
        k.batch = batch;
        k.chunk = batch;
        std::vector<unsigned char> ws1((size_t)batch * n * esz), ws2(ws1.size()), wsc((size_t)batch * 16 * esz);
        k.in = in.data();
        k.out = out.data();
        k.ws1 = ws1.data();
        k.ws2 = ws2.data();
        k.wsc = wsc.data();
        k.ktab = kt.data();
        k.conj_in = conj;
        k.conj_out = conj;
        e = launch_kL(k, nullptr);
    } else if (path == "multipass") {
        // the multi-pass engine with the sub-block size a forced plan takes
        // (several global levels above it), two chunks when the batch allows
        mp_launch m{};
        m.variant = variant;
        m.dtype = dtype;
        m.logn = logn;
        m.sb = std::max(2, std::min(multipass_sb(dtype), logn - 5));
        m.batch = batch;
        m.chunk = batch > 1 ? batch - 1 : 1;
        std::vector<unsigned char> w0((size_t)m.chunk * n * esz), w1(w0.size()), w2(w0.size());
        m.in = in.data();
        m.out = out.data();
        m.ws0 = w0.data();
        m.ws1 = w1.data();
        m.ws2 = w2.data();
        m.ktab = kt.data();
        m.ktab_log2n = logn;
        m.conj_in = conj;
        m.conj_out = conj;
        e = launch_multipass(m, nullptr);
    } else if (path == "large_ip" || path == "large_ip_naive") {
        kl_launch k{};
        k.variant = variant;
        k.dtype = dtype;
        k.logn = logn;
        k.batch = batch;
        k.chunk = batch > 1 ? batch - 1 : 1;  // two chunks when the batch allows
        std::vector<int> tab;
        int nsh = ip_layout_build(logn, tab);
        if (nsh < 0) { std::fprintf(stderr, "no in-place layout\n"); return 2; }
        if (path == "large_ip_naive") {
            // a layout that ignores which chain workgroup reads a slot (slot s
            // in orbit s + 1, nothing shared): the checker must object
            const int w3 = (int)(n / 16);
            for (int q = 0; q < w3 - 1; ++q) tab[q] = q + 1;
            for (int q = 0; q < w3; ++q) tab[w3 + q] = -1;
            tab.resize(2 * w3);
            nsh = 0;
        }
        std::vector<unsigned char> ws2((size_t)k.chunk * (n / 8 + 16) * esz),
            ws3((size_t)k.chunk * (nsh > 0 ? nsh : 1) * 16 * esz), wsc((size_t)k.chunk * 16 * esz);
        std::memcpy(out.data(), in.data(), in.size());
        k.in = out.data();
        k.out = out.data();
        k.ws2 = ws2.data();
        k.ws3 = ws3.data();
        k.wsc = wsc.data();
        k.iptab = tab.data();
        k.ipnsh = nsh;
        k.inplace = 1;
        k.ktab = kt.data();
        k.conj_in = conj;
        k.conj_out = conj;
        e = launch_kL(k, nullptr);
    } else {
        std::fprintf(stderr, "unknown path %s\n", path.c_str());
        return 2;
    }
    if (e != hipSuccess) { std::fprintf(stderr, "launch failed %d\n", (int)e); return 3; }
    if (emu::g_races.load() > 0) { std::fprintf(stderr, "%ld LDS races\n", emu::g_races.load()); return 4; }
    if (emu::g_global_races.load() > 0) {
        std::fprintf(stderr, "%ld cross-workgroup hazards\n", emu::g_global_races.load());
        return 5;
    }
    f = std::fopen(argv[8], "wb");
    if (!f || std::fwrite(out.data(), 1, out.size(), f) != out.size()) { std::fprintf(stderr, "bad output\n"); return 2; }
    std::fclose(f);
    return 0;
}
