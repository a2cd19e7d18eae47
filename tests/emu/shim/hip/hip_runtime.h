// CPU emulation of the HIP device environment the amqft kernels use -- TEST
// INFRASTRUCTURE ONLY (tests/test_emu.py).  Every workgroup runs as
// blockDim.x host threads; __syncthreads is a barrier of those threads;
// lane moves (shuffles, DPP row shifts) exchange through a per-wave buffer
// between two wave barriers; dynamic LDS is a heap block of exactly the
// requested size, filled with NaN bytes before the workgroup starts, so that
// AddressSanitizer sees every access outside it and reads of unwritten words
// come out NaN.  Buffer loads and stores outside their resource abort.
// Workgroups run one after another.
#pragma once
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __align__(n) alignas(n)

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct emu_uint3 {
    unsigned x, y, z;
};
struct alignas(16) double2 { double x, y; };
struct alignas(8) float2 { float x, y; };
struct alignas(16) int4 { int x, y, z, w; };
inline double2 make_double2(double a, double b) { return {a, b}; }
inline float2 make_float2(float a, float b) { return {a, b}; }
struct alignas(8) int2 { int x, y; };
inline int2 make_int2(int a, int b) { return {a, b}; }

typedef enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2, hipErrorInvalidSymbol = 13 } hipError_t;
typedef void* hipStream_t;
enum { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
inline hipError_t hipFuncSetAttribute(const void*, int, int) { return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "emulated"; }

namespace emu {

// Barrier-interval race checker over the LDS accesses made through ldc /
// stc: every 8-byte word remembers the last writer and reader (thread and
// barrier epoch); a write after another thread's read or write, or a read
// after another thread's write, in the same epoch is a race.
struct word_state {
    int w_epoch = -1, w_thread = -1, w_wepoch = -1, r_epoch = -1, r_thread = -1, r_wepoch = -1;
};

struct epoch_tick {
    void operator()() noexcept;
};

struct block_state {
    std::unique_ptr<std::barrier<epoch_tick>> bar;
    std::vector<std::unique_ptr<std::barrier<>>> wave_bar;
    std::vector<uint64_t> xbuf;  // per lane, two words (lane moves of up to 16 bytes)
    unsigned char* lds = nullptr;
    size_t lds_bytes = 0;
    int epoch = 0;
    std::vector<word_state> words;
    std::mutex mu;
};

inline block_state* g_block = nullptr;
inline std::atomic<long> g_races{0};

inline void epoch_tick::operator()() noexcept { ++g_block->epoch; }
inline thread_local emu_uint3 t_threadIdx{0, 0, 0}, t_blockIdx{0, 0, 0};
inline thread_local dim3 t_blockDim{1, 1, 1}, t_gridDim{1, 1, 1};
inline thread_local int t_wave_epoch = 0;  // wave barriers this thread has passed

inline unsigned char* lds_base() { return g_block->lds; }

// Cross-workgroup checker over global memory (enabled by EMU_TRACK_GLOBAL=1;
// accesses made through buffer loads / stores and the in-place path's xld /
// xst): within one launch, every 8-byte word remembers the workgroup that
// wrote it and the one that read it (-2: several); a word written by one
// workgroup and read or written by another is a cross-workgroup hazard --
// workgroups run in no defined order on the GPU.
struct gword {
    int w = -1, r = -1;
};
inline std::mutex g_gmu;
inline std::unordered_map<uintptr_t, gword> g_gwords;
inline std::atomic<long> g_global_races{0};
inline bool g_track = std::getenv("EMU_TRACK_GLOBAL") && std::atoi(std::getenv("EMU_TRACK_GLOBAL")) != 0;
inline thread_local int t_block_id = 0;

inline void global_touch(const void* p, size_t bytes, bool write) {
    if (!g_track) return;
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(p) & ~uintptr_t(7);
    const uintptr_t a1 = reinterpret_cast<uintptr_t>(p) + bytes;
    const int b = t_block_id;
    std::lock_guard<std::mutex> g(g_gmu);
    for (uintptr_t a = a0; a < a1; a += 8) {
        gword& s = g_gwords[a];
        bool bad;
        if (write) {
            bad = (s.w >= 0 && s.w != b) || (s.r != -1 && s.r != b);
            s.w = b;
        } else {
            bad = s.w >= 0 && s.w != b;
            s.r = s.r == -1 || s.r == b ? b : -2;
        }
        if (bad && g_global_races.fetch_add(1) < 8)
            std::fprintf(stderr, "emu: global word %#lx %s by workgroup %d, touched by workgroup %d/%d\n",
                         (unsigned long)a, write ? "written" : "read", b, s.w, s.r);
    }
}

inline void lds_touch(const void* p, size_t bytes, bool write) {
    block_state* b = g_block;
    if (!b || !b->lds) return;
    const unsigned char* c = static_cast<const unsigned char*>(p);
    if (c < b->lds || c >= b->lds + b->lds_bytes) return;  // not LDS
    const int t = (int)t_threadIdx.x, we = t_wave_epoch;
    // two accesses by lanes of one wave on either side of a wave barrier are ordered
    auto ordered = [&](int other, int other_we) {
        return other >= 0 && (other >> 6) == (t >> 6) && other_we != we;
    };
    std::lock_guard<std::mutex> g(b->mu);
    for (size_t w = (size_t)(c - b->lds) / 8; w <= (size_t)(c - b->lds + bytes - 1) / 8; ++w) {
        word_state& s = b->words[w];
        const bool wr = s.w_epoch == b->epoch && s.w_thread != t && !ordered(s.w_thread, s.w_wepoch);
        const bool rd = s.r_epoch == b->epoch && s.r_thread != t && !ordered(s.r_thread, s.r_wepoch);
        const bool race = write ? (wr || rd) : wr;
        if (race && g_races.fetch_add(1) < 10)
            std::fprintf(stderr, "emu: LDS race at byte %zu, block (%u,%u,%u), thread %d %s, epoch %d\n", w * 8,
                         t_blockIdx.x, t_blockIdx.y, t_blockIdx.z, t, write ? "writes" : "reads", b->epoch);
        if (write) {
            s.w_epoch = b->epoch;
            s.w_thread = t;
            s.w_wepoch = we;
        } else if (s.r_epoch == b->epoch && s.r_thread != t && !ordered(s.r_thread, s.r_wepoch)) {
            s.r_thread = -2;  // several unordered readers
        } else {
            s.r_epoch = b->epoch;
            s.r_thread = t;
            s.r_wepoch = we;
        }
    }
}
inline void syncthreads() { g_block->bar->arrive_and_wait(); }
// wave barrier (every lane of the calling wave): orders the wave's LDS accesses
inline void wave_barrier() {
    g_block->wave_bar[t_threadIdx.x >> 6]->arrive_and_wait();
    ++t_wave_epoch;
}
inline int lane() { return (int)(t_threadIdx.x & 63u); }
inline int wave() { return (int)(t_threadIdx.x >> 6); }

// every lane of the wave publishes v; returns the value of lane src(lane)
template <typename T, typename F>
inline T wave_move(T v, F src) {
    static_assert(sizeof(T) <= 16, "lane moves of at most 16 bytes");
    block_state* b = g_block;
    const int w = wave(), l = lane();
    uint64_t* slot = &b->xbuf[(size_t)(w * 64 + l) * 2];
    std::memcpy(slot, &v, sizeof(T));
    b->wave_bar[w]->arrive_and_wait();
    const int s = src(l);
    T r = v;
    if (s >= 0) std::memcpy(&r, &b->xbuf[(size_t)(w * 64 + s) * 2], sizeof(T));
    b->wave_bar[w]->arrive_and_wait();
    return r;
}

struct rsrc {
    const char* base;
    long long nbytes;
};
inline rsrc make_rsrc(const void* p, long long n) { return {static_cast<const char*>(p), n}; }
inline void check_range(const rsrc& r, long long off, int size) {
    if (off < 0 || off + size > r.nbytes) {
        std::fprintf(stderr, "emu: buffer access at byte %lld (+%d) outside a %lld-byte resource\n", off, size,
                     r.nbytes);
        std::abort();
    }
}
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
template <typename T>
inline T buf_load(rsrc r, int vo, int so) {
    check_range(r, (long long)vo + so, (int)sizeof(T));
    global_touch(r.base + vo + so, sizeof(T), false);
    T v;
    std::memcpy(&v, r.base + vo + so, sizeof(T));
    return v;
}
template <typename T>
inline void buf_store(T v, rsrc r, int vo, int so) {
    check_range(r, (long long)vo + so, (int)sizeof(T));
    global_touch(r.base + vo + so, sizeof(T), true);
    std::memcpy(const_cast<char*>(r.base) + vo + so, &v, sizeof(T));
}

// DPP: row_shl:D (0x101..0x10F), row_shr:D (0x111..0x11F) inside rows of 16
// lanes, wave_shl:1 (0x130), wave_shr:1 (0x138); an invalid source lane
// yields `old` (bound_ctrl off)
inline int update_dpp(int old, int src, int ctrl, int, int, bool) {
    int valid_src = 0;
    const int r = wave_move<int>(src, [&](int l) {
        int s = -1;
        if (ctrl >= 0x101 && ctrl <= 0x10F) s = ((l & 15) + (ctrl - 0x100) < 16) ? l + (ctrl - 0x100) : -1;
        else if (ctrl >= 0x111 && ctrl <= 0x11F) s = ((l & 15) - (ctrl - 0x110) >= 0) ? l - (ctrl - 0x110) : -1;
        else if (ctrl == 0x130) s = l + 1 < 64 ? l + 1 : -1;
        else if (ctrl == 0x138) s = l >= 1 ? l - 1 : -1;
        else { std::fprintf(stderr, "emu: DPP control 0x%x not emulated\n", ctrl); std::abort(); }
        valid_src = s >= 0;
        return s;
    });
    return valid_src ? r : old;
}

template <typename... P, typename... A>
void launch(void (*k)(P...), dim3 grid, dim3 block, size_t shmem, hipStream_t, A&&... args) {
    if (block.y != 1 || block.z != 1 || block.x == 0 || block.x > 1024) {
        std::fprintf(stderr, "emu: unsupported block shape\n");
        std::abort();
    }
    const unsigned nt = block.x, nw = (nt + 63) / 64;
    if (g_track) g_gwords.clear();  // hazards are within one launch
    for (unsigned bz = 0; bz < grid.z; ++bz)
        for (unsigned by = 0; by < grid.y; ++by)
            for (unsigned bx = 0; bx < grid.x; ++bx) {
                block_state st;
                st.bar = std::make_unique<std::barrier<epoch_tick>>((std::ptrdiff_t)nt);
                for (unsigned w = 0; w < nw; ++w) {
                    const unsigned lanes = (w + 1) * 64 <= nt ? 64 : nt - w * 64;
                    st.wave_bar.push_back(std::make_unique<std::barrier<>>((std::ptrdiff_t)lanes));
                }
                st.xbuf.assign((size_t)nw * 64 * 2, 0);
                st.lds = shmem ? static_cast<unsigned char*>(std::malloc(shmem)) : nullptr;
                if (shmem) std::memset(st.lds, 0xFF, shmem);  // NaN in FP32 and FP64
                st.lds_bytes = shmem;
                st.words.assign((shmem + 7) / 8, word_state{});
                g_block = &st;
                std::vector<std::thread> th;
                th.reserve(nt);
                for (unsigned t = 0; t < nt; ++t) {
                    th.emplace_back([&, t] {
                        t_threadIdx = {t, 0, 0};
                        t_blockIdx = {bx, by, bz};
                        t_block_id = (int)(bx + grid.x * (by + grid.y * bz));
                        t_blockDim = block;
                        t_gridDim = grid;
                        k(static_cast<P>(args)...);
                        st.wave_bar[t >> 6]->arrive_and_drop();
                        st.bar->arrive_and_drop();
                    });
                }
                for (auto& x : th) x.join();
                g_block = nullptr;
                std::free(st.lds);
            }
}

}  // namespace emu

#define threadIdx (::emu::t_threadIdx)
#define blockIdx (::emu::t_blockIdx)
#define blockDim (::emu::t_blockDim)
#define gridDim (::emu::t_gridDim)
#define __syncthreads() ::emu::syncthreads()
#define hipLaunchKernelGGL(K, G, B, SH, ST, ...) ::emu::launch(K, G, B, SH, ST, __VA_ARGS__)

inline int __clz(int x) { return x == 0 ? 32 : __builtin_clz((unsigned)x); }
inline int __ffs(int x) { return __builtin_ffs(x); }
inline int __popc(unsigned x) { return __builtin_popcount(x); }
inline float __uint_as_float(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
inline uint32_t __float_as_uint(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
inline double cospi(double x) { return (double)std::cos(3.141592653589793238462643383279502884L * (long double)x); }
inline double sinpi(double x) { return (double)std::sin(3.141592653589793238462643383279502884L * (long double)x); }

template <typename T> inline T __shfl_up(T v, unsigned d) {
    return ::emu::wave_move<T>(v, [&](int l) { return l - (int)d >= 0 ? l - (int)d : l; });
}
template <typename T> inline T __shfl_down(T v, unsigned d) {
    return ::emu::wave_move<T>(v, [&](int l) { return l + (int)d < 64 ? l + (int)d : l; });
}
template <typename T> inline T __shfl_xor(T v, int m) {
    return ::emu::wave_move<T>(v, [&](int l) { return l ^ m; });
}

#define __amdgpu_buffer_rsrc_t ::emu::rsrc
#define __builtin_amdgcn_make_buffer_rsrc(p, stride, n, flags) ::emu::make_rsrc((const void*)(p), (long long)(n))
#define __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, aux) ::emu::buf_load<unsigned>(r, vo, so)
#define __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, aux) ::emu::buf_load<::emu::u32x2>(r, vo, so)
#define __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, aux) ::emu::buf_load<::emu::u32x4>(r, vo, so)
#define __builtin_amdgcn_raw_buffer_store_b32(v, r, vo, so, aux) ::emu::buf_store<unsigned>(v, r, vo, so)
#define __builtin_amdgcn_raw_buffer_store_b64(v, r, vo, so, aux) ::emu::buf_store<::emu::u32x2>(v, r, vo, so)
#define __builtin_amdgcn_raw_buffer_store_b128(v, r, vo, so, aux) ::emu::buf_store<::emu::u32x4>(v, r, vo, so)
#define __builtin_amdgcn_readfirstlane(x) (x)
#define __builtin_amdgcn_readlane(x, l) ::emu::wave_move<int>((int)(x), [&](int) { return (int)(l); })
#define __builtin_amdgcn_wave_barrier() ::emu::wave_barrier()
#define __builtin_amdgcn_fence(order, scope) ((void)0)
#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) ::emu::update_dpp(old, src, ctrl, rm, bm, bc)
