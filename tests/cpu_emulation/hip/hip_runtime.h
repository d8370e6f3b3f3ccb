// CPU execution of the library's HIP kernels, for sanitizer runs in the test suite.
//
// This header stands in for <hip/hip_runtime.h> when fc_kernels.hip is compiled as plain C++
// for the host (tests/cpu_emulation/build.py).  It is never part of the library: the gfx950
// build uses the real HIP runtime.  Semantics modelled:
//   * every GPU thread of a block is a fiber (its own stack, x86-64 context switch) on the host
//     thread; blocks of a grid run one after another;
//   * __syncthreads / __syncthreads_or are block-wide barriers; shuffles and ballots exchange
//     values between the 64 lanes of a wave through a per-wave barrier, so they must be
//     reached by every lane of the wave, as on the GPU; a barrier that cannot complete aborts;
//   * a thread runs until it waits, so the interleaving of threads between barriers is one
//     fixed order (the GPU may pick any), unless EMU_SHUFFLE is set (see below);
//   * atomics are plain host atomics;
//   * __shared__ variables are static; before every block they are overwritten with a poison
//     byte (or, under MemorySanitizer, marked uninitialised), so reading LDS that the block did
//     not write shows up.  With EMU_LDS_REDZONE each __shared__ array is an ordinary static,
//     which AddressSanitizer surrounds with redzones;
//   * device memory is host memory; launches run synchronously.
#pragma once
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define EMU_ASAN_FIBERS 1
#endif
#endif
#ifdef __SANITIZE_ADDRESS__
#define EMU_ASAN_FIBERS 1
#endif
#if EMU_ASAN_FIBERS
#include <sanitizer/asan_interface.h>
#include <sanitizer/common_interface_defs.h>
#endif

#if defined(__has_feature)
#if __has_feature(memory_sanitizer)
#include <sanitizer/msan_interface.h>
#define EMU_MSAN 1
#endif
#endif

// EMU_TRACE (the "trace" build): every load and store of kernel code, struct copies included,
// is checked against the memory a GPU thread may touch (runtime.cpp).  The runtime's own
// functions that run on a thread's fiber are kept out of line and uninstrumented, so only
// kernel code is checked.
#ifdef EMU_TRACE
#define EMU_FN inline __attribute__((noinline, no_sanitize("address")))
#define EMU_FN_ATTR __attribute__((noinline, no_sanitize("address")))
void emu_dev_register(const void *p, size_t n);
void emu_dev_unregister(const void *p);
void emu_check_access(const void *p, size_t n, int store);
#else
#define EMU_FN inline
#define EMU_FN_ATTR
inline void emu_check_access(const void *, size_t, int) {}
#endif

#ifdef EMU_TRACE
#define __global__ __attribute__((noinline))
#else
#define __global__
#endif
#define __device__
#define __align__(n) __attribute__((aligned(n)))
#define __host__
#define __constant__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __restrict__
#ifdef EMU_LDS_REDZONE
#define __shared__ static
#else
#define __shared__ static __attribute__((section("emu_lds")))
#endif

struct int2 { int x, y; };
inline int2 make_int2(int x, int y) { return int2{x, y}; }
struct alignas(16) float4 { float x, y, z, w; };
inline float4 make_float4(float x, float y, float z, float w) { return float4{x, y, z, w}; }

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
typedef void *hipStream_t;
typedef int hipError_t;
#define hipSuccess 0

// ------------------------------------------------------------------ scheduling --
// All GPU threads of a block are fibers on the calling host thread, switched cooperatively at
// barriers (a fiber runs until it waits).  A block in which some live thread can never pass
// the barrier it waits at is reported as a deadlock, the CPU picture of a hung GPU.
struct EmuBarrier {
    int count = 0, arrived = 0;
    unsigned gen = 0;
};
struct EmuBlock {
    EmuBarrier bar;
    std::vector<EmuBarrier> wave_bar;
    std::vector<int64_t> lane_value;
    int or_acc = 0;
};
extern dim3 threadIdx, blockIdx, blockDim, gridDim;
extern EmuBlock *emu_block;
extern void (*emu_after_launch)(const void *kernel);
extern "C" void emu_ctx_switch(void **save_sp, void *next_sp);   // defined in driver.cpp

struct EmuFiber {
    void *sp = nullptr;
    char *stack = nullptr;
    bool done = false;
    EmuBarrier *wait = nullptr;
    unsigned wait_gen = 0;
};
struct EmuSched {
    static constexpr size_t kStack = 256 * 1024;
    static constexpr int kFibers = 1024;
    std::vector<EmuFiber> fib;
    void *main_sp = nullptr;
    const void *main_bottom = nullptr;
    size_t main_size = 0;
    int cur = -1;
    void (*fn)(void *) = nullptr;
    void *ctx = nullptr;
};
inline EmuSched emu_sched;
inline bool emu_in_block = false;               // fibers of a block are running

// EMU_SHUFFLE=<seed>: threads are resumed in a random order on every scheduling pass, and a
// thread may give up its turn at any atomic operation, so that other interleavings between
// barriers are tried as well.
EMU_FN uint64_t emu_shuffle_state() {
    static uint64_t seed = [] {
        const char *e = getenv("EMU_SHUFFLE");
        return e ? (uint64_t)strtoull(e, nullptr, 10) * 2654435761ull + 1 : 0ull;
    }();
    return seed;
}
EMU_FN uint64_t emu_rand() {
    static uint64_t x = emu_shuffle_state();
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    return x;
}

EMU_FN void emu_to_fiber(EmuFiber &f) {
#if EMU_ASAN_FIBERS
    void *fake = nullptr;
    __sanitizer_start_switch_fiber(&fake, f.stack, EmuSched::kStack);
    emu_ctx_switch(&emu_sched.main_sp, f.sp);
    __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#else
    emu_ctx_switch(&emu_sched.main_sp, f.sp);
#endif
}
EMU_FN void emu_to_main(EmuFiber &f, bool dying) {
#if EMU_ASAN_FIBERS
    void *fake = nullptr;
    __sanitizer_start_switch_fiber(dying ? nullptr : &fake, emu_sched.main_bottom, emu_sched.main_size);
    emu_ctx_switch(&f.sp, emu_sched.main_sp);
    __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#else
    (void)dying;
    emu_ctx_switch(&f.sp, emu_sched.main_sp);
#endif
}
[[noreturn]] EMU_FN void emu_fiber_main() {
#if EMU_ASAN_FIBERS
    __sanitizer_finish_switch_fiber(nullptr, &emu_sched.main_bottom, &emu_sched.main_size);
#endif
    EmuFiber &f = emu_sched.fib[emu_sched.cur];
    emu_sched.fn(emu_sched.ctx);
    f.done = true;
    emu_to_main(f, true);
    abort();                                   // a finished fiber is never resumed
}
EMU_FN void emu_maybe_yield() {
    if (!emu_shuffle_state() || emu_sched.cur < 0 || (emu_rand() & 3) != 0) return;
    EmuFiber &f = emu_sched.fib[emu_sched.cur];
    f.wait = nullptr;
    emu_to_main(f, false);
}
EMU_FN void emu_barrier_wait(EmuBarrier &b) {
    const unsigned g = b.gen;
    if (++b.arrived == b.count) {              // the last thread to arrive releases the others
        b.arrived = 0;
        ++b.gen;
        return;
    }
    EmuFiber &f = emu_sched.fib[emu_sched.cur];
    f.wait = &b;
    f.wait_gen = g;
    emu_to_main(f, false);
}
EMU_FN void emu_run_block(unsigned nt, dim3 bid, EmuBlock *blk, void (*fn)(void *), void *ctx) {
    EmuSched &s = emu_sched;
    if (s.fib.empty()) {
        s.fib.resize(EmuSched::kFibers);
        for (auto &f : s.fib) f.stack = (char *)aligned_alloc(64, EmuSched::kStack);
    }
    s.fn = fn;
    s.ctx = ctx;
    for (unsigned t = 0; t < nt; ++t) {
        EmuFiber &f = s.fib[t];
#if EMU_ASAN_FIBERS
        __asan_unpoison_memory_region(f.stack, EmuSched::kStack);
#endif
        uintptr_t top = ((uintptr_t)f.stack + EmuSched::kStack) & ~(uintptr_t)15;
        void **sp = (void **)top;
        *--sp = nullptr;                       // return address of the entry function
        *--sp = (void *)&emu_fiber_main;       // where the first switch returns to
        for (int r = 0; r < 6; ++r) *--sp = nullptr;   // rbp rbx r12 r13 r14 r15
        f.sp = sp;
        f.done = false;
        f.wait = nullptr;
    }
    unsigned left = nt;
    emu_in_block = true;
    std::vector<unsigned> order(nt);
    for (unsigned t = 0; t < nt; ++t) order[t] = t;
    while (left > 0) {
        bool moved = false;
        if (emu_shuffle_state())
            for (unsigned k = nt; k > 1; --k) std::swap(order[k - 1], order[emu_rand() % k]);
        for (unsigned t : order) {
            EmuFiber &f = s.fib[t];
            if (f.done || (f.wait && f.wait->gen == f.wait_gen)) continue;
            f.wait = nullptr;
            s.cur = (int)t;
            threadIdx = dim3(t);
            blockIdx = bid;
            emu_block = blk;
            emu_to_fiber(f);
            moved = true;
            if (f.done) --left;
        }
        s.cur = -1;
        if (!moved) {
            fprintf(stderr, "emulation: deadlock, %u threads wait at a barrier that cannot complete\n", left);
            abort();
        }
    }
    emu_in_block = false;
}

EMU_FN void __syncthreads() { emu_barrier_wait(emu_block->bar); }
// the gfx950 barrier and fence builtins: every emulated barrier orders all memory
#define __builtin_amdgcn_s_barrier() __syncthreads()
#define __builtin_amdgcn_fence(...) ((void)0)
EMU_FN int __syncthreads_or(int x) {
    EmuBlock *b = emu_block;
    emu_barrier_wait(b->bar);
    if (x) b->or_acc = 1;
    emu_barrier_wait(b->bar);
    const int r = b->or_acc;
    emu_barrier_wait(b->bar);
    if (threadIdx.x == 0) b->or_acc = 0;
    emu_barrier_wait(b->bar);
    return r;
}
EMU_FN int __lane_id() { return (int)(threadIdx.x & 63u); }
EMU_FN int emu_wave() { return (int)(threadIdx.x >> 6); }
EMU_FN int64_t emu_read_lane(int64_t v, int src) {
    EmuBlock *b = emu_block;
    EmuBarrier &w = b->wave_bar[emu_wave()];
    b->lane_value[threadIdx.x] = v;
    emu_barrier_wait(w);
    const int64_t got = b->lane_value[(emu_wave() << 6) + src];
    emu_barrier_wait(w);
    return got;
}
EMU_FN int __shfl_up(int v, int d, int = 64) {
    const int l = __lane_id();
    return (int)emu_read_lane(v, l - d < 0 ? l : l - d);
}
EMU_FN int __shfl(int v, int src, int = 64) { return (int)emu_read_lane(v, src & 63); }
// v_mov_b32_dpp with the controls the kernels use: row_shr:1..15 (0x111..0x11F), row_bcast:15
// (0x142) and row_bcast:31 (0x143); a lane of a row or bank left out by the masks, or whose
// source lies outside its row without bound_ctrl, keeps old
EMU_FN int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    const int l = __lane_id(), row = l >> 4, p = l & 15;
    int s = -1;
    if (ctrl >= 0x111 && ctrl <= 0x11F) s = p >= ctrl - 0x110 ? l - (ctrl - 0x110) : -1;
    else if (ctrl == 0x142) s = row >= 1 ? 16 * row - 1 : -1;
    else if (ctrl == 0x143) s = row >= 2 ? 31 : -1;
    else { fprintf(stderr, "emulation: update_dpp control 0x%x not emulated\n", ctrl); abort(); }
    const int v = (int)emu_read_lane(src, s < 0 ? l : s);     // every lane takes part
    if (!((row_mask >> row) & 1) || !((bank_mask >> (p >> 2)) & 1)) return old;
    if (s < 0) return bound_ctrl ? 0 : old;
    return v;
}
EMU_FN int __shfl_xor(int v, int m, int = 64) { return (int)emu_read_lane(v, (__lane_id() ^ m) & 63); }
EMU_FN unsigned long long __ballot(int pred) {
    EmuBlock *b = emu_block;
    EmuBarrier &w = b->wave_bar[emu_wave()];
    b->lane_value[threadIdx.x] = pred ? 1 : 0;
    emu_barrier_wait(w);
    unsigned long long m = 0;
    for (int l = 0; l < 64 && (emu_wave() << 6) + l < (int)b->lane_value.size(); ++l)
        if (b->lane_value[(emu_wave() << 6) + l]) m |= 1ull << l;
    emu_barrier_wait(w);
    return m;
}
inline int __popc(unsigned x) { return __builtin_popcount(x); }
// v_perm_b32: byte i of the result is chosen by byte i of sel from the eight bytes of
// {hi, lo}: 0..7 a byte, 8..11 the sign of bytes 1, 3, 5, 7 replicated, 12 zero, 13.. 0xFF
inline unsigned __builtin_amdgcn_perm(unsigned hi, unsigned lo, unsigned sel) {
    const unsigned long long d = ((unsigned long long)hi << 32) | lo;
    unsigned out = 0;
    for (int i = 0; i < 4; ++i) {
        const unsigned s = (sel >> (8 * i)) & 0xFFu;
        unsigned b;
        if (s < 8) b = (unsigned)(d >> (8 * s)) & 0xFFu;
        else if (s < 12) b = ((d >> (16 * (s - 8) + 15)) & 1u) ? 0xFFu : 0u;
        else b = s == 12 ? 0u : 0xFFu;
        out |= b << (8 * i);
    }
    return out;
}
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline unsigned __float_as_uint(float f) { unsigned u; memcpy(&u, &f, 4); return u; }
inline float __int_as_float(int i) { float f; memcpy(&f, &i, 4); return f; }

template <typename T> EMU_FN T atomicAdd(T *p, T v) {
    emu_check_access(p, sizeof(T), 1);
    emu_maybe_yield();
    return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
EMU_FN float atomicAdd(float *p, float v) {
    emu_check_access(p, sizeof(float), 1);
    emu_maybe_yield();
    float old, nw;
    __atomic_load(p, &old, __ATOMIC_SEQ_CST);
    do { nw = old + v; } while (!__atomic_compare_exchange(p, &old, &nw, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST));
    return old;
}
template <typename T> EMU_FN T atomicMin(T *p, T v) {
    emu_check_access(p, sizeof(T), 1);
    emu_maybe_yield();
    T old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (v < old && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return old;
}
template <typename T> EMU_FN T atomicXor(T *p, T v) {
    emu_check_access(p, sizeof(T), 1);
    emu_maybe_yield();
    return __atomic_fetch_xor(p, v, __ATOMIC_SEQ_CST);
}
template <typename T> EMU_FN T atomicAnd(T *p, T v) {
    emu_check_access(p, sizeof(T), 1);
    emu_maybe_yield();
    return __atomic_fetch_and(p, v, __ATOMIC_SEQ_CST);
}
template <typename T> EMU_FN T atomicOr(T *p, T v) {
    emu_check_access(p, sizeof(T), 1);
    emu_maybe_yield();
    return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST);
}
template <typename T> EMU_FN T atomicMax(T *p, T v) {
    emu_check_access(p, sizeof(T), 1);
    emu_maybe_yield();
    T old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (v > old && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return old;
}
template <typename T> EMU_FN T atomicCAS(T *p, T cmp, T v) {
    emu_check_access(p, sizeof(T), 1);
    emu_maybe_yield();
    __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
    return cmp;
}
#ifdef __clang__
#ifndef __HIP_MEMORY_SCOPE_AGENT
#define __HIP_MEMORY_SCOPE_WORKGROUP 2
#define __HIP_MEMORY_SCOPE_AGENT 3
#endif
#else
#define __HIP_MEMORY_SCOPE_WORKGROUP 0
#define __HIP_MEMORY_SCOPE_AGENT 0
template <typename T> inline T __hip_atomic_load(T *p, int, int) {
    emu_maybe_yield();
    return __atomic_load_n(p, __ATOMIC_SEQ_CST);
}
template <typename T> inline void __hip_atomic_store(T *p, T v, int, int) {
    emu_maybe_yield();
    __atomic_store_n(p, v, __ATOMIC_SEQ_CST);
}
#endif

// host API subset
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated error"; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
enum { hipDeviceAttributeMaxSharedMemoryPerBlock = 1, hipDeviceAttributeMaxThreadsPerBlock = 2 };
inline hipError_t hipDeviceGetAttribute(int *v, int a, int) { *v = a == 1 ? 163840 : 1024; return hipSuccess; }
struct hipFuncAttributes { size_t sharedSizeBytes; int numRegs; int maxThreadsPerBlock; };
inline hipError_t hipFuncGetAttributes(hipFuncAttributes *at, const void *) {
    at->sharedSizeBytes = 0; at->numRegs = 0; at->maxThreadsPerBlock = 1024;
    return hipSuccess;
}
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
#ifdef EMU_ISA
// EMU_ISA (the "isa" build): kernel launches and device allocations are handed to hooks that
// the Python interpreter of the library's gfx950 code object installs (runtime.cpp); the host
// C++ bodies of the kernels are never run.
extern void (*emu_isa_launch)(const char *kernel, const unsigned *dims, const void *args, size_t len);
extern void (*emu_isa_alloc)(void *p, size_t n, int is_free);
#endif
inline hipError_t hipMalloc(void **p, size_t n) {
    *p = malloc(n ? n : 1);
#ifdef EMU_TRACE
    if (*p) emu_dev_register(*p, n);
#endif
#ifdef EMU_ISA
    if (*p && emu_isa_alloc) emu_isa_alloc(*p, n ? n : 1, 0);
#endif
    return *p ? hipSuccess : 2;
}
inline hipError_t hipFree(void *p) {
#ifdef EMU_TRACE
    if (p) emu_dev_unregister(p);
#endif
#ifdef EMU_ISA
    if (p && emu_isa_alloc) emu_isa_alloc(p, 0, 1);
#endif
    free(p);
    return hipSuccess;
}
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { memcpy(d, s, n); return hipSuccess; }
// A file-scope __device__ array is an ordinary host array here.  Its address is registered as
// device memory (once) the first time the library asks for it, like a hipMalloc allocation.
#define HIP_SYMBOL(x) ((const void *)&(x)), sizeof(x)
inline hipError_t hipGetSymbolAddress(void **p, const void *sym, size_t n) {
    static std::vector<const void *> seen;
    bool fresh = true;
    for (const void *q : seen) fresh &= q != sym;
    if (fresh) {
        seen.push_back(sym);
#ifdef EMU_TRACE
        emu_dev_register(sym, n);
#endif
#ifdef EMU_ISA
        if (emu_isa_alloc) emu_isa_alloc((void *)sym, n, 0);
#endif
    }
    *p = (void *)sym;
    return hipSuccess;
}
typedef struct EmuEvent { double t; } *hipEvent_t;
inline double emu_now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = new EmuEvent{0}; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { e->t = emu_now_ms(); return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) { *ms = (float)(b->t - a->t); return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }

#ifndef EMU_LDS_REDZONE
extern "C" char __start_emu_lds[], __stop_emu_lds[];
#endif
inline void emu_poison_lds() {
#ifndef EMU_LDS_REDZONE
    const char *e = getenv("EMU_POISON");
    memset(__start_emu_lds, e ? atoi(e) : 0x4F, (size_t)(__stop_emu_lds - __start_emu_lds));
#ifdef EMU_MSAN
    __msan_poison(__start_emu_lds, (size_t)(__stop_emu_lds - __start_emu_lds));
#endif
#endif
}

#ifdef EMU_ISA
#include <dlfcn.h>
template <typename T> void emu_pack(std::vector<unsigned char> &buf, const T &x) {
    size_t at = (buf.size() + alignof(T) - 1) / alignof(T) * alignof(T);
    buf.resize(at + sizeof(T));
    memcpy(buf.data() + at, &x, sizeof(T));
}
template <typename K, typename... A>
void emu_launch(K kern, dim3 g, dim3 b, A... args) {
    Dl_info info;
    if (!dladdr((void *)kern, &info) || !info.dli_sname) { fprintf(stderr, "emulation: kernel has no symbol\n"); abort(); }
    std::vector<unsigned char> buf;
    (emu_pack(buf, args), ...);
    const unsigned dims[6] = {g.x, g.y, g.z, b.x, b.y, b.z};
    if (!emu_isa_launch) { fprintf(stderr, "emulation: no launch hook\n"); abort(); }
    emu_isa_launch(info.dli_sname, dims, buf.data(), buf.size());
}
#else
template <typename K, typename... A>
void emu_launch(K kern, dim3 g, dim3 b, A... args) {
    gridDim = g;
    blockDim = b;
    const unsigned nt = b.x * b.y * b.z;
    if (nt == 0 || nt > (unsigned)EmuSched::kFibers) { fprintf(stderr, "emulation: bad block size\n"); abort(); }
    auto call = [&]() EMU_FN_ATTR { kern(args...); };
    using Call = decltype(call);
    for (unsigned bz = 0; bz < g.z; ++bz)
        for (unsigned by = 0; by < g.y; ++by)
            for (unsigned bx = 0; bx < g.x; ++bx) {
                emu_poison_lds();
                EmuBlock blk;
                blk.bar.count = (int)nt;
                blk.wave_bar.resize((nt + 63) / 64);
                for (unsigned w = 0; w < blk.wave_bar.size(); ++w) blk.wave_bar[w].count = (int)std::min(64u, nt - 64 * w);
                blk.lane_value.assign(nt, 0);
                emu_run_block(nt, dim3(bx, by, bz), &blk, [](void *c) EMU_FN_ATTR { (*(Call *)c)(); }, &call);
            }
    if (emu_after_launch) emu_after_launch((const void *)kern);
}
#endif
#define hipLaunchKernelGGL(K, G, B, SH, ST, ...) emu_launch(K, G, B, __VA_ARGS__)
