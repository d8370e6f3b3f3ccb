// Globals of the emulated HIP runtime (hip/hip_runtime.h in this folder) and its fiber switch.
#include "hip/hip_runtime.h"

dim3 threadIdx, blockIdx, blockDim, gridDim;
EmuBlock *emu_block = nullptr;
void (*emu_after_launch)(const void *) = nullptr;

#ifdef EMU_ISA
void (*emu_isa_launch)(const char *, const unsigned *, const void *, size_t) = nullptr;
void (*emu_isa_alloc)(void *, size_t, int) = nullptr;
extern "C" void emu_isa_set_hooks(void (*launch)(const char *, const unsigned *, const void *, size_t),
                                  void (*alloc)(void *, size_t, int)) {
    emu_isa_launch = launch;
    emu_isa_alloc = alloc;
}
#endif

// Fiber switch (x86-64 System V): push the callee-saved registers, save the stack pointer to
// *save_sp, load next_sp, pop the same registers and return into the other fiber.
asm(R"(
    .text
    .globl emu_ctx_switch
    .type emu_ctx_switch, @function
emu_ctx_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
    .size emu_ctx_switch, .-emu_ctx_switch
)");

#ifdef EMU_TRACE
// ------------------------------------------------------------------ access check --
// The trace build compiles with AddressSanitizer's outlined instrumentation renamed to the
// __emu_ hooks below, so every load, store and struct copy of kernel code calls one of them.
// While a GPU thread runs (a fiber is current), the bytes touched must lie in memory that
// thread may touch on the GPU:
//   * a live device allocation (hipMalloc), inside its bounds;
//   * LDS (the emu_lds section);
//   * the thread's own private memory (its fiber stack);
//   * the thread and block indices and grid sizes (registers and dispatch data on the GPU);
//   * for loads only, constant data of the program's read-only segments.
// Host memory (host stacks, heap objects not made by hipMalloc, writable host globals) and
// another thread's private memory are reported and the run aborts, as are bytes that
// AddressSanitizer holds poisoned.  EMU_LOCKSTEP=1 also hands control to the next thread after
// every access, so the threads of a block advance one memory operation at a time instead of
// running from barrier to barrier.
#include <dlfcn.h>
#include <execinfo.h>
#include <link.h>
#include <sanitizer/asan_interface.h>

#include <map>

#define EMU_NOSAN __attribute__((no_sanitize("address")))

namespace {
std::map<uintptr_t, size_t> g_dev;                 // start -> bytes of each live device allocation
std::vector<std::pair<uintptr_t, uintptr_t>> g_ro; // read-only segments of the loaded objects
bool g_ro_ready = false;
int g_lockstep = -1;

EMU_NOSAN int collect_ro(struct dl_phdr_info *info, size_t, void *) {
    for (int k = 0; k < info->dlpi_phnum; ++k) {
        const ElfW(Phdr) &ph = info->dlpi_phdr[k];
        if (ph.p_type == PT_LOAD && !(ph.p_flags & PF_W))
            g_ro.emplace_back(info->dlpi_addr + ph.p_vaddr, info->dlpi_addr + ph.p_vaddr + ph.p_memsz);
    }
    return 0;
}

EMU_NOSAN bool in(uintptr_t a, size_t n, const void *lo, size_t len) {
    const uintptr_t b = (uintptr_t)lo;
    return a >= b && a + n <= b + len;
}

[[noreturn]] __attribute__((noinline)) EMU_NOSAN void report(const char *what, uintptr_t a, size_t n, int store) {
    fprintf(stderr, "emulation: %s: %s of %zu bytes at %p by thread %d of block (%u,%u,%u)\n", what,
            store ? "store" : "load", n, (void *)a, emu_sched.cur, blockIdx.x, blockIdx.y, blockIdx.z);
    auto it = g_dev.upper_bound(a);
    if (it != g_dev.begin()) {
        --it;
        fprintf(stderr, "emulation: nearest device allocation below: %p, %zu bytes (access at +%ld)\n",
                (void *)it->first, it->second, (long)(a - it->first));
    }
    void *bt[16];
    const int k = backtrace(bt, 16);
    backtrace_symbols_fd(bt, k, 2);
    abort();
}

bool g_busy = false;      // the check's own library calls are instrumented too: no recursion

__attribute__((noinline)) EMU_NOSAN void check(uintptr_t a, size_t n, int store) {
    if (!emu_in_block || emu_sched.cur < 0 || n == 0 || g_busy) return;   // host code
    struct Busy {
        Busy() { g_busy = true; }
        ~Busy() { g_busy = false; }
    } busy;
    const EmuFiber &f = emu_sched.fib[emu_sched.cur];
    bool ok = in(a, n, f.stack, EmuSched::kStack);
#ifndef EMU_LDS_REDZONE
    ok = ok || in(a, n, __start_emu_lds, (size_t)(__stop_emu_lds - __start_emu_lds));
#endif
    ok = ok || in(a, n, &threadIdx, sizeof threadIdx) || in(a, n, &blockIdx, sizeof blockIdx) ||
         in(a, n, &blockDim, sizeof blockDim) || in(a, n, &gridDim, sizeof gridDim);
    if (!ok) {
        auto it = g_dev.upper_bound(a);
        if (it != g_dev.begin()) {
            --it;
            if (a >= it->first && a < it->first + it->second) {
                if (a + n > it->first + it->second) report("access runs past a device allocation", a, n, store);
                ok = true;
            }
        }
    }
    if (!ok && !store) {
        if (!g_ro_ready) {
            dl_iterate_phdr(collect_ro, nullptr);
            g_ro_ready = true;
        }
        for (const auto &r : g_ro)
            if (a >= r.first && a + n <= r.second) { ok = true; break; }
    }
    if (!ok) {
        for (int t = 0; t < (int)emu_sched.fib.size(); ++t)
            if (emu_sched.fib[t].stack && in(a, n, emu_sched.fib[t].stack, EmuSched::kStack))
                report("access to another thread's private memory", a, n, store);
        report("access outside device memory", a, n, store);
    }
    if (__asan_region_is_poisoned((void *)a, n)) report("access to poisoned bytes", a, n, store);
    if (g_lockstep < 0) {
        const char *e = getenv("EMU_LOCKSTEP");
        g_lockstep = e && e[0] == '1';
    }
    if (g_lockstep) {
        EmuFiber &cf = emu_sched.fib[emu_sched.cur];
        cf.wait = nullptr;
        g_busy = false;
        emu_to_main(cf, false);
        g_busy = true;
    }
}
}  // namespace

EMU_NOSAN void emu_dev_register(const void *p, size_t n) { g_dev[(uintptr_t)p] = n ? n : 1; }
EMU_NOSAN void emu_dev_unregister(const void *p) { g_dev.erase((uintptr_t)p); }
EMU_NOSAN void emu_check_access(const void *p, size_t n, int store) { check((uintptr_t)p, n, store); }

extern "C" {
#define EMU_HOOK(N)                                                              \
    EMU_NOSAN void __emu_load##N(uintptr_t a) { check(a, N, 0); }               \
    EMU_NOSAN void __emu_store##N(uintptr_t a) { check(a, N, 1); }
EMU_HOOK(1)
EMU_HOOK(2)
EMU_HOOK(4)
EMU_HOOK(8)
EMU_HOOK(16)
EMU_NOSAN void __emu_loadN(uintptr_t a, uintptr_t n) { check(a, n, 0); }
EMU_NOSAN void __emu_storeN(uintptr_t a, uintptr_t n) { check(a, n, 1); }
EMU_NOSAN void *__emu_memcpy(void *d, const void *s, uintptr_t n) {
    check((uintptr_t)s, n, 0);
    check((uintptr_t)d, n, 1);
    return memcpy(d, s, n);
}
EMU_NOSAN void *__emu_memmove(void *d, const void *s, uintptr_t n) {
    check((uintptr_t)s, n, 0);
    check((uintptr_t)d, n, 1);
    return memmove(d, s, n);
}
EMU_NOSAN void *__emu_memset(void *d, int c, uintptr_t n) {
    check((uintptr_t)d, n, 1);
    return memset(d, c, n);
}
}
#endif
